// sasa_internal.h -- device-side data layout shared by the HIP kernels and the
// host side of the library (not part of the public C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sasa {

// Per-atom capacities of the star kernel (local data in LDS).
constexpr int NB_CAP = 160;  // overlapping neighbours of one atom in the fast pass
constexpr int NB_CAP_WIDE = 512;  // ... in the second pass (large probes on dense molecules)
constexpr int V_CAP = 128;   // vertices of the clipped power cell (two slots per lane)
// Per-atom capacities of the kept complex (HBM).
// A cell kept per atom between the frames of a trajectory: up to 64 facets and
// 64 vertices (a simple polytope with 64 vertices has 34 facets); a larger
// cell keeps no vertices and at most 64 facets (the facets only order the
// clipping and the vertices are verified before use, so no hint changes a
// result).
constexpr int FAC_CAP = 64;
constexpr int KN_CAP = 64;    // K-edges at an atom (bit mask of exterior edges is one u64)
constexpr int KT_CAP = 160;   // K-tetrahedra at an atom
constexpr int KTR_CAP = 160;  // exterior K-triangles at an atom
constexpr int ROW = KN_CAP + 1;  // gradient row: one block per K-neighbour + the atom itself

// Counter slots (unsigned long long) on the device.
enum Counter {
  C_VERT = 0,      // vertices in K
  C_EDGE,          // edges in K (counted once, by the lowest atom index)
  C_TRI,           // triangles in K
  C_TET,           // tetrahedra in K
  C_EXT_VERT,      // exterior vertices
  C_EXT_EDGE,      // exterior edges
  C_EXT_TRI,       // exterior triangles
  C_MAX_NB,        // max overlapping neighbours (atomicMax)
  C_MAX_V,         // max polytope vertices (atomicMax)
  C_NEAR_TIE,      // near-degenerate decisions
  C_OVERFLOW,      // atoms past NB_CAP_WIDE / V_CAP / KN_CAP / KT_CAP / KTR_CAP
  C_BAD_INPUT,     // NaN / Inf / radius <= 0
  C_LOST_PAIR,     // K-edge seen from one side only (gather)
  C_RMAX_BITS,     // bits of max R (positive doubles order like integers)
  C_CELLS,         // grid cells used by all molecules
  C_EX_EDGE,       // export cursors
  C_EX_TRI,
  C_EX_TET,
  C_PLANE_TESTS,   // algorithmic work counters of the star kernel
  C_NEW_VERTS,
  C_CANDIDATES,
  C_PLANES_USED,   // planes the clipping loop visited (sum and max over atoms)
  C_MAX_PLANES,
  C_PLANES_GT64,   // atoms whose clipping visited more than 64 planes
  C_WIDE,          // atoms queued for the star kernel's wide pass
  C_REUSED,        // atoms whose previous-frame cell was verified and kept
  C_MOVED,         // incremental calls: atoms moved since the previous call (queue cursor)
  C_SKIPPED,       // ... atoms whose star was kept
  C_COUNT
};
// Counters sit 128 bytes apart, so that atomics on different counters never
// queue on one L2 line; counter k is ctr[ctr_slot(k)].
constexpr int CTR_STRIDE = 16;
constexpr int ctr_slot(int k) { return k * CTR_STRIDE; }
constexpr size_t CTR_BYTES = (size_t)C_COUNT * CTR_STRIDE * sizeof(unsigned long long);

// Per-atom record of the star kernel (plain stores, one per atom), summed into
// the counters by k_stats: a wavefront never issues a device-scope atomic on
// the shared counters, which would serialise every wavefront on one L2 line.
enum Stat {
  S_NN = 0,   // overlapping neighbours (max)
  S_VMAX,     // largest polytope while clipping (max)
  S_CAND,     // neighbour candidates read
  S_TESTS,    // (vertex, plane) side tests
  S_NEWV,     // vertices created
  S_TIES,     // near-degenerate decisions
  S_BAD,      // capacity exceeded or broken star (bit 0); previous-frame cell kept (bit 1);
              // star kept from the previous call (bit 2)
  S_VERT,     // atom is a vertex of K
  S_EXTV,     // ... an exterior one
  S_TET,      // owned simplices (lowest index)
  S_TRI,
  S_EXTTRI,
  S_EDGE,
  S_EXTEDGE,
  S_KSTOP,    // planes the clipping loop visited
  S_COUNT
};
constexpr int STAT_STRIDE = 16;  // ints per atom record

// Vertex flags.
constexpr uint8_t VF_IN = 1, VF_EXT = 2;

struct Bufs {
  int n = 0;
  int nmol = 0;
  int cell_cap = 0;      // grid cells available to all molecules together
  // inputs staged or borrowed
  const double* xyz = nullptr;
  const double* radii = nullptr;
  double probe = 0;
  const int64_t* offsets = nullptr;  // nmol + 1 (device)
  // cell list: one dense grid per molecule, cells numbered x fastest, so the
  // atoms of a run of cells along x are one contiguous range of `sorted`
  double4* pos = nullptr;    // x, y, z, R (original order)
  int* mol = nullptr;        // molecule id (original order)
  int* cellid = nullptr;     // grid cell of each atom (original order)
  unsigned long long* mol_box = nullptr;  // per molecule: ordered bits of min x, y, z and -max x, y, z
  double4* mol_geo = nullptr;  // per molecule: grid origin x, y, z and cell side
  int4* mol_dim = nullptr;     // per molecule: cells along x, y, z and the first cell's index
  int* cnt = nullptr;        // atoms per cell (cell_cap)
  int* start = nullptr;      // exclusive scan of cnt (cell_cap + 1)
  int* scan_tmp = nullptr;   // block sums of the scan
  int* sorted = nullptr;     // atom ids grouped by cell
  double4* spos = nullptr;   // positions in cell order (coalesced neighbour loads)
  int2* smc = nullptr;       // molecule id and cell in cell order
  // kept complex
  uint8_t* vflag = nullptr;
  int* kn_cnt = nullptr;
  int* knbr = nullptr;                 // n * KN_CAP, ascending global ids
  unsigned long long* kn_ext = nullptr;  // exterior-edge mask
  int* kt_cnt = nullptr;
  unsigned* ktet = nullptr;            // n * KT_CAP, 3 x 8-bit K-neighbour slots
  int* ktr_cnt = nullptr;
  unsigned* ktri = nullptr;            // n * KTR_CAP, 2 x 8-bit slots + n_tet << 16
  int* stat = nullptr;       // n * STAT_STRIDE per-atom records of the star kernel
  int* wide = nullptr;       // cell-ordered positions queued for the star's wide pass (n)
  // each atom's cell in the previous call of a trajectory (null when the
  // context does not keep them): its facet neighbours (ids, FAC_CAP per atom),
  // its vertices as triples of facet-list positions (FAC_CAP per atom), and
  // the two counts (facets | vertices << 8)
  int* fac = nullptr;
  unsigned* vtx = nullptr;
  int* hint_n = nullptr;
  // incremental calls (null otherwise): each atom's weighted point in the
  // previous call (x, y, z, R), the moved atoms (ids and previous points, in
  // queue order), the atoms whose star is rebuilt (1) or kept (0; read by the
  // star and terms kernels only when set), and each atom's last area
  double4* prev = nullptr;
  int* mv_id = nullptr;
  double4* mv_old = nullptr;
  uint8_t* dirty = nullptr;
  double* area_keep = nullptr;
  // results
  double* area = nullptr;
  double* rows = nullptr;    // n * ROW * 3
  unsigned long long* ctr = nullptr;
  // pinned host words that the terms kernel of a compute fills from the
  // counters: [0] input errors, [1] capacity failures, [2] = 1 (written)
  unsigned long long* status = nullptr;
  // export (optional)
  int export_on = 0;
  int64_t ex_cap_e = 0, ex_cap_t = 0, ex_cap_q = 0;
  int* ex_edges = nullptr;
  int* ex_tris = nullptr;
  uint8_t* ex_ntet = nullptr;
  int* ex_tets = nullptr;
};

// Launchers (kernels.hip).
void launch_prep(const Bufs& b, hipStream_t s);
void launch_grid(const Bufs& b, hipStream_t s);
void launch_count(const Bufs& b, hipStream_t s);
void launch_scan(const Bufs& b, hipStream_t s);
void launch_scatter(const Bufs& b, hipStream_t s);
void launch_cells_one(const Bufs& b, hipStream_t s);
void launch_star(const Bufs& b, hipStream_t s);        // fast pass over all atoms
void launch_star_wide(const Bufs& b, hipStream_t s);   // atoms the fast pass queued
// Largest single molecule whose cell list is built by one block.
constexpr int64_t ONE_BLOCK_MAX_ATOMS = 8192;
void launch_stats(const Bufs& b, hipStream_t s);
// Incremental calls (incremental.hip), after the cell list: atoms whose point
// changed since the previous call (b.prev updated; with `mark`, dirty[i] set
// to whether atom i moved and the moved atoms queued), then every atom that
// overlaps a queued atom at its old or new point marked too (all atoms when
// more than a quarter moved).
void launch_moved(const Bufs& b, bool mark, hipStream_t s);
void launch_mark(const Bufs& b, hipStream_t s);
void launch_terms(const Bufs& b, int precision, int with_grad, hipStream_t s);
// out[m] (+)= scale sum_i u_i dA_i/dp_m (accumulate: added to out, else stored)
void launch_gather(const Bufs& b, const double* u, double* out, double scale, hipStream_t s, int accumulate = 0);
// The crease part of the integrated mean curvature per atom into b.area, and
// (with_grad) its gradient blocks into b.rows; FP64.
void launch_terms_crease(const Bufs& b, int with_grad, hipStream_t s);
// out[i] = u[i] / R_i (u may be NULL: 1 / R_i).
void launch_recip_radius(const Bufs& b, const double* u, double* out, hipStream_t s);
// Per-atom cell volumes and the molecular-volume gradient (needs b.area in FP64),
// and with curv the per-atom integrated mean curvature of the surface.
void launch_volume(const Bufs& b, double* vol, double* grad, hipStream_t s, double* curv = nullptr);
// out[m] = sum_i u_i dV_i/dp_m (faces' areas and first moments).
void launch_volume_vjp(const Bufs& b, const double* u, double* out, hipStream_t s);

// Unique triangles of the kept complex by sorting the faces of its
// tetrahedra (the paper's extraction, for comparison with the stars).
// nfaces = 4 x owned K-tetrahedra, cap_free >= owned tetrahedron-free
// K-triangles; cursors (2) and nruns start at 0; tris / ntet hold
// nfaces + cap_free entries.
struct SortedFaces {
  unsigned long long* faces = nullptr;      // nfaces keys (emitted)
  unsigned long long* sorted = nullptr;     // nfaces keys (sorted)
  unsigned long long* uniq = nullptr;       // nfaces (runs)
  unsigned* counts = nullptr;               // nfaces (run lengths = n_t)
  unsigned* nruns = nullptr;                // 1
  unsigned long long* free_tris = nullptr;  // cap_free keys
  unsigned long long* cursors = nullptr;    // 2
  int* tris = nullptr;                      // 3 (nfaces + cap_free)
  uint8_t* ntet = nullptr;                  // nfaces + cap_free
  void* temp = nullptr;
  size_t temp_bytes = 0;
  long long nfaces = 0, cap_free = 0;
};
size_t sorted_faces_temp_bytes(int64_t nfaces);
hipError_t launch_sorted_faces(const Bufs& b, const SortedFaces& w, hipStream_t s);

// Buffers of the sorted extraction of unique edges and vertices (grown on demand).
struct SortedEV {
  unsigned long long* keys = nullptr;   // candidates: edge (a << 21 | b) or vertex id
  unsigned* vals = nullptr;             // bit 0: on a triangle (edge) / an edge (vertex); bit 1: an exterior one
  unsigned long long* skeys = nullptr;  // sorted
  unsigned* svals = nullptr;
  unsigned long long* uniq = nullptr;  // unique keys
  unsigned* agg = nullptr;             // OR of the values of each key
  unsigned* nuniq = nullptr;           // 1
  unsigned long long* cursor = nullptr;  // 1
  int* out_ids = nullptr;                // 2 per edge / 1 per vertex
  uint8_t* out_ext = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  long long cap = -1;  // candidate capacity of every array above
};
size_t sorted_ev_temp_bytes(int64_t n);
// Unique edges: candidates from the m unique triangles (3 each) and from the
// stars (each K-edge once, by its lower atom), sorted and reduced.
hipError_t launch_sorted_edges(const Bufs& b, const int* tris, const uint8_t* ntet, long long m, long long ncand,
                               const SortedEV& w, hipStream_t s);
// Unique vertices: candidates from the ue unique edges (2 each) and from the
// stars (every atom in K), sorted and reduced.
hipError_t launch_sorted_vertices(const Bufs& b, const unsigned long long* edges, const unsigned* eagg, long long ue,
                                  long long ncand, const SortedEV& w, hipStream_t s);
// Unique keys and their OR-ed values to ids and exterior flags (edges: 2 ids).
void launch_ev_unpack(const SortedEV& w, long long count, int ids_per_key, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);
int scan_blocks(unsigned hb);
// Grid cells a batch of n atoms may use: a molecule of m > 0 atoms gets at most
// 8 m + 8 cells (empty molecules none), so all molecules together at most 16 n.
inline int64_t cell_capacity(int64_t n) { return 16 * n + 64; }

}  // namespace sasa
