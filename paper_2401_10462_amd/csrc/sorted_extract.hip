// sorted_extract.hip -- the paper's GPU extraction of unique triangles, edges
// and vertices, as an A/B against the per-atom classification of the star
// kernel.
//
// The paper (GPU section, extraction of exterior simplices) starts from the
// global list of tetrahedra, lists all four faces of every tetrahedron, sorts
// the list lexicographically so that equal triangles are adjacent, and counts
// each run: a triangle belongs to one or two tetrahedra, and it is exterior
// when it belongs to at most one.  Here the tetrahedra are those of the kept
// complex, each listed once by its lowest atom (the stars hold every
// tetrahedron four times); a triangle is one 63-bit key (three ascending atom
// ids of 21 bits), sorted by rocPRIM's radix sort and counted by its run-length
// encoding.  K-triangles on no K-tetrahedron are not faces of anything, so
// they come from the stars directly (owned by their lowest atom).  The star
// kernel decides the same n_t locally, as the number of the cell edge's two
// vertices inside the ball.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce_by_key.hpp>
#include <rocprim/device/device_run_length_encode.hpp>

#include "sasa_internal.h"

namespace sasa {
namespace {

__device__ inline unsigned long long tri_key(unsigned a, unsigned b, unsigned c) {
  unsigned t;
  if (a > b) t = a, a = b, b = t;
  if (b > c) t = b, b = c, c = t;
  if (a > b) t = a, a = b, b = t;
  return ((unsigned long long)a << 42) | ((unsigned long long)b << 21) | (unsigned long long)c;  // lexicographic
}

// Wave-aggregated slot reservation: one atomic per wavefront.
__device__ inline unsigned long long reserve(unsigned long long* cursor, int count) {
  int pre = count;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(pre, off, 64);
    if ((int)(threadIdx.x & 63) >= off) pre += t;
  }
  const int total = __shfl(pre, 63, 64);
  unsigned long long base = 0;
  if ((threadIdx.x & 63) == 63 && total > 0) base = atomicAdd(cursor, (unsigned long long)total);
  base = __shfl(base, 63, 64);
  return base + (unsigned long long)(pre - count);
}

// One thread per atom: the four faces of each K-tetrahedron it owns, and the
// tetrahedron-free exterior K-triangles it owns.
__global__ __launch_bounds__(64) void k_emit_faces(Bufs b, unsigned long long* faces, unsigned long long* free_tris,
                                                   unsigned long long* cursors, long long cap_faces,
                                                   long long cap_free) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  int nt = 0, nr = 0;
  const int* nb = nullptr;
  if (i < b.n && (b.vflag[i] & VF_IN)) {
    nt = min(b.kt_cnt[i], KT_CAP);
    nr = min(b.ktr_cnt[i], KTR_CAP);
    nb = b.knbr + (size_t)i * KN_CAP;
  }
  int own_t = 0, own_r = 0;
  for (int t = 0; t < nt; ++t) {
    const unsigned w = b.ktet[(size_t)i * KT_CAP + t];
    const int a = nb[w & 255u], c2 = nb[(w >> 8) & 255u], d = nb[(w >> 16) & 255u];
    own_t += i < a && i < c2 && i < d;
  }
  for (int t = 0; t < nr; ++t) {
    const unsigned w = b.ktri[(size_t)i * KTR_CAP + t];
    const int a = nb[w & 255u], c2 = nb[(w >> 8) & 255u];
    own_r += (w >> 16) == 0u && i < a && i < c2;
  }
  unsigned long long pf = reserve(&cursors[0], 4 * own_t);
  unsigned long long pr = reserve(&cursors[1], own_r);
  for (int t = 0; t < nt; ++t) {
    const unsigned w = b.ktet[(size_t)i * KT_CAP + t];
    const unsigned a = (unsigned)nb[w & 255u], c2 = (unsigned)nb[(w >> 8) & 255u], d = (unsigned)nb[(w >> 16) & 255u];
    if (!((unsigned)i < a && (unsigned)i < c2 && (unsigned)i < d)) continue;
    const unsigned long long k4[4] = {tri_key(i, a, c2), tri_key(i, a, d), tri_key(i, c2, d), tri_key(a, c2, d)};
    for (int f = 0; f < 4; ++f, ++pf)
      if ((long long)pf < cap_faces) faces[pf] = k4[f];
  }
  for (int t = 0; t < nr; ++t) {
    const unsigned w = b.ktri[(size_t)i * KTR_CAP + t];
    const unsigned a = (unsigned)nb[w & 255u], c2 = (unsigned)nb[(w >> 8) & 255u];
    if ((w >> 16) != 0u || !((unsigned)i < a && (unsigned)i < c2)) continue;
    if ((long long)pr < cap_free) free_tris[pr] = tri_key(i, a, c2);
    ++pr;
  }
}

// Runs of the sorted faces (n_t = run length), then the tetrahedron-free
// triangles (n_t = 0): three atom ids and n_t per triangle.
__global__ void k_unpack(const unsigned long long* uniq, const unsigned* counts, const unsigned* nruns,
                         const unsigned long long* free_tris, const unsigned long long* cursors, long long cap_free,
                         int* tris, uint8_t* ntet) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nu = (long long)*nruns;
  const long long nf = (long long)cursors[1] < cap_free ? (long long)cursors[1] : cap_free;
  if (q >= nu + nf) return;
  const unsigned long long k = q < nu ? uniq[q] : free_tris[q - nu];
  tris[3 * q] = (int)(k >> 42);
  tris[3 * q + 1] = (int)((k >> 21) & 0x1fffffull);
  tris[3 * q + 2] = (int)(k & 0x1fffffull);
  ntet[q] = q < nu ? (uint8_t)counts[q] : (uint8_t)0;
}

// Edges and vertices, the same way one dimension down (GPU section, extraction
// of exterior simplices: unique simplices by lexicographic sorts of the
// candidates, then classification).  Every unique triangle lists its three
// edges with its exterior flag (n_t <= 1); every K-edge is also listed once
// from the star of its lower atom with no flag, so that an edge on no triangle
// still appears.  Sorting by the edge and OR-ing the flags of each run gives,
// per unique edge, whether it lies on a triangle and on an exterior one; it is
// exterior iff on an exterior triangle or on none (the classification rule
// read from the paper's text).  Vertices: every unique edge lists its two atoms
// with its exterior flag, every atom in K is listed once with none, and a
// vertex is exterior iff it has an exterior edge or no edge.
constexpr unsigned EV_ON = 1u, EV_EXT = 2u;

__device__ inline unsigned long long edge_key(unsigned a, unsigned b) {
  return a < b ? ((unsigned long long)a << 21) | b : ((unsigned long long)b << 21) | a;
}

__global__ void k_edges_from_tris(const int* tris, const uint8_t* ntet, long long m, unsigned long long* keys,
                                  unsigned* vals) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const unsigned a = (unsigned)tris[3 * q], b = (unsigned)tris[3 * q + 1], c = (unsigned)tris[3 * q + 2];
  const unsigned v = EV_ON | (ntet[q] <= 1 ? EV_EXT : 0u);
  keys[3 * q] = edge_key(a, b), keys[3 * q + 1] = edge_key(a, c), keys[3 * q + 2] = edge_key(b, c);
  vals[3 * q] = vals[3 * q + 1] = vals[3 * q + 2] = v;
}

// One thread per atom: its K-edges to higher atoms, after the triangles' 3m
// candidates (slots by wave-aggregated reservation; the sort makes the order
// immaterial).
__global__ __launch_bounds__(64) void k_edges_from_stars(Bufs b, long long base, long long cap,
                                                         unsigned long long* cursor, unsigned long long* keys,
                                                         unsigned* vals) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  int nk = 0, own = 0;
  const int* nb = nullptr;
  if (i < b.n && (b.vflag[i] & VF_IN)) {
    nk = min(b.kn_cnt[i], KN_CAP);
    nb = b.knbr + (size_t)i * KN_CAP;
    for (int k = 0; k < nk; ++k) own += i < nb[k];
  }
  unsigned long long p = base + reserve(cursor, own);
  for (int k = 0; k < nk; ++k) {
    if (!(i < nb[k])) continue;
    if ((long long)p < cap) keys[p] = edge_key((unsigned)i, (unsigned)nb[k]), vals[p] = 0u;
    ++p;
  }
}

__global__ void k_vertices_from_edges(const unsigned long long* edges, const unsigned* eagg, const unsigned* nue,
                                      unsigned long long* keys, unsigned* vals) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)*nue) return;
  const unsigned long long e = edges[q];
  const unsigned f = eagg[q];
  const bool ext = !(f & EV_ON) || (f & EV_EXT);
  const unsigned v = EV_ON | (ext ? EV_EXT : 0u);
  keys[2 * q] = e >> 21, keys[2 * q + 1] = e & 0x1fffffull;
  vals[2 * q] = vals[2 * q + 1] = v;
}

__global__ __launch_bounds__(64) void k_vertices_from_stars(Bufs b, const unsigned* nue, long long cap,
                                                            unsigned long long* cursor, unsigned long long* keys,
                                                            unsigned* vals) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int own = (i < b.n && (b.vflag[i] & VF_IN)) ? 1 : 0;
  const unsigned long long p = 2ull * *nue + reserve(cursor, own);
  if (own && (long long)p < cap) keys[p] = (unsigned long long)i, vals[p] = 0u;
}

// Unique keys to ids and exterior flags.
__global__ void k_ev_unpack(const unsigned long long* uniq, const unsigned* agg, long long count, int ids_per_key,
                            int* ids, uint8_t* ext) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const unsigned long long k = uniq[q];
  if (ids_per_key == 2) ids[2 * q] = (int)(k >> 21), ids[2 * q + 1] = (int)(k & 0x1fffffull);
  else ids[q] = (int)k;
  const unsigned f = agg[q];
  ext[q] = (!(f & EV_ON) || (f & EV_EXT)) ? 1 : 0;
}

struct BitOr {
  __host__ __device__ unsigned operator()(unsigned a, unsigned b) const { return a | b; }
};

hipError_t sort_and_reduce(const SortedEV& w, long long ncand, unsigned end_bit, hipStream_t s) {
  if (ncand <= 0) return hipSuccess;
  size_t bytes = w.temp_bytes;
  hipError_t e = rocprim::radix_sort_pairs(w.temp, bytes, w.keys, w.skeys, w.vals, w.svals, (size_t)ncand, 0u,
                                           end_bit, s);
  if (e != hipSuccess) return e;
  bytes = w.temp_bytes;
  return rocprim::reduce_by_key(w.temp, bytes, w.skeys, w.svals, (size_t)ncand, w.uniq, w.agg, w.nuniq, BitOr(),
                                rocprim::equal_to<unsigned long long>(), s);
}

}  // namespace

size_t sorted_ev_temp_bytes(int64_t n) {
  size_t a = 0, c = 0;
  const unsigned long long* k = nullptr;
  unsigned long long* o = nullptr;
  const unsigned* v = nullptr;
  unsigned* u = nullptr;
  size_t a2 = 0;
  (void)rocprim::radix_sort_pairs(nullptr, a, k, o, v, u, (size_t)n, 0u, 42u);
  (void)rocprim::radix_sort_pairs(nullptr, a2, k, o, v, u, (size_t)n, 0u, 21u);
  (void)rocprim::reduce_by_key(nullptr, c, k, v, (size_t)n, o, u, u, BitOr(), rocprim::equal_to<unsigned long long>());
  return std::max(std::max(a, a2), c);
}

hipError_t launch_sorted_edges(const Bufs& b, const int* tris, const uint8_t* ntet, long long m, long long ncand,
                               const SortedEV& w, hipStream_t s) {
  if (m > 0) k_edges_from_tris<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(tris, ntet, m, w.keys, w.vals);
  if (b.n) k_edges_from_stars<<<(b.n + 63) / 64, 64, 0, s>>>(b, 3 * m, w.cap, w.cursor, w.keys, w.vals);
  hipError_t e = sort_and_reduce(w, ncand, 42u, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_sorted_vertices(const Bufs& b, const unsigned long long* edges, const unsigned* eagg, long long ue,
                                  long long ncand, const SortedEV& w, hipStream_t s) {
  if (ue > 0) k_vertices_from_edges<<<(unsigned)((ue + 255) / 256), 256, 0, s>>>(edges, eagg, w.nuniq, w.keys, w.vals);
  if (b.n) k_vertices_from_stars<<<(b.n + 63) / 64, 64, 0, s>>>(b, w.nuniq, w.cap, w.cursor, w.keys, w.vals);
  hipError_t e = sort_and_reduce(w, ncand, 21u, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

void launch_ev_unpack(const SortedEV& w, long long count, int ids_per_key, hipStream_t s) {
  if (count > 0)
    k_ev_unpack<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(w.uniq, w.agg, count, ids_per_key, w.out_ids,
                                                                w.out_ext);
}

size_t sorted_faces_temp_bytes(int64_t nfaces) {
  size_t a = 0, c = 0;
  const unsigned long long* k = nullptr;
  unsigned long long* o = nullptr;
  unsigned* u = nullptr;
  (void)rocprim::radix_sort_keys(nullptr, a, k, o, (unsigned)nfaces, 0, 63);
  (void)rocprim::run_length_encode(nullptr, c, k, (unsigned)nfaces, o, u, u);
  return a > c ? a : c;
}

hipError_t launch_sorted_faces(const Bufs& b, const SortedFaces& w, hipStream_t s) {
  if (b.n) k_emit_faces<<<(b.n + 63) / 64, 64, 0, s>>>(b, w.faces, w.free_tris, w.cursors, w.nfaces, w.cap_free);
  if (w.nfaces > 0) {
    size_t bytes = w.temp_bytes;
    hipError_t e = rocprim::radix_sort_keys(w.temp, bytes, w.faces, w.sorted, (unsigned)w.nfaces, 0, 63, s);
    if (e != hipSuccess) return e;
    bytes = w.temp_bytes;
    e = rocprim::run_length_encode(w.temp, bytes, w.sorted, (unsigned)w.nfaces, w.uniq, w.counts, w.nruns, s);
    if (e != hipSuccess) return e;
  }
  const long long total = w.nfaces + w.cap_free;
  if (total > 0)
    k_unpack<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(w.uniq, w.counts, w.nruns, w.free_tris, w.cursors,
                                                             w.cap_free, w.tris, w.ntet);
  return hipGetLastError();
}

}  // namespace sasa
