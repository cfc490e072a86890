// incremental.hip -- which stars an incremental call rebuilds.
//
// The star of atom i in the alpha = 0 dual complex (Methods, Steps 1-2) is
// read off the power cell of i clipped to its ball, and that cell is cut only
// by the radical planes of atoms whose balls overlap the ball of i (a plane of
// a disjoint ball misses it).  The star kernel reads nothing else: the
// neighbours are ranked by the distance of their planes, ties by atom id, and
// every side test is certified, so the star is a function of the points of i
// and of its overlapping neighbours alone.  Between two calls it can therefore
// change only if i moved, or an atom that overlaps i at its old or at its new
// point moved.  The area terms (Eq. 1) and gradient blocks (Eq. 2) of i read
// the star and the points of its K-neighbours, a subset of those atoms.
#include <hip/hip_runtime.h>

#include "sasa_internal.h"

namespace sasa {
namespace {

constexpr int MOVED_T = 256;
constexpr int MARK_BLOCKS = 2048;

__device__ inline bool same_point(const double4& a, const double4& b) {
  return __double_as_longlong(a.x) == __double_as_longlong(b.x) &&
         __double_as_longlong(a.y) == __double_as_longlong(b.y) &&
         __double_as_longlong(a.z) == __double_as_longlong(b.z) &&
         __double_as_longlong(a.w) == __double_as_longlong(b.w);
}

// One thread per atom: the weighted point of this call (from the cell-list
// stage) against the previous call's, bit for bit (without `mark` the previous
// points belong to no kept call: every atom counts as moved).  A wavefront
// reserves the queue slots of its moved atoms with one atomic.
__global__ __launch_bounds__(MOVED_T) void k_moved(Bufs b, int mark) {
  const int i = blockIdx.x * MOVED_T + threadIdx.x;
  const int lane = threadIdx.x & 63;
  bool mv = false;
  double4 old = make_double4(0.0, 0.0, 0.0, 0.0);
  if (i < b.n) {
    const double4 cur = b.pos[i];
    if (mark) old = b.prev[i];
    mv = !mark || !same_point(cur, old);
    if (mv) b.prev[i] = cur;
    if (mark) b.dirty[i] = mv ? 1 : 0;
  }
  const unsigned long long m = __ballot(mv);
  if (m == 0ull) return;
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0ull;
  if (lane == leader) base = atomicAdd(&b.ctr[ctr_slot(C_MOVED)], (unsigned long long)__popcll(m));
  base = __shfl(base, leader, 64);
  if (mv && mark) {
    const unsigned long long q = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
    b.mv_id[q] = i;
    b.mv_old[q] = old;
  }
}

// One wavefront per (moved atom, old or new point) c: every atom a whose ball
// overlaps the ball at c is marked.  Candidates are the atoms of the grid
// cells within R_c + h of c along each axis (the cell side h is at least the
// largest radius); lane r takes row r of those cells (cells along x are one
// contiguous range of the cell order) and tests its atoms eight at a time.
// The test is the star kernel's overlap test, widened, so it marks a superset.
__global__ __launch_bounds__(64) void k_mark(Bufs b) {
  const int cnt = (int)b.ctr[ctr_slot(C_MOVED)];
  const int lane = threadIdx.x;
  if (4ll * cnt > (long long)b.n) {  // rebuilding everything is cheaper than marking
    for (int i = blockIdx.x * 64 + lane; i < b.n; i += gridDim.x * 64) b.dirty[i] = 1;
    return;
  }
  const double4 gg = b.mol_geo[0];
  const int4 gd = b.mol_dim[0];
  const double h = gg.w, inv = 1.0 / h;
  const int dim[3] = {gd.x, gd.y, gd.z};
  for (int q = blockIdx.x; q < 2 * cnt; q += gridDim.x) {
    const double4 c = (q & 1) ? b.mv_old[q >> 1] : b.pos[b.mv_id[q >> 1]];
    const double reach = (c.w + h) * (1.0 + 1e-9) + 1e-9;
    const double rel[3] = {c.x - gg.x, c.y - gg.y, c.z - gg.z};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      // clamped in double first: an old point may lie far outside this grid
      lo[a] = (int)fmin(fmax(floor((rel[a] - reach) * inv), 0.0), (double)dim[a]);
      hi[a] = (int)fmin(fmax(floor((rel[a] + reach) * inv), -1.0), (double)(dim[a] - 1));
    }
    if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]) continue;
    const int ny = hi[1] - lo[1] + 1;
    const int nrow = ny * (hi[2] - lo[2] + 1);
    for (int r = lane; r < nrow; r += 64) {
      const int y = lo[1] + r % ny, z = lo[2] + r / ny;
      const int c0 = gd.w + (z * gd.y + y) * gd.x;
      const int e = b.start[c0 + hi[0] + 1];
      for (int k0 = b.start[c0 + lo[0]]; k0 < e; k0 += 8) {
        double4 p[8];
        int id[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          id[u] = -1;
          if (k0 + u < e) p[u] = b.spos[k0 + u], id[u] = b.sorted[k0 + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (id[u] < 0) continue;
          const double dx = p[u].x - c.x, dy = p[u].y - c.y, dz = p[u].z - c.z;
          const double rr = p[u].w + c.w;
          if (dx * dx + dy * dy + dz * dz < rr * rr * (1.0 + 1e-9) + 1e-9) b.dirty[id[u]] = 1;
        }
      }
    }
  }
}

inline unsigned blocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_moved(const Bufs& b, bool mark, hipStream_t s) {
  if (b.n) k_moved<<<blocks(b.n, MOVED_T), MOVED_T, 0, s>>>(b, mark ? 1 : 0);
}

void launch_mark(const Bufs& b, hipStream_t s) {
  if (b.n) k_mark<<<std::min<unsigned>(MARK_BLOCKS, blocks(b.n, 2)), 64, 0, s>>>(b);
}

}  // namespace sasa
