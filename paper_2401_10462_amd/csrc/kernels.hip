// kernels.hip -- HIP kernels (gfx950, wave64) of the exact analytic SASA path.
//
// Pipeline for one batch of molecules (each molecule is one segment of atoms):
//   k_cells_one one molecule of up to 8,192 atoms: the whole cell-list stage
//               below in one block (weights, box, grid, counts, scan, scatter)
//   k_prep      weights R_i = r_i + probe, molecule ids, input checks, R_max and
//               each molecule's bounding box
//   k_grid      one dense cell grid per molecule (cell side >= R_max)
//   k_count     cell of every atom, atoms per cell
//   k_scan*     exclusive scan of the cell counts
//   k_scatter   atoms grouped by cell; positions copied in that order so that
//               neighbour loads are coalesced
//   k_star      one wavefront per atom: its power (Laguerre) cell clipped by the
//               radical planes of its overlapping neighbours, restricted to its
//               ball; yields the atom's star in the dual complex K, the
//               exterior classification, and a per-atom statistics record
//               (a trajectory's calls start from the previous frame's cell)
//   k_star_wide the atoms whose cell outgrew the fast pass, with full capacities
//   k_stats     the statistics records folded into the counters (on demand:
//               diagnostics and complex counts, not every call)
//   k_terms     one wavefront per exterior atom: Eq. 1 area from the star and,
//               on request, the gradient blocks dA_i/dp_m of Eq. 2
//   k_gather    16 lanes per atom: segmented sum over its K-neighbours of
//               u_i dA_i/dp_m (deterministic order)
#include <hip/hip_runtime.h>

#include "exact_side.h"
#include "sasa_internal.h"

namespace sasa {

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline int prefix_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ inline double rmax_of(const unsigned long long* ctr) {
  return __longlong_as_double((long long)ctr[ctr_slot(C_RMAX_BITS)]);
}

// Order-preserving map of doubles to unsigned integers (for atomicMax on
// coordinates); the box of a molecule keeps max(~ord(x)) for its minimum and
// max(ord(x)) for its maximum, so a zero-filled box is the empty box.
__device__ inline unsigned long long ord_bits(double d) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double from_ord(unsigned long long u) {
  return __longlong_as_double((long long)((u >> 63) ? (u & 0x7fffffffffffffffull) : ~u));
}

__device__ inline double wave_min_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_max_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// ------------------------------------------------------------------ prep
constexpr int PREP_T = 1024;

// molecule of atom a: largest k with offsets[k] <= a
__device__ inline int mol_of(const Bufs& b, int a) {
  int lo = 0, hi = b.nmol - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.offsets[mid] <= a) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Weights R_i = r_i + probe, molecule ids, R_max and each molecule's bounding
// box, kept by atomicMax on the shared counters and boxes.
__global__ __launch_bounds__(PREP_T) void k_prep(Bufs b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool live = i < b.n;
  double x = 0.0, y = 0.0, z = 0.0, R = 0.0;
  int m = -1;
  if (live) {
    x = b.xyz[3 * i], y = b.xyz[3 * i + 1], z = b.xyz[3 * i + 2];
    double r = b.radii[i];
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(r) && r > 0.0;
    if (!ok) {
      atomicAdd(&b.ctr[ctr_slot(C_BAD_INPUT)], 1ull);
      x = y = z = 0.0;
      r = 1.0;
    }
    R = r + b.probe;
    b.pos[i] = make_double4(x, y, z, R);
    m = mol_of(b, i);
    b.mol[i] = m;
  }
  // a block inside one molecule (the common case) merges its wavefronts in
  // LDS and issues one set of atomics; otherwise each wavefront issues one set
  // per molecule it holds
  __shared__ double part[PREP_T / 64][7];
  const int first = blockIdx.x * PREP_T, last = min(b.n - 1, first + PREP_T - 1);
  const bool one_mol = b.nmol == 1 || mol_of(b, first) == mol_of(b, last);
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  if (one_mol) {
    const double v[7] = {wave_min_d(live ? x : inf), wave_min_d(live ? y : inf), wave_min_d(live ? z : inf),
                         wave_max_d(live ? x : -inf), wave_max_d(live ? y : -inf), wave_max_d(live ? z : -inf),
                         wave_max_d(R)};
    if (lane == 0)
      for (int q = 0; q < 7; ++q) part[threadIdx.x >> 6][q] = v[q];
    __syncthreads();
    if (threadIdx.x < 7) {
      const int q = threadIdx.x;
      double r = part[0][q];
      for (int w = 1; w < PREP_T / 64; ++w) r = q < 3 ? fmin(r, part[w][q]) : fmax(r, part[w][q]);
      if (q == 6) {
        if (r > 0.0) atomicMax(&b.ctr[ctr_slot(C_RMAX_BITS)], (unsigned long long)__double_as_longlong(r));
      } else {
        unsigned long long* box = b.mol_box + 6 * (size_t)mol_of(b, first);
        atomicMax(&box[q], q < 3 ? ~ord_bits(r) : ord_bits(r));
      }
    }
    return;
  }
  const double rmax = wave_max_d(R);
  if (lane == 0 && rmax > 0.0) atomicMax(&b.ctr[ctr_slot(C_RMAX_BITS)], (unsigned long long)__double_as_longlong(rmax));
  unsigned long long pend = __ballot(live);
  while (pend) {
    const int leader = (int)__builtin_ctzll(pend);
    const int mm = __shfl(m, leader, 64);
    const bool mine = live && m == mm;
    const unsigned long long grp = __ballot(mine);
    const double x0 = wave_min_d(mine ? x : inf), y0 = wave_min_d(mine ? y : inf), z0 = wave_min_d(mine ? z : inf);
    const double x1 = wave_max_d(mine ? x : -inf), y1 = wave_max_d(mine ? y : -inf), z1 = wave_max_d(mine ? z : -inf);
    if (lane == leader) {
      unsigned long long* box = b.mol_box + 6 * (size_t)mm;
      atomicMax(&box[0], ~ord_bits(x0));
      atomicMax(&box[1], ~ord_bits(y0));
      atomicMax(&box[2], ~ord_bits(z0));
      atomicMax(&box[3], ord_bits(x1));
      atomicMax(&box[4], ord_bits(y1));
      atomicMax(&box[5], ord_bits(z1));
    }
    pend &= ~grp;
  }
}

// Grid over the box [lo, hi] of a molecule of na atoms: cell side R_max,
// enlarged by factors of 1.25 until the grid has at most 8 na + 8 cells.
__device__ inline int grid_dims(double lx, double ly, double lz, double hx, double hy, double hz, int64_t na,
                                double rmax, double4& geo, int& nx, int& ny, int& nz) {
  const double ex = hx - lx, ey = hy - ly, ez = hz - lz;
  const double cap = 8.0 * (double)na + 8.0;
  double s = rmax;
  double fx, fy, fz;
  for (;;) {
    fx = floor(ex / s) + 1.0, fy = floor(ey / s) + 1.0, fz = floor(ez / s) + 1.0;
    if (fx * fy * fz <= cap) break;
    s *= 1.25;
  }
  nx = (int)fx, ny = (int)fy, nz = (int)fz;
  geo = make_double4(lx, ly, lz, s);
  return nx * ny * nz;
}

// One dense grid per molecule over its bounding box.  The cell side is R_max
// (so every overlapping pair lies within two cells along each axis), enlarged
// for sparse, elongated molecules until the grid has at most 8 n_m + 8 cells;
// the cells of all molecules are numbered consecutively.
__global__ __launch_bounds__(1024) void k_grid(Bufs b) {
  __shared__ int lds[1024];
  const double rmax = rmax_of(b.ctr);
  int carry = 0;
  for (int k0 = 0; k0 < b.nmol; k0 += 1024) {
    const int k = k0 + (int)threadIdx.x;
    int cells = 0;
    double4 geo = make_double4(0.0, 0.0, 0.0, rmax);
    int nx = 0, ny = 0, nz = 0;
    if (k < b.nmol) {
      const int64_t na = b.offsets[k + 1] - b.offsets[k];
      if (na > 0) {
        const unsigned long long* box = b.mol_box + 6 * (size_t)k;
        const double lx = from_ord(~box[0]), ly = from_ord(~box[1]), lz = from_ord(~box[2]);
        cells = grid_dims(lx, ly, lz, from_ord(box[3]), from_ord(box[4]), from_ord(box[5]), na, rmax, geo, nx, ny,
                          nz);
      }
    }
    // exclusive scan of the cell counts over this chunk of molecules
    lds[threadIdx.x] = cells;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int v = (int)threadIdx.x >= off ? lds[threadIdx.x - off] : 0;
      __syncthreads();
      lds[threadIdx.x] += v;
      __syncthreads();
    }
    const int incl = lds[threadIdx.x], total = lds[1023];
    __syncthreads();
    if (k < b.nmol) {
      b.mol_geo[k] = geo;
      b.mol_dim[k] = make_int4(nx, ny, nz, carry + incl - cells);
    }
    carry += total;
  }
  if (threadIdx.x == 0) b.ctr[ctr_slot(C_CELLS)] = (unsigned long long)carry;
}

__device__ inline int cell_index(double v, double lo, double inv_s, int n) {
  const int c = (int)floor((v - lo) * inv_s);
  return min(max(c, 0), n - 1);
}

__global__ void k_count(Bufs b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int m = b.mol[i];
  const double4 g = b.mol_geo[m];
  const int4 d = b.mol_dim[m];
  const double4 p = b.pos[i];
  const double inv_s = 1.0 / g.w;
  const int cx = cell_index(p.x, g.x, inv_s, d.x), cy = cell_index(p.y, g.y, inv_s, d.y),
            cz = cell_index(p.z, g.z, inv_s, d.z);
  const int c = d.w + (cz * d.y + cy) * d.x + cx;
  b.cellid[i] = c;
  atomicAdd(&b.cnt[c], 1);
}

// ------------------------------------------------------------------ scan
constexpr int SCAN_T = 1024;
constexpr int SCAN_E = 2 * SCAN_T;

__device__ int block_scan2(int a0, int a1, int* lds, int* total) {
  const int t = threadIdx.x;
  const int s = a0 + a1;
  lds[t] = s;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    const int v = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += v;
    __syncthreads();
  }
  const int incl = lds[t];
  *total = lds[SCAN_T - 1];
  __syncthreads();
  return incl - s;
}

__global__ __launch_bounds__(SCAN_T) void k_scan1(const int* cnt, int* start, int* sums, int hb) {
  __shared__ int lds[SCAN_T];
  const int base = blockIdx.x * SCAN_E + 2 * threadIdx.x;
  const int a0 = base < hb ? cnt[base] : 0;
  const int a1 = base + 1 < hb ? cnt[base + 1] : 0;
  int total;
  const int ex = block_scan2(a0, a1, lds, &total);
  if (base < hb) start[base] = ex;
  if (base + 1 < hb) start[base + 1] = ex + a0;
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of the block sums, in chunks of SCAN_E with a running carry
__global__ __launch_bounds__(SCAN_T) void k_scan2(int* sums, int nb, int* start, int hb) {
  __shared__ int lds[SCAN_T];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += SCAN_E) {
    const int base = c0 + 2 * threadIdx.x;
    const int a0 = base < nb ? sums[base] : 0;
    const int a1 = base + 1 < nb ? sums[base + 1] : 0;
    int total;
    const int ex = carry + block_scan2(a0, a1, lds, &total);
    if (base < nb) sums[base] = ex;
    if (base + 1 < nb) sums[base + 1] = ex + a0;
    carry += total;
  }
  if (threadIdx.x == 0) start[hb] = carry;
}

__global__ void k_scan3(int* start, const int* sums, int hb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < hb) start[k] += sums[k / SCAN_E];
}

__global__ void k_scatter(Bufs b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int c = b.cellid[i];
  const int slot = b.start[c] + atomicSub(&b.cnt[c], 1) - 1;
  b.sorted[slot] = i;
  b.spos[slot] = b.pos[i];
  b.smc[slot] = make_int2(b.mol[i], c);
}

// ------------------------------------------------------------------ one molecule
// The whole cell-list stage of a call with one molecule in one block: clears
// the counters, weights + box, grid, per-cell counts (in LDS when the grid
// fits), their scan and the scatter into cell order.  It replaces the ten
// launches of the batched path for the common single-molecule call.  Its
// memory traffic all goes through one CU, so the scatter into cell order is
// staged in LDS and leaves in coalesced stores (a direct scatter touches one
// cache line per atom and store, and the CU's address unit then sets the pace).
constexpr int ONE_T = 1024;
constexpr int ONE_LDS_CELLS = 32768;
// atoms per staging pass: a 32-byte position and two ints each in the count array's LDS
constexpr int ONE_STAGE = ONE_LDS_CELLS * (int)sizeof(int) / 40;

// A double moved N lanes up within each row of 16 lanes (DPP); a lane with no
// source in its row keeps its own value, which min and max ignore.
template <int N>
__device__ inline double row_shr(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = (int)(u & 0xffffffffll), hi = (int)(u >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, 0x110 + N, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, 0x110 + N, 0xf, 0xf, false);
  return __longlong_as_double(((long long)h2 << 32) | (unsigned)l2);
}
// min (or max) over the 64 lanes, in every lane: four DPP steps leave each
// row's result in its last lane, and the four rows meet in scalar reads
template <bool MAX>
__device__ inline double wave_minmax(double x) {
  auto op = [](double a, double c) { return MAX ? fmax(a, c) : fmin(a, c); };
  x = op(x, row_shr<1>(x));
  x = op(x, row_shr<2>(x));
  x = op(x, row_shr<4>(x));
  x = op(x, row_shr<8>(x));
  const long long u = __double_as_longlong(x);
  const int lo = (int)(u & 0xffffffffll), hi = (int)(u >> 32);
  double r = 0.0;
#pragma unroll
  for (int l = 15; l < 64; l += 16) {
    const double y = __longlong_as_double(((long long)__builtin_amdgcn_readlane(hi, l) << 32) |
                                          (unsigned)__builtin_amdgcn_readlane(lo, l));
    r = l == 15 ? y : op(r, y);
  }
  return r;
}

// Every atom of the call stays in the registers of one thread (n <= PER * NT,
// NT threads); larger molecules take the multi-kernel cell list, which spreads
// over the whole GPU.  Small molecules take fewer waves and fewer atoms per
// thread: the block's barriers then wait on fewer waves, and less code runs.
template <int PER, int NT>
__global__ __launch_bounds__(NT) void k_cells_one(Bufs b) {
  static_assert(PER > 0, "atoms in registers");
  constexpr int R = PER;
  __shared__ __align__(32) int lcnt[ONE_LDS_CELLS];
  __shared__ double red[NT / 64][7];
  __shared__ int scan_lds[NT / 64];
  const int t = threadIdx.x, lane = t & 63;
  for (int k = t; k < C_COUNT * CTR_STRIDE; k += NT) b.ctr[k] = 0ull;
  // weights, box and R_max
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  double v[7] = {inf, inf, inf, -inf, -inf, -inf, 0.0};
  double rx[R], ry[R], rz[R], rr[R];
  int rc[R];
  int bad = 0;
  // Every phase issues all of a thread's loads before its first store: the
  // compiler cannot prove that the output arrays do not alias the inputs, so a
  // load after a store would wait for it (one memory round trip per atom).
  auto load = [&](int i, double& x, double& y, double& z, double& r) {
    x = b.xyz[3 * i], y = b.xyz[3 * i + 1], z = b.xyz[3 * i + 2];
    r = b.radii[i];
  };
  auto weigh = [&](int i, double& x, double& y, double& z, double& r) {  // r becomes R_i
    if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(r) && r > 0.0)) {
      ++bad;
      x = y = z = 0.0;
      r = 1.0;
    }
    r += b.probe;
    b.pos[i] = make_double4(x, y, z, r);
    v[0] = fmin(v[0], x), v[1] = fmin(v[1], y), v[2] = fmin(v[2], z);
    v[3] = fmax(v[3], x), v[4] = fmax(v[4], y), v[5] = fmax(v[5], z);
    v[6] = fmax(v[6], r);
  };
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t + k * NT;
    if (i < b.n) load(i, rx[k], ry[k], rz[k], rr[k]);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t + k * NT;
    if (i < b.n) weigh(i, rx[k], ry[k], rz[k], rr[k]);
  }
  // box and R_max: each wave reduces its lanes, and after the barrier every
  // wave reduces the waves' results itself (no second barrier to hand them out)
  auto minmax7 = [&](double* w) {
#pragma unroll
    for (int q = 0; q < 3; ++q) w[q] = wave_minmax<false>(w[q]);
#pragma unroll
    for (int q = 3; q < 7; ++q) w[q] = wave_minmax<true>(w[q]);
  };
  minmax7(v);
  if (lane == 0)
    for (int q = 0; q < 7; ++q) red[t >> 6][q] = v[q];
  __syncthreads();  // also orders the counter clearing before the stores below
  if (bad) atomicAdd(&b.ctr[ctr_slot(C_BAD_INPUT)], (unsigned long long)bad);
#pragma unroll
  for (int q = 0; q < 7; ++q) v[q] = lane < NT / 64 ? red[lane][q] : (q < 3 ? inf : -inf);
  minmax7(v);
  const double rmax = v[6];
  double4 geo;
  int dx, dy, dz;
  const int cells = grid_dims(v[0], v[1], v[2], v[3], v[4], v[5], b.n, rmax, geo, dx, dy, dz);
  if (t == 0) {
    b.ctr[ctr_slot(C_RMAX_BITS)] = (unsigned long long)__double_as_longlong(rmax);
    b.mol_geo[0] = geo;
    b.mol_dim[0] = make_int4(dx, dy, dz, 0);
    b.ctr[ctr_slot(C_CELLS)] = (unsigned long long)cells;
  }
  const bool in_lds = cells <= ONE_LDS_CELLS;
  int* cnt = in_lds ? lcnt : b.cnt;
  for (int c = t; c < cells; c += NT) cnt[c] = 0;
  const double gx = geo.x, gy = geo.y, gz = geo.z, inv_s = 1.0 / geo.w;
  __syncthreads();
  auto cell_of = [&](double x, double y, double z) {
    return (cell_index(z, gz, inv_s, dz) * dy + cell_index(y, gy, inv_s, dy)) * dx + cell_index(x, gx, inv_s, dx);
  };
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t + k * NT;
    if (i < b.n) {
      rc[k] = cell_of(rx[k], ry[k], rz[k]);
      atomicAdd(&cnt[rc[k]], 1);
    }
  }
  __syncthreads();
  // exclusive scan: thread t owns the contiguous cells [t*per, (t+1)*per)
  const int per = (cells + NT - 1) / NT;
  const int c0 = min(t * per, cells), c1 = min(c0 + per, cells);
  int sum = 0;
  for (int c = c0; c < c1; ++c) sum += cnt[c];
  // inclusive scan of the threads' sums: within each wave by lane shifts, then
  // across the waves' totals (two barriers in all)
  int incl = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const int x = __shfl_up(incl, off, 64);
    if (lane >= off) incl += x;
  }
  if (lane == 63) scan_lds[t >> 6] = incl;
  __syncthreads();
  for (int w = 0; w < (t >> 6); ++w) incl += scan_lds[w];
  int run = incl - sum;
  for (int c = c0; c < c1; ++c) {
    const int k = cnt[c];
    if (!in_lds) b.start[c] = run;
    cnt[c] = run;  // becomes the fill cursor of the cell
    run += k;
  }
  if (t == NT - 1) b.start[cells] = incl;
  __syncthreads();
  if (in_lds) {  // the cell starts leave LDS in coalesced stores (a thread's own cells are strided)
    for (int c = t; c < cells; c += NT) b.start[c] = lcnt[c];
    __syncthreads();
  }
  // every slot first (the cursor atomics then are all in flight together)
  int slot[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t + k * NT;
    slot[k] = i < b.n ? atomicAdd(&cnt[rc[k]], 1) : -1;
  }
  // then the scatter, ONE_STAGE slots per pass: each atom of the pass's slot
  // range goes to LDS (the counts are no longer needed), and the range leaves
  // in slot order
  double4* st_pos = reinterpret_cast<double4*>(lcnt);
  int* st_id = reinterpret_cast<int*>(st_pos + ONE_STAGE);
  int* st_cell = st_id + ONE_STAGE;
  for (int base = 0; base < b.n; base += ONE_STAGE) {
    __syncthreads();  // the slot atomics, or the last pass's stores, have read LDS
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int i = t + k * NT;
      const int j = slot[k] - base;
      if (i < b.n && j >= 0 && j < ONE_STAGE) {
        st_pos[j] = make_double4(rx[k], ry[k], rz[k], rr[k]);
        st_id[j] = i;
        st_cell[j] = rc[k];
      }
    }
    __syncthreads();
    const int m = min(ONE_STAGE, b.n - base);
    for (int j = t; j < m; j += NT) {
      b.sorted[base + j] = st_id[j];
      b.spos[base + j] = st_pos[j];
      b.smc[base + j] = make_int2(0, st_cell[j]);
    }
  }
}

// ------------------------------------------------------------------ star
// Plane ids inside one star: 0..5 are the faces of the starting cube
// (+x, -x, +y, -y, +z, -z), 6 + q is the radical plane of neighbour slot q.
// A plane keeps n . x <= b (x relative to p_i).  For neighbour q with
// a = p_q - p_i: pi_i(x) <= pi_q(x)  <=>  2 a . x <= |a|^2 - w_q + w_i.
// Cell vertices are simple (three planes each), stored as the three plane ids
// packed 10 bits apiece in ascending order; two vertices are joined by a cell
// edge iff they share two plane ids.
struct Pl {
  double x, y, z, b;
};

__device__ inline unsigned pack3(unsigned a, unsigned b, unsigned c) {
  // sort three ids ascending
  unsigned t;
  if (a > b) t = a, a = b, b = t;
  if (b > c) t = b, b = c, c = t;
  if (a > b) t = a, a = b, b = t;
  return a | (b << 10) | (c << 20);
}
__device__ inline unsigned pid0(unsigned p) { return p & 1023u; }
__device__ inline unsigned pid1(unsigned p) { return (p >> 10) & 1023u; }
__device__ inline unsigned pid2(unsigned p) { return p >> 20; }

constexpr int EH_BITS = 8, EH_SIZE = 1 << EH_BITS;  // > 2 x the 1.5 VC edges of a cell

// LDS of one star: NBC overlapping neighbours, VC cell vertices, the planes of
// the NPL nearest neighbours (farther ones are recomputed when needed).
template <int NBC, int VC, int NPL>
struct StarLds {
  static_assert(VC <= 128 && NBC % 4 == 0 && NPL <= NBC, "vertex slots are 7 bits in the edge table");
  static constexpr int kPlanes = NPL;
  int idx[NBC];  // neighbour global ids, slot order = clipping order (nearest plane first)
  double nx[NPL], ny[NPL], nz[NPL], nb[NPL];  // plane n = 2a, offset b
  union {
    unsigned char b[NBC];  // per-slot flags (facet present, K-triangles, K-edge ...)
    unsigned w[NBC / 4];   // the same four to a word (atomic OR)
  } sf;
  signed char kidx[NBC];  // slot -> K-neighbour index or -1
  union alignas(16) {
    struct {  // candidates in arrival order (neighbour search and ranking only)
      double key[NBC];  // signed distance of the radical plane from p_i
      int id[NBC];
    } app;
    struct {  // the cell across a cut, then the star's lists
      double vx[VC], vy[VC], vz[VC];
      unsigned vp[VC];
      signed char vt[VC];  // side-test bound of each vertex (thr_code)
      union {
        alignas(16) unsigned pairs[3 * VC];  // edges of the removed vertices of one cut
        struct {                 // cell edges by plane pair: code << 7 | first end, second end
          unsigned key[EH_SIZE];
          unsigned char second[EH_SIZE];
        } eh;
        struct {
          unsigned tri[2 * VC];  // triangle candidates: slot a | slot b << 10 | n_tet << 20
          int kslot[KN_CAP];     // K-edge slots in slot order
        } st;
      } w;
    } cl;
  } u;
};

template <class LT>
__device__ inline void sf_or(LT& L, int s, unsigned f) {
  atomicOr(&L.sf.w[s >> 2], f << ((s & 3) * 8));
}

enum SFlag : unsigned { SF_FACET = 1, SF_KTRI = 2, SF_EXTTRI = 4, SF_KEDGE = 8, SF_EXTEDGE = 16 };

// Radical plane of neighbour j (position pj, weight R_j^2) seen from p_i:
// n = 2 (p_j - p_i), b = |p_j - p_i|^2 - w_j + w_i, in a fixed order of
// correctly rounded operations so that every evaluation gives the same bits.
// (exact::radd / rsub / rmul: no contraction into fused operations)
__device__ inline Pl radical_plane(const double4& pi, double wi, const double4& pj) {
  using exact::radd, exact::rsub, exact::rmul;
  const double ax = rsub(pj.x, pi.x), ay = rsub(pj.y, pi.y), az = rsub(pj.z, pi.z);
  const double a2 = radd(radd(rmul(ax, ax), rmul(ay, ay)), rmul(az, az));
  return {2.0 * ax, 2.0 * ay, 2.0 * az, radd(rsub(a2, rmul(pj.w, pj.w)), wi)};
}

// Plane of neighbour slot q: from LDS, or recomputed for slots past the
// stored ones.
template <class LT>
__device__ inline Pl slot_plane(const LT& L, const Bufs& b, const double4& pi, double wi, int q) {
  if (__builtin_expect(q < LT::kPlanes, 1)) return {L.nx[q], L.ny[q], L.nz[q], L.nb[q]};
  return radical_plane(pi, wi, b.pos[L.idx[q]]);
}

// Plane of id pid (a cube face or a neighbour slot) for a per-lane id: the
// cube faces come from selects and the stored planes from an LDS read that
// every lane makes (its index clamped into range), so that the reads of a
// vertex solve's two planes are in flight together; only a slot past the
// stored planes takes a branch.
template <class LT>
__device__ inline Pl plane_of(const LT& L, const Bufs& b, const double4& pi, double wi, unsigned pid, double half) {
  const bool cube = pid < 6;
  const int q = cube ? 0 : (int)pid - 6;
  const int qs = q < LT::kPlanes ? q : LT::kPlanes - 1;
  Pl p = {L.nx[qs], L.ny[qs], L.nz[qs], L.nb[qs]};
  if (q >= LT::kPlanes) p = radical_plane(pi, wi, b.pos[L.idx[q]]);
  if (cube) {
    const double s = (pid & 1) ? -1.0 : 1.0;
    const unsigned ax = pid >> 1;
    p = {ax == 0 ? s : 0.0, ax == 1 ? s : 0.0, ax == 2 ? s : 0.0, half};
  }
  return p;
}

// Vertex of three planes.  thr (optional) receives a bound on the rounding
// error of any side test at this vertex: the planes' own coefficients carry
// rounding (relative ~8 u for the offsets), and the solve divides by the
// determinant, so the vertex is off by at most E |1/det| with E a per-atom
// constant, and a side test b_m - n_m . v by at most P E |1/det| + T (see
// star_atom, where E, P and T are set).
__device__ inline void solve3(const Pl& A, const Pl& B, const Pl& C, double& x, double& y, double& z,
                              double* thr = nullptr, double thrP = 0.0, double thrT = 0.0) {
  const double bcx = B.y * C.z - B.z * C.y, bcy = B.z * C.x - B.x * C.z, bcz = B.x * C.y - B.y * C.x;
  const double cax = C.y * A.z - C.z * A.y, cay = C.z * A.x - C.x * A.z, caz = C.x * A.y - C.y * A.x;
  const double abx = A.y * B.z - A.z * B.y, aby = A.z * B.x - A.x * B.z, abz = A.x * B.y - A.y * B.x;
  // 1 / det from the hardware estimate and two Newton steps (a fixed sequence,
  // so a vertex still has one value however it is reached)
  const double det = A.x * bcx + A.y * bcy + A.z * bcz;
  double inv = __builtin_amdgcn_rcp(det);
  inv = fma(inv, fma(-det, inv, 1.0), inv);
  inv = fma(inv, fma(-det, inv, 1.0), inv);
  x = (A.b * bcx + B.b * cax + C.b * abx) * inv;
  y = (A.b * bcy + B.b * cay + C.b * aby) * inv;
  z = (A.b * bcz + B.b * caz + C.b * abz) * inv;
  if (thr) *thr = fma(fabs(inv), thrP, thrT);  // inf when det = 0: every test at it is undecided
}

// A side-test bound kept in LDS as the exponent of a power of two above it.
__device__ inline signed char thr_code(double t) {
  if (!(t < 1e30)) return (signed char)127;
  return (signed char)max(-126, __builtin_amdgcn_frexp_exp(t));  // t < 2^e
}
__device__ inline double thr_value(signed char e) { return ldexp(1.0, (int)e); }

// value of lane l (wave-uniform l)
__device__ inline double rdl(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline int rdl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// The clipping's security-radius test is made at every this many slots.
constexpr int kSecurityStride = 16;

// Lowers the ranking key of a neighbour that was a facet in the previous frame
// (plane distances are a few Angstrom; the shifted keys keep their order to
// well below 1e-9 A, and exact ties fall back to the atom id).
constexpr double kFirstShift = 1.0e6;

// Clipping order of a candidate as one 64-bit integer: its plane distance
// rounded to float (as order-preserving bits) above its atom id, so that
// nearest plane comes first and ties go by atom id, and ranking compares one
// lane pair per candidate.  Rounding to float can only reorder planes whose
// distances agree to about 1e-7 relative; the stopping test keeps a margin
// above that.
__device__ inline unsigned long long order_key(double key, int id) {
  const unsigned u = __float_as_uint((float)key);
  const unsigned o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((unsigned long long)o << 32) | (unsigned)id;
}

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Exact sign of the side test of plane slot k at the vertex with plane ids pv
// (exact_side.h), evaluated by the calling lane alone in the work space W.
// (These helpers take the positions array, not the whole buffer set: a
// non-inlined function taking the kernel's argument block by reference would
// make every block copy that block to scratch memory on entry.)
template <class LT>
__device__ __noinline__ int exact_side_at(const double4* pos, const double4& pi, double half, const LT& L,
                                          exact::Work& W, unsigned pv, int k) {
  const unsigned ids[4] = {pid0(pv), pid1(pv), pid2(pv), 6u + (unsigned)k};
  for (int q = 0; q < 4; ++q) {
    if (ids[q] < 6) {
      exact::cube_face(ids[q], half, W.pl[q]);
    } else {
      const double4 pj = pos[L.idx[ids[q] - 6]];
      if (!exact::radical(pi.x, pi.y, pi.z, pi.w, pj.x, pj.y, pj.z, pj.w, W.pl[q], W)) return 2;
    }
  }
  return exact::side(W);
}

// Side test of plane slot k at the vertex with plane ids pv in double-double
// (each lane its own; 0 if that does not decide it).
template <class LT>
__device__ __noinline__ int dd_side_at(const double4* pos, const double4& pi, double half, const LT& L, unsigned pv,
                                       int k) {
  exact::DPl P[4];
  const unsigned ids[4] = {pid0(pv), pid1(pv), pid2(pv), 6u + (unsigned)k};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (ids[q] < 6) {
      P[q] = exact::dd_cube(ids[q], half);
    } else {
      const double4 pj = pos[L.idx[ids[q] - 6]];
      P[q] = exact::dd_radical(pi.x, pi.y, pi.z, pi.w, pj.x, pj.y, pj.z, pj.w);
    }
  }
  return exact::dd_side(P);
}

// Sign of det[n_a; n_b; n_c] of the vertex with plane ids pv (the orientation
// of the tetrahedron (i, a, b, c)): double-double, each lane its own; 0 if that
// does not decide it.
template <class LT>
__device__ __noinline__ int dd_orient_at(const double4* pos, const double4& pi, double half, const LT& L, unsigned pv) {
  exact::DPl P[3];
  const unsigned ids[3] = {pid0(pv), pid1(pv), pid2(pv)};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (ids[q] < 6) {
      P[q] = exact::dd_cube(ids[q], half);
    } else {
      const double4 pj = pos[L.idx[ids[q] - 6]];
      P[q] = exact::dd_radical(pi.x, pi.y, pi.z, pi.w, pj.x, pj.y, pj.z, pj.w);
    }
  }
  double m;
  const exact::DD d = exact::dd_det3(P[0], P[1], P[2], m);
  const double v = d.hi + d.lo;
  return fabs(v) > 1e-27 * m ? (v > 0.0 ? 1 : -1) : 0;
}

// The same sign from the expansions, by the calling lane alone in W.
template <class LT>
__device__ __noinline__ int exact_orient_at(const double4* pos, const double4& pi, double half, const LT& L,
                                            exact::Work& W, unsigned pv) {
  const unsigned ids[3] = {pid0(pv), pid1(pv), pid2(pv)};
  for (int q = 0; q < 3; ++q) {
    if (ids[q] < 6) {
      exact::cube_face(ids[q], half, W.pl[q]);
    } else {
      const double4 pj = pos[L.idx[ids[q] - 6]];
      if (!exact::radical(pi.x, pi.y, pi.z, pi.w, pj.x, pj.y, pj.z, pj.w, W.pl[q], W)) return 2;
    }
  }
  if (!exact::det3(W.pl[0], W.pl[1], W.pl[2], W)) return 2;
  return exact::sign(W.det3);
}

// The vertex of plane ids pv solved exactly (exact_side.h), by the calling lane
// alone in the work space W.  False on failure.
template <class LT>
__device__ __noinline__ bool exact_vertex_at(const double4* pos, const double4& pi, double half, const LT& L,
                                             exact::Work& W, unsigned pv, double* v) {
  const unsigned ids[3] = {pid0(pv), pid1(pv), pid2(pv)};
  for (int q = 0; q < 3; ++q) {
    if (ids[q] < 6) {
      exact::cube_face(ids[q], half, W.pl[q]);
    } else {
      const double4 pj = pos[L.idx[ids[q] - 6]];
      if (!exact::radical(pi.x, pi.y, pi.z, pi.w, pj.x, pj.y, pj.z, pj.w, W.pl[q], W)) return false;
    }
  }
  return exact::vertex(W, v);
}

// The star of the atom at cell-ordered position sidx.  Returns false when the
// atom needs more than NBC neighbours or VC cell vertices, or (without EXACT)
// when a clipping side test is too close to zero for its rounding bound, and
// `last` is not set: it is then left to the second pass (larger capacities,
// exact side tests; nothing is written).  With `last` an atom over capacity is
// reported as a capacity overflow.
//
// Ties.  A side test that rounding cannot decide is decided exactly (EXACT);
// a vertex exactly on the plane is kept.  Keeping every tie is the clipping of
// the cell whose planes are each moved outwards by an infinitesimal that grows
// with the clipping order (later planes more), a valid perturbation of the
// neighbours' weights: the cell is a consistent simple polytope, and Eq. 1 over
// its star gives the atom's exact area in the limit.  Each atom's cell is its
// own perturbation, so on tied inputs the stars of two atoms need not agree on a
// shared simplex, while every atom's area (unique) and gradient (unique where
// the area is differentiable) do.
template <bool HINTS, bool EXACT, int NBC, int VC, int NPL>
__device__ bool star_atom(const Bufs& b, StarLds<NBC, VC, NPL>& L, int sidx, bool last, exact::Work* W) {
  // atoms in cell order (neighbouring blocks share neighbours in cache); the
  // atom's id, position, molecule and cell come from the cell-ordered copies
  const int i = b.sorted[sidx];
  const int lane = threadIdx.x;
  const double4 pi = b.spos[sidx];
  const int2 mc = b.smc[sidx];
  const int mi = mc.x;
  const double Ri = pi.w, wi = Ri * Ri;
  const int4 gd = b.mol_dim[mi];
  const double4 gg = b.mol_geo[mi];
  const double rmax = rmax_of(b.ctr);
  const double h = gg.w;  // cell side of i's molecule (>= R_max)
  int cx, cy, cz;
  {
    const int c = mc.y - gd.w;
    cx = c % gd.x;
    cy = (c / gd.x) % gd.y;
    cz = c / (gd.x * gd.y);
  }

  // ---- 1. overlapping neighbours.  Candidates lie within R_i + R_max <= 2h
  // of p_i: in the rows (cy + dy, cz + dz), |dy|, |dz| <= 2, of x-cells
  // cx - 2 .. cx + 2, pruned to the chord of that sphere.  Lane r < 25 finds
  // row r's range of `sorted` (cells along x are contiguous); the rows are
  // then read as one flat, coalesced candidate list.
  const double reach = Ri + rmax;
  const double reach2 = reach * reach * (1.0 + 1e-12) + 1e-12;  // widened: a cell is never lost to rounding
  int row_a = 0, row_n = 0;
  if (lane < 25) {
    const int y = cy + lane % 5 - 2, z = cz + lane / 5 - 2;
    if (y >= 0 && y < gd.y && z >= 0 && z < gd.z) {
      const double ylo = gg.y + y * h, zlo = gg.z + z * h;
      const double ty = pi.y < ylo ? ylo - pi.y : (pi.y > ylo + h ? pi.y - ylo - h : 0.0);
      const double tz = pi.z < zlo ? zlo - pi.z : (pi.z > zlo + h ? pi.z - zlo - h : 0.0);
      const double t2 = ty * ty + tz * tz;
      if (t2 < reach2) {
        const double half = sqrt(reach2 - t2);
        const double inv_s = 1.0 / h;
        const int x0 = max(max(cx - 2, 0), (int)floor((pi.x - half - gg.x) * inv_s));
        const int x1 = min(min(cx + 2, gd.x - 1), (int)floor((pi.x + half - gg.x) * inv_s));
        if (x0 <= x1) {
          const int c0 = gd.w + (z * gd.y + y) * gd.x;
          row_a = b.start[c0 + x0];
          row_n = b.start[c0 + x1 + 1] - row_a;
        }
      }
    }
  }
  int pre = row_n;  // inclusive prefix over the rows
  for (int off = 1; off < 32; off <<= 1) {
    const int t = __shfl_up(pre, off, 64);
    if (lane >= off) pre += t;
  }
  const int total = __shfl(pre, 24, 64);
  const int row_s = pre - row_n;     // first flat index of the row
  const int row_d = row_a - row_s;   // sorted index = flat index + row_d of its row
  // this atom's cell in the previous frame of a trajectory (loaded now, used
  // once the candidates are ranked): facet neighbour ids and vertex triples.
  // fslot maps a facet's list position to its slot in this frame (0xff: the
  // neighbour is no longer a candidate).
  int npf = 0, nvh = 0, pf = -1;
  unsigned vh = 0u;
  unsigned char* fslot = L.u.cl.w.eh.second;  // free until the star is read off
  if constexpr (HINTS) {
    const int hn = __builtin_amdgcn_readfirstlane(b.hint_n[i]);
    npf = min(hn & 255, FAC_CAP);
    nvh = min((hn >> 8) & 255, FAC_CAP);
    if (lane < npf) pf = b.fac[(size_t)i * FAC_CAP + lane], fslot[lane] = 0xff;
    if (lane < nvh) vh = b.vtx[(size_t)i * FAC_CAP + lane];
  }
  int nn = 0;
  bool overflow = false;
  long long plane_tests = 0, new_verts = 0;
  // four chunks of 64 candidates per round: all their loads are in flight together
  for (int base = 0; base < total; base += 256) {
    int j[4];
    double4 pj[4];
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2) {
      const int f = base + 64 * h2 + lane;
      j[h2] = -1;
      // its row: the last of lanes 0..31 whose first flat index is <= f (the
      // starts ascend; lanes 25..31 start at total), by binary search
      int r = 0;
#pragma unroll
      for (int step = 16; step >= 1; step >>= 1)
        if (__shfl(row_s, r + step, 64) <= f) r += step;
      const int d = __shfl(row_d, r, 64);
      if (f < total) {
        const int k = f + d;
        j[h2] = b.sorted[k];
        pj[h2] = b.spos[k];
      }
    }
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2) {
      bool take = false;
      double dx = 0.0, dy = 0.0, dz = 0.0, d2 = 0.0;
      if (j[h2] >= 0) {
        dx = pj[h2].x - pi.x, dy = pj[h2].y - pi.y, dz = pj[h2].z - pi.z;
        d2 = dx * dx + dy * dy + dz * dz;
        const double rr = Ri + pj[h2].w;
        take = (j[h2] != i) && (d2 < rr * rr);
      }
      // two balls with one centre and one radius have one cell between them:
      // the input is refused (a smaller ball on the centre of a larger one is
      // hidden by the clipping: its plane 0 . x <= w_i - w_j removes the cell)
      if (__builtin_expect(__ballot(take && d2 == 0.0 && pj[h2].w == Ri) != 0ull, 0) && lane == 0)
        atomicAdd(&b.ctr[ctr_slot(C_BAD_INPUT)], 1ull);
      const unsigned long long m = __ballot(take);
      if (take) {
        const int at = nn + prefix_below(m);
        if (at < NBC) {
          // distance of the radical plane from p_i: (d^2 + w_i - w_j) / (2 d); a
          // neighbour at the same centre has no plane (it empties the cell or
          // cuts nothing) and goes first
          L.u.app.id[at] = j[h2];
          L.u.app.key[at] = d2 > 0.0 ? (d2 + wi - pj[h2].w * pj[h2].w) / (2.0 * sqrt(d2)) : -1e300;
        }
      }
      nn += __popcll(m);
    }
  }
  if (nn > NBC) {
    overflow = true;
    nn = NBC;
  }
  nn = __builtin_amdgcn_readfirstlane(nn);  // wave-uniform: keeps the loops over slots scalar
  __syncthreads();
  // ---- slots in clipping order: nearest plane first, ties by atom id.  Lane
  // s holds candidates s, s + 64, s + 128 in registers, ranks each against all
  // others (their order keys read back from LDS) and writes its plane at its
  // rank; the candidates' positions are fetched while the ranks are counted.
  constexpr int SL = (NBC + 63) / 64;  // candidates per lane
  int nfirst = 0;
  if constexpr (SL > 3) {
    // the wide pass's larger capacity: the same ranking over SL candidates
    // per lane (s, s + 64, ...); their positions are fetched at the end
    double ck[SL];
    int ci[SL], ft[SL], rk[SL];
    unsigned long long ok[SL];
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      ck[q] = 0.0, ci[q] = -1, ft[q] = -1, rk[q] = 0;
      if (lane + 64 * q < nn) ck[q] = L.u.app.key[lane + 64 * q], ci[q] = L.u.app.id[lane + 64 * q];
    }
    if (HINTS && npf > 0) {
      for (int t = 0; t < npf; ++t) {
        const int id = rdl(pf, t);
#pragma unroll
        for (int q = 0; q < SL; ++q)
          if (ci[q] >= 0 && id == ci[q]) ft[q] = t;
      }
#pragma unroll
      for (int q = 0; q < SL; ++q) {
        if (ft[q] >= 0) ck[q] -= kFirstShift;
        nfirst += __popcll(__ballot(ft[q] >= 0));
      }
    }
#pragma unroll
    for (int q = 0; q < SL; ++q) ok[q] = order_key(ck[q], ci[q]);
    unsigned long long* okey = reinterpret_cast<unsigned long long*>(L.u.app.key);
#pragma unroll
    for (int q = 0; q < SL; ++q)
      if (lane + 64 * q < nn) okey[lane + 64 * q] = ok[q];
    if (lane == 0 && (nn & 1)) okey[nn] = ~0ull;
    __syncthreads();
    const ulonglong2* okp = reinterpret_cast<const ulonglong2*>(okey);
    const int npair = (nn + 1) >> 1;
    for (int t = 0; t < npair; ++t) {
      const ulonglong2 kt = okp[t];
#pragma unroll
      for (int q = 0; q < SL; ++q) rk[q] += (kt.x < ok[q]) + (kt.y < ok[q]);
    }
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      if (ci[q] < 0) continue;
      const int r = rk[q];
      L.idx[r] = ci[q];
      if (r < NPL) {
        const Pl pl = radical_plane(pi, wi, b.pos[ci[q]]);
        L.nx[r] = pl.x, L.ny[r] = pl.y, L.nz[r] = pl.z, L.nb[r] = pl.b;
      }
      L.sf.b[r] = 0;
      L.kidx[r] = -1;
      if (ft[q] >= 0) fslot[ft[q]] = (unsigned char)r;
    }
  } else {
    const int nsets = (nn + 63) >> 6;
    double ck0 = 0.0, ck1 = 0.0, ck2 = 0.0;
    int ci0 = -1, ci1 = -1, ci2 = -1;
    if (lane < nn) ck0 = L.u.app.key[lane], ci0 = L.u.app.id[lane];
    if (lane + 64 < nn) ck1 = L.u.app.key[lane + 64], ci1 = L.u.app.id[lane + 64];
    if (lane + 128 < nn) ck2 = L.u.app.key[lane + 128], ci2 = L.u.app.id[lane + 128];
    double4 cp0 = make_double4(0.0, 0.0, 0.0, 0.0), cp1 = cp0, cp2 = cp0;
    if (ci0 >= 0) cp0 = b.pos[ci0];
    if (ci1 >= 0) cp1 = b.pos[ci1];
    if (ci2 >= 0) cp2 = b.pos[ci2];
    // a neighbour whose plane bounded the previous frame's cell is clipped before
    // all others: its key is lowered by far more than any plane distance (the
    // order among such neighbours stays nearest plane first, ties by atom id).
    // The cell is the same in any clipping order; this one makes few cuts and
    // few vertices that a later cut removes.
    int ft0 = -1, ft1 = -1, ft2 = -1;  // facet-list position of each candidate
    if (HINTS && npf > 0) {
      for (int t = 0; t < npf; ++t) {
        const int id = rdl(pf, t);
        if (id == ci0) ft0 = t;
        if (id == ci1) ft1 = t;
        if (id == ci2) ft2 = t;
      }
      if (ci0 < 0) ft0 = -1;
      if (ci1 < 0) ft1 = -1;
      if (ci2 < 0) ft2 = -1;
      if (ft0 >= 0) ck0 -= kFirstShift;
      if (ft1 >= 0) ck1 -= kFirstShift;
      if (ft2 >= 0) ck2 -= kFirstShift;
      nfirst = __popcll(__ballot(ft0 >= 0)) + __popcll(__ballot(ft1 >= 0)) + __popcll(__ballot(ft2 >= 0));
    }
    const unsigned long long ok0 = order_key(ck0, ci0), ok1 = order_key(ck1, ci1), ok2 = order_key(ck2, ci2);
    // The keys go to LDS (each lane overwrites the arrival slots it has just
    // read), padded to an even count with a key above every candidate's; each
    // lane then counts the keys below its own, two keys per (broadcast) read.
    unsigned long long* okey = reinterpret_cast<unsigned long long*>(L.u.app.key);
    if (lane < nn) okey[lane] = ok0;
    if (lane + 64 < nn) okey[lane + 64] = ok1;
    if (lane + 128 < nn) okey[lane + 128] = ok2;
    if (lane == 0 && (nn & 1)) okey[nn] = ~0ull;
    __syncthreads();
    const ulonglong2* okp = reinterpret_cast<const ulonglong2*>(okey);
    const int npair = (nn + 1) >> 1;
    int rk0 = 0, rk1 = 0, rk2 = 0;
    if (nsets == 1) {
      for (int t = 0; t < npair; ++t) {
        const ulonglong2 kt = okp[t];
        rk0 += (kt.x < ok0) + (kt.y < ok0);
      }
    } else if (nsets == 2) {
      for (int t = 0; t < npair; ++t) {
        const ulonglong2 kt = okp[t];
        rk0 += (kt.x < ok0) + (kt.y < ok0);
        rk1 += (kt.x < ok1) + (kt.y < ok1);
      }
    } else {
      for (int t = 0; t < npair; ++t) {
        const ulonglong2 kt = okp[t];
        rk0 += (kt.x < ok0) + (kt.y < ok0);
        rk1 += (kt.x < ok1) + (kt.y < ok1);
        rk2 += (kt.x < ok2) + (kt.y < ok2);
      }
    }
    for (int hb = 0; hb < 3; ++hb) {
      const int id = hb == 0 ? ci0 : (hb == 1 ? ci1 : ci2);
      if (id < 0) continue;
      const int r = hb == 0 ? rk0 : (hb == 1 ? rk1 : rk2);
      L.idx[r] = id;
      if (r < NPL) {
        const Pl q = radical_plane(pi, wi, hb == 0 ? cp0 : (hb == 1 ? cp1 : cp2));
        L.nx[r] = q.x, L.ny[r] = q.y, L.nz[r] = q.z, L.nb[r] = q.b;
      }
      L.sf.b[r] = 0;
      L.kidx[r] = -1;
      const int ft = hb == 0 ? ft0 : (hb == 1 ? ft1 : ft2);
      if (ft >= 0) fslot[ft] = (unsigned char)r;
    }
  }
  // ---- 2. clip the cube [-h, h]^3 (h = 1.1 R_i, so it holds B_i strictly) by
  // the planes in order.  Each lane keeps cell vertices lane and lane + 64 in
  // registers; LDS holds the cell only across a cut.
  const double half = 1.1 * Ri;
  // Rounding bounds of the side tests.  Every plane has |n| <= P (neighbours
  // overlap, so |p_j - p_i| < R_i + R_max; cube faces |n| = 1) and an offset
  // computed with error <= 8 u Bo; every vertex has |v| <= V.  A vertex solved
  // from three planes is then off by at most E |1/det|, E = 128 u P^2 (Bo + P V)
  // (the offsets' errors and the normals' through adj(M) / det, the rounding of
  // the cross products, of the numerators and of det), and a side test
  // b_m - n_m . v by at most P E |1/det| + 12 u (Bo + P V) (the plane's own
  // errors and the dot product's rounding).
  constexpr double kU = 1.1102230246251565e-16;  // 2^-53
  const double Pn = fmax(2.0 * (Ri + rmax), 1.0);
  const double Bo = (Ri + rmax) * (Ri + rmax) + rmax * rmax + wi + half;
  const double Vv = 1.7320508075688772 * half;
  const double thrE = 1.01 * 128.0 * kU * Pn * Pn * (Bo + Pn * Vv);
  const double thrP = Pn * thrE;
  const double thrT = 1.01 * 12.0 * kU * (Bo + Pn * Vv);
  const double invPn = 1.0 / Pn;
  // The star is read off the vertices' positions (inside B_i or not; where a
  // cell edge passes).  The fast pass certifies each such decision with the
  // vertex's bound and leaves the atom to the second pass if one is too close
  // to call; the second pass solves every vertex whose position bound passes
  // 1e-9 A exactly (planes close to parallel, as where a cut crosses an edge
  // lying almost in its plane: 4 ulp per coordinate), and a kept trajectory
  // vertex is used only within that bound.
  const double thrCap = fma(Pn, 1e-9, thrT);
  const double thrSolved = fma(Pn, 7.0 * kU * Vv, thrT);
  // |v|^2 bound of a vertex with side-test bound t (its position error is at most t / P)
  auto vr2 = [&](double x, double y, double z, double t) {
    const double ev = t * invPn;
    const double r = fma(ev, 2.0 * Vv + ev, x * x + y * y + z * z);
    return r <= 1e300 ? r : 1e300;  // (a non-finite vertex never lets the clipping stop)
  };
  long long exact_tests = 0;
  bool exact_fail = false;
  int nv = 8;
  double x0 = 0, y0 = 0, z0 = 0, x1 = 0, y1 = 0, z1 = 0;
  double t0 = thrT, t1 = thrT;  // side-test bounds (the cube's corners are exact)
  unsigned p0 = 0, p1 = 0;
  if (lane < 8) {
    x0 = (lane & 1) ? -half : half;
    y0 = (lane & 2) ? -half : half;
    z0 = (lane & 4) ? -half : half;
    p0 = ((lane & 1) ? 1u : 0u) | (((lane & 2) ? 3u : 2u) << 10) | (((lane & 4) ? 5u : 4u) << 20);
  }
  double rho2 = 3.0 * half * half;  // bound on |v|^2 over the cell (exact when rho_exact)
  double rs2 = rho2 * (1.0 + 1e-6) + 1e-12;  // the same with the security test's margin
  bool rho_exact = true;
  bool empty = false;
  int vmax = 8;
  int kstop = nn;  // planes visited
  __syncthreads();
  // ---- 2a. a trajectory's previous cell.  Its facet neighbours are the
  // first nfirst slots; its vertices (plane triples, now in this frame's
  // slots) are solved afresh.  If each lies inside every one of those planes
  // (and the cube's) that it is not on, the set is closed under the edges of
  // their intersection Q (the segment between two feasible vertices on one
  // line lies in Q), so it is Q's whole vertex set: Q is exactly what clipping
  // the cube by the first nfirst planes would give, and the clipping goes on
  // from there with the remaining planes.  Otherwise it starts from the cube.
  bool reused = false;
  int k0 = 0;
  if (HINTS && nvh > 0 && nvh <= 64 && nvh <= VC && nfirst > 0 && !overflow) {
    bool ok = true;
    double vx = 0.0, vy = 0.0, vz = 0.0, vt = 0.0;
    unsigned vp = 0u;
    if (lane < nvh) {
      unsigned q[3];
      for (int c = 0; c < 3; ++c) {
        const unsigned hc = (vh >> (7 * c)) & 127u;
        q[c] = hc;
        if (hc >= 6) {
          const unsigned sl = hc - 6 < (unsigned)npf ? fslot[hc - 6] : 0xffu;
          if (sl == 0xffu) ok = false;
          q[c] = 6u + sl;
        }
      }
      vp = pack3(q[0], q[1], q[2]);
      if (ok && pid0(vp) != pid1(vp) && pid1(vp) != pid2(vp)) {
        solve3(plane_of(L, b, pi, wi, pid0(vp), half), plane_of(L, b, pi, wi, pid1(vp), half),
               plane_of(L, b, pi, wi, pid2(vp), half), vx, vy, vz, &vt, thrP, thrT);
        ok = isfinite(vx) && isfinite(vy) && isfinite(vz) && (!EXACT || vt <= thrCap);
        for (unsigned c = 0; c < 6 && ok; ++c) {  // the cube's planes (strictly inside, beyond rounding)
          if (pid0(vp) == c || pid1(vp) == c || pid2(vp) == c) continue;
          const double sg = (c & 1) ? -1.0 : 1.0;
          const double t = (c >> 1) == 0 ? vx : ((c >> 1) == 1 ? vy : vz);
          ok = half - sg * t >= vt;
        }
      } else {
        ok = false;
      }
    }
    // the previous facets' planes (slots 0 .. nfirst - 1, all in LDS), one
    // vertex per lane, the same side test as the clipping
    for (int k = 0; k < nfirst && __ballot(!ok) == 0ull; ++k) {
      const Pl qk = slot_plane(L, b, pi, wi, k);
      const unsigned pk = 6u + (unsigned)k;
      if (lane < nvh && pid0(vp) != pk && pid1(vp) != pk && pid2(vp) != pk)
        ok = qk.b - (qk.x * vx + qk.y * vy + qk.z * vz) >= vt;
    }
    plane_tests += (long long)nfirst * nvh;
    if (__ballot(!ok) == 0ull) {
      reused = true;
      k0 = nfirst;
      nv = nvh;
      vmax = nvh;
      new_verts += nvh;
      x0 = vx, y0 = vy, z0 = vz, p0 = vp, t0 = vt;
      rho2 = wave_max(lane < nvh ? vr2(vx, vy, vz, vt) : 0.0);
      rs2 = rho2 * (1.0 + 1e-6) + 1e-12;
      rho_exact = true;
      // the star is read off LDS if no plane cuts Q further
      if (lane < nvh)
        L.u.cl.vx[lane] = vx, L.u.cl.vy[lane] = vy, L.u.cl.vz[lane] = vz, L.u.cl.vp[lane] = vp,
        L.u.cl.vt[lane] = thr_code(vt);
      __syncthreads();
    }
  }
  for (int k = k0; k < nn && !overflow; ++k) {
    const Pl qk = slot_plane(L, b, pi, wi, k);
    const double qx = qk.x, qy = qk.y, qz = qk.z, qb = qk.b;
    // security radius: the plane's signed distance from p_i is b / |n| (its
    // ranking key); once it reaches the largest |v| of the cell, no plane from
    // here on can cut it.  Tested without a root or division as b >= 0 and
    // b^2 >= rho^2 |n|^2, with a margin (1e-6 on the squares) above the float
    // rounding of the ranking key, which may put a plane up to about 1e-7
    // nearer after this one.  A neighbour at the same centre (n = 0)
    // has no plane and never ends the loop.  rho^2 is kept as an upper bound
    // (a cut never moves a vertex away from p_i) and made exact only when the
    // bound would end the loop.  The test is made at every kSecurityStride-th
    // slot only: the loop then ends at most that many planes late (planes that
    // cut nothing), and the planes in between are spared it.
    // (k >= nfirst: the rest is in plane order.  The plane and rho^2 are the
    // same in every lane; voting on the tests makes their branches scalar.)
    if (__builtin_expect(k >= nfirst && k % kSecurityStride == 0, 0)) {
      const double qn2 = qx * qx + qy * qy + qz * qz;
      if (__ballot(qn2 > 0.0 && qb >= 0.0 && qb * qb >= rs2 * qn2) != 0ull) {
        if (!rho_exact) {
          double r2 = 0.0;
          if (lane < nv) r2 = vr2(x0, y0, z0, t0);
          if ((VC > 64 && lane + 64 < nv)) r2 = fmax(r2, vr2(x1, y1, z1, t1));
          rho2 = wave_max(r2);
          rs2 = rho2 * (1.0 + 1e-6) + 1e-12;
          rho_exact = true;
        }
        if (__ballot(qb * qb >= rs2 * qn2) != 0ull) {
          kstop = k;
          break;
        }
      }
    }
    const double g0 = qb - (qx * x0 + qy * y0 + qz * z0);
    const double g1 = VC > 64 ? qb - (qx * x1 + qy * y1 + qz * z1) : 0.0;
    bool r0 = lane < nv && g0 < 0.0;
    bool r1 = (VC > 64 && lane + 64 < nv) && g1 < 0.0;
    plane_tests += nv;
    {
      // side tests within their rounding bound: the fast pass leaves the atom to
      // the second pass, which decides them exactly (ties keep the vertex)
      // (negated tests: a vertex with a non-finite coordinate is undecided too)
      const bool u0 = lane < nv && !(fabs(g0) >= t0);
      const bool u1 = (VC > 64 && lane + 64 < nv) && !(fabs(g1) >= t1);
      if (__builtin_expect(__ballot(u0 || u1) != 0ull, 0)) {
        if constexpr (!EXACT) {
          if (!last) return false;
        } else {
          // double-double first, each lane its own test; then the remaining
          // ones (exact ties, in practice) in expansions, one lane at a time
          bool v0 = u0, v1 = u1;
          if (v0) {
            const int sg = dd_side_at(b.pos, pi, half, L, p0, k);
            if (sg != 0) r0 = sg < 0, v0 = false;
          }
          if (VC > 64 && v1) {
            const int sg = dd_side_at(b.pos, pi, half, L, p1, k);
            if (sg != 0) r1 = sg < 0, v1 = false;
          }
          exact_tests += __popcll(__ballot(u0)) + __popcll(__ballot(u1));
          for (int h = 0; h < 2; ++h) {
            unsigned long long um = __ballot(h ? v1 : v0);
            while (um) {
              const int l = __builtin_ctzll(um);
              um &= um - 1ull;
              const unsigned pv = (unsigned)__builtin_amdgcn_readlane((int)(h ? p1 : p0), l);
              int sg = 0;
              if (lane == 0) sg = exact_side_at(b.pos, pi, half, L, *W, pv, k);
              sg = __shfl(sg, 0, 64);
              exact_fail |= sg == 2;
              if (lane == l) {
                if (h) r1 = sg < 0;
                else r0 = sg < 0;
              }
            }
          }
        }
      }
    }
    const unsigned long long m0 = __ballot(r0), m1 = __ballot(r1);
    const int nr0 = __popcll(m0);
    const int nrem = nr0 + __popcll(m1);
    if (__builtin_expect(nrem == 0, 1)) continue;
    if (__builtin_expect(nrem == nv, 0)) {
      empty = true;
      kstop = k + 1;
      break;
    }
    const unsigned pid = 6u + (unsigned)k;
    // removed vertices list their three edges (plane pairs)
    if (r0) {
      const int rk = prefix_below(m0);
      L.u.cl.w.pairs[3 * rk + 0] = pid1(p0) | (pid2(p0) << 10);
      L.u.cl.w.pairs[3 * rk + 1] = pid0(p0) | (pid2(p0) << 10);
      L.u.cl.w.pairs[3 * rk + 2] = pid0(p0) | (pid1(p0) << 10);
    }
    if (r1) {
      const int rk = nr0 + prefix_below(m1);
      L.u.cl.w.pairs[3 * rk + 0] = pid1(p1) | (pid2(p1) << 10);
      L.u.cl.w.pairs[3 * rk + 1] = pid0(p1) | (pid2(p1) << 10);
      L.u.cl.w.pairs[3 * rk + 2] = pid0(p1) | (pid1(p1) << 10);
    }
    // padded to a multiple of four with a code no plane pair has (nrem < nv
    // <= VC, so the pad stays inside the array)
    if (lane < 3 && 3 * nrem + lane < ((3 * nrem + 3) & ~3)) L.u.cl.w.pairs[3 * nrem + lane] = 0xffffffffu;
    __syncthreads();
    const int nkeep = nv - nrem;
    // kept vertices move to their compacted slots (old LDS contents are dead:
    // every lane holds its vertices in registers)
    const unsigned long long k0 = __ballot(lane < nv && !r0), k1 = __ballot((VC > 64 && lane + 64 < nv) && !r1);
    if (lane < nv && !r0) {
      const int d = prefix_below(k0);
      L.u.cl.vx[d] = x0, L.u.cl.vy[d] = y0, L.u.cl.vz[d] = z0, L.u.cl.vp[d] = p0, L.u.cl.vt[d] = thr_code(t0);
    }
    if ((VC > 64 && lane + 64 < nv) && !r1) {
      const int d = __popcll(k0) + prefix_below(k1);
      L.u.cl.vx[d] = x1, L.u.cl.vy[d] = y1, L.u.cl.vz[d] = z1, L.u.cl.vp[d] = p1, L.u.cl.vt[d] = thr_code(t1);
    }
    // an edge with exactly one removed end crosses the plane: new vertex on it,
    // solved from its three planes in ascending id order (canonical)
    // (lane e holds edge e and counts its copies, four pairs per broadcast
    // read of the list)
    const int ne = 3 * nrem;
    const int nq = (ne + 3) >> 2;
    const uint4* pq = reinterpret_cast<const uint4*>(L.u.cl.w.pairs);
    int ncross = 0;
    for (int base = 0; base < ne; base += 64) {
      const int e = base + lane;
      const unsigned pr = e < ne ? L.u.cl.w.pairs[e] : 0xfffffffeu;  // (no pair and not the pad)
      int c = 0;
      for (int t = 0; t < nq; ++t) {
        const uint4 q = pq[t];
        c += (q.x == pr) + (q.y == pr) + (q.z == pr) + (q.w == pr);
      }
      const bool cross = e < ne && c == 1;
      const unsigned long long cm = __ballot(cross);
      bool bad_v = false;
      int my_slot = -1;
      if (cross) {
        const int slot = nkeep + ncross + prefix_below(cm);
        if (slot < VC) {
          my_slot = slot;
          // the pair is stored ascending and the cutting plane has the highest id
          // so far, so the triple is already in ascending order
          const unsigned tri3 = pr | (pid << 20);
          double x, y, z, t;
          solve3(plane_of(L, b, pi, wi, pr & 1023u, half), plane_of(L, b, pi, wi, pr >> 10, half), qk, x, y, z, &t,
                 thrP, thrT);
          L.u.cl.vx[slot] = x;
          L.u.cl.vy[slot] = y;
          L.u.cl.vz[slot] = z;
          L.u.cl.vp[slot] = tri3;
          L.u.cl.vt[slot] = thr_code(t);
          bad_v = EXACT && !(t <= thrCap);
        }
      }
      if constexpr (EXACT) {
        if (__builtin_expect(__ballot(bad_v) != 0ull, 0)) {
          unsigned long long bm = __ballot(bad_v);
          while (bm) {
            const int l = __builtin_ctzll(bm);
            bm &= bm - 1ull;
            const unsigned tv = (unsigned)__builtin_amdgcn_readlane((int)(pr | (pid << 20)), l);
            const int sl = __builtin_amdgcn_readlane(my_slot, l);
            if (lane == 0) {
              double v[3];
              if (exact_vertex_at(b.pos, pi, half, L, *W, tv, v)) {
                L.u.cl.vx[sl] = v[0], L.u.cl.vy[sl] = v[1], L.u.cl.vz[sl] = v[2];
                L.u.cl.vt[sl] = thr_code(thrSolved);
              } else {
                exact_fail = true;
              }
            }
          }
          exact_fail = __shfl(exact_fail ? 1 : 0, 0, 64) != 0;
        }
      }
      ncross += __popcll(cm);
    }
    new_verts += ncross;
    nv = nkeep + ncross;
    if (nv > VC) {
      overflow = true;
      break;
    }
    vmax = max(vmax, nv);
    __syncthreads();
    x0 = y0 = z0 = x1 = y1 = z1 = 0.0;
    p0 = p1 = 0u;
    if (lane < nv)
      x0 = L.u.cl.vx[lane], y0 = L.u.cl.vy[lane], z0 = L.u.cl.vz[lane], p0 = L.u.cl.vp[lane],
      t0 = thr_value(L.u.cl.vt[lane]);
    if ((VC > 64 && lane + 64 < nv))
      x1 = L.u.cl.vx[lane + 64], y1 = L.u.cl.vy[lane + 64], z1 = L.u.cl.vz[lane + 64], p1 = L.u.cl.vp[lane + 64],
      t1 = thr_value(L.u.cl.vt[lane + 64]);
    rho_exact = false;
    __syncthreads();  // the next cut overwrites pairs / vertices only after everyone has read
  }
  overflow |= exact_fail;  // an expansion outgrew its array (inputs far outside Angstrom scales)
  int* st = b.stat + (size_t)i * STAT_STRIDE;
  if (lane == 0) {
    st[S_NN] = nn;
    st[S_VMAX] = vmax;
    st[S_CAND] = total;
    st[S_TESTS] = (int)plane_tests;
    st[S_NEWV] = (int)new_verts;
    st[S_KSTOP] = kstop;
  }
  if (overflow) {
    if (!last) return false;
    if (lane == 0) {
      for (int q = S_TIES; q < S_COUNT; ++q) st[q] = 0;
      st[S_BAD] = 1;
      atomicAdd(&b.ctr[ctr_slot(C_OVERFLOW)], 1ull);  // counted here: the record sums run on demand
      if (HINTS) b.hint_n[i] = 0;
      b.vflag[i] = 0;
      b.kn_cnt[i] = 0;
      b.kt_cnt[i] = 0;
      b.ktr_cnt[i] = 0;
    }
    return true;
  }
  if (empty) nv = 0;
  if (lane >= nv) x0 = y0 = z0 = 0.0, p0 = 0u;
  if ((VC <= 64 || lane + 64 >= nv)) x1 = y1 = z1 = 0.0, p1 = 0u;

  // ---- 3. the star: K-tetrahedra (cell vertices in B_i), K-triangles (cell
  // edges meeting B_i), K-edges (facets meeting B_i)
  int ties = lane == 0 ? (int)exact_tests : 0;  // side tests decided exactly
  // |v|^2 - w_i is off by at most e (2 V + e) + rounding for a vertex off by e
  auto near_sphere = [&](double m, double t) {
    const double e = t * invPn;
    return !(fabs(m) > fma(e, 2.0 * Vv + e, 8.0 * kU * (Vv * Vv + wi)));
  };
  bool in0 = false, in1 = false, unsure = false;
  if (lane < nv) {
    const double m = x0 * x0 + y0 * y0 + z0 * z0 - wi;
    in0 = m <= 0.0 && pid0(p0) >= 6;
    unsure |= pid0(p0) >= 6 && near_sphere(m, t0);
  }
  if ((VC > 64 && lane + 64 < nv)) {
    const double m = x1 * x1 + y1 * y1 + z1 * z1 - wi;
    in1 = m <= 0.0 && pid0(p1) >= 6;
    unsure |= pid0(p1) >= 6 && near_sphere(m, t1);
  }
  // facets present
  for (int h = 0; h < 2; ++h) {
    const int v = lane + 64 * h;
    if (v < nv) {
      const unsigned p = h ? p1 : p0;
      const unsigned ids[3] = {pid0(p), pid1(p), pid2(p)};
      for (int c = 0; c < 3; ++c)
        if (ids[c] >= 6) sf_or(L, (int)ids[c] - 6, (unsigned)SF_FACET);
    }
  }
  __syncthreads();
  if constexpr (HINTS) {  // the cell for the next frame: facets in slot order, vertices
    int nf = 0;
    unsigned long long fm[(NBC + 63) / 64];
#pragma unroll
    for (int w = 0; w < (NBC + 63) / 64; ++w) {
      const int s = 64 * w + lane;
      const bool f = s < nn && (L.sf.b[s] & SF_FACET);
      fm[w] = __ballot(f);
      if (f) {
        const int at = nf + prefix_below(fm[w]);
        if (at < FAC_CAP) b.fac[(size_t)i * FAC_CAP + at] = L.idx[s];
      }
      nf += __popcll(fm[w]);
    }
    const bool keepv = nf <= FAC_CAP && nv <= FAC_CAP;
    if (keepv && lane < nv) {
      unsigned code = 0u;
      for (int c = 0; c < 3; ++c) {
        const unsigned pc = c == 0 ? pid0(p0) : (c == 1 ? pid1(p0) : pid2(p0));
        unsigned hc = pc;
        if (pc >= 6) {  // its position in the facet list
          const int sl = (int)pc - 6;
          int f = 0;
#pragma unroll
          for (int w = 0; w < (NBC + 63) / 64; ++w)
            if (64 * w + 64 <= sl) f += __popcll(fm[w]);
            else if (64 * w <= sl) f += __popcll(fm[w] & ((1ull << (sl - 64 * w)) - 1ull));
          hc = 6u + (unsigned)f;
        }
        code |= hc << (7 * c);
      }
      b.vtx[(size_t)i * FAC_CAP + lane] = code;
    }
    if (lane == 0) b.hint_n[i] = min(nf, FAC_CAP) | ((keepv ? nv : 0) << 8);
  }
  // cell edges: the two end vertices of an edge (a plane pair) meet in a small
  // LDS hash table keyed by the pair: the first to arrive claims an entry
  // (atomic compare-and-swap), the second finds it and leaves its slot there.
  // An edge is handled by its lower vertex; triangles are appended in a fixed
  // (vertex, pair) order so that the star is deterministic.
  unsigned* ht = L.u.cl.w.eh.key;
  unsigned char* ht2 = L.u.cl.w.eh.second;
  for (int q = lane; q < EH_SIZE; q += 64) ht[q] = 0xffffffffu, ht2[q] = 0xffu;
  __syncthreads();
  int partner[2][3] = {{-1, -1, -1}, {-1, -1, -1}};
  int claimed[2][3] = {{-1, -1, -1}, {-1, -1, -1}};
  for (int h = 0; h < 2; ++h) {
    const int v = lane + 64 * h;
    if (v >= nv) continue;
    const unsigned p = h ? p1 : p0;
    for (int c = 0; c < 3; ++c) {
      const unsigned code = c == 0 ? (pid1(p) | (pid2(p) << 10)) : c == 1 ? (pid0(p) | (pid2(p) << 10))
                                                                          : (pid0(p) | (pid1(p) << 10));
      const unsigned mine = (code << 7) | (unsigned)v;
      unsigned hsh = (code * 2654435761u) >> (32 - EH_BITS);
      for (int probe = 0; probe < EH_SIZE; ++probe) {
        const unsigned old = atomicCAS(&ht[hsh], 0xffffffffu, mine);
        if (old == 0xffffffffu) {
          claimed[h][c] = (int)hsh;
          break;
        }
        if ((old >> 7) == code) {
          partner[h][c] = (int)(old & 127u);
          ht2[hsh] = (unsigned char)v;
          break;
        }
        hsh = (hsh + 1) & (EH_SIZE - 1);
      }
    }
  }
  __syncthreads();
  for (int h = 0; h < 2; ++h)
    for (int c = 0; c < 3; ++c)
      if (claimed[h][c] >= 0) {
        const unsigned u = ht2[claimed[h][c]];
        partner[h][c] = u == 0xffu ? -1 : (int)u;
      }
  __syncthreads();  // the table's LDS is reused by the triangle list
  int ntri = 0;
  for (int h = 0; h < 2; ++h) {
    const int v = lane + 64 * h;
    const unsigned p = h ? p1 : p0;
    const double vx = h ? x1 : x0, vy = h ? y1 : y0, vz = h ? z1 : z0;
    const double vtt = h ? t1 : t0;
    const bool vin = h ? in1 : in0;
    for (int c = 0; c < 3; ++c) {
      const unsigned pa = c == 0 ? pid1(p) : pid0(p);
      const unsigned pb = c == 2 ? pid1(p) : pid2(p);
      const int u = partner[h][c];
      bool hit = false;
      unsigned word = 0;
      if (v < nv && u > v && pa >= 6 && pb >= 6) {
        const double ux = L.u.cl.vx[u], uy = L.u.cl.vy[u], uz = L.u.cl.vz[u];
        const unsigned pu = L.u.cl.vp[u];
        const double u2 = ux * ux + uy * uy + uz * uz;
        const bool uin = (u2 - wi <= 0.0) && pid0(pu) >= 6;
        // closest point of the segment to p_i
        const double dx = ux - vx, dy = uy - vy, dz = uz - vz;
        const double dd = dx * dx + dy * dy + dz * dz;
        double t = dd > 0.0 ? -(vx * dx + vy * dy + vz * dz) / dd : 0.0;
        t = fmin(fmax(t, 0.0), 1.0);
        const double qx = vx + t * dx, qy = vy + t * dy, qz = vz + t * dz;
        const double m = qx * qx + qy * qy + qz * qz - wi;
        // (the distance of a segment from p_i moves by at most the larger
        // displacement of its ends)
        unsure |= !vin && !uin && near_sphere(m, fmax(vtt, thr_value(L.u.cl.vt[u])));
        // an edge with an end vertex in B_i meets B_i (so that n_t and the
        // triangle's presence never disagree through rounding)
        if (m <= 0.0 || vin || uin) {
          hit = true;
          const unsigned nt = (unsigned)vin + (unsigned)uin;
          word = (pa - 6) | ((pb - 6) << 10) | (nt << 20);
          const unsigned f = SF_KTRI | (nt <= 1 ? SF_EXTTRI : 0u);
          sf_or(L, (int)pa - 6, f);
          sf_or(L, (int)pb - 6, f);
        }
      }
      const unsigned long long hm = __ballot(hit);
      if (hit) {
        const int at = ntri + prefix_below(hm);
        if (at < 2 * VC) L.u.cl.w.st.tri[at] = word;
      }
      ntri += __popcll(hm);
    }
  }
  ntri = min(ntri, 2 * VC);
  if constexpr (!EXACT) {
    if (__builtin_expect(__ballot(unsure) != 0ull, 0) && !last) return false;
  }
  __syncthreads();
  // facets without a K-triangle: K-edge iff the disk centre lies in the cell
  for (int s = lane; s < nn; s += 64) {
    unsigned f = L.sf.b[s];
    bool kedge = (f & SF_KTRI) != 0;
    if (!kedge && (f & SF_FACET)) {
      const Pl qs = slot_plane(L, b, pi, wi, s);
      const double nx = qs.x, ny = qs.y, nz = qs.z, nb = qs.b;
      const double sc = nb / (nx * nx + ny * ny + nz * nz);
      const double yx = sc * nx, yy = sc * ny, yz = sc * nz;
      const double se = yx * yx + yy * yy + yz * yz - wi;
      bool inside = se <= 0.0;
      for (int t = 0; t < nn && inside; ++t) {
        if (t == s) continue;
        const Pl qt = slot_plane(L, b, pi, wi, t);
        const double g = qt.b - (qt.x * yx + qt.y * yy + qt.z * yz);
        inside = g >= 0.0;
      }
      kedge = inside;
    }
    if (kedge) {
      f |= SF_KEDGE;
      if (!(f & SF_KTRI) || (f & SF_EXTTRI)) f |= SF_EXTEDGE;
    }
    L.sf.b[s] = (unsigned char)f;
  }
  // origin in the cell (used when there is no K-edge)
  bool origin_in = true;
  for (int s = lane; s < nn; s += 64) origin_in &= slot_plane(L, b, pi, wi, s).b >= 0.0;
  origin_in = __ballot(!origin_in) == 0ull;
  __syncthreads();
  // K-edges in slot order, then K-neighbour indices by ascending atom id
  int nk = 0;
  for (int base = 0; base < nn; base += 64) {
    const int s = base + lane;
    const bool ke = s < nn && (L.sf.b[s] & SF_KEDGE);
    const unsigned long long m = __ballot(ke);
    if (ke) {
      const int kk = nk + prefix_below(m);
      if (kk < KN_CAP) L.u.cl.w.st.kslot[kk] = s;
    }
    nk += __popcll(m);
  }
  __syncthreads();
  unsigned long long extmask = 0ull;
  if (lane < nk && lane < KN_CAP) {
    const int s = L.u.cl.w.st.kslot[lane];
    const int id = L.idx[s];
    int rank = 0;
    const int lim = min(nk, KN_CAP);
    for (int t = 0; t < lim; ++t) rank += L.idx[L.u.cl.w.st.kslot[t]] < id;
    L.kidx[s] = (signed char)rank;
    b.knbr[(size_t)i * KN_CAP + rank] = id;
    if (L.sf.b[s] & SF_EXTEDGE) extmask = 1ull << rank;
  }
  {
    unsigned lo = (unsigned)extmask, hi = (unsigned)(extmask >> 32);
    for (int off = 32; off > 0; off >>= 1) {
      lo |= (unsigned)__shfl_xor((int)lo, off, 64);
      hi |= (unsigned)__shfl_xor((int)hi, off, 64);
    }
    extmask = (unsigned long long)lo | ((unsigned long long)hi << 32);
  }
  const int next = __popcll(extmask);
  const bool inK = !empty && (nk > 0 || origin_in);
  const bool ext = inK && (nk == 0 || next > 0);
  __syncthreads();

  // orientation of each K-tetrahedron (i, a, b, c): the sign of det[n_a; n_b;
  // n_c] in plane-id order.  The angle terms take |det| as that sign times det,
  // which for a nearly flat tetrahedron fixes the branch of their derivatives
  // that rounding could flip; it is taken from the vertex's normals when their
  // rounding (relative u in n = 2 (p_j - p_i)) cannot reach it, else exactly
  // (the fast pass leaves such an atom to the second pass).
  int osg0 = 1, osg1 = 1;
  bool ounsure0 = false, ounsure1 = false;
  for (int h = 0; h < 2; ++h) {
    const bool vin = h ? in1 : in0;
    if (!vin) continue;
    const unsigned p = h ? p1 : p0;
    const Pl A = plane_of(L, b, pi, wi, pid0(p), half), B = plane_of(L, b, pi, wi, pid1(p), half),
             C = plane_of(L, b, pi, wi, pid2(p), half);
    const double d = A.x * (B.y * C.z - B.z * C.y) + A.y * (B.z * C.x - B.x * C.z) + A.z * (B.x * C.y - B.y * C.x);
    const double m = (fabs(A.x) + fabs(A.y) + fabs(A.z)) * (fabs(B.x) + fabs(B.y) + fabs(B.z)) *
                     (fabs(C.x) + fabs(C.y) + fabs(C.z));
    const bool sure = fabs(d) > 24.0 * kU * m;
    if (h) osg1 = d < 0.0 ? -1 : 1, ounsure1 = !sure;
    else osg0 = d < 0.0 ? -1 : 1, ounsure0 = !sure;
  }
  if (__builtin_expect(__ballot(ounsure0 || ounsure1) != 0ull, 0)) {
    if constexpr (!EXACT) {
      if (!last) return false;
    } else {
      for (int h = 0; h < 2; ++h) {
        bool u = h ? ounsure1 : ounsure0;
        if (u) {
          const int sg = dd_orient_at(b.pos, pi, half, L, h ? p1 : p0);
          if (sg != 0) {
            if (h) osg1 = sg;
            else osg0 = sg;
            u = false;
          }
        }
        unsigned long long um = __ballot(u);
        while (um) {
          const int l = __builtin_ctzll(um);
          um &= um - 1ull;
          const unsigned pv = (unsigned)__builtin_amdgcn_readlane((int)(h ? p1 : p0), l);
          int sg = 0;
          if (lane == 0) sg = exact_orient_at(b.pos, pi, half, L, *W, pv);
          sg = __shfl(sg, 0, 64);
          exact_fail |= sg == 2 || sg == 0;
          if (lane == l) {
            if (h) osg1 = sg < 0 ? -1 : 1;
            else osg0 = sg < 0 ? -1 : 1;
          }
        }
      }
    }
  }
  if (exact_fail) {  // an expansion outgrew its array: reported as a capacity overflow
    if (lane == 0) {
      st[S_BAD] = 1;
      atomicAdd(&b.ctr[ctr_slot(C_OVERFLOW)], 1ull);
      if (HINTS) b.hint_n[i] = 0;
      b.vflag[i] = 0;
      b.kn_cnt[i] = 0;
      b.kt_cnt[i] = 0;
      b.ktr_cnt[i] = 0;
    }
    return true;
  }
  // tetrahedra at i (cell vertices inside B_i)
  const unsigned long long tm0 = __ballot(in0), tm1 = __ballot(in1);
  const int ntet = __popcll(tm0) + __popcll(tm1);
  bool bad = nk > KN_CAP || ntet > KT_CAP;
  bool bad_lane = false;  // a cell vertex in B_i whose facets were not all found (broken star)
  int own_tet = 0;
  for (int h = 0; h < 2; ++h) {
    const bool vin = h ? in1 : in0;
    if (!vin) continue;
    const unsigned p = h ? p1 : p0;
    const int at = h ? __popcll(tm0) + prefix_below(tm1) : prefix_below(tm0);
    const int sa = (int)pid0(p) - 6, sb = (int)pid1(p) - 6, sc = (int)pid2(p) - 6;
    const int ka = L.kidx[sa], kb = L.kidx[sb], kc = L.kidx[sc];
    if (ka < 0 || kb < 0 || kc < 0 || ka >= KN_CAP || kb >= KN_CAP || kc >= KN_CAP) {
      bad_lane = true;
    } else if (at < KT_CAP) {  // K-neighbour indices ascending: the terms do not depend on the clipping order
      const unsigned k3 = pack3(ka, kb, kc);
      // orientation in that order: the plane-id order's, flipped by an odd sort
      const int inv = (ka > kb) + (ka > kc) + (kb > kc);
      const int osg = (h ? osg1 : osg0) * ((inv & 1) ? -1 : 1);
      b.ktet[(size_t)i * KT_CAP + at] =
          pid0(k3) | (pid1(k3) << 8) | (pid2(k3) << 16) | (osg < 0 ? (1u << 24) : 0u);
    }
    int ja = L.idx[sa], jb = L.idx[sb], jc = L.idx[sc];
    if (i < ja && i < jb && i < jc) {
      ++own_tet;
      if (b.export_on) {
        // ascending ids
        int t;
        if (ja > jb) t = ja, ja = jb, jb = t;
        if (jb > jc) t = jb, jb = jc, jc = t;
        if (ja > jb) t = ja, ja = jb, jb = t;
        const unsigned long long at2 = atomicAdd(&b.ctr[ctr_slot(C_EX_TET)], 1ull);
        if ((int64_t)at2 < b.ex_cap_q) {
          int* o = b.ex_tets + 4 * at2;
          o[0] = i, o[1] = ja, o[2] = jb, o[3] = jc;
        }
      }
    }
  }
  // triangles at i: exterior ones are kept, owned ones counted / exported
  int own_tri = 0, own_ext_tri = 0, next_tri = 0;
  for (int base = 0; base < ntri; base += 64) {
    const int r = base + lane;
    bool keep = false;
    unsigned word = 0;
    if (r < ntri) {
      const unsigned t = L.u.cl.w.st.tri[r];
      const int sa = (int)(t & 1023u), sb = (int)((t >> 10) & 1023u);
      const unsigned nt = t >> 20;
      const int ka = L.kidx[sa], kb = L.kidx[sb];
      keep = nt <= 1;
      if (ka < 0 || kb < 0 || ka >= KN_CAP || kb >= KN_CAP) bad_lane = true, keep = false;
      word = (unsigned)min(ka, kb) | ((unsigned)max(ka, kb) << 8) | (nt << 16);
      const int ja = L.idx[sa], jb = L.idx[sb];
      if (i < ja && i < jb) {
        ++own_tri;
        own_ext_tri += keep;
        if (b.export_on) {
          const unsigned long long at2 = atomicAdd(&b.ctr[ctr_slot(C_EX_TRI)], 1ull);
          if ((int64_t)at2 < b.ex_cap_t) {
            int* o = b.ex_tris + 3 * at2;
            o[0] = i, o[1] = min(ja, jb), o[2] = max(ja, jb);
            b.ex_ntet[at2] = (uint8_t)nt;
          }
        }
      }
    }
    const unsigned long long km = __ballot(keep);
    if (keep) {
      const int at = next_tri + prefix_below(km);
      if (at < KTR_CAP) b.ktri[(size_t)i * KTR_CAP + at] = word;
    }
    next_tri += __popcll(km);
  }
  bad |= next_tri > KTR_CAP;
  bad |= __ballot(bad_lane) != 0ull;
  // owned edges
  int own_edge = 0, own_ext_edge = 0;
  for (int s = lane; s < nn; s += 64) {
    const unsigned f = L.sf.b[s];
    if ((f & SF_KEDGE) && i < L.idx[s]) {
      ++own_edge;
      own_ext_edge += (f & SF_EXTEDGE) != 0;
      if (b.export_on) {
        const unsigned long long at2 = atomicAdd(&b.ctr[ctr_slot(C_EX_EDGE)], 1ull);
        if ((int64_t)at2 < b.ex_cap_e) {
          b.ex_edges[2 * at2] = i;
          b.ex_edges[2 * at2 + 1] = L.idx[s];
        }
      }
    }
  }
  // wave sums
  for (int off = 32; off > 0; off >>= 1) {
    own_tet += __shfl_xor(own_tet, off, 64);
    own_tri += __shfl_xor(own_tri, off, 64);
    own_ext_tri += __shfl_xor(own_ext_tri, off, 64);
    own_edge += __shfl_xor(own_edge, off, 64);
    own_ext_edge += __shfl_xor(own_ext_edge, off, 64);
    ties += __shfl_xor(ties, off, 64);
  }
  if (lane == 0) {
    if (bad) {
      b.vflag[i] = 0;
      b.kn_cnt[i] = 0;
      b.kt_cnt[i] = 0;
      b.ktr_cnt[i] = 0;
    } else {
      b.vflag[i] = (inK ? VF_IN : 0) | (ext ? VF_EXT : 0);
      b.kn_cnt[i] = nk;
      b.kn_ext[i] = extmask;
      b.kt_cnt[i] = ntet;
      b.ktr_cnt[i] = next_tri;
    }
    st[S_TIES] = ties;
    st[S_BAD] = (bad ? 1 : 0) | (reused ? 2 : 0);
    if (bad) atomicAdd(&b.ctr[ctr_slot(C_OVERFLOW)], 1ull);
    st[S_VERT] = inK ? 1 : 0;
    st[S_EXTV] = ext ? 1 : 0;
    st[S_TET] = own_tet;
    st[S_TRI] = own_tri;
    st[S_EXTTRI] = own_ext_tri;
    st[S_EDGE] = own_edge;
    st[S_EXTEDGE] = own_ext_edge;
  }
  return true;
}

// Fast pass over all atoms with LDS sized for 20 wavefronts per CU (planes of
// the 128 nearest neighbours in LDS, cells of up to 64 vertices); the rare
// atoms whose cell grows past 64 vertices are queued for the wide pass.
// HINTS: a trajectory's calls (the previous frame's cells are kept).
constexpr int V_FAST = 64, NPL_FAST = 128;

template <bool HINTS>
__global__ __launch_bounds__(64, 5) void k_star(Bufs b) {
  __shared__ StarLds<NB_CAP, V_FAST, NPL_FAST> L;
  if ((int)blockIdx.x >= b.n) return;
  if (b.dirty) {
    // incremental call: an atom whose star cannot have changed keeps it (and
    // its record's sizes and simplex counts); the work counts become zero
    const int i = b.sorted[blockIdx.x];
    if (!b.dirty[i]) {
      if (threadIdx.x == 0) {
        int* st = b.stat + (size_t)i * STAT_STRIDE;
        st[S_VMAX] = 0;
        st[S_CAND] = 0;
        st[S_TESTS] = 0;
        st[S_NEWV] = 0;
        st[S_TIES] = 0;
        st[S_BAD] = 4;
        st[S_KSTOP] = 0;
      }
      return;
    }
  }
  if (!star_atom<HINTS, false>(b, L, blockIdx.x, false, nullptr) && threadIdx.x == 0) {
    const unsigned long long q = atomicAdd(&b.ctr[ctr_slot(C_WIDE)], 1ull);
    b.wide[q] = (int)blockIdx.x;
  }
}

// Second pass: the queued atoms (cells past 64 vertices, or a side test
// within its rounding bound), with the full capacities and exact side tests,
// a fixed grid looping over the queue (it returns at once when the queue is
// empty).  The exact work space is in LDS, used by one lane at a time.
constexpr int WIDE_BLOCKS = 64;

template <bool HINTS>
__global__ __launch_bounds__(64) void k_star_wide(Bufs b) {
  __shared__ StarLds<NB_CAP_WIDE, V_CAP, NB_CAP_WIDE> L;
  __shared__ exact::Work W;
  const int cnt = (int)b.ctr[ctr_slot(C_WIDE)];
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    __syncthreads();
    star_atom<HINTS, true>(b, L, b.wide[q], true, &W);
  }
}

// ------------------------------------------------------------------ stats
// Sums (maxima for the sizes) of the star kernel's per-atom records into the
// counters: one atom per thread (a record is four int4 loads), a block folds
// its 256 records and one thread per counter issues the block's atomic.  It
// runs when the counts are asked for, after the call that wrote the records.
constexpr int STATS_T = 256;

__device__ inline int stat_counter(int q) {
  switch (q) {
    case S_NN: return C_MAX_NB;
    case S_VMAX: return C_MAX_V;
    case S_CAND: return C_CANDIDATES;
    case S_TESTS: return C_PLANE_TESTS;
    case S_NEWV: return C_NEW_VERTS;
    case S_TIES: return C_NEAR_TIE;
    case S_BAD: return C_OVERFLOW;
    case S_VERT: return C_VERT;
    case S_EXTV: return C_EXT_VERT;
    case S_TET: return C_TET;
    case S_TRI: return C_TRI;
    case S_EXTTRI: return C_EXT_TRI;
    case S_EDGE: return C_EDGE;
    case S_KSTOP: return C_PLANES_USED;
    default: return C_EXT_EDGE;
  }
}

__global__ __launch_bounds__(STATS_T) void k_stats(Bufs b) {
  static_assert(STAT_STRIDE == 16 && S_COUNT < 16, "a record is four int4 with one spare slot");
  constexpr int S_KMAX = 15;  // spare slot: the largest S_KSTOP of the block
  constexpr int S_KGT = 16;   // extra slot: atoms that visited more than 64 planes
  constexpr int S_REUSE = 17;  // extra slot: atoms that kept their previous-frame cell
  constexpr int S_SKIP = 18;   // extra slot: atoms that kept their previous call's star
  constexpr int NV = 19;
  __shared__ int part[STATS_T / 64][NV];
  const int a = blockIdx.x * STATS_T + threadIdx.x;
  int v[NV];
  if (a < b.n) {
    const int4* r = (const int4*)(b.stat + (size_t)a * STAT_STRIDE);
    for (int c = 0; c < 4; ++c) {
      const int4 t = r[c];
      v[4 * c] = t.x, v[4 * c + 1] = t.y, v[4 * c + 2] = t.z, v[4 * c + 3] = t.w;
    }
  } else {
    for (int q = 0; q < 16; ++q) v[q] = 0;
  }
  v[S_KMAX] = v[S_KSTOP];
  v[S_KGT] = v[S_KSTOP] > 64 ? 1 : 0;
  v[S_REUSE] = (v[S_BAD] >> 1) & 1;
  v[S_SKIP] = (v[S_BAD] >> 2) & 1;
  v[S_BAD] &= 1;
  auto is_max = [](int q) { return q == S_NN || q == S_VMAX || q == S_KMAX; };
  for (int q = 0; q < NV; ++q)
    for (int off = 32; off > 0; off >>= 1) {
      const int o = __shfl_xor(v[q], off, 64);
      v[q] = is_max(q) ? max(v[q], o) : v[q] + o;
    }
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < NV; ++q) part[threadIdx.x >> 6][q] = v[q];
  __syncthreads();
  // (capacity failures are counted by the star kernel itself)
  if (threadIdx.x < NV && threadIdx.x != S_BAD && (threadIdx.x < S_COUNT || threadIdx.x >= S_KMAX)) {
    const int q = threadIdx.x;
    long long t = part[0][q];
    for (int w = 1; w < STATS_T / 64; ++w) t = is_max(q) ? max(t, (long long)part[w][q]) : t + part[w][q];
    const int ctr = q == S_KMAX   ? C_MAX_PLANES
                    : q == S_KGT  ? C_PLANES_GT64
                    : q == S_REUSE ? C_REUSED
                    : q == S_SKIP ? C_SKIPPED
                                  : stat_counter(q);
    if (is_max(q)) atomicMax(&b.ctr[ctr_slot(ctr)], (unsigned long long)t);
    else if (t) atomicAdd(&b.ctr[ctr_slot(ctr)], (unsigned long long)t);
  }
}

// ------------------------------------------------------------------ terms
template <typename T>
struct V3 {
  T x, y, z;
};
template <typename T>
__device__ inline V3<T> operator+(V3<T> a, V3<T> b) {
  return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename T>
__device__ inline V3<T> operator-(V3<T> a, V3<T> b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename T>
__device__ inline V3<T> operator*(V3<T> a, T s) {
  return {a.x * s, a.y * s, a.z * s};
}
template <typename T>
__device__ inline T dot(V3<T> a, V3<T> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ inline V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ inline T norm(V3<T> a) {
  return sqrt(dot(a, a));
}

template <typename T>
__device__ inline V3<double> dbl3(V3<T> a) {
  return {(double)a.x, (double)a.y, (double)a.z};
}

__device__ inline float tatan2(float y, float x) { return atan2f(y, x); }
__device__ inline double tatan2(double y, double x) { return atan2(y, x); }

// Normalised solid angle at the origin of the tetrahedron (0, a, b, c) (Van
// Oosterom--Strackee, atan2 form) and its gradient with respect to a, b, c.
// osg (if not 0) is the sign of det[a; b; c], known exactly: |a.(b x c)| is then
// taken as osg a.(b x c), which for a nearly flat tetrahedron keeps the
// derivative on the branch of its true orientation.
template <typename T>
__device__ T solid_angle(V3<T> a, V3<T> b, V3<T> c, V3<T>* ga, V3<T>* gb, V3<T>* gc, bool grad, int osg = 0) {
  const T la = norm(a), lb = norm(b), lc = norm(c);
  const V3<T> bxc = cross(b, c);
  const T tp = dot(a, bxc);
  const T N = osg ? T(osg) * tp : fabs(tp);
  const T ab = dot(a, b), ac = dot(a, c), bc = dot(b, c);
  const T D = la * lb * lc + ab * lc + ac * lb + bc * la;
  const T inv2pi = T(1.0 / (2.0 * kPi));
  const T om = tatan2(N, D) * inv2pi;
  if (grad) {
    const T k = inv2pi / (N * N + D * D);
    const T dN = D * k * (osg ? T(osg) : (tp >= T(0) ? T(1) : T(-1)));
    const T dD = -N * k;
    *ga = cross(b, c) * dN + (a * ((lb * lc + bc) / la) + b * lc + c * lb) * dD;
    *gb = cross(c, a) * dN + (b * ((la * lc + ac) / lb) + a * lc + c * la) * dD;
    *gc = cross(a, b) * dN + (c * ((la * lb + ab) / lc) + a * lb + b * la) * dD;
  }
  return om;
}

// Normalised dihedral angle along the edge (0, e) between the faces (0, e, u)
// and (0, e, v), and its gradient with respect to e, u, v.  The wing
// gradients are normal to their faces; the edge end takes the lever share
// that keeps the angle invariant under translation and rotation.  With osg
// (if not 0) the sign of det[e; u; v], known exactly, |n_k x n_l| is taken as
// osg |e| det[e; u; v] (n_k x n_l = det[e; u; v] e) and the wings' side from it.
// The face normals e x u, e x v and det[e; u; v] are formed in double from
// double inputs in both precisions: for a wing nearly along the edge they are
// small differences of large products, and the gradient divides by |n|^2, so
// in float they would carry an error of u_f / sin^2 of the wing's angle.
template <typename T>
__device__ T dihedral(V3<double> ed, V3<double> ud, V3<double> vd, V3<T>* ge, V3<T>* gu, V3<T>* gv, bool grad,
                      int osg = 0) {
  const V3<double> nkd = cross(ed, ud), nld = cross(ed, vd);
  const V3<T> e = {T(ed.x), T(ed.y), T(ed.z)}, u = {T(ud.x), T(ud.y), T(ud.z)}, v = {T(vd.x), T(vd.y), T(vd.z)};
  const V3<T> nk = {T(nkd.x), T(nkd.y), T(nkd.z)}, nl = {T(nld.x), T(nld.y), T(nld.z)};
  const T inv2pi = T(1.0 / (2.0 * kPi));
  const T num = osg ? T(osg) * norm(e) * T(dot(nkd, vd)) : norm(cross(nk, nl));
  const T ph = tatan2(num, dot(nk, nl)) * inv2pi;
  if (grad) {
    const T le2 = dot(e, e), le = sqrt(le2);
    const T sg = osg ? T(osg) : (dot(nk, v) >= T(0) ? T(1) : T(-1));
    *gu = nk * (-sg * le / dot(nk, nk) * inv2pi);
    *gv = nl * (sg * le / dot(nl, nl) * inv2pi);
    const T tu = dot(u, e) / le2, tv = dot(v, e) / le2;
    *ge = (*gu) * (-tu) + (*gv) * (-tv);
  }
  return ph;
}

// Cap of sphere i (centre at the origin, radius R) inside ball (a, Ra):
// S = 2 pi R h, h = R - (d^2 + R^2 - Ra^2) / (2d); gradient with respect to a.
template <typename T>
__device__ T cap_area(V3<T> a, T R, T Ra, V3<T>* g, bool grad) {
  const T d = norm(a);
  const T dw = R * R - Ra * Ra;
  const T h = R - (d * d + dw) / (T(2) * d);
  if (grad) *g = a * (T(-2.0 * kPi) * R * (T(0.5) - dw / (T(2) * d * d)) / d);
  return T(2.0 * kPi) * R * h;
}

// Crease weight of the circle where sphere i (radius R, centre at the origin)
// meets sphere a (centre a, radius Ra): W = (pi / 2) rho gamma, rho the
// circle's radius and gamma the angle between the two spheres' outward normals
// along it (sin gamma = d rho / (R Ra), cos gamma = (R^2 + Ra^2 - d^2) /
// (2 R Ra)), and its gradient with respect to a.  The integrated mean
// curvature of the surface has, besides the spheres' A_i / R_i, the part
// -1/4 L gamma of each exposed crease arc of length L = rho theta per atom;
// with theta / 2 pi = Phi - sum_t c_t 2 phi(T_x) (the exposed share of the
// circle, as the volume kernel uses it) that part is the Eq. 1 edge and
// triangle sums with W in place of the cap areas and no vertex term.  With
// dgamma/dd = 1 / rho, dW/dd = (pi / 2) (gamma drho/dd + 1).
__device__ inline double crease_weight(V3<double> a, double R, double Ra, V3<double>* g, bool grad) {
  const double d2 = dot(a, a), d = sqrt(d2), w = R * R, wa = Ra * Ra;
  const double h = (d2 + w - wa) / (2.0 * d);
  const double rho = sqrt(fmax(w - h * h, 0.0));
  const double gam = atan2(d * rho, 0.5 * (w + wa - d2));
  if (grad) {
    const double dh = 0.5 * (1.0 - (w - wa) / d2);
    const double drho = rho > 0.0 ? -h * dh / rho : 0.0;
    *g = a * (0.5 * kPi * (gam * drho + 1.0) / d);
  }
  return 0.5 * kPi * rho * gam;
}

// Edge weight of the terms: the cap area (the area, Eq. 1), or the crease
// weight (CR: the mean curvature's crease part).
template <bool CR>
__device__ inline double edge_weight(V3<double> a, double R, double Ra, V3<double>* g, bool grad) {
  if constexpr (CR) return crease_weight(a, R, Ra, g, grad);
  else return cap_area<double>(a, R, Ra, g, grad);
}

struct TermsLds {
  double px[KN_CAP], py[KN_CAP], pz[KN_CAP], pR[KN_CAP];
  unsigned tet[KT_CAP];
  unsigned tri[KTR_CAP];
  double S[KN_CAP];                 // cap areas of exterior edges
  union {
    struct {
      double phi[64][3];    // dihedral fractions along (i,a), (i,b), (i,c) of one chunk of tetrahedra
      double tg[64][3][3];  // their contributions to a, b, c
    } t;
    double rg[64][2][3];    // contributions of one chunk of triangles to a, b
  } c;
};

template <typename T>
__device__ inline V3<T> ld(const TermsLds& L, int k) {
  return {T(L.px[k]), T(L.py[k]), T(L.pz[k])};
}

// One K-tetrahedron (i, a, b, c) at atom i (i at the origin): the solid angle
// at i, the three dihedral fractions along (i,a), (i,b), (i,c), and -- with
// grad -- its contributions to dA_i/dp for a, b, c: -4 pi w_i d(omega) from the
// vertex term and +S_e d(phi_e) for each exterior edge e at i (Eqs. 3, 5).
template <typename T>
__device__ double tet_item(const TermsLds& L, const int ks[3], int osg, unsigned long long extm, double Si, bool grad,
                           double phi[3], double acc_out[3][3]) {
  const V3<double> PD[3] = {ld<double>(L, ks[0]), ld<double>(L, ks[1]), ld<double>(L, ks[2])};
  // The vertex term 4 pi w_i omega is the largest single term and cancels
  // against its neighbours' for nearly buried atoms: its solid angle is always
  // evaluated in double, and every contribution is summed in double.
  V3<double> g[3], acc[3];
  const double om = solid_angle<double>(PD[0], PD[1], PD[2], &g[0], &g[1], &g[2], grad, osg);
  for (int c = 0; c < 3; ++c) acc[c] = g[c] * (-Si);
  for (int c = 0; c < 3; ++c) {
    const int o1 = (c + 1) % 3, o2 = (c + 2) % 3;
    V3<T> ge, g1, g2;
    const T ph = dihedral<T>(PD[c], PD[o1], PD[o2], &ge, &g1, &g2, grad, osg);  // cyclic: same orientation
    phi[c] = (double)ph;
    if (grad && ((extm >> ks[c]) & 1ull)) {
      const double Se = L.S[ks[c]];
      acc[c] = acc[c] + dbl3(ge) * Se;
      acc[o1] = acc[o1] + dbl3(g1) * Se;
      acc[o2] = acc[o2] + dbl3(g2) * Se;
    }
  }
  if (grad)
    for (int c = 0; c < 3; ++c) acc_out[c][0] = acc[c].x, acc_out[c][1] = acc[c].y, acc_out[c][2] = acc[c].z;
  return om;
}

// One exterior K-triangle (i, a, b) at atom i, Eq. 6: S/2 = phi_ia(T_x) S_ia +
// phi_ib(T_x) S_ib - omega_i(T_x) 4 pi w_i with T_x = (p_i, p_a, p_b, x); its
// gradient (Eq. 7) includes the chain rule through the triple point x, whose
// derivative follows from |x - p_m|^2 = w_m:  M dx = [(x - p_m) . dp_m]_m with
// rows of M = (x - p_m)^T, so dS/dp_m += lambda_m (x - p_m), M^T lambda = dS/dx.
template <typename T, bool CR = false>
__device__ double tri_item(const TermsLds& L, int ka, int kb, double X0, double X1, double X2, double Ri,
                           double Si, bool grad, double G[2][3]) {
  V3<T> g1e, g1u, g1v, g2e, g2u, g2v;
  // caps in double: they multiply the angles' derivatives, and a buried atom's
  // area is the small difference of many of them
  V3<double> gSa, gSb;
  const double Sa = edge_weight<CR>(ld<double>(L, ka), Ri, L.pR[ka], &gSa, grad);
  const double Sb = edge_weight<CR>(ld<double>(L, kb), Ri, L.pR[kb], &gSb, grad);
  const V3<double> AD = ld<double>(L, ka), BD = ld<double>(L, kb), XD = {X0, X1, X2};
  const T ph1 = dihedral<T>(AD, BD, XD, &g1e, &g1u, &g1v, grad);  // along (i,a)
  const T ph2 = dihedral<T>(BD, AD, XD, &g2e, &g2u, &g2v, grad);  // along (i,b)
  // solid angle in double, as in tet_item
  V3<double> hwa, hwb, hwx;
  const double om = solid_angle<double>(ld<double>(L, ka), ld<double>(L, kb), V3<double>{X0, X1, X2}, &hwa, &hwb,
                                        &hwx, grad);
  const double p1 = (double)ph1, p2 = (double)ph2;
  const double St = 2.0 * (p1 * Sa + p2 * Sb - om * Si);
  if (grad) {
    // the angles' derivatives in T; the caps, the sums, the solid angle's
    // share and the chain rule through x in double (M^-T amplifies rounding)
    V3<double> dA = dbl3(g1e) * Sa + gSa * p1 + dbl3(g2u) * Sb - hwa * Si;
    V3<double> dB = dbl3(g1u) * Sa + dbl3(g2e) * Sb + gSb * p2 - hwb * Si;
    const V3<double> dX = dbl3(g1v) * Sa + dbl3(g2v) * Sb - hwx * Si;
    const V3<double> Xd = {X0, X1, X2};
    const V3<double> r0 = Xd, r1 = Xd - ld<double>(L, ka), r2 = Xd - ld<double>(L, kb);
    const V3<double> c0 = cross(r1, r2), c1 = cross(r2, r0), c2 = cross(r0, r1);
    const double idet = 1.0 / dot(r0, c0);
    const double l1 = dot(c1, dX) * idet, l2 = dot(c2, dX) * idet;
    dA = dA + r1 * l1;
    dB = dB + r2 * l2;
    G[0][0] = 2.0 * dA.x, G[0][1] = 2.0 * dA.y, G[0][2] = 2.0 * dA.z;
    G[1][0] = 2.0 * dB.x, G[1][1] = 2.0 * dB.y, G[1][2] = 2.0 * dB.z;
  }
  return St;
}

// Conditioning of a tetrahedron seen from the origin, |a.(b x c)| / (|a||b||c|),
// small for slivers, whose angle derivatives lose accuracy in float: true when
// it is below q (compared squared, without a root or a division).
__device__ inline bool tet_below(double ax, double ay, double az, double bx, double by, double bz, double cx,
                                 double cy, double cz, double q) {
  const double tp = ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
  const double l2 = (ax * ax + ay * ay + az * az) * (bx * bx + by * by + bz * bz) * (cx * cx + cy * cy + cz * cz);
  return tp * tp < q * q * l2;
}

// In MIXED precision, items below these qualities are evaluated in double.
// With the face normals formed in double (dihedral), what float still loses on
// a sliver is the rounding of the wing vectors themselves, relative u_f /
// sin theta; the quality bounds sin theta from below.  Largest gradient error
// on a drifted 20,000-atom MD frame (bar 1e-4): 2.9e-5 at a bound of 0.2
// (5.7e-5 with the normals in float), 4.6e-5 at 0.05, 5.0e-5 at 0.01 and
// 2.6e-4 with no item promoted; large probes (larger caps) reached 1.01e-4 at
// 0.01, so 0.2 is kept.  One item below the bound puts its wavefront's whole
// chunk of 64 items in double: with item-wise promotion the wavefront ran both
// paths whenever one lane needed double, which was nearly always, and FP64
// runs at the FP32 rate on this GPU, so the double path costs no more than the
// float one (terms of the 5,000-atom globule 38.9 -> 33.3 us, and the errors
// only fall).
constexpr double kTetQualityMin = 0.2;
constexpr double kTripleDepthMin = 0.1;  // -s_t / w_i: triple points close to the centres' plane

// CR: the crease part of the integrated mean curvature instead of the area
// (edge weights W, no vertex term; b.area receives the per-atom part).
template <typename T, bool CR = false>
__global__ __launch_bounds__(64) void k_terms(Bufs b, int with_grad) {
  __shared__ TermsLds L;
  if ((int)blockIdx.x >= b.n) return;
  if (b.status && blockIdx.x == 0 && threadIdx.x == 0) {
    // the call's error counts are final here (cells and stars are done): the
    // host reads them after its wait instead of copying the counters back
    b.status[0] = b.ctr[ctr_slot(C_BAD_INPUT)];
    b.status[1] = b.ctr[ctr_slot(C_OVERFLOW)];
    b.status[2] = 1ull;
  }
  const int i = b.sorted[blockIdx.x];  // cell order, as in k_star
  const int lane = threadIdx.x;
  if (b.dirty && !b.dirty[i]) {  // incremental call: star kept, so are its area and blocks
    if (lane == 0) b.area[i] = b.area_keep[i];
    return;
  }
  const uint8_t vf = b.vflag[i];
  if (!(vf & VF_EXT)) {
    if (lane == 0) {
      b.area[i] = 0.0;
      if (b.area_keep) b.area_keep[i] = 0.0;
    }
    return;
  }
  const bool grad = with_grad != 0;
  const double4 pi = b.pos[i];
  const double Ri = pi.w, wi = Ri * Ri;
  const int nk = b.kn_cnt[i], nt = b.kt_cnt[i], nr = b.ktr_cnt[i];
  const unsigned long long extm = b.kn_ext[i];
  for (int k = lane; k < nk; k += 64) {
    const double4 pj = b.pos[b.knbr[(size_t)i * KN_CAP + k]];
    L.px[k] = pj.x - pi.x;
    L.py[k] = pj.y - pi.y;
    L.pz[k] = pj.z - pi.z;
    L.pR[k] = pj.w;
  }
  for (int t = lane; t < nt; t += 64) L.tet[t] = b.ktet[(size_t)i * KT_CAP + t];
  for (int t = lane; t < nr; t += 64) L.tri[t] = b.ktri[(size_t)i * KTR_CAP + t];
  __syncthreads();
  const double Si = CR ? 0.0 : 4.0 * kPi * wi;
  // edges: cap areas, in double in both precisions (they multiply the
  // dihedral angles and their derivatives, and a buried atom's area is the
  // small difference of many of them)
  V3<double> gS = {0.0, 0.0, 0.0};
  double Sk = 0.0;
  const int k = lane;  // one K-neighbour per lane (KN_CAP = 64)
  const bool kext = k < nk && ((extm >> k) & 1ull);
  if (kext) {
    Sk = edge_weight<CR>(ld<double>(L, k), Ri, L.pR[k], &gS, grad);
    L.S[k] = Sk;
  }
  __syncthreads();
  // tetrahedra, in chunks of 64 (one per lane): solid angle at i, dihedral
  // angles along the three edges at i and their gradient contributions; after
  // each chunk, lane k adds the entries that touch K-neighbour k, in order
  double omega_sum = 0.0, phi_sum = 0.0;
  double gx = 0.0, gy = 0.0, gz = 0.0;  // gradient block of K-neighbour k
  for (int c0 = 0; c0 < nt; c0 += 64) {
    const int t = c0 + lane;
    if (t < nt) {
      const unsigned w = L.tet[t];
      const int ks[3] = {(int)(w & 255u), (int)((w >> 8) & 255u), (int)((w >> 16) & 255u)};
      if (ks[0] >= nk || ks[1] >= nk || ks[2] >= nk) {  // never produced by k_star; keeps LDS reads in range
        L.c.t.phi[lane][0] = L.c.t.phi[lane][1] = L.c.t.phi[lane][2] = 0.0;
        for (int c = 0; c < 3; ++c) L.c.t.tg[lane][c][0] = L.c.t.tg[lane][c][1] = L.c.t.tg[lane][c][2] = 0.0;
      } else {
        bool dbl = sizeof(T) == sizeof(double);
        if (!dbl)  // one poorly shaped tetrahedron puts the wave's whole chunk in double (see below)
          dbl = __ballot(tet_below(L.px[ks[0]], L.py[ks[0]], L.pz[ks[0]], L.px[ks[1]], L.py[ks[1]], L.pz[ks[1]],
                                   L.px[ks[2]], L.py[ks[2]], L.pz[ks[2]], kTetQualityMin)) != 0ull;
        double ph[3];
        const int osg = (w >> 24) & 1u ? -1 : 1;  // orientation of (i, ks[0], ks[1], ks[2]), decided exactly
        const double om = dbl ? tet_item<double>(L, ks, osg, extm, Si, grad, ph, L.c.t.tg[lane])
                              : tet_item<T>(L, ks, osg, extm, Si, grad, ph, L.c.t.tg[lane]);
        omega_sum += om;
        L.c.t.phi[lane][0] = ph[0], L.c.t.phi[lane][1] = ph[1], L.c.t.phi[lane][2] = ph[2];
      }
    }
    __syncthreads();
    if (k < nk) {
      const int lim = min(64, nt - c0);
      for (int q = 0; q < lim; ++q) {
        const unsigned w = L.tet[c0 + q];
        const int a = (int)(w & 255u), bb = (int)((w >> 8) & 255u), c = (int)((w >> 16) & 255u);
        const int pos = a == k ? 0 : bb == k ? 1 : c == k ? 2 : -1;
        if (pos < 0) continue;
        phi_sum += L.c.t.phi[q][pos];
        if (grad) gx += L.c.t.tg[q][pos][0], gy += L.c.t.tg[q][pos][1], gz += L.c.t.tg[q][pos][2];
      }
    }
    __syncthreads();
  }
  // edges: outer dihedral coefficient Phi = 1 - sum of the K-tet dihedral fractions
  double area_part = 0.0;
  if (kext) {
    const double Phi = 1.0 - phi_sum;
    area_part -= Phi * Sk;
    gx -= Phi * gS.x;
    gy -= Phi * gS.y;
    gz -= Phi * gS.z;
  }
  // exterior triangles: Eq. 6 through the triple point, in chunks of 64
  for (int c0 = 0; c0 < nr; c0 += 64) {
    const int r = c0 + lane;
    if (r < nr) {
      const unsigned w = L.tri[r];
      const int ka = (int)(w & 255u), kb = (int)((w >> 8) & 255u);
      double St = 0.0;
      double G[2][3] = {{0, 0, 0}, {0, 0, 0}};
      double ct = 0.0;
      if (ka < nk && kb < nk) {  // always true for k_star's output; keeps LDS reads in range
        ct = 1.0 - 0.5 * (double)(w >> 16);
        // triple point in double: y in the plane of the centres, x = y + sqrt(-s) n
        const double ax = L.px[ka], ay = L.py[ka], az = L.pz[ka];
        const double bx = L.px[kb], by = L.py[kb], bz = L.pz[kb];
        const double wa = L.pR[ka] * L.pR[ka], wb = L.pR[kb] * L.pR[kb];
        const double aa = ax * ax + ay * ay + az * az, bb2 = bx * bx + by * by + bz * bz,
                     ab = ax * bx + ay * by + az * bz;
        const double ra = aa - wa + wi, rb = bb2 - wb + wi;
        const double det = 2.0 * (aa * bb2 - ab * ab);
        const double al = (ra * bb2 - rb * ab) / det, be = (aa * rb - ab * ra) / det;
        const double yx = al * ax + be * bx, yy = al * ay + be * by, yz = al * az + be * bz;
        const double s = yx * yx + yy * yy + yz * yz - wi;
        if (s < 0.0) {
          const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
          const double f = sqrt(-s / (nx * nx + ny * ny + nz * nz));
          const double X0 = yx + f * nx, X1 = yy + f * ny, X2 = yz + f * nz;
          bool dbl = sizeof(T) == sizeof(double);
          if (!dbl)
            dbl = __ballot((-s < kTripleDepthMin * wi) ||
                           tet_below(ax, ay, az, bx, by, bz, X0, X1, X2, kTetQualityMin)) != 0ull;
          St = dbl ? tri_item<double, CR>(L, ka, kb, X0, X1, X2, Ri, Si, grad, G)
                   : tri_item<T, CR>(L, ka, kb, X0, X1, X2, Ri, Si, grad, G);
        }
      }
      area_part += ct * St;
      if (grad)
        for (int c = 0; c < 3; ++c) L.c.rg[lane][0][c] = ct * G[0][c], L.c.rg[lane][1][c] = ct * G[1][c];
    }
    if (!grad) continue;
    __syncthreads();
    if (k < nk) {
      const int lim = min(64, nr - c0);
      for (int q = 0; q < lim; ++q) {
        const unsigned w = L.tri[c0 + q];
        const int a = (int)(w & 255u), bb = (int)((w >> 8) & 255u);
        const int pos = a == k ? 0 : bb == k ? 1 : -1;
        if (pos >= 0) gx += L.c.rg[q][pos][0], gy += L.c.rg[q][pos][1], gz += L.c.rg[q][pos][2];
      }
    }
    __syncthreads();
  }
  // area: Omega_i 4 pi w_i - sum Phi S + sum c S_t  (deterministic butterfly sums)
  double os = omega_sum, ap = area_part;
  for (int off = 32; off > 0; off >>= 1) {
    os += __shfl_xor(os, off, 64);
    ap += __shfl_xor(ap, off, 64);
  }
  if (lane == 0) {
    const double a = (1.0 - os) * Si + ap;
    b.area[i] = a;
    if (b.area_keep) b.area_keep[i] = a;
  }
  if (!grad) return;
  // gradient block of K-neighbour k: edge + tetrahedra + triangles containing k
  if (k < nk) {
    double* row = b.rows + ((size_t)i * ROW + k) * 3;
    row[0] = gx, row[1] = gy, row[2] = gz;
  } else {
    gx = gy = gz = 0.0;
  }
  // the atom's own block: every term is translation invariant
  for (int off = 32; off > 0; off >>= 1) {
    gx += __shfl_xor(gx, off, 64);
    gy += __shfl_xor(gy, off, 64);
    gz += __shfl_xor(gz, off, 64);
  }
  if (lane == 0) {
    double* row = b.rows + ((size_t)i * ROW + KN_CAP) * 3;
    row[0] = -gx, row[1] = -gy, row[2] = -gz;
  }
}

// ------------------------------------------------------------------ gather
// 16 lanes per receiving atom m (4 atoms per wavefront): lane l takes the
// K-neighbours l, l + 16, ... of m, finds m among each neighbour i's sorted
// K-neighbours and adds u_i dA_i/dp_m; a fixed xor tree sums the 16 partials,
// so the result does not depend on scheduling.  The search compares 16 entries
// of i's list at a time, loaded together with i's flag and count (the rows are
// KN_CAP entries wide and 16-byte aligned), so that finding m takes one memory
// round trip for lists of up to 16 entries instead of a chain of dependent loads.
__device__ inline double sum16(double v) {
  for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// the slot of m among entries [c, c + 16) of a K-list of nk entries, or s
__device__ inline int find16(const int4 (&q)[4], int m, int c, int nk, int s) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int j = c + 4 * e;
    if (q[e].x == m && j < nk) s = j;
    if (q[e].y == m && j + 1 < nk) s = j + 1;
    if (q[e].z == m && j + 2 < nk) s = j + 2;
    if (q[e].w == m && j + 3 < nk) s = j + 3;
  }
  return s;
}

__global__ __launch_bounds__(64) void k_gather(Bufs b, const double* u, double* out, double scale, int accumulate) {
  const int sub = threadIdx.x & 15;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 4);
  double gx = 0, gy = 0, gz = 0;
  int lost = 0;
  if (m < b.n) {
    if (sub == 0 && (b.vflag[m] & VF_EXT)) {
      const double um = u ? u[m] : 1.0;
      const double* row = b.rows + ((size_t)m * ROW + KN_CAP) * 3;
      gx = um * row[0], gy = um * row[1], gz = um * row[2];
    }
    const int nk = b.kn_cnt[m];
    for (int k = sub; k < nk; k += 16) {
      const int i = b.knbr[(size_t)m * KN_CAP + k];
      const int4* li = reinterpret_cast<const int4*>(b.knbr + (size_t)i * KN_CAP);
      const uint8_t fl = b.vflag[i];
      const int nki = b.kn_cnt[i];
      int4 q[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) q[e] = li[e];
      if (!(fl & VF_EXT)) continue;
      int s = find16(q, m, 0, nki, -1);
      for (int c = 16; s < 0 && c < nki; c += 16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) q[e] = li[c / 4 + e];
        s = find16(q, m, c, nki, s);
      }
      if (s < 0) {
        ++lost;
        continue;
      }
      const double ui = u ? u[i] : 1.0;
      const double* row = b.rows + ((size_t)i * ROW + s) * 3;
      gx += ui * row[0], gy += ui * row[1], gz += ui * row[2];
    }
  }
  gx = sum16(gx);
  gy = sum16(gy);
  gz = sum16(gz);
  for (int off = 8; off > 0; off >>= 1) lost += __shfl_xor(lost, off, 64);
  if (m < b.n && sub == 0) {
    if (accumulate) {
      out[3 * m] += scale * gx;
      out[3 * m + 1] += scale * gy;
      out[3 * m + 2] += scale * gz;
    } else {
      out[3 * m] = scale * gx;
      out[3 * m + 1] = scale * gy;
      out[3 * m + 2] = scale * gz;
    }
    if (lost) atomicAdd(&b.ctr[ctr_slot(C_LOST_PAIR)], (unsigned long long)lost);
  }
}

// out[i] = u[i] / R_i (u = NULL: 1 / R_i): the weights that turn the area
// VJP into that of sum_i u_i A_i / R_i.
__global__ void k_recip_radius(Bufs b, const double* u, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < b.n) out[i] = (u ? u[i] : 1.0) / b.pos[i].w;
}

__global__ void k_zero(unsigned* p, size_t words) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < words) p[k] = 0u;
}

inline unsigned blocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int scan_blocks(unsigned hb) { return (int)((hb + SCAN_E - 1) / SCAN_E); }

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  if (words) k_zero<<<blocks(words, 256), 256, 0, s>>>((unsigned*)p, words);
}
void launch_prep(const Bufs& b, hipStream_t s) {
  if (b.n) k_prep<<<blocks(b.n, PREP_T), PREP_T, 0, s>>>(b);
}
void launch_grid(const Bufs& b, hipStream_t s) {
  if (b.n) k_grid<<<1, 1024, 0, s>>>(b);
}
void launch_count(const Bufs& b, hipStream_t s) {
  if (b.n) k_count<<<blocks(b.n, 256), 256, 0, s>>>(b);
}
void launch_scan(const Bufs& b, hipStream_t s) {
  const int hb = b.cell_cap;
  const int nb = scan_blocks((unsigned)hb);
  k_scan1<<<nb, SCAN_T, 0, s>>>(b.cnt, b.start, b.scan_tmp, hb);
  k_scan2<<<1, SCAN_T, 0, s>>>(b.scan_tmp, nb, b.start, hb);
  k_scan3<<<blocks(hb, 256), 256, 0, s>>>(b.start, b.scan_tmp, hb);
}
void launch_scatter(const Bufs& b, hipStream_t s) {
  if (b.n) k_scatter<<<blocks(b.n, 256), 256, 0, s>>>(b);
}
void launch_cells_one(const Bufs& b, hipStream_t s) {
  if (!b.n) return;
  static_assert(ONE_BLOCK_MAX_ATOMS <= 8 * ONE_T, "one block holds its atoms in registers");
  if (b.n <= 512) k_cells_one<2, 256><<<1, 256, 0, s>>>(b);
  else if (b.n <= ONE_T) k_cells_one<1, ONE_T><<<1, ONE_T, 0, s>>>(b);
  else if (b.n <= 2 * ONE_T) k_cells_one<2, ONE_T><<<1, ONE_T, 0, s>>>(b);
  else if (b.n <= 5 * ONE_T) k_cells_one<5, ONE_T><<<1, ONE_T, 0, s>>>(b);
  else k_cells_one<8, ONE_T><<<1, ONE_T, 0, s>>>(b);
}
void launch_star(const Bufs& b, hipStream_t s) {
  if (!b.n) return;
  if (b.fac) k_star<true><<<b.n, 64, 0, s>>>(b);
  else k_star<false><<<b.n, 64, 0, s>>>(b);
}
void launch_star_wide(const Bufs& b, hipStream_t s) {
  if (!b.n) return;
  if (b.fac) k_star_wide<true><<<min(b.n, WIDE_BLOCKS), 64, 0, s>>>(b);
  else k_star_wide<false><<<min(b.n, WIDE_BLOCKS), 64, 0, s>>>(b);
}
void launch_stats(const Bufs& b, hipStream_t s) {
  if (b.n) k_stats<<<blocks(b.n, STATS_T), STATS_T, 0, s>>>(b);
}
void launch_terms(const Bufs& b, int precision, int with_grad, hipStream_t s) {
  if (!b.n) return;
  if (precision == 1) k_terms<float><<<b.n, 64, 0, s>>>(b, with_grad);
  else k_terms<double><<<b.n, 64, 0, s>>>(b, with_grad);
}
void launch_gather(const Bufs& b, const double* u, double* out, double scale, hipStream_t s, int accumulate) {
  if (b.n) k_gather<<<blocks(b.n, 4), 64, 0, s>>>(b, u, out, scale, accumulate);
}
void launch_terms_crease(const Bufs& b, int with_grad, hipStream_t s) {
  if (b.n) k_terms<double, true><<<b.n, 64, 0, s>>>(b, with_grad);
}
void launch_recip_radius(const Bufs& b, const double* u, double* out, hipStream_t s) {
  if (b.n) k_recip_radius<<<blocks(b.n, 256), 256, 0, s>>>(b, u, out);
}

}  // namespace sasa
