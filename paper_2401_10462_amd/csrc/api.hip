// api.hip -- host side of the C-ABI declared in include/sasa.h.
//
// A context owns its device buffers (grown on demand, never shrunk), a small
// pinned block for the device counters, and the complex kept from its last
// compute.  All work of a call is enqueued on the caller's stream; synchronous
// calls end with one stream synchronisation that also brings the counters
// (errors, capacity, diagnostics) back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sasa.h"
#include "sasa_internal.h"

using namespace sasa;

// The context behind the C-ABI's opaque handle.
struct sasa_context {
  int device = 0;
  int precision = SASA_FP64;
  uint32_t flags = 0;
  int64_t cap_n = 0;
  int64_t cap_cells = 0;
  int cap_mol = 0;
  Bufs b;                 // device pointers (capacity-sized)
  double* xyz_d = nullptr;  // staging of host inputs
  double* rad_d = nullptr;
  double* area_d = nullptr;
  double* out_d = nullptr;  // n*3
  double* u_d = nullptr;
  int64_t* off_d = nullptr;
  int64_t* off_h = nullptr;  // pinned
  unsigned long long* ctr_h = nullptr;  // pinned copy of the counters
  unsigned long long* status_h = nullptr;  // pinned words the terms kernel of a compute writes (Bufs::status)
  unsigned long long* status_d = nullptr;  // ... their device address
  // export buffers
  int64_t ex_cap_e = 0, ex_cap_t = 0, ex_cap_q = 0;
  // kept state
  bool kept = false;
  int64_t n = 0;
  int nmol = 0;
  double probe = 0;
  bool pending = false;  // an async call whose counters were not read yet
  bool stats_due = false;  // the star records of the last compute are not summed into the counters yet
  hipStream_t last_stream = nullptr;  // stream of the last call (pending counters are read there)
  hipEvent_t ev[6] = {};  // stage boundaries (SASA_FLAG_TIMING)
  bool timed = false;     // events of the last call were recorded
  int64_t fac_atoms = -1;  // atom count of the call that wrote the facet hints (-1: none)
  SortedFaces sf;           // buffers of the sorted-face extraction (grown on demand)
  int64_t sf_cap_faces = -1, sf_cap_free = -1;
  SortedEV se, sv;          // the same for unique edges and vertices
  // SASA_FLAG_INCREMENTAL: buffers (capacity-sized) and whether the last call
  // left stars, areas (and, with inc_grad, gradient blocks) of every atom that
  // the next call of the same system may keep
  double4* prev_d = nullptr;
  int* mv_id_d = nullptr;
  double4* mv_old_d = nullptr;
  uint8_t* dirty_d = nullptr;
  double* area_keep_d = nullptr;
  bool inc_valid = false;
  bool inc_grad = false;
  sasa_diag diag{};
  std::string err;
};

namespace {

using Ctx = sasa_context;

thread_local std::string g_err;

// Largest batch: keeps every cell and scan index in 32 bits (16 n + 64 cells).
constexpr int64_t kMaxAtoms = 100000000;

int fail(Ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      return fail(ctx, e_ == hipErrorOutOfMemory ? SASA_E_NOMEM : SASA_E_DEVICE,        \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    }                                                                                   \
  } while (0)

// Allocation failure injection for the tests of the capacity bookkeeping:
// with SASA_TEST_FAIL_ALLOC=k in the environment, the k-th buffer allocation
// from then on (counted per process) reports out-of-memory without calling
// the allocator.
bool injected_alloc_failure() {
  static long counter = 0;
  const char* v = std::getenv("SASA_TEST_FAIL_ALLOC");
  if (!v || !*v) {
    counter = 0;
    return false;
  }
  return ++counter == std::atol(v);
}

template <typename T>
hipError_t grow(T** p, size_t count) {
  if (*p) {
    hipError_t e = hipFree(*p);
    *p = nullptr;
    if (e != hipSuccess) return e;
  }
  if (count && injected_alloc_failure()) return hipErrorOutOfMemory;
  return count ? hipMalloc((void**)p, count * sizeof(T)) : hipSuccess;
}

// Each group of buffers records its capacity only once all of them exist: a
// grow frees a buffer before allocating its replacement, so the capacity is
// zeroed first, and an allocation that fails part-way leaves 0 behind and the
// next call grows the whole group again (never writing through a freed or
// missing buffer).
constexpr int64_t kPresizedMolecules = 8192;

int ensure(Ctx* c, int64_t n, int nmol) {
  Bufs& b = c->b;
  if (n > c->cap_n) {
    const int64_t cap = std::max<int64_t>(n, c->cap_n + c->cap_n / 2);
    c->cap_n = 0;
    HIP_TRY(c, grow(&b.pos, cap));
    HIP_TRY(c, grow(&b.mol, cap));
    HIP_TRY(c, grow(&b.cellid, cap));
    HIP_TRY(c, grow(&b.sorted, cap));
    HIP_TRY(c, grow(&b.spos, cap));
    HIP_TRY(c, grow(&b.smc, cap));
    HIP_TRY(c, grow(&b.vflag, cap));
    HIP_TRY(c, grow(&b.stat, cap * STAT_STRIDE));
    HIP_TRY(c, grow(&b.wide, cap));
    HIP_TRY(c, grow(&b.kn_cnt, cap));
    HIP_TRY(c, grow(&b.knbr, cap * KN_CAP));
    HIP_TRY(c, grow(&b.kn_ext, cap));
    HIP_TRY(c, grow(&b.kt_cnt, cap));
    HIP_TRY(c, grow(&b.ktet, cap * KT_CAP));
    HIP_TRY(c, grow(&b.ktr_cnt, cap));
    HIP_TRY(c, grow(&b.ktri, cap * KTR_CAP));
    HIP_TRY(c, grow(&c->area_d, cap));
    HIP_TRY(c, grow(&b.rows, cap * ROW * 3));
    HIP_TRY(c, grow(&c->xyz_d, cap * 3));
    HIP_TRY(c, grow(&c->rad_d, cap));
    HIP_TRY(c, grow(&c->out_d, cap * 3));
    HIP_TRY(c, grow(&c->u_d, cap));
    if (c->flags & SASA_FLAG_FRAMES) {
      HIP_TRY(c, grow(&b.fac, cap * FAC_CAP));
      HIP_TRY(c, grow(&b.vtx, cap * FAC_CAP));
      HIP_TRY(c, grow(&b.hint_n, cap));
    }
    c->inc_valid = false;
    if (c->flags & SASA_FLAG_INCREMENTAL) {
      HIP_TRY(c, grow(&c->prev_d, cap));
      HIP_TRY(c, grow(&c->mv_id_d, cap));
      HIP_TRY(c, grow(&c->mv_old_d, cap));
      HIP_TRY(c, grow(&c->dirty_d, cap));
      HIP_TRY(c, grow(&c->area_keep_d, cap));
    }
    c->fac_atoms = -1;
    c->cap_n = cap;
  }
  const int64_t cells = cell_capacity(n);
  if (cells > c->cap_cells) {
    const int64_t cap = std::max<int64_t>(cells, c->cap_cells + c->cap_cells / 2);
    c->cap_cells = 0;
    HIP_TRY(c, grow(&b.cnt, cap));
    HIP_TRY(c, grow(&b.start, (size_t)cap + 1));
    HIP_TRY(c, grow(&b.scan_tmp, (size_t)scan_blocks((unsigned)cap) + 1));
    c->cap_cells = cap;
  }
  b.cell_cap = (int)cells;
  if (nmol + 1 > c->cap_mol) {
    const int cap = std::max(nmol + 1, 2 * c->cap_mol);
    c->cap_mol = 0;
    HIP_TRY(c, grow(&c->off_d, cap));
    HIP_TRY(c, grow(&b.mol_box, (size_t)cap * 6));
    HIP_TRY(c, grow(&b.mol_geo, cap));
    HIP_TRY(c, grow(&b.mol_dim, cap));
    if (c->off_h) HIP_TRY(c, hipHostFree(c->off_h));
    c->off_h = nullptr;
    HIP_TRY(c, hipHostMalloc((void**)&c->off_h, cap * sizeof(int64_t)));
    c->cap_mol = cap;
  }
  return SASA_OK;
}

bool host_inputs_ok(int64_t n, const double* xyz, const double* radii) {
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return false;
  for (int64_t i = 0; i < n; ++i)
    if (!(radii[i] > 0.0) || !std::isfinite(radii[i])) return false;
  return true;
}

// Stage times of the last call (SASA_FLAG_TIMING), once its stream is done.
void read_times(Ctx* c) {
  if (!c->timed) return;
  c->timed = false;
  float ms[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < 5; ++k)
    if (hipEventElapsedTime(&ms[k], c->ev[k], c->ev[k + 1]) != hipSuccess) ms[k] = -1.0f;
  c->diag.ms_cells = ms[0];
  c->diag.ms_star = ms[1];
  c->diag.ms_star_wide = ms[2];
  c->diag.ms_terms = ms[3];
  c->diag.ms_gather = ms[4];
}

int check_errors(Ctx* c, unsigned long long bad_input, unsigned long long overflow) {
  if (bad_input || overflow) c->inc_valid = false;
  if (bad_input) {
    c->kept = false;
    return fail(c, SASA_E_INVAL,
                "NaN/Inf coordinate, radius <= 0, or two atoms with the same centre and radius in the input");
  }
  if (overflow) {
    c->kept = false;
    return fail(c, SASA_E_CAPACITY, "an atom exceeds the per-atom neighbour / cell-vertex / star capacity");
  }
  return SASA_OK;
}

// Waits for the stream of the last call and reports its errors.  full: copies
// all counters back (diagnostics, complex counts); otherwise only the error
// counts that the call's terms kernel wrote to pinned host memory are read
// (a compute with no atoms has none).
int read_counters(Ctx* c, hipStream_t s, bool full = true) {
  if (!full) {
    HIP_TRY(c, hipStreamSynchronize(s));
    c->pending = false;
    const volatile unsigned long long* st = c->status_h;
    if (c->n > 0 && st[2] != 1ull) return fail(c, SASA_E_DEVICE, "the call's status words were not written");
    const unsigned long long bad_input = c->n > 0 ? st[0] : 0ull, overflow = c->n > 0 ? st[1] : 0ull;
    c->diag.input_errors = (int64_t)bad_input;
    c->diag.overflow = (int64_t)overflow;
    read_times(c);
    return check_errors(c, bad_input, overflow);
  }
  HIP_TRY(c, hipMemcpyAsync(c->ctr_h, c->b.ctr, CTR_BYTES, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->pending = false;
  const unsigned long long* h = c->ctr_h;
  c->diag.max_neighbours = (int64_t)h[ctr_slot(C_MAX_NB)];
  c->diag.max_cell_vertices = (int64_t)h[ctr_slot(C_MAX_V)];
  c->diag.near_ties = (int64_t)h[ctr_slot(C_NEAR_TIE)];
  c->diag.lost_pairs = (int64_t)h[ctr_slot(C_LOST_PAIR)];
  c->diag.input_errors = (int64_t)h[ctr_slot(C_BAD_INPUT)];
  c->diag.overflow = (int64_t)h[ctr_slot(C_OVERFLOW)];
  c->diag.plane_tests = (int64_t)h[ctr_slot(C_PLANE_TESTS)];
  c->diag.new_vertices = (int64_t)h[ctr_slot(C_NEW_VERTS)];
  c->diag.candidates = (int64_t)h[ctr_slot(C_CANDIDATES)];
  c->diag.planes_used = (int64_t)h[ctr_slot(C_PLANES_USED)];
  c->diag.max_planes_used = (int64_t)h[ctr_slot(C_MAX_PLANES)];
  c->diag.atoms_over_64_planes = (int64_t)h[ctr_slot(C_PLANES_GT64)];
  c->diag.reused_cells = (int64_t)h[ctr_slot(C_REUSED)];
  c->diag.second_pass_atoms = (int64_t)h[ctr_slot(C_WIDE)];
  c->diag.moved_atoms = (int64_t)h[ctr_slot(C_MOVED)];
  c->diag.skipped_atoms = (int64_t)h[ctr_slot(C_SKIPPED)];
  read_times(c);
  return check_errors(c, h[ctr_slot(C_BAD_INPUT)], h[ctr_slot(C_OVERFLOW)]);
}

// The star kernel's per-atom records of the last compute, summed into the
// counters when they are asked for (diagnostics, complex counts) rather than
// by a launch in every call.  Capacity failures are counted by the star kernel
// itself and were reported by the compute; only a HIP error is returned here.
int sum_stats(Ctx* c) {
  if (!c->stats_due) return SASA_OK;
  c->stats_due = false;
  Bufs b = c->b;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  HIP_TRY(c, hipSetDevice(c->device));
  launch_stats(b, c->last_stream);
  HIP_TRY(c, hipGetLastError());
  const int rc = read_counters(c, c->last_stream);
  return rc == SASA_E_DEVICE ? rc : SASA_OK;
}

int run(Ctx* c, int nmol, const int64_t* offsets, const double* xyz, const double* radii, double probe,
        double* area, double* dA_dx, int mem, hipStream_t s, double scale = 1.0) {
  const auto t0 = std::chrono::steady_clock::now();
  if (nmol < 0 || !offsets) return fail(c, SASA_E_INVAL, "nmol < 0 or offsets == NULL");
  if (!(probe >= 0.0) || !std::isfinite(probe)) return fail(c, SASA_E_INVAL, "probe must be finite and >= 0");
  if (mem != SASA_MEM_HOST && mem != SASA_MEM_DEVICE) return fail(c, SASA_E_INVAL, "bad mem");
  if (offsets[0] != 0) return fail(c, SASA_E_INVAL, "offsets[0] must be 0");
  for (int k = 0; k < nmol; ++k)
    if (offsets[k + 1] < offsets[k]) return fail(c, SASA_E_INVAL, "offsets must be non-decreasing");
  const int64_t n = offsets[nmol];
  if (n > kMaxAtoms) return fail(c, SASA_E_INVAL, "too many atoms (at most 100,000,000 per call)");
  if (n > 0 && (!xyz || !radii)) return fail(c, SASA_E_INVAL, "xyz / radii must not be NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  if (c->pending) {
    int rc = read_counters(c, c->last_stream, false);
    (void)rc;
  }
  c->kept = false;
  c->stats_due = false;  // the buffers may be reallocated below
  // an incremental call keeps what the previous call of the same system left
  // (checked before anything of this call can fail; set again once it is enqueued)
  const bool inc = (c->flags & SASA_FLAG_INCREMENTAL) && nmol == 1 && n > 0;
  bool inc_keep = inc && c->inc_valid && c->n == n && c->nmol == 1 && c->probe == probe;
  c->inc_valid = false;
  if (mem == SASA_MEM_HOST && n > 0 && !host_inputs_ok(n, xyz, radii))
    return fail(c, SASA_E_INVAL, "NaN/Inf coordinate or radius <= 0 in the input");
  int rc = ensure(c, n, nmol);
  if (rc) return rc;
  Bufs b = c->b;
  b.n = (int)n;
  b.nmol = std::max(nmol, 1);
  b.probe = probe;
  b.export_on = 0;
  // the single-block cell list of a one-molecule call never reads the offsets
  const bool one_block = nmol <= 1 && n <= ONE_BLOCK_MAX_ATOMS;
  if (!one_block) {
    std::memcpy(c->off_h, offsets, (size_t)(nmol + 1) * sizeof(int64_t));
    if (nmol == 0) c->off_h[1] = 0;
    HIP_TRY(c, hipMemcpyAsync(c->off_d, c->off_h, (size_t)(b.nmol + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  }
  b.offsets = c->off_d;
  if (mem == SASA_MEM_HOST) {
    if (n) {
      HIP_TRY(c, hipMemcpyAsync(c->xyz_d, xyz, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_TRY(c, hipMemcpyAsync(c->rad_d, radii, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    }
    b.xyz = c->xyz_d;
    b.radii = c->rad_d;
  } else {
    b.xyz = xyz;
    b.radii = radii;
  }
  b.area = (mem == SASA_MEM_DEVICE && area) ? area : c->area_d;
  double* out = (mem == SASA_MEM_DEVICE && dA_dx) ? dA_dx : c->out_d;
  const bool timing = (c->flags & SASA_FLAG_TIMING) != 0;
  b.status = c->status_d;
  c->status_h[0] = c->status_h[1] = c->status_h[2] = 0ull;  // no kernel of this context is in flight
  if (timing) HIP_TRY(c, hipEventRecord(c->ev[0], s));
  if (b.fac && c->fac_atoms != n) {  // hints of another system: start without
    if (n) launch_zero(b.hint_n, (size_t)n * sizeof(int), s);
    c->fac_atoms = n;
  }
  if (one_block) {
    launch_cells_one(b, s);  // also clears the counters
    if (!n) launch_zero(b.ctr, CTR_BYTES, s);
  } else {
    launch_zero(b.ctr, CTR_BYTES, s);
    launch_zero(b.cnt, (size_t)b.cell_cap * sizeof(int), s);
    launch_zero(b.mol_box, (size_t)b.nmol * 6 * sizeof(unsigned long long), s);
    launch_prep(b, s);
    launch_grid(b, s);
    launch_count(b, s);
    launch_scan(b, s);
    launch_scatter(b, s);
  }
  if (inc) {
    // atoms that moved since the previous call, and the stars they can reach
    b.prev = c->prev_d;
    b.mv_id = c->mv_id_d;
    b.mv_old = c->mv_old_d;
    b.dirty = c->dirty_d;
    b.area_keep = c->area_keep_d;
    launch_moved(b, inc_keep, s);
    if (inc_keep) launch_mark(b, s);
    else b.dirty = nullptr;  // every star is rebuilt
  }
  if (timing) HIP_TRY(c, hipEventRecord(c->ev[1], s));
  launch_star(b, s);
  if (timing) HIP_TRY(c, hipEventRecord(c->ev[2], s));
  launch_star_wide(b, s);
  if (timing) HIP_TRY(c, hipEventRecord(c->ev[3], s));
  {
    // kept stars keep their area, and their gradient blocks when the previous
    // call wrote them too (the context's precision never changes)
    Bufs bt = b;
    if (c->inc_grad != (dA_dx != nullptr)) bt.dirty = nullptr;
    launch_terms(bt, c->precision, dA_dx != nullptr, s);
  }
  if (timing) HIP_TRY(c, hipEventRecord(c->ev[4], s));
  if (dA_dx) launch_gather(b, nullptr, out, scale, s);
  if (timing) HIP_TRY(c, hipEventRecord(c->ev[5], s));
  c->timed = timing;
  c->stats_due = true;
  HIP_TRY(c, hipGetLastError());
  if (mem == SASA_MEM_HOST && n) {
    if (area) HIP_TRY(c, hipMemcpyAsync(area, b.area, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    if (dA_dx) HIP_TRY(c, hipMemcpyAsync(dA_dx, out, (size_t)n * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  c->n = n;
  c->nmol = nmol;
  c->probe = probe;
  c->diag.n_atoms = n;
  c->diag.n_mol = nmol;
  const bool async = (c->flags & SASA_FLAG_ASYNC) && mem == SASA_MEM_DEVICE;
  c->kept = true;
  c->inc_valid = inc;  // cleared again if the call reports an error
  c->inc_grad = dA_dx != nullptr;
  c->last_stream = s;
  if (async) {
    c->pending = true;
    return SASA_OK;
  }
  rc = read_counters(c, s, false);
  c->diag.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

// Sorts m tuples of K atom ids (row-major) lexicographically, carrying one
// byte per tuple along (if given).
template <int K>
void sort_tuples(int32_t* ids, uint8_t* tag, int64_t m) {
  std::vector<int64_t> ord((size_t)m);
  for (int64_t k = 0; k < m; ++k) ord[(size_t)k] = k;
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(ids + a * K, ids + a * K + K, ids + b * K, ids + b * K + K);
  });
  std::vector<int32_t> t(ids, ids + m * K);
  std::vector<uint8_t> g;
  if (tag) g.assign(tag, tag + m);
  for (int64_t k = 0; k < m; ++k) {
    std::memcpy(ids + k * K, t.data() + ord[(size_t)k] * K, K * sizeof(int32_t));
    if (tag) tag[k] = g[(size_t)ord[(size_t)k]];
  }
}

}  // namespace

extern "C" {

int sasa_create(const sasa_options* opt, sasa_context** ctx_out) {
  if (!ctx_out) return fail(nullptr, SASA_E_INVAL, "ctx_out == NULL");
  *ctx_out = nullptr;
  auto* c = new (std::nothrow) Ctx;
  if (!c) return fail(nullptr, SASA_E_NOMEM, "host allocation failed");
  if (opt) {
    c->device = opt->device;
    c->precision = opt->precision;
    c->flags = opt->flags;
    if (c->precision != SASA_FP64 && c->precision != SASA_MIXED) {
      delete c;
      return fail(nullptr, SASA_E_INVAL, "precision must be SASA_FP64 or SASA_MIXED");
    }
    constexpr uint32_t kKnownFlags = SASA_FLAG_ASYNC | SASA_FLAG_TIMING | SASA_FLAG_FRAMES | SASA_FLAG_INCREMENTAL;
    if ((opt->flags & ~kKnownFlags) || opt->reserved) {
      delete c;
      return fail(nullptr, SASA_E_INVAL, "unknown flag bits or non-zero reserved field in sasa_options");
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev) {
    delete c;
    return fail(nullptr, SASA_E_DEVICE, "no such HIP device");
  }
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipMalloc((void**)&c->b.ctr, CTR_BYTES);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->ctr_h, CTR_BYTES);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->status_h, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->status_d, c->status_h, 0);
  if (e != hipSuccess) {
    sasa_destroy(c);
    return fail(nullptr, SASA_E_DEVICE, std::string("context set-up: ") + hipGetErrorString(e));
  }
  std::memset(c->ctr_h, 0, CTR_BYTES);
  std::memset(c->status_h, 0, 4 * sizeof(unsigned long long));
  if (c->flags & SASA_FLAG_TIMING)
    for (auto& ev : c->ev)
      if (hipEventCreate(&ev) != hipSuccess) {
        sasa_destroy(c);
        return fail(nullptr, SASA_E_DEVICE, "hipEventCreate failed");
      }
  if (opt && opt->max_atoms > 0) {
    // the per-molecule arrays too, for batches of up to min(max_atoms, 8,192)
    // molecules: growing them later frees pinned and device memory, which
    // waits for the device (tens of milliseconds inside a serving loop)
    int rc = ensure(c, opt->max_atoms, (int)std::min<int64_t>(opt->max_atoms, kPresizedMolecules));
    if (rc) {
      sasa_destroy(c);
      return rc;
    }
  }
  *ctx_out = c;
  return SASA_OK;
}

void sasa_destroy(sasa_context* ctx) {
  Ctx* c = ctx;
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  Bufs& b = c->b;
  void* dev[] = {b.pos,  b.mol,   b.cellid,   b.cnt,      b.start,  b.scan_tmp, b.sorted, b.spos, b.smc,
                 b.mol_box, b.mol_geo, b.mol_dim, b.vflag, b.stat, b.wide, b.kn_cnt, b.knbr, b.kn_ext, b.kt_cnt, b.ktet, b.ktr_cnt,
                 b.ktri, b.rows,  b.ctr,      b.ex_edges, b.ex_tris, b.ex_ntet, b.ex_tets, b.fac, b.vtx, b.hint_n,
                 c->sf.faces, c->sf.sorted, c->sf.uniq, c->sf.counts, c->sf.nruns, c->sf.free_tris, c->sf.cursors,
                 c->sf.tris, c->sf.ntet, c->sf.temp, c->xyz_d, c->prev_d, c->mv_id_d, c->mv_old_d, c->dirty_d,
                 c->area_keep_d,
                 c->rad_d, c->area_d, c->out_d, c->u_d, c->off_d};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  for (SortedEV* w : {&c->se, &c->sv}) {
    void* ev[] = {w->keys, w->vals, w->skeys, w->svals, w->uniq, w->agg, w->nuniq, w->cursor, w->out_ids, w->out_ext,
                  w->temp};
    for (void* p : ev)
      if (p) (void)hipFree(p);
  }
  if (c->off_h) (void)hipHostFree(c->off_h);
  for (auto& ev : c->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->ctr_h) (void)hipHostFree(c->ctr_h);
  if (c->status_h) (void)hipHostFree(c->status_h);
  delete c;
}

int sasa_compute(sasa_context* ctx, int64_t n, const double* xyz, const double* radii, double probe, double* area,
                 double* dA_dx, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (n < 0) return fail(c, SASA_E_INVAL, "n < 0");
  const int64_t off[2] = {0, n};
  return run(c, 1, off, xyz, radii, probe, area, dA_dx, mem, (hipStream_t)hip_stream);
}

int sasa_compute_batch(sasa_context* ctx, int32_t nmol, const int64_t* offsets, const double* xyz, const double* radii,
                       double probe, double* area, double* dA_dx, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  return run(c, nmol, offsets, xyz, radii, probe, area, dA_dx, mem, (hipStream_t)hip_stream);
}

int sasa_compute_forces(sasa_context* ctx, int64_t n, const double* xyz, const double* radii, double probe, double gamma,
                        double* area, double* forces, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (n < 0) return fail(c, SASA_E_INVAL, "n < 0");
  if (!std::isfinite(gamma)) return fail(c, SASA_E_INVAL, "gamma must be finite");
  if (n > 0 && !forces) return fail(c, SASA_E_INVAL, "forces must not be NULL");
  const int64_t off[2] = {0, n};
  return run(c, 1, off, xyz, radii, probe, area, forces, mem, (hipStream_t)hip_stream, -gamma);
}

int sasa_backward(sasa_context* ctx, const double* dL_dA, double* dL_dx, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (!c->kept) return fail(c, SASA_E_STATE, "no kept compute on this context");
  if (mem != SASA_MEM_HOST && mem != SASA_MEM_DEVICE) return fail(c, SASA_E_INVAL, "bad mem");
  if (c->n > 0 && (!dL_dA || !dL_dx)) return fail(c, SASA_E_INVAL, "dL_dA / dL_dx must not be NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(c, hipSetDevice(c->device));
  Bufs b = c->b;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  b.area = c->area_d;
  const double* u = dL_dA;
  double* out = dL_dx;
  if (mem == SASA_MEM_HOST && c->n) {
    HIP_TRY(c, hipMemcpyAsync(c->u_d, dL_dA, (size_t)c->n * sizeof(double), hipMemcpyHostToDevice, s));
    u = c->u_d;
    out = c->out_d;
  }
  launch_terms(b, c->precision, 1, s);
  launch_gather(b, u, out, 1.0, s);
  HIP_TRY(c, hipGetLastError());
  if (mem == SASA_MEM_HOST && c->n) {
    HIP_TRY(c, hipMemcpyAsync(dL_dx, out, (size_t)c->n * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  } else if (!(c->flags & SASA_FLAG_ASYNC)) {
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return SASA_OK;
}

int sasa_volume(sasa_context* ctx, double* volume, double* dV_dx, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (!c->kept) return fail(c, SASA_E_STATE, "no kept compute on this context");
  if (mem != SASA_MEM_HOST && mem != SASA_MEM_DEVICE) return fail(c, SASA_E_INVAL, "bad mem");
  if (c->n > 0 && (!volume || !dV_dx)) return fail(c, SASA_E_INVAL, "volume / dV_dx must not be NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(c, hipSetDevice(c->device));
  Bufs b = c->b;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  b.area = c->area_d;  // the areas again, in FP64, for R_i A_i
  double* vol = volume;
  double* grad = dV_dx;
  if (mem == SASA_MEM_HOST) {
    vol = c->u_d;
    grad = c->out_d;
  }
  launch_terms(b, SASA_FP64, 0, s);
  launch_volume(b, vol, grad, s);
  HIP_TRY(c, hipGetLastError());
  if (mem == SASA_MEM_HOST && c->n) {
    HIP_TRY(c, hipMemcpyAsync(volume, vol, (size_t)c->n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(dV_dx, grad, (size_t)c->n * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  } else if (!(c->flags & SASA_FLAG_ASYNC)) {
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return SASA_OK;
}

int sasa_volume_backward(sasa_context* ctx, const double* dL_dV, double* dL_dx, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (!c->kept) return fail(c, SASA_E_STATE, "no kept compute on this context");
  if (mem != SASA_MEM_HOST && mem != SASA_MEM_DEVICE) return fail(c, SASA_E_INVAL, "bad mem");
  if (c->n > 0 && (!dL_dV || !dL_dx)) return fail(c, SASA_E_INVAL, "dL_dV / dL_dx must not be NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(c, hipSetDevice(c->device));
  Bufs b = c->b;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  const double* u = dL_dV;
  double* out = dL_dx;
  if (mem == SASA_MEM_HOST && c->n) {
    HIP_TRY(c, hipMemcpyAsync(c->u_d, dL_dV, (size_t)c->n * sizeof(double), hipMemcpyHostToDevice, s));
    u = c->u_d;
    out = c->out_d;
  }
  launch_volume_vjp(b, u, out, s);
  HIP_TRY(c, hipGetLastError());
  if (mem == SASA_MEM_HOST && c->n) {
    HIP_TRY(c, hipMemcpyAsync(dL_dx, out, (size_t)c->n * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  } else if (!(c->flags & SASA_FLAG_ASYNC)) {
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return SASA_OK;
}

int sasa_curvature(sasa_context* ctx, double* mean, int64_t* euler, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (!c->kept) return fail(c, SASA_E_STATE, "no kept compute on this context");
  if (mem != SASA_MEM_HOST && mem != SASA_MEM_DEVICE) return fail(c, SASA_E_INVAL, "bad mem");
  if (c->n > 0 && !mean && !euler) return fail(c, SASA_E_INVAL, "mean and euler must not both be NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(c, hipSetDevice(c->device));
  if (mean && c->n) {
    Bufs b = c->b;
    b.n = (int)c->n;
    b.nmol = std::max(c->nmol, 1);
    b.area = c->area_d;  // the areas again, in FP64
    double* cv = mem == SASA_MEM_HOST ? c->u_d : mean;
    // the volume kernel walks the same exposed arcs; its volumes go to scratch
    // (the input staging of the last compute, no longer needed)
    launch_terms(b, SASA_FP64, 0, s);
    launch_volume(b, c->xyz_d, c->out_d, s, cv);
    HIP_TRY(c, hipGetLastError());
    if (mem == SASA_MEM_HOST)
      HIP_TRY(c, hipMemcpyAsync(mean, cv, (size_t)c->n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  if (euler) {
    int64_t cnt[8];
    int rc = sasa_complex_counts(ctx, cnt);
    if (rc) return rc;
    *euler = cnt[0] - cnt[1] + cnt[2] - cnt[3];
  }
  return SASA_OK;
}

int sasa_curvature_backward(sasa_context* ctx, const double* dL_dC, double* dL_dx, int32_t mem, void* hip_stream) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  if (!c->kept) return fail(c, SASA_E_STATE, "no kept compute on this context");
  if (mem != SASA_MEM_HOST && mem != SASA_MEM_DEVICE) return fail(c, SASA_E_INVAL, "bad mem");
  if (c->n > 0 && (!dL_dC || !dL_dx)) return fail(c, SASA_E_INVAL, "dL_dC / dL_dx must not be NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(c, hipSetDevice(c->device));
  c->inc_valid = false;  // the gradient blocks are rewritten below
  if (c->n) {
    Bufs b = c->b;
    b.n = (int)c->n;
    b.nmol = std::max(c->nmol, 1);
    b.area = c->area_d;
    const double* u = dL_dC;
    double* out = dL_dx;
    if (mem == SASA_MEM_HOST) {
      HIP_TRY(c, hipMemcpyAsync(c->u_d, dL_dC, (size_t)c->n * sizeof(double), hipMemcpyHostToDevice, s));
      u = c->u_d;
      out = c->out_d;
    }
    // sum_i u_i / R_i dA_i/dp (the spheres), then + sum_i u_i dC_i^crease/dp;
    // scratch: the input staging buffers of the last compute
    double* ur = c->xyz_d;
    launch_recip_radius(b, u, ur, s);
    launch_terms(b, SASA_FP64, 1, s);
    launch_gather(b, ur, out, 1.0, s);
    Bufs bc = b;
    bc.area = c->rad_d;
    launch_terms_crease(bc, 1, s);
    launch_gather(bc, u, out, 1.0, s, 1);
    HIP_TRY(c, hipGetLastError());
    if (mem == SASA_MEM_HOST)
      HIP_TRY(c, hipMemcpyAsync(dL_dx, out, (size_t)c->n * 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  if (mem == SASA_MEM_HOST || !(c->flags & SASA_FLAG_ASYNC)) HIP_TRY(c, hipStreamSynchronize(s));
  return SASA_OK;
}

int sasa_triangles_by_sort(sasa_context* ctx, int32_t* tris, uint8_t* tri_ntet, int64_t capacity, int64_t* count,
                           float* ms) {
  Ctx* c = ctx;
  if (!c || !count) return fail(c, SASA_E_INVAL, "NULL argument");
  int64_t cnt[8];
  int rc = sasa_complex_counts(ctx, cnt);
  if (rc) return rc;
  if (c->n >= (int64_t)1 << 21) return fail(c, SASA_E_INVAL, "the sorted extraction packs atom ids in 21 bits");
  HIP_TRY(c, hipSetDevice(c->device));
  SortedFaces& w = c->sf;
  const int64_t nfaces = 4 * cnt[3], cap_free = cnt[6];
  if (nfaces > c->sf_cap_faces || cap_free > c->sf_cap_free) {
    const int64_t nf = std::max<int64_t>(nfaces, 1), nz = std::max<int64_t>(cap_free, 1);
    c->sf_cap_faces = c->sf_cap_free = -1;  // set again once every buffer exists
    HIP_TRY(c, grow(&w.faces, nf));
    HIP_TRY(c, grow(&w.sorted, nf));
    HIP_TRY(c, grow(&w.uniq, nf));
    HIP_TRY(c, grow(&w.counts, nf));
    HIP_TRY(c, grow(&w.free_tris, nz));
    HIP_TRY(c, grow(&w.tris, 3 * (nf + nz)));
    HIP_TRY(c, grow(&w.ntet, nf + nz));
    if (!w.nruns) HIP_TRY(c, grow(&w.nruns, 4));
    if (!w.cursors) HIP_TRY(c, grow(&w.cursors, 2));
    const size_t tb = sorted_faces_temp_bytes(nf);
    if (tb > w.temp_bytes) {
      w.temp_bytes = 0;
      HIP_TRY(c, grow((char**)&w.temp, tb));
      w.temp_bytes = tb;
    }
    c->sf_cap_faces = nfaces;
    c->sf_cap_free = cap_free;
  }
  w.nfaces = nfaces;
  w.cap_free = cap_free;
  Bufs b = c->b;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  launch_zero(w.cursors, 2 * sizeof(unsigned long long), s);
  launch_zero(w.nruns, sizeof(unsigned), s);
  HIP_TRY(c, hipEventRecord(e0, s));
  const hipError_t le = launch_sorted_faces(b, w, s);
  HIP_TRY(c, hipEventRecord(e1, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  float t = 0.0f;
  HIP_TRY(c, hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(c, le);
  unsigned nruns = 0;
  unsigned long long cur[2] = {0, 0};
  HIP_TRY(c, hipMemcpy(&nruns, w.nruns, sizeof(unsigned), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(cur, w.cursors, sizeof(cur), hipMemcpyDeviceToHost));
  if ((int64_t)cur[0] != nfaces || (int64_t)cur[1] > cap_free)
    return fail(c, SASA_E_DEVICE, "sorted extraction: face count differs from the complex's counters");
  const int64_t m = (int64_t)nruns + (int64_t)cur[1];
  *count = m;
  if (ms) *ms = t;
  if (!tris || !tri_ntet) return SASA_OK;  // size query
  if (m > capacity) return fail(c, SASA_E_CAPACITY, "sorted extraction: output capacity too small");
  if (m) {
    HIP_TRY(c, hipMemcpy(tris, w.tris, (size_t)m * 3 * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(tri_ntet, w.ntet, (size_t)m, hipMemcpyDeviceToHost));
  }
  return SASA_OK;
}

namespace {
// Work buffers of one sorted edge / vertex extraction for n candidates (a
// failed allocation leaves cap at -1, so the next call grows them all again).
int ensure_ev(Ctx* c, SortedEV& w, int64_t n) {
  n = std::max<int64_t>(n, 1);
  if (n <= w.cap) return SASA_OK;
  w.cap = -1;
  HIP_TRY(c, grow(&w.keys, n));
  HIP_TRY(c, grow(&w.vals, n));
  HIP_TRY(c, grow(&w.skeys, n));
  HIP_TRY(c, grow(&w.svals, n));
  HIP_TRY(c, grow(&w.uniq, n));
  HIP_TRY(c, grow(&w.agg, n));
  HIP_TRY(c, grow(&w.out_ids, 2 * n));
  HIP_TRY(c, grow(&w.out_ext, n));
  if (!w.nuniq) HIP_TRY(c, grow(&w.nuniq, 1));
  if (!w.cursor) HIP_TRY(c, grow(&w.cursor, 1));
  const size_t tb = sorted_ev_temp_bytes(n);
  if (tb > w.temp_bytes) {
    w.temp_bytes = 0;
    HIP_TRY(c, grow((char**)&w.temp, tb));
    w.temp_bytes = tb;
  }
  w.cap = n;
  return SASA_OK;
}
}  // namespace

int sasa_edges_vertices_by_sort(sasa_context* ctx, int32_t* edges, uint8_t* edge_ext, int64_t edge_capacity,
                                int64_t* edge_count, int32_t* verts, uint8_t* vert_ext, int64_t vert_capacity,
                                int64_t* vert_count, float* ms) {
  Ctx* c = ctx;
  if (!c || !edge_count || !vert_count) return fail(c, SASA_E_INVAL, "NULL argument");
  int64_t m = 0;
  float t_tri = 0.0f;
  int rc = sasa_triangles_by_sort(ctx, nullptr, nullptr, 0, &m, &t_tri);  // unique triangles, kept on the device
  if (rc) return rc;
  int64_t cnt[8];
  rc = sasa_complex_counts(ctx, cnt);
  if (rc) return rc;
  HIP_TRY(c, hipSetDevice(c->device));
  const int64_t ne_cand = 3 * m + cnt[1];
  rc = ensure_ev(c, c->se, ne_cand);
  if (rc) return rc;
  Bufs b = c->b;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  hipStream_t s = nullptr;
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  for (auto& ev : e) HIP_TRY(c, hipEventCreate(&ev));
  auto done = [&](int code) {
    for (auto& ev : e)
      if (ev) (void)hipEventDestroy(ev);
    return code;
  };
  // edges
  launch_zero(c->se.cursor, sizeof(unsigned long long), s);
  launch_zero(c->se.nuniq, sizeof(unsigned), s);
  HIP_TRY(c, hipEventRecord(e[0], s));
  hipError_t le = launch_sorted_edges(b, c->sf.tris, c->sf.ntet, m, ne_cand, c->se, s);
  if (le != hipSuccess) return done(fail(c, SASA_E_DEVICE, hipGetErrorString(le)));
  HIP_TRY(c, hipStreamSynchronize(s));
  unsigned ue = 0;
  unsigned long long cur = 0;
  HIP_TRY(c, hipMemcpy(&ue, c->se.nuniq, sizeof(unsigned), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&cur, c->se.cursor, sizeof(cur), hipMemcpyDeviceToHost));
  if ((int64_t)cur != cnt[1] || (int64_t)ue != cnt[1])
    return done(fail(c, SASA_E_DEVICE, "sorted extraction: edge count differs from the complex's counters"));
  launch_ev_unpack(c->se, ue, 2, s);
  // vertices, from the unique edges
  const int64_t nv_cand = 2 * (int64_t)ue + cnt[0];
  rc = ensure_ev(c, c->sv, nv_cand);
  if (rc) return done(rc);
  launch_zero(c->sv.cursor, sizeof(unsigned long long), s);
  launch_zero(c->sv.nuniq, sizeof(unsigned), s);
  HIP_TRY(c, hipEventRecord(e[1], s));
  // (the vertex candidates from edges read the edge step's unique count first)
  HIP_TRY(c, hipMemcpyAsync(c->sv.nuniq, c->se.nuniq, sizeof(unsigned), hipMemcpyDeviceToDevice, s));
  le = launch_sorted_vertices(b, c->se.uniq, c->se.agg, ue, nv_cand, c->sv, s);
  if (le != hipSuccess) return done(fail(c, SASA_E_DEVICE, hipGetErrorString(le)));
  HIP_TRY(c, hipEventRecord(e[2], s));
  HIP_TRY(c, hipStreamSynchronize(s));
  unsigned uv = 0;
  HIP_TRY(c, hipMemcpy(&uv, c->sv.nuniq, sizeof(unsigned), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&cur, c->sv.cursor, sizeof(cur), hipMemcpyDeviceToHost));
  if ((int64_t)cur != cnt[0] || (int64_t)uv != cnt[0])
    return done(fail(c, SASA_E_DEVICE, "sorted extraction: vertex count differs from the complex's counters"));
  launch_ev_unpack(c->sv, uv, 1, s);
  HIP_TRY(c, hipStreamSynchronize(s));
  float t_e = 0.0f, t_v = 0.0f;
  HIP_TRY(c, hipEventElapsedTime(&t_e, e[0], e[1]));
  HIP_TRY(c, hipEventElapsedTime(&t_v, e[1], e[2]));
  *edge_count = ue;
  *vert_count = uv;
  if (ms) *ms = t_tri + t_e + t_v;
  if (edges || edge_ext || verts || vert_ext) {
    if (!edges || !edge_ext || !verts || !vert_ext)
      return done(fail(c, SASA_E_INVAL, "sorted extraction: give all four output arrays or none"));
    if ((int64_t)ue > edge_capacity || (int64_t)uv > vert_capacity)
      return done(fail(c, SASA_E_CAPACITY, "sorted extraction: output capacity too small"));
    if (ue) {
      HIP_TRY(c, hipMemcpy(edges, c->se.out_ids, (size_t)ue * 2 * sizeof(int), hipMemcpyDeviceToHost));
      HIP_TRY(c, hipMemcpy(edge_ext, c->se.out_ext, (size_t)ue, hipMemcpyDeviceToHost));
    }
    if (uv) {
      HIP_TRY(c, hipMemcpy(verts, c->sv.out_ids, (size_t)uv * sizeof(int), hipMemcpyDeviceToHost));
      HIP_TRY(c, hipMemcpy(vert_ext, c->sv.out_ext, (size_t)uv, hipMemcpyDeviceToHost));
    }
  }
  return done(SASA_OK);
}

int sasa_complex_counts(sasa_context* ctx, int64_t counts[8]) {
  Ctx* c = ctx;
  if (!c || !counts) return fail(c, SASA_E_INVAL, "NULL argument");
  if (!c->kept) return fail(c, SASA_E_STATE, "no kept compute on this context");
  if (c->pending) {
    int rc = read_counters(c, c->last_stream);
    if (rc) return rc;
  }
  int rc = sum_stats(c);
  if (rc) return rc;
  const unsigned long long* h = c->ctr_h;
  counts[0] = (int64_t)h[ctr_slot(C_VERT)];
  counts[1] = (int64_t)h[ctr_slot(C_EDGE)];
  counts[2] = (int64_t)h[ctr_slot(C_TRI)];
  counts[3] = (int64_t)h[ctr_slot(C_TET)];
  counts[4] = (int64_t)h[ctr_slot(C_EXT_VERT)];
  counts[5] = (int64_t)h[ctr_slot(C_EXT_EDGE)];
  counts[6] = (int64_t)h[ctr_slot(C_EXT_TRI)];
  counts[7] = c->n;
  return SASA_OK;
}

int sasa_complex_export(sasa_context* ctx, int32_t* edges, int32_t* tris, uint8_t* tri_ntet, int32_t* tets,
                        uint8_t* vert_flags) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  int64_t cnt[8];
  int rc = sasa_complex_counts(ctx, cnt);
  if (rc) return rc;
  HIP_TRY(c, hipSetDevice(c->device));
  Bufs& B = c->b;
  if (cnt[1] > c->ex_cap_e) {
    c->ex_cap_e = 0;
    HIP_TRY(c, grow(&B.ex_edges, (size_t)cnt[1] * 2));
    c->ex_cap_e = cnt[1];
  }
  if (cnt[2] > c->ex_cap_t) {
    c->ex_cap_t = 0;
    HIP_TRY(c, grow(&B.ex_tris, (size_t)cnt[2] * 3));
    HIP_TRY(c, grow(&B.ex_ntet, (size_t)cnt[2]));
    c->ex_cap_t = cnt[2];
  }
  if (cnt[3] > c->ex_cap_q) {
    c->ex_cap_q = 0;
    HIP_TRY(c, grow(&B.ex_tets, (size_t)cnt[3] * 4));
    c->ex_cap_q = cnt[3];
  }
  // re-run the (deterministic) star kernel with export on; the cell list of the
  // last compute is still in place
  Bufs b = B;
  b.n = (int)c->n;
  b.nmol = std::max(c->nmol, 1);
  b.export_on = 1;
  b.fac = nullptr;  // the export leaves the trajectory's hints alone
  b.vtx = nullptr;
  b.hint_n = nullptr;
  b.ex_cap_e = c->ex_cap_e;
  b.ex_cap_t = c->ex_cap_t;
  b.ex_cap_q = c->ex_cap_q;
  hipStream_t s = nullptr;
  // keep R_max (needed for the cell size), clear everything else
  unsigned long long rmax_bits = c->ctr_h[ctr_slot(C_RMAX_BITS)];
  launch_zero(b.ctr, CTR_BYTES, s);
  HIP_TRY(c, hipMemcpyAsync(b.ctr + ctr_slot(C_RMAX_BITS), &rmax_bits, sizeof(rmax_bits), hipMemcpyHostToDevice, s));
  launch_star(b, s);
  launch_star_wide(b, s);
  launch_stats(b, s);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(s));
  c->timed = false;
  c->stats_due = false;
  rc = read_counters(c, s);
  if (rc) return rc;
  // the kernels emit in arrival order; the lists are returned sorted
  if (edges && cnt[1]) {
    HIP_TRY(c, hipMemcpy(edges, b.ex_edges, (size_t)cnt[1] * 2 * sizeof(int), hipMemcpyDeviceToHost));
    sort_tuples<2>(edges, nullptr, cnt[1]);
  }
  if ((tris || tri_ntet) && cnt[2]) {
    std::vector<int32_t> t((size_t)cnt[2] * 3);
    std::vector<uint8_t> nt((size_t)cnt[2]);
    HIP_TRY(c, hipMemcpy(t.data(), b.ex_tris, t.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(nt.data(), b.ex_ntet, nt.size(), hipMemcpyDeviceToHost));
    sort_tuples<3>(t.data(), nt.data(), cnt[2]);
    if (tris) std::memcpy(tris, t.data(), t.size() * sizeof(int32_t));
    if (tri_ntet) std::memcpy(tri_ntet, nt.data(), nt.size());
  }
  if (tets && cnt[3]) {
    HIP_TRY(c, hipMemcpy(tets, b.ex_tets, (size_t)cnt[3] * 4 * sizeof(int), hipMemcpyDeviceToHost));
    sort_tuples<4>(tets, nullptr, cnt[3]);
  }
  if (vert_flags && c->n) HIP_TRY(c, hipMemcpy(vert_flags, b.vflag, (size_t)c->n, hipMemcpyDeviceToHost));
  return SASA_OK;
}

int sasa_diagnostics(sasa_context* ctx, sasa_diag* out, int64_t size) {
  Ctx* c = ctx;
  if (!c || !out || size < 0) return fail(c, SASA_E_INVAL, "NULL argument");
  int rc = SASA_OK;
  if (c->pending) rc = read_counters(c, c->last_stream);
  if (!rc) rc = sum_stats(c);
  std::memcpy(out, &c->diag, (size_t)std::min<int64_t>(size, sizeof(sasa_diag)));
  return rc;
}

int sasa_status(sasa_context* ctx) {
  Ctx* c = ctx;
  if (!c) return fail(nullptr, SASA_E_INVAL, "ctx == NULL");
  return c->pending ? read_counters(c, c->last_stream, false) : SASA_OK;
}

int sasa_footprint(int64_t n, int64_t* bytes) {
  if (n < 0 || !bytes) return fail(nullptr, SASA_E_INVAL, "n < 0 or bytes == NULL");
  // per atom: positions (2 orders), molecule / cell / sorted ids, the star's
  // statistics record, flags, the
  // kept complex, gradient blocks, area and the staging of inputs and outputs;
  // per molecule (at most one per atom): offsets, box, grid geometry
  const int64_t per_atom = sizeof(double4) * 2 + sizeof(int2) + sizeof(int) * (4 + STAT_STRIDE) + 1 + sizeof(int) * (KN_CAP + 3) +
                           sizeof(unsigned long long) + sizeof(unsigned) * (KT_CAP + KTR_CAP) +
                           sizeof(double) * (ROW * 3 + 1 + 3 + 3 + 1 + 1);
  const int64_t per_mol = sizeof(int64_t) * 2 + sizeof(unsigned long long) * 6 + sizeof(double4) + sizeof(int4);
  *bytes = n * (per_atom + per_mol) + cell_capacity(n) * 2 * (int64_t)sizeof(int) + 4096;
  return SASA_OK;
}

void sasa_capacity(int64_t caps[2]) {
  if (!caps) return;
  caps[0] = NB_CAP_WIDE;
  caps[1] = V_CAP;
}

const char* sasa_strerror(int32_t code) {
  switch (code) {
    case SASA_OK: return "ok";
    case SASA_E_INVAL: return "invalid argument";
    case SASA_E_NOMEM: return "out of device memory";
    case SASA_E_DEVICE: return "HIP device error";
    case SASA_E_STATE: return "no kept compute on this context";
    case SASA_E_CAPACITY: return "per-atom capacity exceeded";
  }
  return "unknown error";
}

const char* sasa_last_error(sasa_context* ctx) {
  Ctx* c = ctx;
  return c ? c->err.c_str() : g_err.c_str();
}

}  // extern "C"

// ------------------------------------------------------------ no allocation
// sasa_compute_noalloc's work space: one fixed array in the library's device
// code (allocated on each GPU when the code is loaded there, held until the
// process ends).  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// ever handed to kernels.
namespace {
constexpr size_t kNoAllocBytes = (size_t)16 << 20;  // 16 MiB: SASA_NOALLOC_MAX_ATOMS atoms with room to spare
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kMaxDevices] = {};

// Consecutive 256-byte-aligned arrays carved from a base address (with a null
// base it only counts the bytes).
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// The buffers of a one-molecule compute of n atoms; returns the bytes used.
size_t noalloc_layout(unsigned char* base, int64_t n, Bufs& b, double** area_ws, unsigned long long** status) {
  Carve c{base};
  const size_t N = (size_t)n;
  const int64_t cells = cell_capacity(n);
  b.pos = c.take<double4>(N);
  b.mol = c.take<int>(N);
  b.cellid = c.take<int>(N);
  b.offsets = c.take<int64_t>(2);  // (not read by the one-block cell list)
  b.mol_box = c.take<unsigned long long>(6);
  b.mol_geo = c.take<double4>(1);
  b.mol_dim = c.take<int4>(1);
  b.cnt = c.take<int>((size_t)cells);
  b.start = c.take<int>((size_t)cells + 1);
  b.scan_tmp = c.take<int>((size_t)scan_blocks((unsigned)cells) + 1);
  b.sorted = c.take<int>(N);
  b.spos = c.take<double4>(N);
  b.smc = c.take<int2>(N);
  b.vflag = c.take<uint8_t>(N);
  b.kn_cnt = c.take<int>(N);
  b.knbr = c.take<int>(N * KN_CAP);
  b.kn_ext = c.take<unsigned long long>(N);
  b.kt_cnt = c.take<int>(N);
  b.ktet = c.take<unsigned>(N * KT_CAP);
  b.ktr_cnt = c.take<int>(N);
  b.ktri = c.take<unsigned>(N * KTR_CAP);
  b.stat = c.take<int>(N * STAT_STRIDE);
  b.wide = c.take<int>(N);
  b.rows = c.take<double>(N * ROW * 3);
  b.ctr = c.take<unsigned long long>((size_t)C_COUNT * CTR_STRIDE);
  *area_ws = c.take<double>(N);
  *status = c.take<unsigned long long>(3);
  return c.off;
}

}  // namespace

extern "C" int sasa_compute_noalloc(int device, int64_t n, const double* xyz, const double* radii, double probe,
                                    double* area, double* dA_dx, int precision, void* hip_stream) {
  if (n < 0) return fail(nullptr, SASA_E_INVAL, "n < 0");
  if (n > SASA_NOALLOC_MAX_ATOMS)
    return fail(nullptr, SASA_E_INVAL, "n exceeds SASA_NOALLOC_MAX_ATOMS (the fixed work space of this entry point)");
  if (n > 0 && (!xyz || !radii)) return fail(nullptr, SASA_E_INVAL, "xyz / radii must not be NULL");
  if (!(probe >= 0.0) || !std::isfinite(probe)) return fail(nullptr, SASA_E_INVAL, "probe must be finite and >= 0");
  if (precision != SASA_FP64 && precision != SASA_MIXED)
    return fail(nullptr, SASA_E_INVAL, "precision must be SASA_FP64 or SASA_MIXED");
  if (device < 0 || device >= kMaxDevices) return fail(nullptr, SASA_E_INVAL, "bad device ordinal");
  if (n == 0) return SASA_OK;
  int prev = 0;
  HIP_TRY(nullptr, hipGetDevice(&prev));
  if (prev != device) HIP_TRY(nullptr, hipSetDevice(device));
  int rc = SASA_OK;
  do {
    unsigned char* base = nullptr;
    {
      std::lock_guard<std::mutex> lock(g_noalloc_mu);
      if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
          rc = fail(nullptr, SASA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
          break;
        }
        g_noalloc_ptr[device] = (unsigned char*)p;
      }
      base = g_noalloc_ptr[device];
    }
    Bufs b;
    double* area_ws = nullptr;
    unsigned long long* status = nullptr;
    if (noalloc_layout(nullptr, n, b, &area_ws, &status) > kNoAllocBytes) {
      rc = fail(nullptr, SASA_E_INVAL, "n does not fit the fixed work space");
      break;
    }
    noalloc_layout(base, n, b, &area_ws, &status);
    b.n = (int)n;
    b.nmol = 1;
    b.cell_cap = (int)cell_capacity(n);
    b.xyz = xyz;
    b.radii = radii;
    b.probe = probe;
    b.area = area ? area : area_ws;
    b.status = status;
    hipStream_t s = (hipStream_t)hip_stream;
    // k_cells_one clears the counters (everything else is written before it
    // is read); the last call's contents are never used
    launch_cells_one(b, s);
    launch_star(b, s);
    launch_star_wide(b, s);
    launch_terms(b, precision, dA_dx != nullptr, s);
    if (dA_dx) launch_gather(b, nullptr, dA_dx, 1.0, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      rc = fail(nullptr, SASA_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
      break;
    }
    unsigned long long st[3] = {0, 0, 0};
    e = hipMemcpyAsync(st, status, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rc = fail(nullptr, SASA_E_DEVICE, std::string("status read: ") + hipGetErrorString(e));
      break;
    }
    if (st[2] != 1ull) {
      rc = fail(nullptr, SASA_E_DEVICE, "the call's status words were not written");
    } else if (st[0]) {
      rc = fail(nullptr, SASA_E_INVAL,
                "NaN/Inf coordinate, radius <= 0, or two atoms with the same centre and radius in the input");
    } else if (st[1]) {
      rc = fail(nullptr, SASA_E_CAPACITY, "an atom exceeds the per-atom neighbour / cell-vertex / star capacity");
    }
  } while (false);
  if (prev != device) (void)hipSetDevice(prev);
  return rc;
}
