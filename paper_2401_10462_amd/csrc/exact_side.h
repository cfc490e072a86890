// exact_side.h -- exact sign of a cell-clipping side test (host and device).
//
// A vertex of the power cell of atom i is the intersection of three planes
// n_q . x = b_q (x relative to p_i): the radical plane of a neighbour q,
// n_q = 2 (p_q - p_i), b_q = |p_q - p_i|^2 - R_q^2 + R_i^2, or a face of the
// starting cube, n = +-e_axis, b = h.  Whether a later plane m keeps the
// vertex v is the sign of g_m(v) = b_m - n_m . v.  With M the matrix of the
// vertex's three normals and beta its offsets, the Schur complement gives
//   det [[M, beta], [n_m^T, b_m]] = det(M) (b_m - n_m^T M^-1 beta) = det(M) g_m(v),
// so sign(g_m(v)) = sign(det4) * sign(det3(M)), both exact polynomials in the
// input doubles.  They are evaluated here without rounding in floating-point
// expansion arithmetic (a value is the exact sum of non-overlapping doubles;
// Shewchuk, "Adaptive precision floating-point arithmetic and fast robust
// geometric predicates", DCG 18, 1997: Two-Sum, Two-Product by fused
// multiply-add, Grow-Expansion, Scale-Expansion and Compress).  Intermediate
// results are compressed after every product, which keeps them at a handful of
// doubles for inputs in Angstrom; every array is bounded and an expansion
// that would outgrow it makes the routine report failure (2) instead.
#pragma once
#include <hip/hip_runtime.h>

namespace sasa {
namespace exact {

constexpr int CAP = 64;  // doubles per expansion

// Correctly rounded operations that the compiler may not fuse: HIP's
// __dadd_rn and friends are plain operators unless OCML's rounded operations
// are enabled, and the default contraction would fuse a product into a later
// sum across inlined calls, breaking Two-Sum and Two-Product.  With
// contraction off here, the IR operations carry no contract flag and stay
// separate wherever they are inlined.
__host__ __device__ inline double radd(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}
__host__ __device__ inline double rsub(double a, double b) {
#pragma clang fp contract(off)
  return a - b;
}
__host__ __device__ inline double rmul(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

struct Ex {
  int n;
  double v[CAP];  // increasing magnitude, non-overlapping, no zeros (n = 0: the value 0)
};

__host__ __device__ inline void two_sum(double a, double b, double& x, double& y) {
  x = radd(a, b);
  const double bv = rsub(x, a);
  const double av = rsub(x, bv);
  y = radd(rsub(a, av), rsub(b, bv));
}
// |a| >= |b| (or a = 0)
__host__ __device__ inline void fast_two_sum(double a, double b, double& x, double& y) {
  x = radd(a, b);
  y = rsub(b, rsub(x, a));
}
__host__ __device__ inline void two_prod(double a, double b, double& x, double& y) {
  x = rmul(a, b);
  y = fma(a, b, -x);
}

__host__ __device__ inline void copy(Ex& dst, const Ex& src) {
  dst.n = src.n;
  for (int t = 0; t < src.n; ++t) dst.v[t] = src.v[t];
}

__host__ __device__ inline void set(Ex& e, double d) {
  e.n = 0;
  if (d != 0.0) e.v[e.n++] = d;
}

// h = e + d (Grow-Expansion, zero-eliminating); false if h would overflow.
// h may be e: each output term goes to a slot whose input was already read.
__host__ __device__ inline bool grow(const Ex& e, double d, Ex& h) {
  if (e.n + 1 > CAP) return false;
  double q = d;
  int k = 0;
  for (int t = 0; t < e.n; ++t) {
    double s, r;
    two_sum(q, e.v[t], s, r);
    q = s;
    if (r != 0.0) h.v[k++] = r;
  }
  if (q != 0.0 || k == 0) h.v[k++] = q;
  if (k == 1 && h.v[0] == 0.0) k = 0;
  h.n = k;
  return true;
}

// h = e + f (f added term by term, in place in h); h may be e, not f
__host__ __device__ inline bool add(const Ex& e, const Ex& f, Ex& h) {
  if (&h != &e) copy(h, e);
  for (int t = 0; t < f.n; ++t)
    if (!grow(h, f.v[t], h)) return false;
  return true;
}

__host__ __device__ inline void negate(Ex& e) {
  for (int t = 0; t < e.n; ++t) e.v[t] = -e.v[t];
}

// h = e * d (Scale-Expansion, zero-eliminating)
__host__ __device__ inline bool scale(const Ex& e, double d, Ex& h) {
  if (e.n == 0 || d == 0.0) {
    h.n = 0;
    return true;
  }
  if (2 * e.n > CAP) return false;
  int k = 0;
  double q, r;
  two_prod(e.v[0], d, q, r);
  if (r != 0.0) h.v[k++] = r;
  for (int t = 1; t < e.n; ++t) {
    double p1, p0, s, u;
    two_prod(e.v[t], d, p1, p0);
    two_sum(q, p0, s, u);
    if (u != 0.0) h.v[k++] = u;
    fast_two_sum(p1, s, q, u);
    if (u != 0.0) h.v[k++] = u;
  }
  if (q != 0.0 || k == 0) h.v[k++] = q;
  if (k == 1 && h.v[0] == 0.0) k = 0;
  h.n = k;
  return true;
}

// Compress (two sweeps of Fast-Two-Sum), in place: the first sweep writes
// only slots it has already read, the second only slots below the one it reads.
__host__ __device__ inline void compress(Ex& e) {
  if (e.n <= 1) return;
  int bottom = e.n - 1;
  double q = e.v[e.n - 1];
  for (int t = e.n - 2; t >= 0; --t) {
    double s, r;
    fast_two_sum(q, e.v[t], s, r);
    if (r != 0.0) {
      e.v[bottom--] = s;
      q = r;
    } else {
      q = s;
    }
  }
  e.v[bottom] = q;
  int top = 0;
  for (int t = bottom + 1; t < e.n; ++t) {
    double s, r;
    fast_two_sum(e.v[t], q, s, r);
    q = s;
    if (r != 0.0) e.v[top++] = r;
  }
  e.v[top++] = q;
  e.n = (top == 1 && e.v[0] == 0.0) ? 0 : top;
}

// h = e * f, compressed (h distinct from e, f and t1)
__host__ __device__ inline bool mul(const Ex& e, const Ex& f, Ex& h, Ex& t1) {
  h.n = 0;
  for (int t = 0; t < f.n; ++t) {
    if (!scale(e, f.v[t], t1)) return false;
    if (!add(h, t1, h)) return false;
    compress(h);
  }
  return true;
}

__host__ __device__ inline int sign(const Ex& e) {
  return e.n == 0 ? 0 : (e.v[e.n - 1] > 0.0 ? 1 : -1);
}

// One plane, exactly: normal components and offset as expansions.
struct Plane {
  Ex n[3];
  Ex b;
};

// Work space of one evaluation.
struct Work {
  Plane pl[4];
  Ex m1, m2, det3, prod, acc, t1;
};

// Radical plane of neighbour (x, y, z, R) seen from atom (xi, yi, zi, Ri).
__host__ __device__ inline bool radical(double xi, double yi, double zi, double Ri, double x, double y, double z,
                                        double R, Plane& p, Work& w) {
  const double pj[3] = {x, y, z}, pi[3] = {xi, yi, zi};
  Ex& a2 = w.acc;
  a2.n = 0;
  for (int c = 0; c < 3; ++c) {
    double hi, lo;
    two_sum(pj[c], -pi[c], hi, lo);  // p_j - p_i exactly
    Ex& a = w.m1;
    a.n = 0;
    if (lo != 0.0) a.v[a.n++] = lo;
    if (hi != 0.0) a.v[a.n++] = hi;
    // n = 2 a (exact)
    p.n[c].n = a.n;
    for (int t = 0; t < a.n; ++t) p.n[c].v[t] = 2.0 * a.v[t];
    if (!mul(a, a, w.prod, w.t1)) return false;
    if (!add(a2, w.prod, a2)) return false;
  }
  // b = |a|^2 - R^2 + Ri^2
  double q, r;
  two_prod(R, R, q, r);
  Ex& rr = w.m2;
  rr.n = 0;
  if (r != 0.0) rr.v[rr.n++] = -r;
  if (q != 0.0) rr.v[rr.n++] = -q;
  if (!add(a2, rr, a2)) return false;
  two_prod(Ri, Ri, q, r);
  rr.n = 0;
  if (r != 0.0) rr.v[rr.n++] = r;
  if (q != 0.0) rr.v[rr.n++] = q;
  if (!add(a2, rr, p.b)) return false;
  compress(p.b);
  return true;
}

// Face of the starting cube: id 0..5 = +x, -x, +y, -y, +z, -z at distance h.
__host__ __device__ inline void cube_face(unsigned id, double h, Plane& p) {
  for (int c = 0; c < 3; ++c) p.n[c].n = 0;
  set(p.n[id >> 1], (id & 1) ? -1.0 : 1.0);
  set(p.b, h);
}

// Entry (row p, column col) of the matrix of normals whose column repl (if
// any) is replaced by the offsets (Cramer's rule).
__host__ __device__ inline const Ex& entry(const Plane& p, int col, int repl) { return col == repl ? p.b : p.n[col]; }

// det3 of normals (rows u, v, s; column repl replaced by the offsets) into w.det3
__host__ __device__ inline bool det3(const Plane& u, const Plane& v, const Plane& s, Work& w, int repl = -1) {
  w.det3.n = 0;
  for (int c = 0; c < 3; ++c) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    // minor = v[c1] s[c2] - v[c2] s[c1]
    if (!mul(entry(v, c1, repl), entry(s, c2, repl), w.m1, w.t1)) return false;
    if (!mul(entry(v, c2, repl), entry(s, c1, repl), w.m2, w.t1)) return false;
    negate(w.m2);
    if (!add(w.m1, w.m2, w.m1)) return false;
    compress(w.m1);
    if (!mul(entry(u, c, repl), w.m1, w.prod, w.t1)) return false;
    if (!add(w.det3, w.prod, w.det3)) return false;
    compress(w.det3);
  }
  return true;
}

// Value of an expansion rounded (summed from the smallest term up: within two
// units in the last place).
__host__ __device__ inline double approx(const Ex& e) {
  double s = 0.0;
  for (int t = 0; t < e.n; ++t) s += e.v[t];
  return s;
}

// The vertex of planes pl[0..2] by Cramer's rule with exact determinants,
// each coordinate within a few units in the last place however close the
// planes are to parallel.  False if an expansion outgrew its array or the
// planes meet in no single point.
__host__ __device__ inline bool vertex(Work& w, double v[3]) {
  if (!det3(w.pl[0], w.pl[1], w.pl[2], w)) return false;
  const double d = approx(w.det3);
  if (d == 0.0) return false;
  for (int c = 0; c < 3; ++c) {
    if (!det3(w.pl[0], w.pl[1], w.pl[2], w, c)) return false;
    v[c] = approx(w.det3) / d;
  }
  return true;
}

// Sign of g_m at the vertex of planes pl[0..2], with pl[3] the plane m:
// +1 kept, -1 cut away, 0 on the plane; 2 if an expansion outgrew its array.
__host__ __device__ inline int side(Work& w) {
  int sdet = 0;
  w.acc.n = 0;
  for (int r = 0; r < 4; ++r) {
    const Plane* o[3];
    int k = 0;
    for (int q = 0; q < 4; ++q)
      if (q != r) o[k++] = &w.pl[q];
    if (!det3(*o[0], *o[1], *o[2], w)) return 2;
    if (r == 3) sdet = sign(w.det3);
    // cofactor sign along the last column: - + - +
    if (!mul(w.pl[r].b, w.det3, w.prod, w.t1)) return 2;
    if ((r & 1) == 0) negate(w.prod);
    if (!add(w.acc, w.prod, w.acc)) return 2;
    compress(w.acc);
  }
  return sign(w.acc) * sdet;
}

// ------------------------------------------------------------------------
// First stage: the same determinants in double-double arithmetic (about 106
// bits; Dekker's pairs with the accurate sum and the fused-multiply-add
// product of Joldes, Muller and Popescu, ACM TOMS 44, 2017: relative error per
// operation below 6e-32).  The normals 2 (p_j - p_i) are exact pairs and the
// offsets carry a relative error of about 1e-31 of |p_j - p_i|^2 + R_j^2 + R_i^2,
// so the error of det4 is far below 1e-27 times the same expansion evaluated on
// magnitudes; past that bound the sign is certain, and only a side test closer
// to zero than that (an exact tie, in practice) needs the expansions above.

struct DD {
  double hi, lo;
};
__host__ __device__ inline DD dd_add(DD a, DD b) {
  double s, e, t, f;
  two_sum(a.hi, b.hi, s, e);
  two_sum(a.lo, b.lo, t, f);
  e = radd(e, t);
  fast_two_sum(s, e, s, e);
  e = radd(e, f);
  fast_two_sum(s, e, s, e);
  return {s, e};
}
__host__ __device__ inline DD dd_sub(DD a, DD b) { return dd_add(a, {-b.hi, -b.lo}); }
__host__ __device__ inline DD dd_mul(DD a, DD b) {
  double p, e;
  two_prod(a.hi, b.hi, p, e);
  e = fma(a.hi, b.lo, e);
  e = fma(a.lo, b.hi, e);
  fast_two_sum(p, e, p, e);
  return {p, e};
}

// A plane in double-double with the magnitudes of its entries (for the bound).
struct DPl {
  DD n[3], b;
  double an[3], ab;
};

__host__ __device__ inline DPl dd_radical(double xi, double yi, double zi, double Ri, double x, double y, double z,
                                          double R) {
  DPl p;
  const double pj[3] = {x, y, z}, pi[3] = {xi, yi, zi};
  DD a2 = {0.0, 0.0};
  double m2 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    DD a;
    two_sum(pj[c], -pi[c], a.hi, a.lo);
    p.n[c] = {2.0 * a.hi, 2.0 * a.lo};
    p.an[c] = fabs(p.n[c].hi);
    a2 = dd_add(a2, dd_mul(a, a));
    m2 += a.hi * a.hi;
  }
  DD r2, q2;
  two_prod(R, R, r2.hi, r2.lo);
  two_prod(Ri, Ri, q2.hi, q2.lo);
  p.b = dd_add(dd_sub(a2, r2), q2);
  p.ab = 1.01 * (m2 + R * R + Ri * Ri);
  return p;
}

__host__ __device__ inline DPl dd_cube(unsigned id, double h) {
  DPl p;
#pragma unroll
  for (int c = 0; c < 3; ++c) p.n[c] = {0.0, 0.0}, p.an[c] = 0.0;
  const double sg = (id & 1) ? -1.0 : 1.0;
  const int ax = (int)(id >> 1);
  p.n[ax == 0 ? 0 : (ax == 1 ? 1 : 2)] = {sg, 0.0};
  p.an[ax == 0 ? 0 : (ax == 1 ? 1 : 2)] = 1.0;
  p.b = {h, 0.0};
  p.ab = h;
  return p;
}

// det3 of the normals of u, v, s and its magnitude bound
__host__ __device__ inline DD dd_det3(const DPl& u, const DPl& v, const DPl& s, double& mag) {
  const DD cx = dd_sub(dd_mul(v.n[1], s.n[2]), dd_mul(v.n[2], s.n[1]));
  const DD cy = dd_sub(dd_mul(v.n[2], s.n[0]), dd_mul(v.n[0], s.n[2]));
  const DD cz = dd_sub(dd_mul(v.n[0], s.n[1]), dd_mul(v.n[1], s.n[0]));
  mag = u.an[0] * (v.an[1] * s.an[2] + v.an[2] * s.an[1]) + u.an[1] * (v.an[2] * s.an[0] + v.an[0] * s.an[2]) +
        u.an[2] * (v.an[0] * s.an[1] + v.an[1] * s.an[0]);
  return dd_add(dd_add(dd_mul(u.n[0], cx), dd_mul(u.n[1], cy)), dd_mul(u.n[2], cz));
}

// Sign of g_m at the vertex of P[0..2] (P[3] the plane m) if double-double
// decides it, else 0.
__host__ __device__ inline int dd_side(const DPl* P) {
  double m0, m1, m2, m3;
  const DD d0 = dd_det3(P[1], P[2], P[3], m0);
  const DD d1 = dd_det3(P[0], P[2], P[3], m1);
  const DD d2 = dd_det3(P[0], P[1], P[3], m2);
  const DD d3 = dd_det3(P[0], P[1], P[2], m3);
  const DD det4 = dd_add(dd_add(dd_sub(dd_mul(P[1].b, d1), dd_mul(P[0].b, d0)), dd_mul(P[3].b, d3)),
                         dd_mul(P[2].b, DD{-d2.hi, -d2.lo}));
  const double mag4 = P[0].ab * m0 + P[1].ab * m1 + P[2].ab * m2 + P[3].ab * m3;
  const double v4 = det4.hi + det4.lo, v3 = d3.hi + d3.lo;
  if (!(fabs(v4) > 1e-27 * mag4) || !(fabs(v3) > 1e-27 * m3)) return 0;
  return ((v4 > 0.0) == (v3 > 0.0)) ? 1 : -1;
}

}  // namespace exact
}  // namespace sasa
