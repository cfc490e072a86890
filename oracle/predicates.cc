// predicates.cc -- exact, symbolically perturbed predicates (TEST
// INFRASTRUCTURE ONLY; see predicates.h for what is decided and why).
//
// Two number types evaluate the same polynomial expressions:
//   Flt    an FP64 value with a running bound on its rounding error; a value
//          larger than twice its bound has the exact sign;
//   Exact  sign * magnitude * 2^exp with an arbitrary-precision integer
//          magnitude: every double is such a number, and sums and products
//          of them are computed without rounding.
#include "predicates.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace oracle_pred {
namespace {

// ---------------------------------------------------------------- Flt
// A running error bound: the inputs (doubles) are exact, and every rounded
// operation adds u |result| to the propagated bound (Wilkinson's running
// error analysis), so |v - exact| <= e up to the rounding of e itself.
constexpr double kU = 1.1102230246251565e-16;  // 2^-53
struct Flt {
  double v = 0.0, e = 0.0;
  Flt() = default;
  explicit Flt(double d) : v(d), e(0.0) {}
  Flt(double v_, double e_) : v(v_), e(e_) {}
};
inline Flt operator+(const Flt& a, const Flt& b) {
  const double v = a.v + b.v;
  return {v, a.e + b.e + kU * std::fabs(v)};
}
inline Flt operator-(const Flt& a, const Flt& b) {
  const double v = a.v - b.v;
  return {v, a.e + b.e + kU * std::fabs(v)};
}
inline Flt operator*(const Flt& a, const Flt& b) {
  const double v = a.v * b.v;
  return {v, std::fabs(a.v) * b.e + std::fabs(b.v) * a.e + a.e * b.e + kU * std::fabs(v)};
}
// Sign of the exact value if the bound decides it (with a factor 2 for the
// rounding of the bound), else 2.
inline int certain_sign(const Flt& f) {
  if (!std::isfinite(f.v) || !std::isfinite(f.e)) return 2;
  if (std::fabs(f.v) > 2.0 * f.e + 1e-290) return f.v > 0 ? 1 : -1;
  return 2;
}

// ---------------------------------------------------------------- Exact
// Magnitudes are little-endian vectors of 32-bit limbs without leading zero
// limbs; the empty vector is zero.
using Mag = std::vector<uint32_t>;

void trim(Mag& a) {
  while (!a.empty() && a.back() == 0) a.pop_back();
}

int cmp_mag(const Mag& a, const Mag& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t k = a.size(); k-- > 0;)
    if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
  return 0;
}

Mag add_mag(const Mag& a, const Mag& b) {
  Mag r(std::max(a.size(), b.size()) + 1, 0);
  uint64_t carry = 0;
  for (size_t k = 0; k < r.size(); ++k) {
    uint64_t s = carry;
    if (k < a.size()) s += a[k];
    if (k < b.size()) s += b[k];
    r[k] = (uint32_t)s;
    carry = s >> 32;
  }
  trim(r);
  return r;
}

// a - b for a >= b
Mag sub_mag(const Mag& a, const Mag& b) {
  Mag r(a.size(), 0);
  int64_t borrow = 0;
  for (size_t k = 0; k < a.size(); ++k) {
    int64_t s = (int64_t)a[k] - borrow - (k < b.size() ? (int64_t)b[k] : 0);
    borrow = 0;
    if (s < 0) {
      s += (int64_t)1 << 32;
      borrow = 1;
    }
    r[k] = (uint32_t)s;
  }
  trim(r);
  return r;
}

Mag mul_mag(const Mag& a, const Mag& b) {
  if (a.empty() || b.empty()) return {};
  Mag r(a.size() + b.size(), 0);
  for (size_t x = 0; x < a.size(); ++x) {
    uint64_t carry = 0;
    for (size_t y = 0; y < b.size(); ++y) {
      const uint64_t t = (uint64_t)a[x] * b[y] + r[x + y] + carry;
      r[x + y] = (uint32_t)t;
      carry = t >> 32;
    }
    size_t k = x + b.size();
    while (carry) {
      const uint64_t t = (uint64_t)r[k] + carry;
      r[k] = (uint32_t)t;
      carry = t >> 32;
      ++k;
    }
  }
  trim(r);
  return r;
}

// a * 2^s, s >= 0
Mag shl(const Mag& a, int s) {
  if (a.empty() || s == 0) return a;
  const int limbs = s / 32, bits = s % 32;
  Mag r(a.size() + limbs + 1, 0);
  for (size_t k = 0; k < a.size(); ++k) {
    const uint64_t v = (uint64_t)a[k] << bits;
    r[k + limbs] |= (uint32_t)v;
    r[k + limbs + 1] |= (uint32_t)(v >> 32);
  }
  trim(r);
  return r;
}

class Exact {
 public:
  Exact() = default;
  explicit Exact(double d) {
    if (d == 0.0) return;
    int ex = 0;
    const double f = std::frexp(std::fabs(d), &ex);  // |d| = f 2^ex, f in [0.5, 1)
    uint64_t mant = (uint64_t)std::ldexp(f, 53);      // exact: 53-bit integer
    int e = ex - 53;
    while ((mant & 1u) == 0) mant >>= 1, ++e;
    s_ = d < 0 ? -1 : 1;
    m_ = {(uint32_t)mant, (uint32_t)(mant >> 32)};
    trim(m_);
    e_ = e;
  }
  int sign() const { return s_; }

  friend Exact operator+(const Exact& a, const Exact& b) {
    if (a.s_ == 0) return b;
    if (b.s_ == 0) return a;
    const int e = std::min(a.e_, b.e_);
    const Mag A = shl(a.m_, a.e_ - e), B = shl(b.m_, b.e_ - e);
    Exact r;
    r.e_ = e;
    if (a.s_ == b.s_) {
      r.m_ = add_mag(A, B);
      r.s_ = a.s_;
    } else {
      const int c = cmp_mag(A, B);
      if (c == 0) return Exact();
      r.m_ = c > 0 ? sub_mag(A, B) : sub_mag(B, A);
      r.s_ = c > 0 ? a.s_ : b.s_;
    }
    r.normalise();
    return r;
  }
  friend Exact operator-(const Exact& a, const Exact& b) {
    Exact nb = b;
    nb.s_ = -nb.s_;
    return a + nb;
  }
  friend Exact operator*(const Exact& a, const Exact& b) {
    Exact r;
    if (a.s_ == 0 || b.s_ == 0) return r;
    r.s_ = a.s_ * b.s_;
    r.m_ = mul_mag(a.m_, b.m_);
    r.e_ = a.e_ + b.e_;
    r.normalise();
    return r;
  }

 private:
  // drop whole zero limbs at the bottom (keeps the numbers short)
  void normalise() {
    size_t z = 0;
    while (z < m_.size() && m_[z] == 0) ++z;
    if (z == m_.size()) {
      *this = Exact();
      return;
    }
    if (z) {
      m_.erase(m_.begin(), m_.begin() + z);
      e_ += 32 * (int)z;
    }
  }
  int s_ = 0;
  Mag m_;
  int e_ = 0;
};

inline int sgn(const Exact& x) { return x.sign(); }

// ------------------------------------------------------------ polynomials
template <class N>
struct V {
  N x, y, z;
};
template <class N>
V<N> vsub(const V<N>& a, const V<N>& b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class N>
V<N> vadd(const V<N>& a, const V<N>& b) {
  return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class N>
V<N> vscl(const V<N>& a, const N& s) {
  return {a.x * s, a.y * s, a.z * s};
}
template <class N>
N vdot(const V<N>& a, const V<N>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class N>
V<N> vcrs(const V<N>& a, const V<N>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class N>
V<N> pos(const Atom& a) {
  return {N(a.x), N(a.y), N(a.z)};
}
template <class N>
N weight(const Atom& a) {
  return N(a.R) * N(a.R);
}

// Quantities relative to the base atom i: a_q = p_q - p_i and
// b_q = |a_q|^2 - w_q + w_i, so that pi_q(x) - pi_i(x) = b_q - 2 a_q . (x - p_i).
template <class N>
struct Rel {
  V<N> a;
  N b;
};
template <class N>
Rel<N> rel(const Atom& i, const Atom& q) {
  Rel<N> r;
  r.a = vsub(pos<N>(q), pos<N>(i));
  r.b = vdot(r.a, r.a) - weight<N>(q) + weight<N>(i);
  return r;
}

// Tetrahedron (i, j, k, l).  With c_j = a_k x a_l, c_k = a_l x a_j,
// c_l = a_j x a_k and D = a_j . c_j the orthocentre is
// y = p_i + U / (2 D), U = b_j c_j + b_k c_k + b_l c_l.
//   size  (2D)^2 pi_i(y)         = U.U - 4 D^2 w_i
//   side  D (pi_m(y) - pi_i(y))   = D b_m - a_m . U
template <class N>
struct TetP {
  Rel<N> j, k, l;
  V<N> cj, ck, cl, U;
  N D, wi;
  TetP() = default;
  TetP(const Atom& I, const Atom& J, const Atom& K, const Atom& L) {
    j = rel<N>(I, J), k = rel<N>(I, K), l = rel<N>(I, L);
    cj = vcrs(k.a, l.a), ck = vcrs(l.a, j.a), cl = vcrs(j.a, k.a);
    D = vdot(j.a, cj);
    U = vadd(vadd(vscl(cj, j.b), vscl(ck, k.b)), vscl(cl, l.b));
    wi = weight<N>(I);
  }
  N size() const { return vdot(U, U) - N(4.0) * D * D * wi; }
  N side(const Rel<N>& m) const { return D * m.b - vdot(m.a, U); }
};

// Triangle (i, j, k).  With n = a_j x a_k, N2 = n.n, e_j = a_k x n,
// e_k = n x a_j the point of the Laguerre edge's line in the plane of the
// centres is y = p_i + U / (2 N2), U = b_j e_j + b_k e_k.
//   size  (2 N2)^2 pi_i(y)        = U.U - 4 N2^2 w_i
//   side  N2 (pi_m(y) - pi_i(y))   = N2 b_m - a_m . U
template <class N>
struct TriP {
  Rel<N> j, k;
  V<N> n, ej, ek, U;
  N N2, wi;
  TriP() = default;
  TriP(const Atom& I, const Atom& J, const Atom& K) {
    j = rel<N>(I, J), k = rel<N>(I, K);
    n = vcrs(j.a, k.a);
    N2 = vdot(n, n);
    ej = vcrs(k.a, n), ek = vcrs(n, j.a);
    U = vadd(vscl(ej, j.b), vscl(ek, k.b));
    wi = weight<N>(I);
  }
  N size() const { return vdot(U, U) - N(4.0) * N2 * N2 * wi; }
  N side(const Rel<N>& m) const { return N2 * m.b - vdot(m.a, U); }
};

// Edge (i, j).  With L2 = a_j.a_j the centre of the disk where the radical
// plane cuts the balls is y = p_i + b_j a_j / (2 L2).
//   size  4 L2 pi_i(y)            = b_j^2 - 4 L2 w_i
//   side  L2 (pi_m(y) - pi_i(y))   = L2 b_m - b_j (a_m . a_j)
template <class N>
struct EdgeP {
  Rel<N> j;
  N L2, wi;
  EdgeP(const Atom& I, const Atom& J) {
    j = rel<N>(I, J);
    L2 = vdot(j.a, j.a);
    wi = weight<N>(I);
  }
  N size() const { return j.b * j.b - N(4.0) * L2 * wi; }
  N side(const Rel<N>& m) const { return L2 * m.b - j.b * vdot(m.a, j.a); }
};

// Perturbed sign: the value's sign if non-zero, else that of the first
// non-zero weight partial in ascending atom index.
int sos(const Exact& value, std::vector<std::pair<int, Exact>> partials, Stats& st) {
  if (sgn(value) != 0) return sgn(value);
  ++st.sos;
  std::sort(partials.begin(), partials.end(),
            [](const std::pair<int, Exact>& a, const std::pair<int, Exact>& b) { return a.first < b.first; });
  for (const auto& p : partials)
    if (sgn(p.second) != 0) return sgn(p.second);
  return 0;  // unreachable for the predicates here (see predicates.h)
}

const Exact kTwo(2.0), kFour(4.0);

}  // namespace

int orient(const Atom& i, const Atom& j, const Atom& k, const Atom& l, Stats& st) {
  {
    const V<Flt> a = vsub(pos<Flt>(j), pos<Flt>(i)), b = vsub(pos<Flt>(k), pos<Flt>(i)),
                 c = vsub(pos<Flt>(l), pos<Flt>(i));
    const int s = certain_sign(vdot(a, vcrs(b, c)));
    if (s != 2) return s;
  }
  ++st.exact;
  const V<Exact> a = vsub(pos<Exact>(j), pos<Exact>(i)), b = vsub(pos<Exact>(k), pos<Exact>(i)),
                 c = vsub(pos<Exact>(l), pos<Exact>(i));
  return sgn(vdot(a, vcrs(b, c)));
}

bool collinear(const Atom& i, const Atom& j, const Atom& k, Stats& st) {
  {
    const V<Flt> n = vcrs(vsub(pos<Flt>(j), pos<Flt>(i)), vsub(pos<Flt>(k), pos<Flt>(i)));
    if (certain_sign(n.x) != 2 && certain_sign(n.x) != 0) return false;
    if (certain_sign(n.y) != 2 && certain_sign(n.y) != 0) return false;
    if (certain_sign(n.z) != 2 && certain_sign(n.z) != 0) return false;
  }
  ++st.exact;
  const V<Exact> n = vcrs(vsub(pos<Exact>(j), pos<Exact>(i)), vsub(pos<Exact>(k), pos<Exact>(i)));
  return sgn(n.x) == 0 && sgn(n.y) == 0 && sgn(n.z) == 0;
}

// ------------------------------------------------------------ tetrahedron
int tet_size(const Atom& I, const Atom& J, const Atom& K, const Atom& L, Stats& st) {
  {
    const int s = certain_sign(TetP<Flt>(I, J, K, L).size());
    if (s != 2) return s;
  }
  ++st.exact;
  const TetP<Exact> t(I, J, K, L);
  const V<Exact> C = vadd(vadd(t.cj, t.ck), t.cl);
  // d size / d w_q: -2 U.c_q for q = j, k, l; 2 U.C - 4 D^2 for i
  return sos(t.size(),
             {{J.id, Exact() - kTwo * vdot(t.U, t.cj)},
              {K.id, Exact() - kTwo * vdot(t.U, t.ck)},
              {L.id, Exact() - kTwo * vdot(t.U, t.cl)},
              {I.id, kTwo * vdot(t.U, C) - kFour * t.D * t.D}},
             st);
}

int tet_side(const Atom& I, const Atom& J, const Atom& K, const Atom& L, const Atom& M, Stats& st) {
  {
    const TetP<Flt> t(I, J, K, L);
    const int sd = certain_sign(t.D);
    const int s = certain_sign(t.side(rel<Flt>(I, M)));
    if (s != 2 && sd != 2 && sd != 0) return s * sd;
  }
  ++st.exact;
  const TetP<Exact> t(I, J, K, L);
  const Rel<Exact> m = rel<Exact>(I, M);
  const V<Exact> C = vadd(vadd(t.cj, t.ck), t.cl);
  // d side / d w_q: -D for m; a_m.c_q for q = j, k, l; D - a_m.C for i
  const int s = sos(t.side(m),
                    {{M.id, Exact() - t.D},
                     {J.id, vdot(m.a, t.cj)},
                     {K.id, vdot(m.a, t.ck)},
                     {L.id, vdot(m.a, t.cl)},
                     {I.id, t.D - vdot(m.a, C)}},
                    st);
  return s * sgn(t.D);
}

// --------------------------------------------------------------- triangle
int tri_size(const Atom& I, const Atom& J, const Atom& K, Stats& st) {
  {
    const int s = certain_sign(TriP<Flt>(I, J, K).size());
    if (s != 2) return s;
  }
  ++st.exact;
  const TriP<Exact> t(I, J, K);
  const V<Exact> E = vadd(t.ej, t.ek);
  return sos(t.size(),
             {{J.id, Exact() - kTwo * vdot(t.U, t.ej)},
              {K.id, Exact() - kTwo * vdot(t.U, t.ek)},
              {I.id, kTwo * vdot(t.U, E) - kFour * t.N2 * t.N2}},
             st);
}

int tri_side(const Atom& I, const Atom& J, const Atom& K, const Atom& M, Stats& st) {
  {
    const int s = certain_sign(TriP<Flt>(I, J, K).side(rel<Flt>(I, M)));
    if (s != 2) return s;
  }
  ++st.exact;
  const TriP<Exact> t(I, J, K);
  const Rel<Exact> m = rel<Exact>(I, M);
  const V<Exact> E = vadd(t.ej, t.ek);
  return sos(t.side(m),
             {{M.id, Exact() - t.N2},
              {J.id, vdot(m.a, t.ej)},
              {K.id, vdot(m.a, t.ek)},
              {I.id, t.N2 - vdot(m.a, E)}},
             st);
}

// ------------------------------------------------------------------- edge
int edge_size(const Atom& I, const Atom& J, Stats& st) {
  {
    const int s = certain_sign(EdgeP<Flt>(I, J).size());
    if (s != 2) return s;
  }
  ++st.exact;
  const EdgeP<Exact> e(I, J);
  return sos(e.size(), {{J.id, Exact() - kTwo * e.j.b}, {I.id, kTwo * e.j.b - kFour * e.L2}}, st);
}

int edge_side(const Atom& I, const Atom& J, const Atom& M, Stats& st) {
  {
    const int s = certain_sign(EdgeP<Flt>(I, J).side(rel<Flt>(I, M)));
    if (s != 2) return s;
  }
  ++st.exact;
  const EdgeP<Exact> e(I, J);
  const Rel<Exact> m = rel<Exact>(I, M);
  const Exact amaj = vdot(m.a, e.j.a);
  return sos(e.side(m), {{M.id, Exact() - e.L2}, {J.id, amaj}, {I.id, e.L2 - amaj}}, st);
}

// ----------------------------------------------------------------- vertex
int vertex_side(const Atom& I, const Atom& M, Stats& st) {
  {
    const int s = certain_sign(rel<Flt>(I, M).b);
    if (s != 2) return s;
  }
  ++st.exact;
  // d b_m / d w_m = -1, d b_m / d w_i = +1
  return sos(rel<Exact>(I, M).b, {{M.id, Exact(-1.0)}, {I.id, Exact(1.0)}}, st);
}

int exact_sign_test(double a, double b, double c, double d, double e) {
  return sgn(Exact(a) + Exact(b) * Exact(c) - Exact(d) * Exact(e));
}

struct BaseFlt {
  std::vector<Rel<Flt>> rel;  // neighbour q relative to atom i
};
struct TetFlt {
  TetP<Flt> p;
};
struct TriFlt {
  TriP<Flt> p;
};
struct EdgeFlt {
  EdgeP<Flt> p;
};

Base::Base(const Atom* atoms, int i, const int* nb, int nnb, Stats& st)
    : atoms_(atoms), i_(i), nb_(nb), st_(st), f_(new BaseFlt) {
  f_->rel.reserve(nnb);
  for (int q = 0; q < nnb; ++q) f_->rel.push_back(rel<Flt>(atoms[i], atoms[nb[q]]));
}
Base::~Base() { delete f_; }

// The simplex polynomials from the cached relative data (the same operations
// as TetP / TriP / EdgeP on the atoms, in the same order).
template <class N>
TetP<N> tet_from(const Rel<N>& j, const Rel<N>& k, const Rel<N>& l, const N& wi) {
  TetP<N> t;
  t.j = j, t.k = k, t.l = l;
  t.cj = vcrs(k.a, l.a), t.ck = vcrs(l.a, j.a), t.cl = vcrs(j.a, k.a);
  t.D = vdot(j.a, t.cj);
  t.U = vadd(vadd(vscl(t.cj, j.b), vscl(t.ck, k.b)), vscl(t.cl, l.b));
  t.wi = wi;
  return t;
}
template <class N>
TriP<N> tri_from(const Rel<N>& j, const Rel<N>& k, const N& wi) {
  TriP<N> t;
  t.j = j, t.k = k;
  t.n = vcrs(j.a, k.a);
  t.N2 = vdot(t.n, t.n);
  t.ej = vcrs(k.a, t.n), t.ek = vcrs(t.n, j.a);
  t.U = vadd(vscl(t.ej, j.b), vscl(t.ek, k.b));
  t.wi = wi;
  return t;
}

TetTest::TetTest(Base& b, int j, int k, int l) : b_(b), j_(j), k_(k), l_(l) {
  static_assert(sizeof(TetFlt) <= sizeof(buf_), "buffer");
  const auto& R = b.f_->rel;
  f_ = new (buf_) TetFlt{tet_from(R[j], R[k], R[l], weight<Flt>(b.atom(-1)))};
  const int s = certain_sign(f_->p.D);
  sd_ = (s != 2) ? s : oracle_pred::orient(b.atom(-1), b.atom(j), b.atom(k), b.atom(l), b.st_);
}
TetTest::~TetTest() { f_->~TetFlt(); }
int TetTest::size() {
  const int s = certain_sign(f_->p.size());
  return s != 2 ? s : tet_size(b_.atom(-1), b_.atom(j_), b_.atom(k_), b_.atom(l_), b_.st_);
}
int TetTest::side(int m) {
  const int s = certain_sign(f_->p.side(b_.f_->rel[m]));
  return s != 2 ? s * sd_ : tet_side(b_.atom(-1), b_.atom(j_), b_.atom(k_), b_.atom(l_), b_.atom(m), b_.st_);
}

TriTest::TriTest(Base& b, int j, int k) : b_(b), j_(j), k_(k) {
  static_assert(sizeof(TriFlt) <= sizeof(buf_), "buffer");
  const auto& R = b.f_->rel;
  f_ = new (buf_) TriFlt{tri_from(R[j], R[k], weight<Flt>(b.atom(-1)))};
}
TriTest::~TriTest() { f_->~TriFlt(); }
int TriTest::size() {
  const int s = certain_sign(f_->p.size());
  return s != 2 ? s : tri_size(b_.atom(-1), b_.atom(j_), b_.atom(k_), b_.st_);
}
int TriTest::side(int m) {
  const int s = certain_sign(f_->p.side(b_.f_->rel[m]));
  return s != 2 ? s : tri_side(b_.atom(-1), b_.atom(j_), b_.atom(k_), b_.atom(m), b_.st_);
}

EdgeTest::EdgeTest(Base& b, int j) : b_(b), j_(j) {
  static_assert(sizeof(EdgeFlt) <= sizeof(buf_), "buffer");
  EdgeP<Flt> e(b.atom(-1), b.atom(j));
  f_ = new (buf_) EdgeFlt{e};
}
EdgeTest::~EdgeTest() { f_->~EdgeFlt(); }
int EdgeTest::size() {
  const int s = certain_sign(f_->p.size());
  return s != 2 ? s : edge_size(b_.atom(-1), b_.atom(j_), b_.st_);
}
int EdgeTest::side(int m) {
  const int s = certain_sign(f_->p.side(b_.f_->rel[m]));
  return s != 2 ? s : edge_side(b_.atom(-1), b_.atom(j_), b_.atom(m), b_.st_);
}

}  // namespace oracle_pred
