// sasa_oracle.cc -- plain FP64 CPU reference of the dSASA hot path.
//
// TEST INFRASTRUCTURE ONLY (see sasa_oracle.h).  Deliberately simple and slow:
// brute-force neighbour search, the dual complex decided from its definition
// simplex by simplex, and derivatives by forward-mode dual numbers.  It shares
// no code with the HIP library.
//
// Notation follows the paper (arXiv 2401.10462, Methods): p_i atom centre,
// R_i = r_i + probe, weight d_i = R_i^2 (called w here), power distance
// pi_i(x) = |x - p_i|^2 - w_i, Laguerre cell L_i = {x : pi_i(x) <= pi_j(x) all j},
// ball B_i = {pi_i <= 0}.

#include "sasa_oracle.h"

#include "predicates.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- plain vectors
struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 crs(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double nrm2(V3 a) { return dot(a, a); }

// ---------------------------------------------------------- forward-mode duals
// A value with its gradient with respect to the 12 coordinates of (at most)
// four atoms; slot s covers coordinates 3s..3s+2.
constexpr int NG = 12;
struct D {
  double v;
  double g[NG];
};
inline D cst(double v) {
  D r;
  r.v = v;
  std::memset(r.g, 0, sizeof(r.g));
  return r;
}
inline D operator+(const D& a, const D& b) {
  D r;
  r.v = a.v + b.v;
  for (int k = 0; k < NG; ++k) r.g[k] = a.g[k] + b.g[k];
  return r;
}
inline D operator-(const D& a, const D& b) {
  D r;
  r.v = a.v - b.v;
  for (int k = 0; k < NG; ++k) r.g[k] = a.g[k] - b.g[k];
  return r;
}
inline D operator*(const D& a, const D& b) {
  D r;
  r.v = a.v * b.v;
  for (int k = 0; k < NG; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k];
  return r;
}
inline D operator*(const D& a, double s) {
  D r;
  r.v = a.v * s;
  for (int k = 0; k < NG; ++k) r.g[k] = a.g[k] * s;
  return r;
}
inline D operator/(const D& a, const D& b) {
  D r;
  r.v = a.v / b.v;
  for (int k = 0; k < NG; ++k) r.g[k] = (a.g[k] * b.v - a.v * b.g[k]) / (b.v * b.v);
  return r;
}
inline D dsqrt(const D& a) {
  D r;
  r.v = std::sqrt(a.v);
  for (int k = 0; k < NG; ++k) r.g[k] = a.g[k] / (2.0 * r.v);
  return r;
}
inline D datan2(const D& y, const D& x) {
  D r;
  r.v = std::atan2(y.v, x.v);
  const double den = x.v * x.v + y.v * y.v;
  for (int k = 0; k < NG; ++k) r.g[k] = (x.v * y.g[k] - y.v * x.g[k]) / den;
  return r;
}

struct DV {
  D x, y, z;
};
inline DV dsub(const DV& a, const DV& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline DV dadd(const DV& a, const DV& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline DV dscl(const DV& a, const D& s) { return {a.x * s, a.y * s, a.z * s}; }
inline D ddot(const DV& a, const DV& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline DV dcrs(const DV& a, const DV& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline D dnorm(const DV& a) { return dsqrt(ddot(a, a)); }

// A point whose three coordinates are the independent variables of slot s.
inline DV seed(V3 p, int s) {
  DV r{cst(p.x), cst(p.y), cst(p.z)};
  r.x.g[3 * s + 0] = 1.0;
  r.y.g[3 * s + 1] = 1.0;
  r.z.g[3 * s + 2] = 1.0;
  return r;
}
inline DV fixed(V3 p) { return {cst(p.x), cst(p.y), cst(p.z)}; }

// ------------------------------------------------------------ formula pieces

// Normalised inner solid angle at p_i of the tetrahedron (p_i, p_j, p_k, p_l)
// in the Van Oosterom--Strackee form (Methods, solid angle after Eq. 3),
// written with atan2 so that it stays correct past a right angle:
//   omega = atan2(|a.(b x c)|, abc + (a.b)c + (a.c)b + (b.c)a) / (2 pi),
// a = p_j - p_i, b = p_k - p_i, c = p_l - p_i.  omega is the fraction of the
// full sphere around p_i that the tetrahedron subtends.
//
// |a.(b x c)| is taken as s a.(b x c) with s the sign of the tetrahedron's
// orientation det[a; b; c] given by the caller (exactly, for a K-tetrahedron):
// the same value, and for a nearly flat tetrahedron the derivative of the
// right branch, which rounding could otherwise flip.
D solid_angle(const DV& pi, const DV& pj, const DV& pk, const DV& pl, int s) {
  const DV a = dsub(pj, pi), b = dsub(pk, pi), c = dsub(pl, pi);
  const D la = dnorm(a), lb = dnorm(b), lc = dnorm(c);
  const D num = ddot(a, dcrs(b, c)) * (double)s;
  const D den = la * lb * lc + ddot(a, b) * lc + ddot(a, c) * lb + ddot(b, c) * la;
  return datan2(num, den) * (1.0 / (2.0 * kPi));
}

// Normalised inner dihedral angle of the tetrahedron (p_i, p_j, p_k, p_l) along
// its edge p_i p_j, i.e. the angle between the faces (i,j,k) and (i,j,l), over
// 2 pi (Eq. 4).  The normals are n_k = e x (p_k - p_i), n_l = e x (p_l - p_i)
// with e = p_j - p_i, so the angle between them is the interior angle; it is
// taken as atan2(|n_k x n_l|, n_k . n_l) rather than arccos of the normalised
// dot product, which is the same angle without the loss of accuracy near 0, pi.
//
// n_k x n_l = (e . (a_k x a_l)) e for n_k = e x a_k, n_l = e x a_l, so
// |n_k x n_l| = |e| s det[e; a_k; a_l] with s the sign of that orientation,
// given by the caller (exactly, for a K-tetrahedron; see solid_angle).
D dihedral(const DV& pi, const DV& pj, const DV& pk, const DV& pl, int s) {
  const DV e = dsub(pj, pi);
  const DV ak = dsub(pk, pi), al = dsub(pl, pi);
  const DV nk = dcrs(e, ak);
  const DV nl = dcrs(e, al);
  return datan2(dnorm(e) * (ddot(e, dcrs(ak, al)) * (double)s), ddot(nk, nl)) * (1.0 / (2.0 * kPi));
}

// Area of the cap of sphere i that lies inside ball j: S_ij^(i) = 2 pi sqrt(d_i) h_i
// (edge term after Eq. 3).  h_i is the height of that cap: the plane of the
// two spheres' intersection circle lies at distance a_i = (d^2 + w_i - w_j)/(2d)
// from p_i along p_j - p_i, so h_i = R_i - a_i.
D cap_area(const DV& pi, double Ri, const DV& pj, double Rj) {
  const D d = dnorm(dsub(pj, pi));
  const D ai = (d * d + cst(Ri * Ri - Rj * Rj)) / (d * 2.0);
  return (cst(Ri) - ai) * (2.0 * kPi * Ri);
}

// One of the two triple points x common to the spheres i, j, k (Eq. 6): x lies
// on the line of equal power of the three weighted points, at power distance 0.
// y is the point of that line in the plane of the three centres; s = pi_i(y) < 0
// when the three spheres meet; x = y + sqrt(-s) n / |n|, n the plane normal.
// Returns false if the spheres have no common point.
bool triple_point(const DV& pi, double wi, const DV& pj, double wj, const DV& pk, double wk, DV* x) {
  const DV a = dsub(pj, pi), b = dsub(pk, pi);
  // Equal-power conditions relative to p_i: 2 a.y = |a|^2 - w_j + w_i, same for b.
  const D ba = ddot(a, a) + cst(wi - wj);
  const D bb = ddot(b, b) + cst(wi - wk);
  const D aa = ddot(a, a) * 2.0, ab = ddot(a, b) * 2.0, bbb = ddot(b, b) * 2.0;
  const D det = aa * bbb - ab * ab;
  const D alpha = (ba * bbb - bb * ab) / det;
  const D beta = (aa * bb - ab * ba) / det;
  const DV y = dadd(dscl(a, alpha), dscl(b, beta));
  const D s = ddot(y, y) - cst(wi);
  if (!(s.v < 0)) return false;
  const DV n = dcrs(a, b);
  const D t = dsqrt(cst(0.0) - s) / dnorm(n);
  *x = dadd(pi, dadd(y, dscl(n, t)));
  return true;
}

// Contribution S_ijk^(i) of the triple intersection to sphere i (Eq. 6):
//   S/2 = phi_ij(T_x) S_ij^(i) + phi_ik(T_x) S_ik^(i) - omega_i(T_x) 4 pi w_i,
// with T_x = (p_i, p_j, p_k, x), phi_ij(T_x) the normalised dihedral angle of
// T_x along edge ij, omega_i(T_x) its normalised solid angle at p_i.
D triple_term(const DV& pi, double Ri, const DV& pj, double Rj, const DV& pk, double Rk) {
  DV x;
  if (!triple_point(pi, Ri * Ri, pj, Rj * Rj, pk, Rk * Rk, &x)) return cst(0.0);
  // x lies on the side of a x b (a = p_j - p_i, b = p_k - p_i): det[a; b; x - p_i] > 0
  const D phij = dihedral(pi, pj, pk, x, +1);
  const D phik = dihedral(pi, pk, pj, x, -1);
  const D om = solid_angle(pi, pj, pk, x, +1);
  const D half = phij * cap_area(pi, Ri, pj, Rj) + phik * cap_area(pi, Ri, pk, Rk) -
                 om * (4.0 * kPi * Ri * Ri);
  return half * 2.0;
}

// ------------------------------------------------------------------ the run
using Tri = std::array<int, 3>;
using Tet = std::array<int, 4>;

}  // namespace

struct oracle_result {
  int64_t n = 0;
  std::vector<V3> p;
  std::vector<double> R, w;
  std::vector<oracle_pred::Atom> atom;  // the predicates' view of the input
  std::vector<std::vector<int>> nb;     // neighbours (overlapping or touching), ascending
  std::vector<uint8_t> vin, vext;
  std::vector<std::array<int, 2>> edges;
  std::vector<uint8_t> eext;
  std::vector<Tri> tris;
  std::vector<uint8_t> tnt, text;
  std::vector<Tet> tets;
  std::vector<double> area;
  std::vector<std::map<int, V3>> jac;  // jac[i][m] = dA_i/dp_m
  oracle_pred::Stats st;               // predicates decided exactly / by the perturbation
  int64_t flat = 0;                    // candidate simplices with coplanar / collinear centres

  bool ov(int i, int j) const { return std::binary_search(nb[i].begin(), nb[i].end(), j); }
};

namespace {

// Atoms j that can cut L_i cap B_i: for balls that are apart, the radical plane
// separates them, so pi_i < pi_j everywhere in B_i.  The test is widened by a
// relative 1e-9 so that touching balls (whose perturbed weights may overlap)
// are always listed; a listed ball that is apart changes no decision, since
// every decision about a point inside B_i finds it on the far side of that
// ball's plane.
void neighbours(oracle_result& r) {
  const int n = (int)r.n;
  r.nb.assign(n, {});
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = r.R[i] + r.R[j];
      if (nrm2(sub(r.p[j], r.p[i])) <= s * s * (1.0 + 1e-9)) {
        r.nb[i].push_back(j);
        r.nb[j].push_back(i);
      }
    }
  for (auto& v : r.nb) std::sort(v.begin(), v.end());
}

// The alpha = 0 dual complex K (Steps 1-2): sigma is in K iff the Laguerre
// face shared by its atoms' cells meets their balls.  That face lies in an
// affine space whose point y_sigma closest to the centres is the simplex's
// orthocentre.  Either y_sigma itself belongs to the face and lies inside the
// balls (sigma is "unattached" and of size pi(y_sigma) <= 0), or the face meets
// the balls elsewhere and then it meets them where it ends on a face one
// dimension lower, i.e. sigma is a face of a higher simplex of K.  So
// tetrahedra are decided first, then triangles, edges and vertices.  All
// signs are exact and symbolically perturbed (predicates.h), so the complex
// is that of weights moved by an infinitesimal, index-ordered amount: one
// consistent complex also for co-spherical inputs.
//
// An atom m that would cut y_sigma (pi_m(y) < pi_i(y)) while y is inside B_i
// overlaps B_i, so testing the neighbours of i is the whole emptiness test.

// Tetrahedron (i,j,k,l) is in K iff its orthocentre is inside the balls and no
// other atom has lower power there.
void tetrahedra(oracle_result& r) {
  const int n = (int)r.n;
  for (int i = 0; i < n; ++i) {
    const auto& N = r.nb[i];
    oracle_pred::Base B(r.atom.data(), i, N.data(), (int)N.size(), r.st);
    for (size_t a = 0; a < N.size(); ++a) {
      const int j = N[a];
      if (j < i) continue;
      for (size_t b = a + 1; b < N.size(); ++b) {
        const int k = N[b];
        if (!r.ov(j, k)) continue;
        for (size_t c = b + 1; c < N.size(); ++c) {
          const int l = N[c];
          if (!r.ov(j, l) || !r.ov(k, l)) continue;
          oracle_pred::TetTest T(B, (int)a, (int)b, (int)c);
          if (T.orient() == 0) {
            ++r.flat;
            continue;
          }
          if (T.size() > 0) continue;
          bool empty = true;
          for (size_t q = 0; q < N.size(); ++q) {
            if (q == a || q == b || q == c) continue;
            if (T.side((int)q) < 0) {
              empty = false;
              break;
            }
          }
          if (empty) r.tets.push_back({i, j, k, l});
        }
      }
    }
  }
  std::sort(r.tets.begin(), r.tets.end());
}

// Triangle (i,j,k) is in K iff it is a face of a K-tetrahedron, or the point
// of its Laguerre edge's line in the plane of the centres lies on the edge
// (no other atom has lower power there) and inside the balls.
void triangles(oracle_result& r) {
  const int n = (int)r.n;
  std::vector<Tri> faces;
  for (const auto& T : r.tets) {
    faces.push_back({T[1], T[2], T[3]});
    faces.push_back({T[0], T[2], T[3]});
    faces.push_back({T[0], T[1], T[3]});
    faces.push_back({T[0], T[1], T[2]});
  }
  std::sort(faces.begin(), faces.end());
  const auto& A = r.atom;
  for (int i = 0; i < n; ++i) {
    const auto& N = r.nb[i];
    oracle_pred::Base B(A.data(), i, N.data(), (int)N.size(), r.st);
    for (size_t a = 0; a < N.size(); ++a) {
      const int j = N[a];
      if (j < i) continue;
      for (size_t b = a + 1; b < N.size(); ++b) {
        const int k = N[b];
        if (!r.ov(j, k)) continue;
        const Tri t = {i, j, k};
        if (std::binary_search(faces.begin(), faces.end(), t)) {
          r.tris.push_back(t);
          continue;
        }
        if (oracle_pred::collinear(A[i], A[j], A[k], r.st)) {
          ++r.flat;
          continue;
        }
        oracle_pred::TriTest T(B, (int)a, (int)b);
        if (T.size() > 0) continue;
        bool on_edge = true;
        for (size_t q = 0; q < N.size(); ++q) {
          if (q == a || q == b) continue;
          if (T.side((int)q) < 0) {
            on_edge = false;
            break;
          }
        }
        if (on_edge) r.tris.push_back(t);
      }
    }
  }
  std::sort(r.tris.begin(), r.tris.end());
}

// Edge (i,j) is in K iff it lies on a K-triangle, or the centre of the disk
// where the radical plane cuts the balls lies in the Laguerre facet of i and j
// and inside the balls.
void edges(oracle_result& r) {
  const int n = (int)r.n;
  std::vector<std::vector<int>> has_tri(n);  // j in has_tri[i] if (i,j) is on a K-triangle
  for (const auto& t : r.tris) {
    has_tri[t[0]].push_back(t[1]);
    has_tri[t[0]].push_back(t[2]);
    has_tri[t[1]].push_back(t[2]);
  }
  for (auto& v : has_tri) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  const auto& A = r.atom;
  for (int i = 0; i < n; ++i) {
    const auto& N = r.nb[i];
    oracle_pred::Base B(A.data(), i, N.data(), (int)N.size(), r.st);
    for (size_t a = 0; a < N.size(); ++a) {
      const int j = N[a];
      if (j < i) continue;
      if (std::binary_search(has_tri[i].begin(), has_tri[i].end(), j)) {
        r.edges.push_back({i, j});
        continue;
      }
      if (r.p[i].x == r.p[j].x && r.p[i].y == r.p[j].y && r.p[i].z == r.p[j].z) {
        ++r.flat;  // one centre, two radii: the smaller ball has no cell
        continue;
      }
      oracle_pred::EdgeTest E(B, (int)a);
      if (E.size() > 0) continue;
      bool inside = true;
      for (size_t q = 0; q < N.size(); ++q) {
        if (q == a) continue;
        if (E.side((int)q) < 0) {
          inside = false;
          break;
        }
      }
      if (inside) r.edges.push_back({i, j});
    }
  }
  std::sort(r.edges.begin(), r.edges.end());
}

// Vertex i is in K iff L_i cap B_i is not empty: either a facet of L_i meets
// B_i (a K-edge at i), or no facet does and then B_i lies inside L_i, which
// holds iff p_i itself is in L_i (pi_m(p_i) >= -w_i for all m).
void vertices(oracle_result& r) {
  const int n = (int)r.n;
  r.vin.assign(n, 0);
  for (const auto& e : r.edges) r.vin[e[0]] = r.vin[e[1]] = 1;
  for (int i = 0; i < n; ++i) {
    if (r.vin[i]) continue;
    bool inside = true;
    for (int m : r.nb[i]) {
      if (oracle_pred::vertex_side(r.atom[i], r.atom[m], r.st) < 0) {
        inside = false;
        break;
      }
    }
    r.vin[i] = inside;
  }
}

// Classification (GPU section, extraction of exterior simplices).  A triangle
// with at most one K-tetrahedron on it is exterior; its coefficient is
// c_t = 1 - n_t / 2.  An edge is exterior iff it lies on an exterior triangle or
// on no K-triangle at all: otherwise the K-tetrahedra close up around it and
// its outer dihedral coefficient is exactly 0.  A vertex is exterior iff it has
// an exterior K-edge or no K-edge (then it is an isolated ball); otherwise its
// outer solid angle is exactly 0.  Both rules imply the paper's "an edge is
// exterior only if both its vertices are".
void classify(oracle_result& r) {
  const int n = (int)r.n;
  std::map<Tri, int> nt;
  for (const auto& t : r.tris) nt[t] = 0;
  for (const auto& T : r.tets) {
    const Tri faces[4] = {{T[1], T[2], T[3]}, {T[0], T[2], T[3]}, {T[0], T[1], T[3]}, {T[0], T[1], T[2]}};
    for (const auto& f : faces) nt[f] += 1;  // a K-tet's faces are in K
  }
  r.tnt.resize(r.tris.size());
  r.text.resize(r.tris.size());
  std::map<std::array<int, 2>, int> e_state;  // 0: no triangle yet, 1: only interior, 2: exterior
  for (const auto& e : r.edges) e_state[e] = 0;
  for (size_t t = 0; t < r.tris.size(); ++t) {
    const auto& T = r.tris[t];
    r.tnt[t] = (uint8_t)nt[T];
    r.text[t] = r.tnt[t] <= 1;
    const std::array<int, 2> es[3] = {{T[0], T[1]}, {T[0], T[2]}, {T[1], T[2]}};
    for (const auto& e : es) {
      int& s = e_state[e];
      s = std::max(s, r.text[t] ? 2 : 1);
    }
  }
  r.eext.resize(r.edges.size());
  r.vext.assign(n, 0);
  std::vector<uint8_t> has_edge(n, 0);
  for (size_t k = 0; k < r.edges.size(); ++k) {
    const int s = e_state[r.edges[k]];
    r.eext[k] = (s == 0 || s == 2);
    has_edge[r.edges[k][0]] = has_edge[r.edges[k][1]] = 1;
    if (r.eext[k]) r.vext[r.edges[k][0]] = r.vext[r.edges[k][1]] = 1;
  }
  for (int i = 0; i < n; ++i)
    if (r.vin[i] && !has_edge[i]) r.vext[i] = 1;
}

// Exact sign of det[p_b - p_a; p_c - p_a; p_d - p_a] (never 0 for a K-tetrahedron).
int orient_of(oracle_result& r, int a, int b, int c, int d) {
  return oracle_pred::orient(r.atom[a], r.atom[b], r.atom[c], r.atom[d], r.st);
}

void add_grad(std::map<int, V3>& row, int atom, const D& f, int slot, double scale) {
  V3& g = row[atom];
  g.x += scale * f.g[3 * slot + 0];
  g.y += scale * f.g[3 * slot + 1];
  g.z += scale * f.g[3 * slot + 2];
}

// Per-atom area, Eq. 1, and its gradient, Eq. 2:
//   A_i = Omega_i 4 pi w_i - sum_{ext e=ij} Phi_ij S_ij^(i) + sum_{ext t=ijk} c_ijk S_ijk^(i)
//   Omega_i = 1 - sum_{K-tets T at i} omega_i(T)            (Eq. 3)
//   Phi_ij  = 1 - sum_{K-tets T on ij} phi_ij(T)             (Eqs. 4, 5)
// Each piece is a dual number over the atoms it depends on, so the product rule
// of Eq. 2 and the chain rule through the triple point of Eq. 7 are exact.
void areas(oracle_result& r) {
  const int n = (int)r.n;
  r.area.assign(n, 0.0);
  r.jac.assign(n, {});
  std::vector<std::vector<int>> tets_at(n);
  for (size_t t = 0; t < r.tets.size(); ++t)
    for (int v : r.tets[t]) tets_at[v].push_back((int)t);
  std::vector<std::vector<int>> edges_at(n), tris_at(n);
  for (size_t e = 0; e < r.edges.size(); ++e)
    if (r.eext[e]) {
      edges_at[r.edges[e][0]].push_back((int)e);
      edges_at[r.edges[e][1]].push_back((int)e);
    }
  for (size_t t = 0; t < r.tris.size(); ++t)
    if (r.text[t])
      for (int v : r.tris[t]) tris_at[v].push_back((int)t);

  for (int i = 0; i < n; ++i) {
    if (!r.vin[i] || !r.vext[i]) continue;  // interior or hidden atoms: A_i = 0
    auto& row = r.jac[i];
    row[i] = V3{0, 0, 0};
    const double Si = 4.0 * kPi * r.w[i];
    double A = 0.0;
    // Vertex term.
    double Omega = 1.0;
    for (int t : tets_at[i]) {
      const Tet& T = r.tets[t];
      int o[3], c = 0;
      for (int v : T)
        if (v != i) o[c++] = v;
      const D om = solid_angle(seed(r.p[i], 0), seed(r.p[o[0]], 1), seed(r.p[o[1]], 2), seed(r.p[o[2]], 3),
                               orient_of(r, i, o[0], o[1], o[2]));
      Omega -= om.v;
      add_grad(row, i, om, 0, -Si);
      for (int s = 0; s < 3; ++s) add_grad(row, o[s], om, s + 1, -Si);
    }
    A += Omega * Si;
    // Edge terms.
    for (int e : edges_at[i]) {
      const int j = r.edges[e][0] == i ? r.edges[e][1] : r.edges[e][0];
      const D S = cap_area(seed(r.p[i], 0), r.R[i], seed(r.p[j], 1), r.R[j]);
      double Phi = 1.0;
      for (int t : tets_at[i]) {
        const Tet& T = r.tets[t];
        if (std::find(T.begin(), T.end(), j) == T.end()) continue;
        int o[2], c = 0;
        for (int v : T)
          if (v != i && v != j) o[c++] = v;
        const D ph = dihedral(seed(r.p[i], 0), seed(r.p[j], 1), seed(r.p[o[0]], 2), seed(r.p[o[1]], 3),
                              orient_of(r, i, j, o[0], o[1]));
        Phi -= ph.v;
        // d(Phi S) gets -S dphi
        add_grad(row, i, ph, 0, S.v);
        add_grad(row, j, ph, 1, S.v);
        add_grad(row, o[0], ph, 2, S.v);
        add_grad(row, o[1], ph, 3, S.v);
      }
      A -= Phi * S.v;
      add_grad(row, i, S, 0, -Phi);
      add_grad(row, j, S, 1, -Phi);
    }
    // Triangle terms.
    for (int t : tris_at[i]) {
      const Tri& T = r.tris[t];
      int o[2], c = 0;
      for (int v : T)
        if (v != i) o[c++] = v;
      const double ct = 1.0 - 0.5 * r.tnt[t];
      const D St = triple_term(seed(r.p[i], 0), r.R[i], seed(r.p[o[0]], 1), r.R[o[0]], seed(r.p[o[1]], 2),
                               r.R[o[1]]);
      A += ct * St.v;
      add_grad(row, i, St, 0, ct);
      add_grad(row, o[0], St, 1, ct);
      add_grad(row, o[1], St, 2, ct);
    }
    r.area[i] = A;
  }
}

V3 load(const double* q) { return {q[0], q[1], q[2]}; }

}  // namespace

extern "C" {

oracle_result* oracle_run(int64_t n, const double* xyz, const double* radii, double probe) {
  if (n < 0 || (n > 0 && (!xyz || !radii)) || !(probe >= 0) || !std::isfinite(probe)) return nullptr;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return nullptr;
  for (int64_t i = 0; i < n; ++i)
    if (!(radii[i] > 0) || !std::isfinite(radii[i])) return nullptr;
  auto* r = new oracle_result;
  r->n = n;
  r->p.resize(n);
  r->R.resize(n);
  r->w.resize(n);
  r->atom.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    r->p[i] = load(xyz + 3 * i);
    r->R[i] = radii[i] + probe;  // probe-inflated sphere
    r->w[i] = r->R[i] * r->R[i];  // weight d_i = (r_i + probe)^2
    r->atom[i] = {r->p[i].x, r->p[i].y, r->p[i].z, r->R[i], (int)i};
  }
  neighbours(*r);
  // Two balls with one centre and one radius have the same cell: the complex
  // (and each atom's share of the area) is undefined, so such input is refused.
  // With different radii the smaller ball has no cell and is hidden.
  for (int64_t i = 0; i < n; ++i)
    for (int j : r->nb[i])
      if (j > i && r->p[i].x == r->p[j].x && r->p[i].y == r->p[j].y && r->p[i].z == r->p[j].z &&
          r->R[i] == r->R[j]) {
        delete r;
        return nullptr;
      }
  tetrahedra(*r);
  triangles(*r);
  edges(*r);
  vertices(*r);
  classify(*r);
  areas(*r);
  return r;
}

void oracle_free(oracle_result* r) { delete r; }

int64_t oracle_count(const oracle_result* r, int what) {
  switch (what) {
    case 0: return std::count(r->vin.begin(), r->vin.end(), 1);
    case 1: return (int64_t)r->edges.size();
    case 2: return (int64_t)r->tris.size();
    case 3: return (int64_t)r->tets.size();
    case 4: {
      int64_t c = 0;
      for (int64_t i = 0; i < r->n; ++i) c += r->vin[i] && r->vext[i];
      return c;
    }
    case 5: return std::count(r->eext.begin(), r->eext.end(), 1);
    case 6: return std::count(r->text.begin(), r->text.end(), 1);
    case 7: {
      int64_t c = 0;
      for (const auto& row : r->jac) c += (int64_t)row.size();
      return c;
    }
    case 8: return r->st.exact;
    case 9: return r->st.sos;
    case 10: return r->flat;
  }
  return -1;
}

void oracle_area(const oracle_result* r, double* area) {
  std::copy(r->area.begin(), r->area.end(), area);
}

void oracle_vjp(const oracle_result* r, const double* u, double* g) {
  std::fill(g, g + 3 * r->n, 0.0);
  for (int64_t i = 0; i < r->n; ++i)
    for (const auto& kv : r->jac[i]) {
      g[3 * kv.first + 0] += u[i] * kv.second.x;
      g[3 * kv.first + 1] += u[i] * kv.second.y;
      g[3 * kv.first + 2] += u[i] * kv.second.z;
    }
}

void oracle_dadx(const oracle_result* r, double* g) {
  std::vector<double> ones(r->n, 1.0);
  oracle_vjp(r, ones.data(), g);
}

void oracle_jacobian(const oracle_result* r, int32_t* rows, int32_t* cols, double* vals3) {
  int64_t c = 0;
  for (int64_t i = 0; i < r->n; ++i)
    for (const auto& kv : r->jac[i]) {
      rows[c] = (int32_t)i;
      cols[c] = kv.first;
      vals3[3 * c + 0] = kv.second.x;
      vals3[3 * c + 1] = kv.second.y;
      vals3[3 * c + 2] = kv.second.z;
      ++c;
    }
}

void oracle_vertices(const oracle_result* r, uint8_t* in_k, uint8_t* exterior) {
  for (int64_t i = 0; i < r->n; ++i) {
    in_k[i] = r->vin[i];
    exterior[i] = r->vin[i] && r->vext[i];
  }
}

void oracle_edges(const oracle_result* r, int32_t* e2, uint8_t* exterior) {
  for (size_t k = 0; k < r->edges.size(); ++k) {
    e2[2 * k] = r->edges[k][0];
    e2[2 * k + 1] = r->edges[k][1];
    exterior[k] = r->eext[k];
  }
}

void oracle_triangles(const oracle_result* r, int32_t* t3, uint8_t* n_tet, uint8_t* exterior) {
  for (size_t k = 0; k < r->tris.size(); ++k) {
    for (int c = 0; c < 3; ++c) t3[3 * k + c] = r->tris[k][c];
    n_tet[k] = r->tnt[k];
    exterior[k] = r->text[k];
  }
}

void oracle_tetrahedra(const oracle_result* r, int32_t* t4) {
  for (size_t k = 0; k < r->tets.size(); ++k)
    for (int c = 0; c < 4; ++c) t4[4 * k + c] = r->tets[k][c];
}

double oracle_solid_angle(const double* pi, const double* pj, const double* pk, const double* pl) {
  const DV a = fixed(load(pi)), b = fixed(load(pj)), c = fixed(load(pk)), d = fixed(load(pl));
  const D o = ddot(dsub(b, a), dcrs(dsub(c, a), dsub(d, a)));
  return solid_angle(a, b, c, d, o.v < 0 ? -1 : 1).v;
}
double oracle_dihedral(const double* pi, const double* pj, const double* pk, const double* pl) {
  const DV a = fixed(load(pi)), b = fixed(load(pj)), c = fixed(load(pk)), d = fixed(load(pl));
  const D o = ddot(dsub(b, a), dcrs(dsub(c, a), dsub(d, a)));
  return dihedral(a, b, c, d, o.v < 0 ? -1 : 1).v;
}
double oracle_cap_area(const double* pi, double Ri, const double* pj, double Rj) {
  return cap_area(fixed(load(pi)), Ri, fixed(load(pj)), Rj).v;
}
double oracle_triple_term(const double* pi, double Ri, const double* pj, double Rj, const double* pk, double Rk) {
  return triple_term(fixed(load(pi)), Ri, fixed(load(pj)), Rj, fixed(load(pk)), Rk).v;
}

}  // extern "C"
