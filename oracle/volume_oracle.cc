// volume_oracle.cc -- plain FP64 per-atom volumes (TEST INFRASTRUCTURE ONLY).
//
// The volume of atom i is that of its Laguerre intersection cell B_i ∩ L_i,
// the cell the area of Eq. 1 is the spherical boundary of (Methods; the
// Discussion names volumes and their derivatives as the next measure on the
// same cells).  By the divergence theorem applied to x - p_i over that cell,
//   3 V_i = R_i A_i + sum_j h_ij F_ij,
// where h_ij is the signed distance from p_i of the radical plane of i and j
// (positive towards p_j) and F_ij the area of the flat face of the cell on
// that plane.  The gradient of the molecular volume V = sum_i V_i with
// respect to p_i is the flux of a unit translation of sphere i through its
// exposed part, which by the closed boundary of the cell is
//   dV/dp_i = - sum_j F_ij (p_j - p_i) / |p_j - p_i|.
// F_ij is computed here from its definition: the disk where the radical
// plane cuts B_i, clipped by the half-planes pi_i <= pi_k of every other atom
// k whose ball meets B_i (written out in plane coordinates), as an exact
// convex-polygon-with-disk area.  A_i comes from the oracle's Eq. 1.
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

struct P2 {
  double x, y;
};

double cross(P2 a, P2 b) { return a.x * b.y - a.y * b.x; }

// Clip a convex polygon by a s + b t <= c (Sutherland-Hodgman, one edge).
std::vector<P2> clip(const std::vector<P2>& poly, double a, double b, double c) {
  std::vector<P2> out;
  const size_t m = poly.size();
  for (size_t k = 0; k < m; ++k) {
    const P2 p = poly[k], q = poly[(k + 1) % m];
    const double fp = a * p.x + b * p.y - c, fq = a * q.x + b * q.y - c;
    if (fp <= 0.0) out.push_back(p);
    if ((fp < 0.0 && fq > 0.0) || (fp > 0.0 && fq < 0.0)) {
      const double t = fp / (fp - fq);
      out.push_back({p.x + t * (q.x - p.x), p.y + t * (q.y - p.y)});
    }
  }
  return out;
}

// Signed area of the triangle (origin, a, b) intersected with the disk of
// radius r about the origin: the segment ab is split where it crosses the
// circle; pieces inside count as triangles, pieces outside as sectors.
double tri_disk(P2 a, P2 b, double r) {
  const double r2 = r * r;
  const P2 d = {b.x - a.x, b.y - a.y};
  const double A = d.x * d.x + d.y * d.y;
  if (A == 0.0) return 0.0;
  const double B = a.x * d.x + a.y * d.y;
  const double C = a.x * a.x + a.y * a.y - r2;
  double ts[4] = {0.0, 0.0, 0.0, 1.0};
  int nt = 1;
  const double disc = B * B - A * C;
  if (disc > 0.0) {
    const double sq = std::sqrt(disc);
    const double t1 = (-B - sq) / A, t2 = (-B + sq) / A;
    if (t1 > 0.0 && t1 < 1.0) ts[nt++] = t1;
    if (t2 > 0.0 && t2 < 1.0) ts[nt++] = t2;
  }
  ts[nt++] = 1.0;
  double s = 0.0;
  for (int k = 0; k + 1 < nt; ++k) {
    const P2 p = {a.x + ts[k] * d.x, a.y + ts[k] * d.y};
    const P2 q = {a.x + ts[k + 1] * d.x, a.y + ts[k + 1] * d.y};
    const double tm = 0.5 * (ts[k] + ts[k + 1]);
    const P2 m = {a.x + tm * d.x, a.y + tm * d.y};
    if (m.x * m.x + m.y * m.y <= r2) {
      s += 0.5 * cross(p, q);
    } else {
      s += 0.5 * r2 * std::atan2(cross(p, q), p.x * q.x + p.y * q.y);
    }
  }
  return s;
}

// First moment (integral of y over the region, origin at the disk centre) of
// the same signed piece as tri_disk: triangles contribute area x centroid,
// sectors (r^2 / 3) rot(q - p) for the sweep from p to q.
void tri_disk_moment(P2 a, P2 b, double r, double m[2]) {
  const double r2 = r * r;
  const P2 d = {b.x - a.x, b.y - a.y};
  const double A = d.x * d.x + d.y * d.y;
  if (A == 0.0) return;
  const double B = a.x * d.x + a.y * d.y;
  const double C = a.x * a.x + a.y * a.y - r2;
  double ts[4] = {0.0, 0.0, 0.0, 1.0};
  int nt = 1;
  const double disc = B * B - A * C;
  if (disc > 0.0) {
    const double sq = std::sqrt(disc);
    const double t1 = (-B - sq) / A, t2 = (-B + sq) / A;
    if (t1 > 0.0 && t1 < 1.0) ts[nt++] = t1;
    if (t2 > 0.0 && t2 < 1.0) ts[nt++] = t2;
  }
  ts[nt++] = 1.0;
  for (int k = 0; k + 1 < nt; ++k) {
    const P2 p = {a.x + ts[k] * d.x, a.y + ts[k] * d.y};
    const P2 q = {a.x + ts[k + 1] * d.x, a.y + ts[k + 1] * d.y};
    const double tm = 0.5 * (ts[k] + ts[k + 1]);
    const P2 mm = {a.x + tm * d.x, a.y + tm * d.y};
    if (mm.x * mm.x + mm.y * mm.y <= r2) {
      const double ar = 0.5 * cross(p, q);
      m[0] += ar * (p.x + q.x) / 3.0;
      m[1] += ar * (p.y + q.y) / 3.0;
    } else {
      // the sector swept from p to q the short way (as tri_disk's atan2)
      const double ang = std::atan2(cross(p, q), p.x * q.x + p.y * q.y);
      const P2 pu = {p.x * r / std::sqrt(p.x * p.x + p.y * p.y), p.y * r / std::sqrt(p.x * p.x + p.y * p.y)};
      const double c0 = std::atan2(pu.y, pu.x);
      const double c1 = c0 + ang;
      m[0] += r2 * r / 3.0 * (std::sin(c1) - std::sin(c0));
      m[1] += r2 * r / 3.0 * (std::cos(c0) - std::cos(c1));
    }
  }
}

struct Atoms {
  int64_t n;
  const double* x;
  std::vector<double> R, w;
  std::vector<std::vector<int64_t>> nbr;  // atoms whose ball meets B_i (all-pairs search)
};

double facet(const Atoms& at, int64_t i, int64_t j, double* centroid = nullptr) {
  const double* pi = at.x + 3 * i;
  const double* pj = at.x + 3 * j;
  const double u[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
  const double d2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  if (!(d2 > 0.0)) return 0.0;
  const double d = std::sqrt(d2);
  const double wi = at.w[i], wj = at.w[j];
  if (d >= at.R[i] + at.R[j]) return 0.0;
  const double h = (d2 + wi - wj) / (2.0 * d);
  const double rho2 = wi - h * h;
  if (!(rho2 > 0.0)) return 0.0;
  const double rho = std::sqrt(rho2);
  const double n[3] = {u[0] / d, u[1] / d, u[2] / d};
  // orthonormal frame of the plane
  double e1[3];
  if (std::fabs(n[0]) < 0.6) e1[0] = 0.0, e1[1] = -n[2], e1[2] = n[1];
  else e1[0] = n[2], e1[1] = 0.0, e1[2] = -n[0];
  const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (double& v : e1) v /= l1;
  const double e2[3] = {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2], n[0] * e1[1] - n[1] * e1[0]};
  const double c[3] = {h * n[0], h * n[1], h * n[2]};  // disk centre relative to p_i
  const double s = 1.5 * rho;
  std::vector<P2> poly = {{s, s}, {-s, s}, {-s, -s}, {s, -s}};
  for (size_t q = 0; q < at.nbr[i].size() && !poly.empty(); ++q) {
    const int64_t k = at.nbr[i][q];
    if (k == j) continue;
    const double* pk = at.x + 3 * k;
    const double a[3] = {pk[0] - pi[0], pk[1] - pi[1], pk[2] - pi[2]};
    const double a2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    // (an atom whose ball misses B_i is not listed: its half-space holds all of B_i)
    // pi_i(x) <= pi_k(x)  <=>  2 a . y <= |a|^2 - w_k + w_i,  y = x - p_i = c + s e1 + t e2
    const double rhs = a2 - at.w[k] + wi - 2.0 * (a[0] * c[0] + a[1] * c[1] + a[2] * c[2]);
    const double ca = 2.0 * (a[0] * e1[0] + a[1] * e1[1] + a[2] * e1[2]);
    const double cb = 2.0 * (a[0] * e2[0] + a[1] * e2[1] + a[2] * e2[2]);
    if (ca == 0.0 && cb == 0.0) {
      if (rhs < 0.0) poly.clear();
      continue;
    }
    poly = clip(poly, ca, cb, rhs);
  }
  if (poly.size() < 3) return 0.0;
  double area = 0.0, m[2] = {0.0, 0.0};
  for (size_t k = 0; k < poly.size(); ++k) {
    area += tri_disk(poly[k], poly[(k + 1) % poly.size()], rho);
    if (centroid) tri_disk_moment(poly[k], poly[(k + 1) % poly.size()], rho, m);
  }
  if (centroid && area > 0.0)  // absolute position of the face's centroid
    for (int q = 0; q < 3; ++q) centroid[q] = pi[q] + c[q] + (m[0] * e1[q] + m[1] * e2[q]) / area;
  return area;
}

Atoms make(int64_t n, const double* xyz, const double* radii, double probe) {
  Atoms at{n, xyz, std::vector<double>(n), std::vector<double>(n), std::vector<std::vector<int64_t>>(n)};
  for (int64_t i = 0; i < n; ++i) {
    at.R[i] = radii[i] + probe;
    at.w[i] = at.R[i] * at.R[i];
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) {
      if (k == i) continue;
      const double a[3] = {xyz[3 * k] - xyz[3 * i], xyz[3 * k + 1] - xyz[3 * i + 1], xyz[3 * k + 2] - xyz[3 * i + 2]};
      const double rr = at.R[i] + at.R[k];
      if (a[0] * a[0] + a[1] * a[1] + a[2] * a[2] < rr * rr) at.nbr[i].push_back(k);
    }
  return at;
}

}  // namespace

extern "C" {

// F_ij, the flat face of B_i ∩ L_i on the radical plane of i and j (A^2).
double oracle_facet_area(int64_t n, const double* xyz, const double* radii, double probe, int64_t i, int64_t j) {
  const Atoms at = make(n, xyz, radii, probe);
  return facet(at, i, j);
}

// Per-atom volumes (A^3) from the oracle's areas, and dV/dx of their sum (n x 3).
void oracle_volume(int64_t n, const double* xyz, const double* radii, double probe, const double* area, double* vol,
                   double* grad) {
  const Atoms at = make(n, xyz, radii, probe);
  for (int64_t i = 0; i < n; ++i) {
    double s = at.R[i] * area[i];
    double g[3] = {0.0, 0.0, 0.0};
    for (const int64_t j : at.nbr[i]) {
      const double f = facet(at, i, j);
      if (f == 0.0) continue;
      const double u[3] = {xyz[3 * j] - xyz[3 * i], xyz[3 * j + 1] - xyz[3 * i + 1], xyz[3 * j + 2] - xyz[3 * i + 2]};
      const double d2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const double d = std::sqrt(d2);
      s += (d2 + at.w[i] - at.w[j]) / (2.0 * d) * f;
      for (int c = 0; c < 3; ++c) g[c] -= f * u[c] / d;
    }
    vol[i] = s / 3.0;
    for (int c = 0; c < 3; ++c) grad[3 * i + c] = g[c];
  }
}

// Centroid (3 doubles out, absolute) and area of the flat face of B_i ∩ L_i on
// the radical plane of i and j.
double oracle_facet_centroid(int64_t n, const double* xyz, const double* radii, double probe, int64_t i, int64_t j,
                             double* centroid) {
  const Atoms at = make(n, xyz, radii, probe);
  return facet(at, i, j, centroid);
}

// Vector-Jacobian product of the per-atom volumes: out[m] = sum_i u_i dV_i/dp_m.
// Moving p_j moves only the face (i, j) of cell i, with normal speed
// -(x - p_j).delta / d_ij, so dV_i/dp_j = -F_ij (c_ij - p_j) / d_ij (c_ij the
// face centroid); moving p_i moves its sphere rigidly and every face of its
// cell, so dV_i/dp_i = sum_j F_ij [(c_ij - p_i) / d_ij - u_ij].  Together:
//   out[m] = sum_j F_mj [(u_m - u_j) (c_mj - p_m) / d_mj - u_m (p_j - p_m) / d_mj].
void oracle_volume_vjp(int64_t n, const double* xyz, const double* radii, double probe, const double* u,
                       double* out) {
  const Atoms at = make(n, xyz, radii, probe);
  for (int64_t m = 0; m < n; ++m) {
    double g[3] = {0.0, 0.0, 0.0};
    for (const int64_t j : at.nbr[m]) {
      double cen[3];
      const double f = facet(at, m, j, cen);
      if (f == 0.0) continue;
      const double* pm = xyz + 3 * m;
      const double* pj = xyz + 3 * j;
      const double dv[3] = {pj[0] - pm[0], pj[1] - pm[1], pj[2] - pm[2]};
      const double d = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      for (int q = 0; q < 3; ++q) g[q] += f * ((u[m] - u[j]) * (cen[q] - pm[q]) / d - u[m] * dv[q] / d);
    }
    for (int q = 0; q < 3; ++q) out[3 * m + q] = g[q];
  }
}

}  // extern "C"
