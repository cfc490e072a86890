// curvature_oracle.cc -- plain FP64 integrated mean curvature of the solvent
// accessible surface (TEST INFRASTRUCTURE ONLY).
//
// The Introduction cites the extension of the method from areas to volumes
// and to mean and Gaussian curvatures; the paper gives no formula, so this is
// the standard one for a piecewise smooth closed surface.  The boundary of the
// union of the balls B_i (radius R_i = r_i + probe) is made of the exposed
// spherical patches (area A_i, mean curvature 1/R_i), the exposed arcs of the
// circles where two spheres meet (concave creases) and isolated corners (no
// mean curvature).  With H the mean of the principal curvatures and an
// outward normal,
//   C = sum_i A_i / R_i - 1/2 sum_{i<j} L_ij gamma_ij,
// L_ij the exposed length of the circle of spheres i and j and gamma_ij the
// angle between the two spheres' outward normals along it (the normal turns
// by gamma_ij across the crease, which is concave):
//   cos gamma = (R_i^2 + R_j^2 - d^2) / (2 R_i R_j),  sin gamma = d rho / (R_i R_j)
// (rho the circle's radius).  Per atom each arc is shared equally:
//   C_i = A_i / R_i - 1/4 sum_j L_ij gamma_ij.
// L_ij is computed here from its definition: the circle less the open arcs
// that lie inside any third ball, as a union of intervals on the circle.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace {

const double kPi = 3.14159265358979323846264338327950288;

struct Arc {
  double len = 0.0;    // exposed length L_ij
  double gamma = 0.0;  // angle between the outward normals along the circle
  double rho = 0.0;    // radius of the circle (0: the spheres do not cross)
};

// The circle where spheres i and j meet, and its exposed length.
Arc exposed_arc(int64_t n, const double* X, const double* R, int64_t i, int64_t j) {
  Arc out;
  const double dx = X[3 * j] - X[3 * i], dy = X[3 * j + 1] - X[3 * i + 1], dz = X[3 * j + 2] - X[3 * i + 2];
  const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
  const double Ri = R[i], Rj = R[j];
  if (!(d < Ri + Rj) || !(d > std::fabs(Ri - Rj))) return out;  // disjoint, or one ball inside the other
  const double h = (d * d + Ri * Ri - Rj * Rj) / (2.0 * d);      // from p_i to the circle's plane
  const double rho = std::sqrt(std::max(Ri * Ri - h * h, 0.0));
  out.rho = rho;
  out.gamma = std::atan2(d * rho, 0.5 * (Ri * Ri + Rj * Rj - d * d));
  const double u[3] = {dx / d, dy / d, dz / d};
  const double c[3] = {X[3 * i] + h * u[0], X[3 * i + 1] + h * u[1], X[3 * i + 2] + h * u[2]};
  // e1, e2: an orthonormal basis of the circle's plane
  double a[3] = {1.0, 0.0, 0.0};
  if (std::fabs(u[0]) > 0.6) a[0] = 0.0, a[1] = 1.0;
  const double au = a[0] * u[0] + a[1] * u[1] + a[2] * u[2];
  double e1[3] = {a[0] - au * u[0], a[1] - au * u[1], a[2] - au * u[2]};
  const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (double& v : e1) v /= l1;
  const double e2[3] = {u[1] * e1[2] - u[2] * e1[1], u[2] * e1[0] - u[0] * e1[2], u[0] * e1[1] - u[1] * e1[0]};
  // x(t) = c + rho (cos t e1 + sin t e2) lies inside ball k iff
  // |c - p_k|^2 + rho^2 + 2 rho (cos t e1 + sin t e2).(c - p_k) < R_k^2,
  // i.e. A cos t + B sin t < D: an open arc centred opposite atan2(B, A)
  std::vector<std::pair<double, double>> cov;
  for (int64_t k = 0; k < n; ++k) {
    if (k == i || k == j) continue;
    const double w[3] = {c[0] - X[3 * k], c[1] - X[3 * k + 1], c[2] - X[3 * k + 2]};
    const double A = 2.0 * rho * (e1[0] * w[0] + e1[1] * w[1] + e1[2] * w[2]);
    const double B = 2.0 * rho * (e2[0] * w[0] + e2[1] * w[1] + e2[2] * w[2]);
    const double D = R[k] * R[k] - (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) - rho * rho;
    const double M = std::hypot(A, B);
    if (D >= M) return out;  // the whole circle is inside ball k
    if (D <= -M) continue;   // no point of the circle is inside
    const double phi = std::atan2(B, A), off = std::acos(D / M);
    double s = std::fmod(phi + off, 2.0 * kPi);
    if (s < 0.0) s += 2.0 * kPi;
    const double e = s + 2.0 * (kPi - off);  // covered: (phi + off, phi + 2 pi - off)
    if (e <= 2.0 * kPi) {
      cov.push_back({s, e});
    } else {
      cov.push_back({s, 2.0 * kPi});
      cov.push_back({0.0, e - 2.0 * kPi});
    }
  }
  std::sort(cov.begin(), cov.end());
  double covered = 0.0, lo = 0.0, hi = -1.0;
  for (const auto& iv : cov) {
    if (iv.first > hi) {
      if (hi > lo) covered += hi - lo;
      lo = iv.first, hi = iv.second;
    } else {
      hi = std::max(hi, iv.second);
    }
  }
  if (hi > lo) covered += hi - lo;
  out.len = rho * std::max(2.0 * kPi - covered, 0.0);
  return out;
}

std::vector<double> weights(int64_t n, const double* radii, double probe) {
  std::vector<double> R((size_t)n);
  for (int64_t k = 0; k < n; ++k) R[(size_t)k] = radii[k] + probe;
  return R;
}

}  // namespace

extern "C" {

// Exposed length of the circle of spheres i and j; gamma and rho as above.
double oracle_exposed_arc(int64_t n, const double* xyz, const double* radii, double probe, int64_t i, int64_t j,
                          double* gamma, double* rho) {
  const std::vector<double> R = weights(n, radii, probe);
  const Arc a = exposed_arc(n, xyz, R.data(), i, j);
  if (gamma) *gamma = a.gamma;
  if (rho) *rho = a.rho;
  return a.len;
}

// Per-atom integrated mean curvature C_i (A) from the areas A_i (Eq. 1), and
// over all pairs: sums[0] = sum L_ij gamma_ij, sums[1] = sum L_ij tan(gamma_ij / 2).
void oracle_mean_curvature(int64_t n, const double* xyz, const double* radii, double probe, const double* area,
                           double* curv, double* sums) {
  const std::vector<double> R = weights(n, radii, probe);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = 0; i < n; ++i) curv[i] = area[i] / R[(size_t)i];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      const Arc a = exposed_arc(n, xyz, R.data(), i, j);
      if (a.len == 0.0) continue;
      const double lg = a.len * a.gamma;
      curv[i] -= 0.25 * lg;
      curv[j] -= 0.25 * lg;
      s0 += lg;
      s1 += a.len * std::tan(0.5 * a.gamma);
    }
  if (sums) sums[0] = s0, sums[1] = s1;
}

}  // extern "C"
