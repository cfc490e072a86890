// volume.hip -- per-atom volumes of the cells B_i ∩ L_i and the gradient of
// the molecular volume, from the dual complex K kept by the last compute.
//
// The same cells whose spherical boundary gives the area of Eq. 1 give the
// volume (the Discussion names volumes and their derivatives as the next
// measure on them).  The divergence theorem over B_i ∩ L_i with the field
// x - p_i gives
//   3 V_i = R_i A_i + sum_j h_j F_j,
// j over the K-edges at i (the facets that meet B_i), h_j the signed distance
// of the radical plane of i and j from p_i and F_j the area of the flat face.
// On the plane the face is the disk D_j (centre c_j, radius rho_j) cut by the
// cell's edges, and the divergence theorem in the plane with x - c_j gives
//   2 F_j = rho_j^2 theta_j + sum over the face's boundary segments of
//           delta_t l_t,
// theta_j the angle of the exposed arcs of the circle (the circle where
// spheres i and j meet), delta_t the signed distance from c_j of the line of
// the cell edge t = (i, j, k) and l_t the length of its part in B_i.  Both
// come from K by the same inclusion-exclusion as Eq. 1, one dimension down:
//   theta_j / 2 pi = Phi_j - sum_{exterior t = ijk} c_t 2 phi_ij(T_x),
//   sum_t delta_t l_t = sum_{exterior t} c_t delta_t 2 a_t
//                     + sum_{K-tets T at ij} sum_{faces t of T at ij} delta_t sigma_t zeta_t,
// with Phi_j = 1 - sum over K-tetrahedra at ij of phi_ij(T) (Eq. 4), c_t =
// 1 - n_t / 2, phi_ij(T_x) the dihedral fraction along ij between the planes
// (i, j, k) and (i, j, x) for the triple point x (the half-angle of the arc
// of the circle inside B_k), a_t the half-chord of the cell edge's line in
// B_i, zeta_t the position of the tetrahedron's orthocentre on that line
// (from the chord's middle) and sigma_t = +1 or -1 as the fourth vertex lies
// ahead or behind along the line (every cell edge is the chord less the parts
// cut off at its K-tetrahedra; interior triangles are counted through the two
// tetrahedra that share them).
// The gradient of V = sum_i V_i is the flux of a translation of sphere i
// through its exposed part, and the cell's closed boundary turns it into
//   dV/dp_i = - sum_j F_j (p_j - p_i) / |p_j - p_i|,
// so every atom's gradient comes from its own faces: no gather.
// Per-atom derivatives follow from the same flux argument: moving p_j moves
// only the face (i, j) of cell i, with normal speed -(x - p_j).delta / d_ij,
// and moving p_i moves its sphere and all its faces, so for weights u
//   sum_i u_i dV_i/dp_m = sum_j F_mj [(u_m - u_j)(cbar_mj - p_m) - u_m (p_j - p_m)] / d_mj
// with cbar the face's centroid.  Its first moment about the disk centre
// comes from the divergence theorem in the plane with (x - c)(x - c):
//   3 M = rho int_arcs (x - c) ds + sum_t delta_t int_t (x - c) ds,
// where an arc's integral is rho (x_end - x_start) x n (so only the exposed
// triple points count, each with the sign of the arc it ends or starts), and
// each edge's integral is its chord's, 2 a_t (y_t - c), less the parts cut off
// at its K-tetrahedra, through the same decomposition as the lengths.
//
// The same exposed arcs give the integrated mean curvature of the surface
// (the Introduction lists mean curvature beside volume as a measure the method
// extends to; the formula is the standard one for a piecewise smooth surface):
// the spherical patches contribute A_i / R_i, and each exposed arc of a
// circle where two spheres meet, a concave crease of length L = rho theta,
// contributes -L gamma / 2, gamma the angle between the two spheres' outward
// normals along it (sin gamma = d rho / (R_i R_j), cos gamma = (R_i^2 + R_j^2 -
// d^2) / (2 R_i R_j)).  Each arc is shared equally by its two atoms:
//   C_i = A_i / R_i - 1/4 sum_j rho_j theta_j gamma_j.
#include <hip/hip_runtime.h>

#include "sasa_internal.h"

namespace sasa {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct D3 {
  double x, y, z;
};
__device__ inline D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 operator*(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double len(D3 a) { return sqrt(dot(a, a)); }

template <bool MOM>
struct VolLds {
  double px[KN_CAP], py[KN_CAP], pz[KN_CAP], pw[KN_CAP];  // K-neighbours relative to p_i, weights
  unsigned tet[KT_CAP];
  unsigned tri[KTR_CAP];
  double tphi[KT_CAP][3];  // dihedral fraction of each K-tetrahedron along (i,a), (i,b), (i,c)
  double tseg[KT_CAP][3];  // its segment terms for the faces on planes a, b, c
  double rarc[KTR_CAP][2];  // exterior triangle (i,a,b): c_t 2 phi(T_x) along (i,a) and (i,b)
  double rseg[KTR_CAP][2];  // c_t delta 2 a_t on planes a and b
  double tmom[MOM ? KT_CAP : 1][3][3];   // first-moment terms of the tetrahedra's faces on planes a, b, c
  double rmom[MOM ? KTR_CAP : 1][2][3];  // and of the exterior triangles on planes a and b
};

template <class LT>
__device__ inline D3 at(const LT& L, int k) { return {L.px[k], L.py[k], L.pz[k]}; }

// Dihedral fraction along the axis e between the half-planes through u and v.
__device__ inline double dihedral_frac(D3 e, D3 u, D3 v) {
  const D3 n1 = cross(e, u), n2 = cross(e, v);
  return atan2(len(cross(n1, n2)), dot(n1, n2)) / kTwoPi;
}

// Point y of the plane of (0, a, b) with equal power to i, a and b:
// 2 a.y = ra, 2 b.y = rb, y in span(a, b); returns false when degenerate.
__device__ inline bool ortho2(D3 a, D3 b, double ra, double rb, D3& y) {
  const double aa = dot(a, a), bb = dot(b, b), ab = dot(a, b);
  const double det = 2.0 * (aa * bb - ab * ab);
  if (!(det != 0.0)) return false;
  const double al = (ra * bb - rb * ab) / det, be = (aa * rb - ab * ra) / det;
  y = a * al + b * be;
  return true;
}

// Signed distance from the disk centre c_j of plane j to the line of the cell
// edge (i, j, k), whose closest point to c_j is y: positive when c_j lies on
// i's side of plane k.
__device__ inline double delta_of(D3 aj, D3 ak, D3 y, double hj) {
  const double dj = len(aj);
  const D3 nj = aj * (1.0 / dj);
  const D3 m = ak - nj * dot(ak, nj);  // towards k, in the plane of j
  const D3 cj = nj * hj;
  return dot(y - cj, m) / len(m);
}

template <class LT>
__device__ inline double plane_offset(const LT& L, int k, double wi) {
  const double d2 = L.px[k] * L.px[k] + L.py[k] * L.py[k] + L.pz[k] * L.pz[k];
  return (d2 + wi - L.pw[k]) / (2.0 * sqrt(d2));
}

// MOM = false: vol[i] and the molecular-volume gradient grad[i], and (curv not
// null) the integrated mean curvature curv[i].
// MOM = true: grad[i] = sum_k u_k dV_k/dp_i for the weights u (vol unused).
template <bool MOM>
__global__ __launch_bounds__(64) void k_volume(Bufs b, const double* u, double* vol, double* grad, double* curv) {
  __shared__ VolLds<MOM> L;
  const int i = blockIdx.x;
  if (i >= b.n) return;
  const int lane = threadIdx.x;
  const uint8_t vf = b.vflag[i];
  if (!(vf & VF_IN)) {
    if (!MOM && lane == 0) vol[i] = 0.0;
    if (!MOM && curv && lane == 0) curv[i] = 0.0;
    if (lane < 3) grad[3 * (size_t)i + lane] = 0.0;
    return;
  }
  const double4 pi = b.pos[i];
  const double Ri = pi.w, wi = Ri * Ri;
  const int nk = min(b.kn_cnt[i], KN_CAP), nt = min(b.kt_cnt[i], KT_CAP), nr = min(b.ktr_cnt[i], KTR_CAP);
  if (lane < nk) {
    const double4 pj = b.pos[b.knbr[(size_t)i * KN_CAP + lane]];
    L.px[lane] = pj.x - pi.x;
    L.py[lane] = pj.y - pi.y;
    L.pz[lane] = pj.z - pi.z;
    L.pw[lane] = pj.w * pj.w;
  }
  for (int t = lane; t < nt; t += 64) L.tet[t] = b.ktet[(size_t)i * KT_CAP + t];
  for (int t = lane; t < nr; t += 64) L.tri[t] = b.ktri[(size_t)i * KTR_CAP + t];
  __syncthreads();
  // K-tetrahedra (i, a, b, c): dihedral fractions and the segment terms of
  // their three faces at i, each on the two planes it lies in
  for (int t = lane; t < nt; t += 64) {
    const unsigned w = L.tet[t];
    const int ks[3] = {(int)(w & 255u), (int)((w >> 8) & 255u), (int)((w >> 16) & 255u)};
    double ph[3] = {0.0, 0.0, 0.0}, sg[3] = {0.0, 0.0, 0.0};
    D3 mo[3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    if (ks[0] < nk && ks[1] < nk && ks[2] < nk) {
      const D3 P[3] = {at(L, ks[0]), at(L, ks[1]), at(L, ks[2])};
      double r[3], h[3];
      for (int c = 0; c < 3; ++c) {
        r[c] = dot(P[c], P[c]) - L.pw[ks[c]] + wi;
        h[c] = plane_offset(L, ks[c], wi);
      }
      // orthocentre z: 2 P_c . z = r_c
      const D3 bc = cross(P[1], P[2]), ca = cross(P[2], P[0]), ab = cross(P[0], P[1]);
      const double det = 2.0 * dot(P[0], bc);
      const D3 z = (bc * r[0] + ca * r[1] + ab * r[2]) * (1.0 / det);
      for (int c = 0; c < 3; ++c) ph[c] = dihedral_frac(P[c], P[(c + 1) % 3], P[(c + 2) % 3]);
      // face (e, f) with fourth vertex o
      for (int o = 0; o < 3; ++o) {
        const int e = (o + 1) % 3, f = (o + 2) % 3;
        D3 y;
        if (!ortho2(P[e], P[f], r[e], r[f], y)) continue;
        const D3 ul = cross(P[e], P[f]);
        const double zeta = dot(z - y, ul) / len(ul);
        const bool ahead = dot(P[o], ul) > 0.0;  // the fourth vertex's side of the line
        const double sz = ahead ? zeta : -zeta;
        const double de = delta_of(P[e], P[f], y, h[e]), df = delta_of(P[f], P[e], y, h[f]);
        sg[e] += de * sz;
        sg[f] += df * sz;
        if (MOM) {  // the edge's chord, less its part beyond the fourth vertex's plane
          const D3 un = ul * (1.0 / len(ul));
          const double a = sqrt(fmax(wi - dot(y, y), 0.0));
          const double sgn = ahead ? 1.0 : -1.0;
          const double cut = a - sgn * zeta, mid = 0.5 * (zeta + sgn * a);
          const D3 ce = P[e] * (h[e] / len(P[e])), cf = P[f] * (h[f] / len(P[f]));
          const D3 pc = y + un * mid;
          mo[e] = mo[e] + ((y - ce) * a - (pc - ce) * cut) * (de / 3.0);
          mo[f] = mo[f] + ((y - cf) * a - (pc - cf) * cut) * (df / 3.0);
        }
      }
    }
    for (int c = 0; c < 3; ++c) L.tphi[t][c] = ph[c], L.tseg[t][c] = sg[c];
    if (MOM)
      for (int c = 0; c < 3; ++c) L.tmom[t][c][0] = mo[c].x, L.tmom[t][c][1] = mo[c].y, L.tmom[t][c][2] = mo[c].z;
  }
  // exterior K-triangles (i, a, b): the arc of circle (i,a) inside B_b and of
  // (i,b) inside B_a, and the full-chord segment terms, weighted by c_t
  for (int t = lane; t < nr; t += 64) {
    const unsigned w = L.tri[t];
    const int ka = (int)(w & 255u), kb = (int)((w >> 8) & 255u);
    const double ct = 1.0 - 0.5 * (double)(w >> 16);
    double arc_a = 0.0, arc_b = 0.0, seg_a = 0.0, seg_b = 0.0;
    D3 mo_a = {0.0, 0.0, 0.0}, mo_b = {0.0, 0.0, 0.0};
    if (ka < nk && kb < nk) {
      const D3 A = at(L, ka), B = at(L, kb);
      const double ra = dot(A, A) - L.pw[ka] + wi, rb = dot(B, B) - L.pw[kb] + wi;
      D3 y;
      if (ortho2(A, B, ra, rb, y)) {
        const double s = dot(y, y) - wi;
        const double half = s < 0.0 ? sqrt(-s) : 0.0;
        const D3 ul = cross(A, B);
        const D3 un = ul * (1.0 / len(ul));
        const D3 x = y + un * half;  // a triple point (either one)
        arc_a = ct * 2.0 * dihedral_frac(A, B, x);
        arc_b = ct * 2.0 * dihedral_frac(B, A, x);
        const double ha = plane_offset(L, ka, wi), hb = plane_offset(L, kb, wi);
        const double da = delta_of(A, B, y, ha), db = delta_of(B, A, y, hb);
        seg_a = ct * da * 2.0 * half;
        seg_b = ct * db * 2.0 * half;
        if (MOM) {
          // the exposed triple points: both when no K-tetrahedron holds the
          // triangle, else the one inside its tetrahedron's fourth half-space
          bool keep_p = true, keep_m = true;
          if ((w >> 16) == 1u) {
            int kl = -1;
            for (int q = 0; q < nt && kl < 0; ++q) {
              const unsigned tq = L.tet[q];
              const int q0 = (int)(tq & 255u), q1 = (int)((tq >> 8) & 255u), q2 = (int)((tq >> 16) & 255u);
              const bool ha_ = q0 == ka || q1 == ka || q2 == ka, hb_ = q0 == kb || q1 == kb || q2 == kb;
              if (ha_ && hb_) kl = q0 != ka && q0 != kb ? q0 : (q1 != ka && q1 != kb ? q1 : q2);
            }
            if (kl >= 0 && kl < nk) {
              const D3 Pl = at(L, kl);
              const double rl = dot(Pl, Pl) - L.pw[kl] + wi;
              keep_p = 2.0 * dot(Pl, y + un * half) <= rl;
              keep_m = !keep_p;
            }
          }
          const D3 na = A * (1.0 / len(A)), nb = B * (1.0 / len(B));
          const D3 ca = na * ha, cb = nb * hb;
          const double rho2a = fmax(wi - ha * ha, 0.0), rho2b = fmax(wi - hb * hb, 0.0);
          const D3 ta = B - na * dot(B, na), tb = A - nb * dot(A, nb);  // towards the other ball, in each plane
          mo_a = (y - ca) * (ct * da * 2.0 * half / 3.0);
          mo_b = (y - cb) * (ct * db * 2.0 * half / 3.0);
          for (int e = 0; e < 2; ++e) {
            if (!(e == 0 ? keep_p : keep_m)) continue;
            const D3 xe = y + un * (e == 0 ? half : -half);
            // an exposed arc ends (+) or starts (-) at xe, going round the normal
            const double sa = dot(cross(na, xe - ca), ta) > 0.0 ? 1.0 : -1.0;
            const double sb = dot(cross(nb, xe - cb), tb) > 0.0 ? 1.0 : -1.0;
            mo_a = mo_a + cross(xe - ca, na) * (rho2a * sa / 3.0);
            mo_b = mo_b + cross(xe - cb, nb) * (rho2b * sb / 3.0);
          }
        }
      }
    }
    L.rarc[t][0] = arc_a, L.rarc[t][1] = arc_b;
    L.rseg[t][0] = seg_a, L.rseg[t][1] = seg_b;
    if (MOM) {
      L.rmom[t][0][0] = mo_a.x, L.rmom[t][0][1] = mo_a.y, L.rmom[t][0][2] = mo_a.z;
      L.rmom[t][1][0] = mo_b.x, L.rmom[t][1][1] = mo_b.y, L.rmom[t][1][2] = mo_b.z;
    }
  }
  __syncthreads();
  // faces: one K-edge per lane (KN_CAP = 64), sums in a fixed order
  double hv = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, crease = 0.0;
  const int k = lane;
  if (k < nk) {
    double phi = 0.0, seg = 0.0, arc = 0.0;
    D3 mom = {0.0, 0.0, 0.0};
    for (int t = 0; t < nt; ++t) {
      const unsigned w = L.tet[t];
      const int c = (int)(w & 255u) == k ? 0 : (int)((w >> 8) & 255u) == k ? 1 : (int)((w >> 16) & 255u) == k ? 2 : -1;
      if (c >= 0) {
        phi += L.tphi[t][c], seg += L.tseg[t][c];
        if (MOM) mom = mom + D3{L.tmom[t][c][0], L.tmom[t][c][1], L.tmom[t][c][2]};
      }
    }
    for (int t = 0; t < nr; ++t) {
      const unsigned w = L.tri[t];
      const int c = (int)(w & 255u) == k ? 0 : (int)((w >> 8) & 255u) == k ? 1 : -1;
      if (c >= 0) {
        arc += L.rarc[t][c], seg += L.rseg[t][c];
        if (MOM) mom = mom + D3{L.rmom[t][c][0], L.rmom[t][c][1], L.rmom[t][c][2]};
      }
    }
    const D3 P = at(L, k);
    const double d = len(P);
    const double h = plane_offset(L, k, wi);
    const double rho2 = fmax(wi - h * h, 0.0);
    const double theta = kTwoPi * (1.0 - phi - arc);
    const double F = 0.5 * (rho2 * theta + seg);
    hv = h * F;
    if (!MOM && curv) {
      const double rho = sqrt(rho2);
      crease = rho * theta * atan2(d * rho, 0.5 * (wi + L.pw[k] - d * d));
    }
    if (MOM) {
      // F (cbar - p_i) = F c + M, c = h P / d the disk centre
      const double ui = u[i], uj = u[b.knbr[(size_t)i * KN_CAP + k]];
      const D3 g = (P * (F * h / d) + mom) * ((ui - uj) / d) - P * (ui * F / d);
      gx = g.x, gy = g.y, gz = g.z;
    } else {
      gx = -F * P.x / d, gy = -F * P.y / d, gz = -F * P.z / d;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    hv += __shfl_xor(hv, off, 64);
    gx += __shfl_xor(gx, off, 64);
    gy += __shfl_xor(gy, off, 64);
    gz += __shfl_xor(gz, off, 64);
    if (!MOM && curv) crease += __shfl_xor(crease, off, 64);
  }
  if (lane == 0) {
    if (!MOM) vol[i] = (Ri * b.area[i] + hv) / 3.0;
    if (!MOM && curv) curv[i] = b.area[i] / Ri - 0.25 * crease;
    grad[3 * (size_t)i] = gx;
    grad[3 * (size_t)i + 1] = gy;
    grad[3 * (size_t)i + 2] = gz;
  }
}

}  // namespace

void launch_volume(const Bufs& b, double* vol, double* grad, hipStream_t s, double* curv) {
  if (b.n) k_volume<false><<<b.n, 64, 0, s>>>(b, nullptr, vol, grad, curv);
}

void launch_volume_vjp(const Bufs& b, const double* u, double* out, hipStream_t s) {
  if (b.n) k_volume<true><<<b.n, 64, 0, s>>>(b, u, nullptr, out, nullptr);
}

}  // namespace sasa
