"""Plain FP64 CPU oracle of the dSASA hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its Python binding) never does, and shares no code with it.

``run(xyz, radii, probe)`` returns an :class:`OracleResult` holding, for the
weighted points (p_i, (r_i + probe)^2) of arXiv 2401.10462 (Methods):

* the alpha = 0 dual complex K (vertices, edges, triangles, tetrahedra),
  each simplex decided from its definition (Steps 1-2);
* the exterior classification (GPU section, extraction of exterior simplices);
* per-atom SASA by Eq. 1 and the Jacobian dA_i/dp_m by Eq. 2;
* per-atom volumes of the same cells (``volume``) and the integrated mean
  curvature of the surface (``mean_curvature``), the measures the Introduction
  and the Discussion extend the method to.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def lib():
    global _lib
    if _lib is None:
        # SASA_ORACLE_LIB: another build of the same sources (the sanitizer
        # build of the tests), used as is
        path = os.environ.get("SASA_ORACLE_LIB", _build.LIB)
        if path == _build.LIB and (not os.path.exists(path) or os.path.getmtime(path) < max(
                os.path.getmtime(q) for q in _build.SOURCES + _build.HEADERS)):
            _build.build(force=True)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_run.restype = P
        L.oracle_run.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double]
        L.oracle_free.argtypes = [P]
        L.oracle_count.restype = ctypes.c_int64
        L.oracle_count.argtypes = [P, ctypes.c_int]
        for name in ("oracle_area", "oracle_dadx"):
            getattr(L, name).argtypes = [P, dp]
        L.oracle_vjp.argtypes = [P, dp, dp]
        L.oracle_jacobian.argtypes = [P, P, P, dp]
        L.oracle_vertices.argtypes = [P, P, P]
        L.oracle_edges.argtypes = [P, P, P]
        L.oracle_triangles.argtypes = [P, P, P, P]
        L.oracle_tetrahedra.argtypes = [P, P]
        for name in ("oracle_solid_angle", "oracle_dihedral"):
            f = getattr(L, name)
            f.restype = ctypes.c_double
            f.argtypes = [dp, dp, dp, dp]
        L.oracle_cap_area.restype = ctypes.c_double
        L.oracle_cap_area.argtypes = [dp, ctypes.c_double, dp, ctypes.c_double]
        L.oracle_facet_area.restype = ctypes.c_double
        L.oracle_facet_area.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64]
        L.oracle_volume.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, dp, dp, dp]
        L.oracle_facet_centroid.restype = ctypes.c_double
        L.oracle_facet_centroid.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, dp]
        L.oracle_volume_vjp.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, dp, dp]
        L.oracle_exposed_arc.restype = ctypes.c_double
        L.oracle_exposed_arc.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, dp,
                                         dp]
        L.oracle_mean_curvature.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, dp, dp, dp]
        L.oracle_triple_term.restype = ctypes.c_double
        L.oracle_triple_term.argtypes = [dp, ctypes.c_double, dp, ctypes.c_double, dp, ctypes.c_double]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vp(a):
    return ctypes.c_void_p(a.ctypes.data)


def _v3(p):
    return np.ascontiguousarray(p, dtype=np.float64).reshape(3)


class OracleResult:
    """Result of one oracle run; arrays are numpy copies."""

    def __init__(self, xyz, radii, probe):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        if xyz.shape[0] != radii.shape[0]:
            raise ValueError("xyz and radii disagree on the atom count")
        L = lib()
        self.n = n = xyz.shape[0]
        h = L.oracle_run(n, _dp(xyz), _dp(radii), float(probe))
        if not h:
            raise ValueError("invalid oracle input")
        try:
            c = [L.oracle_count(h, k) for k in range(11)]
            self.counts = dict(zip(
                ["vertices", "edges", "triangles", "tetrahedra", "ext_vertices",
                 "ext_edges", "ext_triangles", "jac_nnz", "exact_predicates", "ties_broken",
                 "flat_candidates"], c))
            self.area = np.zeros(n)
            L.oracle_area(h, _dp(self.area))
            self.dadx = np.zeros((n, 3))
            L.oracle_dadx(h, _dp(self.dadx))
            nnz = c[7]
            self.jac_rows = np.zeros(nnz, np.int32)
            self.jac_cols = np.zeros(nnz, np.int32)
            self.jac_vals = np.zeros((nnz, 3))
            L.oracle_jacobian(h, _vp(self.jac_rows), _vp(self.jac_cols), _dp(self.jac_vals))
            self.vert_in = np.zeros(n, np.uint8)
            self.vert_ext = np.zeros(n, np.uint8)
            L.oracle_vertices(h, _vp(self.vert_in), _vp(self.vert_ext))
            self.edges = np.zeros((c[1], 2), np.int32)
            self.edge_ext = np.zeros(c[1], np.uint8)
            L.oracle_edges(h, _vp(self.edges), _vp(self.edge_ext))
            self.tris = np.zeros((c[2], 3), np.int32)
            self.tri_ntet = np.zeros(c[2], np.uint8)
            self.tri_ext = np.zeros(c[2], np.uint8)
            L.oracle_triangles(h, _vp(self.tris), _vp(self.tri_ntet), _vp(self.tri_ext))
            self.tets = np.zeros((c[3], 4), np.int32)
            L.oracle_tetrahedra(h, _vp(self.tets))
        finally:
            L.oracle_free(h)

    def vjp(self, u):
        """sum_i u_i dA_i/dp_m, from the stored Jacobian blocks (n x 3)."""
        u = np.asarray(u, dtype=np.float64).reshape(-1)
        g = np.zeros((self.n, 3))
        np.add.at(g, self.jac_cols, u[self.jac_rows][:, None] * self.jac_vals)
        return g

    def jacobian_dense(self):
        """dA_i/dp_m as an (n, n, 3) array (small n only)."""
        J = np.zeros((self.n, self.n, 3))
        J[self.jac_rows, self.jac_cols] = self.jac_vals
        return J


def run(xyz, radii, probe=1.4):
    """Run the oracle on one molecule."""
    return OracleResult(xyz, radii, probe)


def _run_job(job):
    return OracleResult(*job)


def run_many(jobs, workers=None):
    """Run the oracle on many molecules [(xyz, radii, probe), ...] in worker
    processes (started fresh, not forked, so a caller that holds a GPU context
    passes none of it on); results in job order."""
    import concurrent.futures
    import multiprocessing

    jobs = list(jobs)
    if workers is None:
        workers = min(16, os.cpu_count() or 1, len(jobs))
    if workers <= 1 or len(jobs) <= 1:
        return [OracleResult(*j) for j in jobs]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(_run_job, jobs))


def solid_angle(pi, pj, pk, pl):
    """Normalised solid angle at pi of tetrahedron (pi, pj, pk, pl)."""
    return lib().oracle_solid_angle(*[_dp(_v3(p)) for p in (pi, pj, pk, pl)])


def dihedral(pi, pj, pk, pl):
    """Normalised dihedral angle along edge pi-pj between faces (i,j,k), (i,j,l)."""
    return lib().oracle_dihedral(*[_dp(_v3(p)) for p in (pi, pj, pk, pl)])


def cap_area(pi, Ri, pj, Rj):
    """Area of sphere (pi, Ri) inside ball (pj, Rj)."""
    a, b = _v3(pi), _v3(pj)
    return lib().oracle_cap_area(_dp(a), float(Ri), _dp(b), float(Rj))


def triple_term(pi, Ri, pj, Rj, pk, Rk):
    """Area of sphere i inside both balls j and k (Eq. 6, both halves)."""
    a, b, c = _v3(pi), _v3(pj), _v3(pk)
    return lib().oracle_triple_term(_dp(a), float(Ri), _dp(b), float(Rj), _dp(c), float(Rk))


def volume(xyz, radii, probe=1.4, area=None):
    """Per-atom volumes of the cells B_i ∩ L_i (A^3) and the gradient of their sum (n x 3).

    3 V_i = R_i A_i + sum_j h_ij F_ij (divergence theorem over the cell) with
    A_i from Eq. 1 (``run``, unless given) and each flat face F_ij computed
    from its definition; dV/dp_i = -sum_j F_ij (p_j - p_i) / |p_j - p_i|.
    """
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    if area is None:
        area = run(xyz, radii, probe).area
    area = np.ascontiguousarray(area, dtype=np.float64)
    n = len(radii)
    vol = np.zeros(n)
    grad = np.zeros((n, 3))
    lib().oracle_volume(n, _dp(xyz), _dp(radii), probe, _dp(area), _dp(vol), _dp(grad))
    return vol, grad


def facet_area(xyz, radii, probe, i, j):
    """Area of the flat face of B_i ∩ L_i on the radical plane of atoms i and j."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    return lib().oracle_facet_area(len(radii), _dp(xyz), _dp(radii), probe, int(i), int(j))


def facet_centroid(xyz, radii, probe, i, j):
    """(area, absolute centroid) of the flat face of B_i ∩ L_i on the radical plane of i and j."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    c = np.zeros(3)
    f = lib().oracle_facet_centroid(len(radii), _dp(xyz), _dp(radii), probe, int(i), int(j), _dp(c))
    return f, c


def volume_vjp(xyz, radii, probe, u):
    """sum_i u_i dV_i/dp_m (n x 3) of the per-atom cell volumes, through the faces' areas and centroids."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    out = np.zeros((len(radii), 3))
    lib().oracle_volume_vjp(len(radii), _dp(xyz), _dp(radii), probe, _dp(u), _dp(out))
    return out


def exposed_arc(xyz, radii, probe, i, j):
    """(L_ij, gamma_ij, rho_ij): exposed length of the circle where spheres i and j meet, the angle
    between their outward normals along it and its radius (all 0 when the spheres do not cross)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    g, r = np.zeros(1), np.zeros(1)
    L = lib().oracle_exposed_arc(len(radii), _dp(xyz), _dp(radii), probe, int(i), int(j), _dp(g), _dp(r))
    return L, float(g[0]), float(r[0])


def mean_curvature(xyz, radii, probe=1.4, area=None):
    """Per-atom integrated mean curvature C_i = A_i / R_i - 1/4 sum_j L_ij gamma_ij (A) of the surface
    of the union of the inflated balls, and (sum L gamma, sum L tan(gamma / 2)) over all pairs."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    if area is None:
        area = run(xyz, radii, probe).area
    area = np.ascontiguousarray(area, dtype=np.float64)
    curv = np.zeros(len(radii))
    sums = np.zeros(2)
    lib().oracle_mean_curvature(len(radii), _dp(xyz), _dp(radii), probe, _dp(area), _dp(curv), _dp(sums))
    return curv, (float(sums[0]), float(sums[1]))


def euler_characteristic(res):
    """V - E + T - Q of the dual complex of an oracle result: the Euler characteristic of the union of
    the balls (the complex is homotopy equivalent to it), so its integrated Gaussian curvature is 4 pi
    times this (Gauss-Bonnet)."""
    c = res.counts
    return c["vertices"] - c["edges"] + c["triangles"] - c["tetrahedra"]
