"""Context object over the C-ABI: exact per-atom SASA and its gradient on one GPU."""
import numpy as np

from . import _lib


class SasaContext:
    """One library context (device buffers, the complex kept from the last call).

    precision: "fp64" (everything in double) or "mixed" (area terms in float,
    tetrahedrization predicates and accumulation in double).
    frames: consecutive calls are frames of one trajectory; each atom's cell is
    clipped first by the previous frame's facet neighbours (same results,
    fewer cuts).
    incremental: consecutive one-molecule calls rebuild only the stars that
    the atoms moved since the previous call can reach (the same results; for
    moves of a few atoms in a large molecule).
    """

    def __init__(self, device=0, precision="fp64", max_atoms=0, async_calls=False, timing=False, frames=False,
                 incremental=False):
        prec = {"fp64": _lib.SASA_FP64, "mixed": _lib.SASA_MIXED}[precision]
        self.precision = precision
        self.device = device
        flags = ((_lib.SASA_FLAG_ASYNC if async_calls else 0) | (_lib.SASA_FLAG_TIMING if timing else 0)
                 | (_lib.SASA_FLAG_FRAMES if frames else 0) | (_lib.SASA_FLAG_INCREMENTAL if incremental else 0))
        self._h = _lib.sasa_create(device, prec, max_atoms, flags)
        self._n, self._kind_last = 0, None

    def close(self):
        if self._h is not None:
            _lib.sasa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- compute
    # out: optional (area, gradient) buffers to fill, float64, contiguous, in
    # the inputs' memory space (the gradient may be None with grad=False);
    # a loop that passes the same buffers every call allocates nothing
    def compute(self, xyz, radii, probe=1.4, grad=True, out=None):
        """Per-atom areas (n,) and d(sum A)/dx (n, 3); torch HIP tensors or numpy arrays."""
        n = xyz.shape[0]
        area, dadx = self._outputs(xyz, n, grad, out)
        _lib.sasa_compute(self._h, n, _c(xyz), _c(radii), probe, area, dadx)
        self._n, self._kind_last = n, _kind(xyz)
        return area, dadx

    def compute_batch(self, offsets, xyz, radii, probe=1.4, grad=True, out=None):
        """Many molecules (atoms offsets[k]..offsets[k+1]-1) in one launch sequence."""
        n = xyz.shape[0]
        area, dadx = self._outputs(xyz, n, grad, out)
        _lib.sasa_compute_batch(self._h, offsets, _c(xyz), _c(radii), probe, area, dadx)
        self._n, self._kind_last = n, _kind(xyz)
        return area, dadx

    def forces(self, xyz, radii, gamma, probe=1.4, out=None):
        """Per-atom areas and nonpolar forces F = -gamma dA/dx (one molecule)."""
        n = xyz.shape[0]
        area, f = self._outputs(xyz, n, True, out)
        _lib.sasa_compute_forces(self._h, n, _c(xyz), _c(radii), probe, gamma, area, f)
        self._n, self._kind_last = n, _kind(xyz)
        return area, f

    def backward(self, dL_dA):
        """sum_i dL_dA[i] dA_i/dx of the last compute (geometry recomputed)."""
        n = dL_dA.shape[0]
        out = _like(dL_dA, (n, 3))
        _lib.sasa_backward(self._h, _c(dL_dA), out)
        return out

    def volume(self):
        """Per-atom cell volumes (n,) of the last compute and d(sum V)/dx (n, 3), FP64, like its inputs."""
        n = self._n
        vol, grad = _alloc(self._kind_last, (n,)), _alloc(self._kind_last, (n, 3))
        _lib.sasa_volume(self._h, vol, grad)
        return vol, grad

    def curvature(self):
        """Per-atom integrated mean curvature (n,) of the last compute's surface (A, FP64, like its inputs)
        and the Euler characteristic chi of the union (integrated Gaussian curvature 4 pi chi)."""
        mean = _alloc(self._kind_last, (self._n,))
        chi = _lib.sasa_curvature(self._h, mean)
        return mean, chi

    def curvature_backward(self, dL_dC):
        """sum_i dL_dC[i] dC_i/dx of the last compute's per-atom integrated mean curvature (FP64)."""
        n = dL_dC.shape[0]
        out = _like(dL_dC, (n, 3))
        _lib.sasa_curvature_backward(self._h, _c(dL_dC), out)
        return out

    def volume_backward(self, dL_dV):
        """sum_i dL_dV[i] dV_i/dx of the last compute's cell volumes (FP64)."""
        n = dL_dV.shape[0]
        out = _like(dL_dV, (n, 3))
        _lib.sasa_volume_backward(self._h, _c(dL_dV), out)
        return out

    def triangles_by_sort(self):
        """The kept complex's triangles and n_t by the sorted-face extraction, and its GPU time (ms)."""
        return _lib.sasa_triangles_by_sort(self._h)

    def edges_vertices_by_sort(self):
        """The kept complex's unique edges and vertices with exterior flags by sorted extraction, and its GPU time (ms):
        (edges (m, 2), edge_ext (m,), verts (k,), vert_ext (k,), ms)."""
        return _lib.sasa_edges_vertices_by_sort(self._h)

    def counts(self):
        c = _lib.sasa_complex_counts(self._h)
        keys = ("vertices", "edges", "triangles", "tetrahedra", "ext_vertices", "ext_edges", "ext_triangles", "atoms")
        return dict(zip(keys, (int(v) for v in c)))

    def export(self):
        """The kept complex: edges, triangles, n_tet per triangle, tetrahedra, vertex flags."""
        return _lib.sasa_complex_export(self._h)

    def diagnostics(self):
        return _lib.sasa_diagnostics(self._h)

    def status(self):
        """Raise if the last call failed (for async calls: waits for its stream)."""
        _lib.sasa_status(self._h)

    @staticmethod
    def _outputs(xyz, n, grad, out=None):
        if out is None:
            kind = _kind(xyz)
            return _alloc(kind, (n,)), (_alloc(kind, (n, 3)) if grad else None)
        area, g = out
        if area.shape != (n,) or (grad and (g is None or g.shape != (n, 3))):
            raise ValueError("out buffers must have shapes (n,) and (n, 3)")
        for a in (area, g if grad else None):
            if a is not None and not _is_f64_contiguous(a):
                raise ValueError("out buffers must be contiguous float64")
        return area, (g if grad else None)


def _is_f64_contiguous(a):
    if type(a).__module__.startswith("torch"):
        import torch
        return a.dtype == torch.float64 and a.is_contiguous()
    return a.dtype == np.float64 and a.flags.c_contiguous


def _c(a):
    if type(a).__module__.startswith("torch"):
        import torch
        if a.dtype == torch.float64 and not a.requires_grad and a.is_contiguous():
            return a  # already what the library takes
        return a.detach().to(torch.float64).contiguous()
    return np.ascontiguousarray(a, dtype=np.float64)


def _kind(a):
    """Where results like a's go: None for numpy, else the torch device."""
    return a.device if type(a).__module__.startswith("torch") else None


def _alloc(kind, shape):
    if kind is None:
        return np.empty(shape, dtype=np.float64)
    import torch
    return torch.empty(shape, dtype=torch.float64, device=kind)


def _like(a, shape):
    if type(a).__module__.startswith("torch"):
        import torch
        return torch.empty(shape, dtype=torch.float64, device=a.device)
    return np.empty(shape, dtype=np.float64)
