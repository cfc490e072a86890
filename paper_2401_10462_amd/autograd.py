"""torch.autograd.Function over the library: per-atom SASA with an analytic backward.

Forward calls ``sasa_compute`` / ``sasa_compute_batch`` (areas only); backward
calls ``sasa_backward``, the hand-written VJP kernel that recomputes the
simplex geometry from the complex kept by that forward (Eq. 2 with Eqs. 3-7)
and returns dL/dx = sum_i dL/dA_i dA_i/dx.  Radii and probe get no gradient.

A context keeps exactly one complex, so every forward takes a context from a
pool and holds it until its backward has run (or the graph is freed).
"""
import threading
import weakref

import torch

from .context import SasaContext


class _Pool:
    def __init__(self):
        self._free = {}
        self._lock = threading.Lock()

    def acquire(self, device, precision):
        key = (device, precision)
        with self._lock:
            lst = self._free.setdefault(key, [])
            if lst:
                return lst.pop()
        return SasaContext(device=device, precision=precision)

    def release(self, ctx):
        with self._lock:
            self._free.setdefault((ctx.device, ctx.precision), []).append(ctx)


_pool = _Pool()


class _Held:
    """A pooled context bound to one forward; returned to the pool once."""

    def __init__(self, ctx):
        self.ctx = ctx
        self._fin = weakref.finalize(self, _pool.release, ctx)

    def done(self):
        self._fin()


class SASAFunction(torch.autograd.Function):
    """A = SASAFunction.apply(xyz, radii, probe, offsets, precision) -> per-atom areas (float64)."""

    @staticmethod
    def forward(fctx, xyz, radii, probe=1.4, offsets=None, precision="fp64"):
        if not xyz.is_cuda:
            raise ValueError("SASAFunction needs HIP tensors (the library has no CPU path)")
        dev = xyz.device.index if xyz.device.index is not None else torch.cuda.current_device()
        held = _Held(_pool.acquire(dev, precision))
        x = xyz.detach().to(torch.float64).contiguous()
        r = radii.detach().to(torch.float64, copy=False).contiguous()
        if offsets is None:
            area, _ = held.ctx.compute(x, r, probe, grad=False)
        else:
            area, _ = held.ctx.compute_batch(offsets, x, r, probe, grad=False)
        fctx.held = held
        fctx.dtype = xyz.dtype
        return area

    @staticmethod
    def backward(fctx, grad_area):
        held = fctx.held
        if held is None:
            raise RuntimeError("SASAFunction.backward called twice on one graph (retain_graph is not supported)")
        g = held.ctx.backward(grad_area.detach().to(torch.float64).contiguous())
        fctx.held = None
        held.done()
        return g.to(fctx.dtype), None, None, None, None


def sasa(xyz, radii, probe=1.4, offsets=None, precision="fp64"):
    """Differentiable per-atom SASA (A^2) of one molecule, or of a batch with ``offsets``."""
    return SASAFunction.apply(xyz, radii, probe, offsets, precision)


class VolumeFunction(torch.autograd.Function):
    """V = VolumeFunction.apply(xyz, radii, probe, offsets) -> per-atom cell volumes (float64, A^3).

    Forward computes the complex (``sasa_compute``) and the volumes of the
    cells B_i ∩ L_i (``sasa_volume``); backward is the library's volume VJP
    (``sasa_volume_backward``), from the faces' areas and centroids.  FP64.
    """

    @staticmethod
    def forward(fctx, xyz, radii, probe=1.4, offsets=None):
        if not xyz.is_cuda:
            raise ValueError("VolumeFunction needs HIP tensors (the library has no CPU path)")
        dev = xyz.device.index if xyz.device.index is not None else torch.cuda.current_device()
        held = _Held(_pool.acquire(dev, "fp64"))
        x = xyz.detach().to(torch.float64).contiguous()
        r = radii.detach().to(torch.float64, copy=False).contiguous()
        if offsets is None:
            held.ctx.compute(x, r, probe, grad=False)
        else:
            held.ctx.compute_batch(offsets, x, r, probe, grad=False)
        vol, _ = held.ctx.volume()
        fctx.held = held
        fctx.dtype = xyz.dtype
        return vol

    @staticmethod
    def backward(fctx, grad_vol):
        held = fctx.held
        if held is None:
            raise RuntimeError("VolumeFunction.backward called twice on one graph (retain_graph is not supported)")
        g = held.ctx.volume_backward(grad_vol.detach().to(torch.float64).contiguous())
        fctx.held = None
        held.done()
        return g.to(fctx.dtype), None, None, None


def volume(xyz, radii, probe=1.4, offsets=None):
    """Differentiable per-atom cell volumes (A^3) of one molecule, or of a batch with ``offsets``."""
    return VolumeFunction.apply(xyz, radii, probe, offsets)


class CurvatureFunction(torch.autograd.Function):
    """C = CurvatureFunction.apply(xyz, radii, probe, offsets, precision) -> per-atom integrated mean
    curvature (float64, A) of the accessible surface.

    Forward computes the complex (``sasa_compute``) and C_i = A_i / R_i - 1/4 sum_j L_ij gamma_ij
    (``sasa_curvature``); backward is the library's curvature VJP (``sasa_curvature_backward``).
    The Euler characteristic is a topological invariant and carries no gradient, so it is not an
    output here; ``SasaContext.curvature`` returns it.
    """

    @staticmethod
    def forward(fctx, xyz, radii, probe=1.4, offsets=None, precision="fp64"):
        if not xyz.is_cuda:
            raise ValueError("CurvatureFunction needs HIP tensors (the library has no CPU path)")
        dev = xyz.device.index if xyz.device.index is not None else torch.cuda.current_device()
        held = _Held(_pool.acquire(dev, precision))
        x = xyz.detach().to(torch.float64).contiguous()
        r = radii.detach().to(torch.float64, copy=False).contiguous()
        if offsets is None:
            held.ctx.compute(x, r, probe, grad=False)
        else:
            held.ctx.compute_batch(offsets, x, r, probe, grad=False)
        curv, _ = held.ctx.curvature()
        fctx.held = held
        fctx.dtype = xyz.dtype
        return curv

    @staticmethod
    def backward(fctx, grad_curv):
        held = fctx.held
        if held is None:
            raise RuntimeError("CurvatureFunction.backward called twice on one graph (retain_graph is not supported)")
        g = held.ctx.curvature_backward(grad_curv.detach().to(torch.float64).contiguous())
        fctx.held = None
        held.done()
        return g.to(fctx.dtype), None, None, None, None


def mean_curvature(xyz, radii, probe=1.4, offsets=None, precision="fp64"):
    """Differentiable per-atom integrated mean curvature (A) of one molecule, or of a batch with ``offsets``."""
    return CurvatureFunction.apply(xyz, radii, probe, offsets, precision)
