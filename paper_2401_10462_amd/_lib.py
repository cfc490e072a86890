"""ctypes binding of the C-ABI in include/sasa.h (argument marshalling only).

The names mirror the C entry points.  Arrays may be torch tensors on a HIP
device (passed by data pointer on torch's current stream) or host numpy arrays.
There is no CPU fallback: if the HIP library is missing, loading fails.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsasa_hip.so")

SASA_OK = 0
SASA_E_INVAL = -1
SASA_E_NOMEM = -2
SASA_E_DEVICE = -3
SASA_E_STATE = -4
SASA_E_CAPACITY = -5
SASA_FP64 = 0
SASA_MIXED = 1
SASA_MEM_HOST = 0
SASA_MEM_DEVICE = 1
SASA_FLAG_ASYNC = 1
SASA_FLAG_TIMING = 2
SASA_FLAG_FRAMES = 4
SASA_FLAG_INCREMENTAL = 8

# every entry point of include/sasa.h
EXPORTS = (
    "sasa_create", "sasa_destroy", "sasa_compute", "sasa_compute_batch", "sasa_compute_forces", "sasa_backward",
    "sasa_volume", "sasa_volume_backward", "sasa_triangles_by_sort", "sasa_complex_counts", "sasa_complex_export",
    "sasa_diagnostics", "sasa_status", "sasa_footprint", "sasa_capacity", "sasa_strerror", "sasa_last_error",
    "sasa_compute_noalloc", "sasa_edges_vertices_by_sort", "sasa_curvature", "sasa_curvature_backward",
)


class SasaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class sasa_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_atoms", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class sasa_diag(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n_atoms", "n_mol", "max_neighbours", "max_cell_vertices", "near_ties", "lost_pairs",
        "capacity_retries", "input_errors", "overflow")] + [
        (name, ctypes.c_double) for name in ("ms_total", "ms_cells", "ms_star", "ms_star_wide", "ms_terms",
                                             "ms_gather")] + [
        (name, ctypes.c_int64) for name in ("plane_tests", "new_vertices", "candidates", "planes_used",
                                            "max_planes_used", "atoms_over_64_planes", "reused_cells",
                                            "second_pass_atoms", "moved_atoms", "skipped_atoms")]


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: when torch is installed, its bundled
    # libamdhip64 must be the one this library binds to (torch streams and
    # device pointers are then shared), so torch is loaded first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2401_10462_amd/build.py "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    from . import build as _build
    if os.path.abspath(LIB_PATH) == os.path.abspath(_build.LIB) and _build.stale():
        raise ImportError(f"{LIB_PATH} was built from other sources than the ones in this tree: rebuild it "
                          "with paper_2401_10462_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.sasa_create.argtypes = [ctypes.POINTER(sasa_options), ctypes.POINTER(P)]
    L.sasa_destroy.argtypes = [P]
    L.sasa_destroy.restype = None
    L.sasa_compute.argtypes = [P, I64, P, P, D, P, P, I32, P]
    L.sasa_compute_batch.argtypes = [P, I32, P, P, P, D, P, P, I32, P]
    L.sasa_compute_forces.argtypes = [P, I64, P, P, D, D, P, P, I32, P]
    L.sasa_backward.argtypes = [P, P, P, I32, P]
    L.sasa_volume.argtypes = [P, P, P, I32, P]
    L.sasa_volume_backward.argtypes = [P, P, P, I32, P]
    L.sasa_curvature.argtypes = [P, P, P, I32, P]
    L.sasa_curvature_backward.argtypes = [P, P, P, I32, P]
    L.sasa_triangles_by_sort.argtypes = [P, P, P, I64, P, P]
    L.sasa_edges_vertices_by_sort.argtypes = [P, P, P, I64, P, P, P, I64, P, P]
    L.sasa_complex_counts.argtypes = [P, P]
    L.sasa_complex_export.argtypes = [P, P, P, P, P, P]
    L.sasa_diagnostics.argtypes = [P, ctypes.POINTER(sasa_diag), I64]
    L.sasa_status.argtypes = [P]
    L.sasa_footprint.argtypes = [I64, P]
    L.sasa_footprint.restype = ctypes.c_int
    L.sasa_capacity.argtypes = [P]
    L.sasa_compute_noalloc.argtypes = [I32, I64, P, P, D, P, P, I32, P]
    L.sasa_capacity.restype = None
    L.sasa_strerror.argtypes = [I32]
    L.sasa_strerror.restype = ctypes.c_char_p
    L.sasa_last_error.argtypes = [P]
    L.sasa_last_error.restype = ctypes.c_char_p
    for name in ("sasa_create", "sasa_compute", "sasa_compute_batch", "sasa_compute_forces", "sasa_backward",
                 "sasa_volume", "sasa_volume_backward", "sasa_triangles_by_sort", "sasa_complex_counts",
                 "sasa_complex_export", "sasa_diagnostics", "sasa_status", "sasa_curvature",
                 "sasa_curvature_backward"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc, ctx=None):
    if rc != SASA_OK:
        L = load()
        msg = L.sasa_last_error(ctx).decode()  # (a NULL context: the thread's last message)
        raise SasaError(rc, msg or L.sasa_strerror(rc).decode())
    return rc


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def ptr(a):
    """Raw pointer of a contiguous numpy array / torch tensor (None -> NULL)."""
    if a is None:
        return None
    if _is_torch(a):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


def mem_of(*arrays):
    """SASA_MEM_DEVICE if the arrays are HIP tensors, SASA_MEM_HOST for numpy."""
    dev = [(_is_torch(a) and a.is_cuda) for a in arrays if a is not None]
    if any(dev) and not all(dev):
        raise ValueError("all arrays of one call must be in the same memory space")
    return SASA_MEM_DEVICE if dev and all(dev) else SASA_MEM_HOST


def stream_of(arrays):
    """torch's current stream on the device of the first device tensor (None: host arrays)."""
    for a in arrays:
        if a is not None and _is_torch(a) and a.is_cuda:
            import torch
            raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)  # the handle without a Stream object
            if raw is not None:
                return ctypes.c_void_p(raw(a.device.index))
            return ctypes.c_void_p(torch.cuda.current_stream(a.device).cuda_stream)
    return None


# --------------------------------------------------------------- C names
def sasa_create(device=0, precision=SASA_FP64, max_atoms=0, flags=0):
    L = load()
    opt = sasa_options(device, precision, max_atoms, flags, 0)
    h = ctypes.c_void_p()
    check(L.sasa_create(ctypes.byref(opt), ctypes.byref(h)))
    return h


def sasa_destroy(ctx):
    load().sasa_destroy(ctx)


def sasa_compute(ctx, n, xyz, radii, probe, area, dA_dx, mem=None, stream=None):
    arrs = (xyz, radii, area, dA_dx)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_compute(ctx, int(n), ptr(xyz), ptr(radii), float(probe), ptr(area), ptr(dA_dx),
                                     mem, stream), ctx)


SASA_NOALLOC_MAX_ATOMS = 4096


def sasa_compute_noalloc(device, n, xyz, radii, probe, area, dA_dx, precision=SASA_FP64, stream=None):
    """One molecule of at most SASA_NOALLOC_MAX_ATOMS atoms on device buffers, with
    the library's fixed work space (no device allocation)."""
    arrs = (xyz, radii, area, dA_dx)
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_compute_noalloc(int(device), int(n), ptr(xyz), ptr(radii), float(probe), ptr(area),
                                             ptr(dA_dx), int(precision), stream), None)


def sasa_compute_batch(ctx, offsets, xyz, radii, probe, area, dA_dx, mem=None, stream=None):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    arrs = (xyz, radii, area, dA_dx)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_compute_batch(ctx, len(off) - 1, ctypes.c_void_p(off.ctypes.data), ptr(xyz),
                                           ptr(radii), float(probe), ptr(area), ptr(dA_dx), mem, stream), ctx)


def sasa_compute_forces(ctx, n, xyz, radii, probe, gamma, area, forces, mem=None, stream=None):
    arrs = (xyz, radii, area, forces)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_compute_forces(ctx, int(n), ptr(xyz), ptr(radii), float(probe), float(gamma), ptr(area),
                                            ptr(forces), mem, stream), ctx)


def sasa_backward(ctx, dL_dA, dL_dx, mem=None, stream=None):
    arrs = (dL_dA, dL_dx)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_backward(ctx, ptr(dL_dA), ptr(dL_dx), mem, stream), ctx)


def sasa_volume(ctx, volume, dV_dx, mem=None, stream=None):
    arrs = (volume, dV_dx)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_volume(ctx, ptr(volume), ptr(dV_dx), mem, stream), ctx)


def sasa_volume_backward(ctx, dL_dV, dL_dx, mem=None, stream=None):
    arrs = (dL_dV, dL_dx)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_volume_backward(ctx, ptr(dL_dV), ptr(dL_dx), mem, stream), ctx)


def sasa_curvature(ctx, mean, mem=None, stream=None):
    """Fills mean (n,) with the per-atom integrated mean curvature; returns the Euler characteristic."""
    arrs = (mean,)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    e = ctypes.c_int64(0)
    check(load().sasa_curvature(ctx, ptr(mean), ctypes.byref(e), mem, stream), ctx)
    return int(e.value)


def sasa_curvature_backward(ctx, dL_dC, dL_dx, mem=None, stream=None):
    arrs = (dL_dC, dL_dx)
    mem = mem_of(*arrs) if mem is None else mem
    stream = stream_of(arrs) if stream is None else stream
    return check(load().sasa_curvature_backward(ctx, ptr(dL_dC), ptr(dL_dx), mem, stream), ctx)


def sasa_triangles_by_sort(ctx):
    """(tris (m, 3) int32, n_t (m,) uint8, GPU ms) of the sorted-face extraction."""
    L = load()
    m = ctypes.c_int64(0)
    ms = ctypes.c_float(0.0)
    check(L.sasa_triangles_by_sort(ctx, None, None, 0, ctypes.byref(m), ctypes.byref(ms)), ctx)
    tris = np.zeros((max(m.value, 1), 3), np.int32)
    nt = np.zeros(max(m.value, 1), np.uint8)
    check(L.sasa_triangles_by_sort(ctx, ctypes.c_void_p(tris.ctypes.data), ctypes.c_void_p(nt.ctypes.data),
                                   int(m.value), ctypes.byref(m), ctypes.byref(ms)), ctx)
    return tris[:m.value], nt[:m.value], float(ms.value)


def sasa_edges_vertices_by_sort(ctx):
    L = load()
    ne, nv = ctypes.c_int64(0), ctypes.c_int64(0)
    ms = ctypes.c_float(0.0)
    check(L.sasa_edges_vertices_by_sort(ctx, None, None, 0, ctypes.byref(ne), None, None, 0, ctypes.byref(nv),
                                        ctypes.byref(ms)), ctx)
    e = np.zeros((max(ne.value, 1), 2), np.int32)
    ee = np.zeros(max(ne.value, 1), np.uint8)
    v = np.zeros(max(nv.value, 1), np.int32)
    ve = np.zeros(max(nv.value, 1), np.uint8)
    check(L.sasa_edges_vertices_by_sort(ctx, ctypes.c_void_p(e.ctypes.data), ctypes.c_void_p(ee.ctypes.data),
                                        int(ne.value), ctypes.byref(ne), ctypes.c_void_p(v.ctypes.data),
                                        ctypes.c_void_p(ve.ctypes.data), int(nv.value), ctypes.byref(nv),
                                        ctypes.byref(ms)), ctx)
    return e[:ne.value], ee[:ne.value].astype(bool), v[:nv.value], ve[:nv.value].astype(bool), float(ms.value)


def sasa_complex_counts(ctx):
    c = np.zeros(8, np.int64)
    check(load().sasa_complex_counts(ctx, ctypes.c_void_p(c.ctypes.data)), ctx)
    return c


def sasa_complex_export(ctx):
    c = sasa_complex_counts(ctx)
    e = np.zeros((c[1], 2), np.int32)
    t = np.zeros((c[2], 3), np.int32)
    nt = np.zeros(c[2], np.uint8)
    q = np.zeros((c[3], 4), np.int32)
    vf = np.zeros(c[7], np.uint8)
    check(load().sasa_complex_export(ctx, ptr(e), ptr(t), ptr(nt), ptr(q), ptr(vf)), ctx)
    return e, t, nt, q, vf


def sasa_diagnostics(ctx):
    d = sasa_diag()
    check(load().sasa_diagnostics(ctx, ctypes.byref(d), ctypes.sizeof(d)), ctx)
    return {f: getattr(d, f) for f, _ in d._fields_}


def sasa_status(ctx):
    check(load().sasa_status(ctx), ctx)


def sasa_footprint(n):
    b = np.zeros(1, np.int64)
    check(load().sasa_footprint(int(n), ctypes.c_void_p(b.ctypes.data)))
    return int(b[0])


def sasa_capacity():
    c = np.zeros(2, np.int64)
    load().sasa_capacity(ctypes.c_void_p(c.ctypes.data))
    return c
