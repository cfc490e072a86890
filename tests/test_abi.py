"""The C-ABI library loads and exports every entry point the header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sasa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sasa_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("sasa_create", "sasa_compute", "sasa_compute_batch", "sasa_backward", "sasa_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2401_10462_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.EXPORTS)


def test_capacity_query_needs_no_gpu():
    from paper_2401_10462_amd import _lib
    caps = _lib.sasa_capacity()
    assert caps[0] >= 128 and caps[1] >= 64
    assert _lib.load().sasa_strerror(-1) == b"invalid argument"


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2401_10462_amd import _lib
    with pytest.raises(_lib.SasaError):
        _lib.sasa_create(0)


def test_create_refuses_unknown_options():
    """Unknown flag bits and a non-zero reserved word are refused before any device call."""
    from paper_2401_10462_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    for flags, reserved in ((1 << 10, 0), (0, 1)):
        opt = _lib.sasa_options(0, _lib.SASA_FP64, 0, flags, reserved)
        assert lib.sasa_create(ctypes.byref(opt), ctypes.byref(h)) == -1  # SASA_E_INVAL
        assert not h.value
