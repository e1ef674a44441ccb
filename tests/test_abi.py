"""C-ABI checks that need no GPU: the library loads, exports every function
include/p2m.h declares, and rejects bad arguments before touching a device."""
import ctypes

import pytest

import paper_1610_05266_amd as pkg
from paper_1610_05266_amd import _lib


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    names = pkg.header_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib._SIGS), "binding signatures out of sync with include/p2m.h"


def test_version_and_error_strings():
    lib = pkg.load()
    assert b"gfx950" in lib.p2m_version()
    assert isinstance(lib.p2m_last_error(), bytes)


def test_argument_validation_without_device():
    lib = pkg.load()
    h = ctypes.c_void_p(0)
    # NULL mesh
    assert lib.p2m_build_weights(None, 0.01, ctypes.c_void_p(16), 10, 0, ctypes.byref(h), None) == _lib.P2M_EINVAL
    m = _lib.P2MMesh(0, 4, 0.25, 0.0, 0.0)
    assert lib.p2m_build_weights(ctypes.byref(m), 0.01, ctypes.c_void_p(16), 10, 0, ctypes.byref(h), None) == -1
    m = _lib.P2MMesh(4, 4, 0.25, 0.0, 0.0)
    # h <= 0, misaligned pos, N out of range, unknown flags
    assert lib.p2m_build_weights(ctypes.byref(m), 0.0, ctypes.c_void_p(16), 10, 0, ctypes.byref(h), None) == -1
    assert lib.p2m_build_weights(ctypes.byref(m), 0.1, ctypes.c_void_p(8), 10, 0, ctypes.byref(h), None) == -1
    assert lib.p2m_build_weights(ctypes.byref(m), 0.1, ctypes.c_void_p(16), 2, 0, ctypes.byref(h), None) == -1
    assert lib.p2m_build_weights(ctypes.byref(m), 0.1, ctypes.c_void_p(16), 10, 0x80, ctypes.byref(h), None) == -1
    assert b"flags" in lib.p2m_last_error()
    # M2P: C out of range, unknown dtype, NULL pointers
    assert lib.m2p_interpolate(ctypes.byref(m), ctypes.c_void_p(16), 0, 0, ctypes.c_void_p(16), 5,
                               ctypes.c_void_p(16), None) == -1
    assert lib.m2p_interpolate(ctypes.byref(m), ctypes.c_void_p(16), 3, 7, ctypes.c_void_p(16), 5,
                               ctypes.c_void_p(16), None) == -1
    assert lib.m2p_interpolate(ctypes.byref(m), None, 3, 0, ctypes.c_void_p(16), 5,
                               ctypes.c_void_p(16), None) == -1
    # handle-based calls with a NULL handle
    assert lib.p2m_project(None, ctypes.c_void_p(16), 1, 0, ctypes.c_void_p(16), None) == -1
    d = _lib.P2MDiag()
    assert lib.p2m_weights_diag(None, ctypes.byref(d), None) == -1
    lib.p2m_weights_destroy(None)


def test_options():
    lib = pkg.load()
    assert lib.p2m_set_option(b"region_h", 4.0) == 0
    assert lib.p2m_set_option(b"levels", 3) == 0
    assert lib.p2m_set_option(b"bin_scale", 1.0) == 0
    assert lib.p2m_set_option(b"closure_radius", 4.0) == 0
    assert lib.p2m_set_option(b"closure_radius", 0.5) == -1
    assert lib.p2m_set_option(b"nonsense", 1.0) == -1
    assert lib.p2m_set_option(b"region_h", 1000.0) == -1


def test_get_option_reads_back_and_derives_slots():
    lib = pkg.load()
    v = ctypes.c_double()
    try:
        assert lib.p2m_set_option(b"fast_radius", 2.8) == 0
        assert lib.p2m_get_option(b"fast_radius", ctypes.byref(v)) == 0 and v.value == 2.8
        # pi * 2.8^2 = 24.6 expected candidates fit 8 slots per lane, pi * 3^2 = 28.3 need 10,
        # pi * 2.6^2 = 21.2 fit 7
        assert lib.p2m_get_option(b"fast_slots", ctypes.byref(v)) == 0 and v.value == 8
        assert lib.p2m_set_option(b"fast_radius", 2.6) == 0
        assert lib.p2m_get_option(b"fast_slots", ctypes.byref(v)) == 0 and v.value == 7
        assert lib.p2m_set_option(b"fast_radius", 3.0) == 0
        assert lib.p2m_get_option(b"fast_slots", ctypes.byref(v)) == 0 and v.value == 10
        assert lib.p2m_get_option(b"levels", ctypes.byref(v)) == 0 and v.value == 3
        assert lib.p2m_get_option(b"nonsense", ctypes.byref(v)) == -1
        assert lib.p2m_get_option(b"levels", None) == -1
        assert b"NULL" in lib.p2m_last_error()
    finally:
        lib.p2m_set_option(b"fast_radius", 2.6)


def test_batch_argument_validation_without_device():
    lib = pkg.load()
    out = ctypes.c_void_p(0)
    M = _lib.P2MMesh * 2
    H = ctypes.c_double * 2
    O = ctypes.c_int64 * 3
    meshes = M(_lib.P2MMesh(4, 4, 0.25, 0.0, 0.0), _lib.P2MMesh(2, 3, 0.5, 1.0, 0.0))
    assert lib.p2m_batch_create(meshes, H(0.1, 0.2), 0, O(0, 10, 20), ctypes.byref(out)) == -1
    assert lib.p2m_batch_create(None, H(0.1, 0.2), 2, O(0, 10, 20), ctypes.byref(out)) == -1
    assert lib.p2m_batch_create(meshes, H(0.1, 0.2), 2, O(1, 10, 20), ctypes.byref(out)) == -1
    assert lib.p2m_batch_create(meshes, H(0.1, 0.2), 2, O(0, 10, 12), ctypes.byref(out)) == -1
    assert b"set 1" in lib.p2m_last_error()
    assert lib.p2m_batch_create(meshes, H(0.1, -0.2), 2, O(0, 10, 20), ctypes.byref(out)) == -1
    bad = M(_lib.P2MMesh(4, 4, 0.25, 0.0, 0.0), _lib.P2MMesh(2, 0, 0.5, 1.0, 0.0))
    assert lib.p2m_batch_create(bad, H(0.1, 0.2), 2, O(0, 10, 20), ctypes.byref(out)) == -1
    assert lib.p2m_batch_create(meshes, H(0.1, 0.2), 2, O(0, 10, 20), None) == -1
    assert out.value is None
    assert lib.p2m_build_weights_batched(None, ctypes.c_void_p(16), 0, ctypes.byref(out), None) == -1
    assert lib.m2p_interpolate_batched(None, ctypes.c_void_p(16), 1, 0, ctypes.c_void_p(16),
                                       ctypes.c_void_p(16), None) == -1
    assert lib.p2m_batch_shape(None, None, None, None) == -1
    lib.p2m_batch_destroy(None)


def test_autograd_recompute_refuses_build_flags():
    """The recompute form builds the default weights: a flag that changes
    them must be refused, not dropped (checked before any device call)."""
    import torch
    from paper_1610_05266_amd import autograd, ops
    pos = torch.zeros((4, 2), dtype=torch.float64)
    vals = torch.zeros((4, 1), dtype=torch.float64)
    mesh = ops.Mesh(4, 4, 0.25, 0.0, 0.0)
    for f in (ops.P2M_PERIODIC, ops.P2M_LINEAR):
        with pytest.raises(ValueError):
            autograd.p2m(pos, vals, mesh, 0.1, flags=f, recompute=True)
