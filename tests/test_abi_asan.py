"""The C ABI's host code under AddressSanitizer, on the CPU.

The library is rebuilt with the sanitizer in the host code of its C-ABI
sources (build.build_host_asan: argument checks, handles, workspaces) and
loaded, with the sanitizer's runtime preloaded, in a child process that runs
the device-free ABI tests of test_abi.py and further bad-argument calls on
every kind of entry point.  Every call must return its error code, and the
sanitizer must report nothing (it aborts the child on the first report)."""
import ctypes
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def more_bad_arguments(lib, L):
    """Bad arguments to the entry points test_abi.py does not cover; each
    must be refused before any device is touched."""
    m = L.P2MMesh(8, 8, 0.125, 0.0, 0.0)
    p = ctypes.c_void_p(16)
    out = ctypes.c_void_p(0)
    nan = float("nan")
    calls = [
        lambda: lib.p2m_project_fused(None, 0.1, p, 10, p, 1, 0, p, None),
        lambda: lib.p2m_project_fused(ctypes.byref(m), 0.1, p, 10, None, 1, 0, p, None),
        lambda: lib.p2m_project_fused(ctypes.byref(m), 0.1, p, 10, p, 0, 0, p, None),
        lambda: lib.p2m_project_fused(ctypes.byref(m), 0.1, p, 10, p, 1, 9, p, None),
        lambda: lib.p2m_backward_fused(None, 0.1, p, 10, p, 1, 0, p, p, None, None),
        lambda: lib.p2m_backward_fused(ctypes.byref(m), 0.1, p, 10, p, 1, 0, None, p, None, None),
        lambda: lib.p2m_project_fused_noalloc(ctypes.byref(m), 0.1, p, 1 << 20, p, 1, 0, p, None),
        lambda: lib.p2m_project_fused_noalloc(None, 0.1, p, 10, p, 1, 0, p, None),
        lambda: lib.m2p_interpolate_backward(ctypes.byref(m), p, 0, 0, p, 10, p, p, None, None),
        lambda: lib.m2p_interpolate_backward(None, p, 1, 0, p, 10, p, p, None, None),
        lambda: lib.p2m_advect(None, p, 10, 0.1, 0.01, None),
        lambda: lib.p2m_advect(ctypes.byref(m), p, 10, nan, 0.01, None),
        lambda: lib.p2m_advect_periodic(ctypes.byref(m), None, 10, 0.1, 0.01, None),
        lambda: lib.p2m_mesh_qcsf_create(None, ctypes.byref(out), None),
        lambda: lib.p2m_mesh_qcsf_create(ctypes.byref(m), None, None),
        lambda: lib.m2p_interpolate_qcsf(None, p, 1, 0, p, 10, p, None),
        lambda: lib.p2m_project_backward(None, p, 1, 0, p, p, None, None),
        lambda: lib.p2m_build_weights_backward(None, p, p, p, None),
        lambda: lib.p2m_weights_export(None, p, p, p, p, None),
        lambda: lib.p2m_weights_shape(None, None, None),
        lambda: lib.p2m_set_option(b"no_such_option", 1.0),
        lambda: lib.p2m_set_option(b"fast_radius", nan),
        lambda: lib.p2m_set_option(b"m2p_ppt", 3.0),
        lambda: lib.p2m_get_option(b"fast_radius", None),
        lambda: lib.p2m_get_option(b"no_such_option", ctypes.byref(ctypes.c_double())),
    ]
    for k, call in enumerate(calls):
        rc = call()
        assert rc != L.P2M_OK, f"bad call {k} accepted"
        assert isinstance(lib.p2m_last_error(), bytes)


CHILD = r"""
import sys
sys.path.insert(0, {root!r})
from paper_1610_05266_amd import _lib as L
L.LIB_PATH = {lib!r}
lib = L.load()
import tests.test_abi as T
import tests.test_abi_asan as A
for name in sorted(dir(T)):
    if name.startswith("test_") and name != "test_autograd_recompute_refuses_build_flags":
        getattr(T, name)()
        print("ok", name, flush=True)
A.more_bad_arguments(lib, L)
print("ok more_bad_arguments", flush=True)
"""


def test_c_abi_host_code_under_address_sanitizer():
    from paper_1610_05266_amd import build

    try:
        lib = build.build_host_asan()
        runtime = build.asan_runtime()
    except (RuntimeError, OSError) as e:
        pytest.skip(f"no sanitizer build here: {e}")
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verbosity=1")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env, capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    log = r.stdout + r.stderr
    assert "AddressSanitizer: ERROR" not in log and "ERROR: AddressSanitizer" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
    # the runtime was live in the child (it announces itself at verbosity 1)
    assert "AddressSanitizer" in r.stderr
    assert "ok more_bad_arguments" in r.stdout
