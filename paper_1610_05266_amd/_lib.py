"""ctypes loader for libp2m.so (the HIP library built from csrc/).

There is no fallback: if the library is missing or cannot be loaded, every
operation raises.  Build it with ``python -m paper_1610_05266_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libp2m.so")
HEADER = os.path.join(os.path.dirname(PKG_DIR), "include", "p2m.h")

P2M_OK, P2M_EINVAL, P2M_EDOMAIN, P2M_ECAP, P2M_EGEOM, P2M_EHIP, P2M_ENOMEM = 0, -1, -2, -3, -4, -5, -6
P2M_F64, P2M_F32, P2M_BF16 = 0, 1, 2
P2M_WEIGHTS_F32, P2M_STRICT, P2M_LINEAR, P2M_PERIODIC, P2M_DETERMINISTIC = 0x1, 0x2, 0x4, 0x8, 0x10
MAX_SUPPORT = 63
CLOSURE_K = 12
MAX_SETS = 65536

STATUS_NAMES = {0: "P2M_OK", -1: "P2M_EINVAL", -2: "P2M_EDOMAIN", -3: "P2M_ECAP", -4: "P2M_EGEOM",
                -5: "P2M_EHIP", -6: "P2M_ENOMEM"}


class P2MMesh(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("H", c_double), ("x0", c_double), ("y0", c_double)]


class P2MDiag(ctypes.Structure):
    _fields_ = [
        ("interior_nodes", c_int64),
        ("closure_nodes", c_int64),
        ("outside_hull_nodes", c_int64),
        ("rank_deficient", c_int64),
        ("cap_overflow", c_int64),
        ("escalated_nodes", c_int64),
        ("global_nodes", c_int64),
        ("near_degenerate", c_int64),
        ("bad_particles", c_int64),
        ("failed_nodes", c_int64),
        ("duplicate_pairs", c_int64),
        ("slow_nodes", c_int64),
        ("status", c_int32),
        ("support_max", c_int32),
        ("svd_systems", c_int64),
        ("max_gram_cond", c_double),
        ("bwd_rank_deficient", c_int64),
        ("long_rows", c_int64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class P2MError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_SIGS = {
    "p2m_build_weights": (c_int, [POINTER(P2MMesh), c_double, c_void_p, c_int64, c_int, POINTER(c_void_p), c_void_p]),
    "p2m_weights_diag": (c_int, [c_void_p, POINTER(P2MDiag), c_void_p]),
    "p2m_weights_export": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "p2m_weights_shape": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    "p2m_project": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "m2p_interpolate": (c_int, [POINTER(P2MMesh), c_void_p, c_int, c_int, c_void_p, c_int64, c_void_p, c_void_p]),
    "p2m_advect": (c_int, [POINTER(P2MMesh), c_void_p, c_int64, c_double, c_double, c_void_p]),
    "p2m_advect_periodic": (c_int, [POINTER(P2MMesh), c_void_p, c_int64, c_double, c_double, c_void_p]),
    "m2p_interpolate_backward": (c_int, [POINTER(P2MMesh), c_void_p, c_int, c_int, c_void_p, c_int64, c_void_p,
                                         c_void_p, c_void_p, c_void_p]),
    "p2m_project_backward": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "m2p_interpolate_backward_binned": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                                c_void_p, c_void_p]),
    "p2m_build_weights_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "p2m_weights_destroy": (None, [c_void_p]),
    "p2m_mesh_qcsf_create": (c_int, [POINTER(P2MMesh), POINTER(c_void_p), c_void_p]),
    "p2m_mesh_qcsf_create_periodic": (c_int, [POINTER(P2MMesh), POINTER(c_void_p), c_void_p]),
    "p2m_mesh_qcsf_destroy": (None, [c_void_p]),
    "m2p_interpolate_qcsf": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_int64, c_void_p, c_void_p]),
    "p2m_project_fused": (c_int, [POINTER(P2MMesh), c_double, c_void_p, c_int64, c_void_p, c_int, c_int, c_void_p,
                                  c_void_p]),
    "p2m_backward_fused": (c_int, [POINTER(P2MMesh), c_double, c_void_p, c_int64, c_void_p, c_int, c_int, c_void_p,
                                   c_void_p, c_void_p, c_void_p]),
    "p2m_fused_handle": (c_void_p, []),
    "p2m_project_fused_noalloc": (c_int, [POINTER(P2MMesh), c_double, c_void_p, c_int64, c_void_p, c_int, c_int,
                                          c_void_p, c_void_p]),
    "p2m_batch_create": (c_int, [POINTER(P2MMesh), POINTER(c_double), c_int, POINTER(c_int64), POINTER(c_void_p)]),
    "p2m_batch_shape": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "p2m_batch_destroy": (None, [c_void_p]),
    "p2m_build_weights_batched": (c_int, [c_void_p, c_void_p, c_int, POINTER(c_void_p), c_void_p]),
    "m2p_interpolate_batched": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "m2p_interpolate_backward_batched": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                                 c_void_p, c_void_p]),
    "p2m_last_error": (c_char_p, []),
    "p2m_version": (c_char_p, []),
    "p2m_set_option": (c_int, [c_char_p, c_double]),
    "p2m_get_option": (c_int, [c_char_p, POINTER(c_double)]),
    "p2m_profile_enable": (c_int, [c_int]),
    "p2m_profile_read": (c_int, [c_char_p, POINTER(c_double), POINTER(c_int64)]),
}

_lib = None


def header_symbols(path: str = HEADER):
    """Names of the functions declared in include/p2m.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b((?:p2m|m2p)_\w+)\s*\(", text, flags=re.M)))


def load():
    """Load libp2m.so once and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1610_05266_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != P2M_OK:
        msg = load().p2m_last_error().decode(errors="replace")
        raise P2MError(rc, msg)
