"""MI355X-native particle <-> fixed-mesh projection (P2M / M2P) and adjoints.

The compute lives in libp2m.so (hand-written HIP for gfx950, C ABI declared in
include/p2m.h); this package is its thin binding.  Importing it does not touch
the GPU; the first call loads the library and fails loudly if it is missing.
"""
from ._lib import (P2M_BF16, P2M_DETERMINISTIC, P2M_F32, P2M_F64, P2M_LINEAR, P2M_PERIODIC, P2M_STRICT, P2M_WEIGHTS_F32, MAX_SUPPORT, CLOSURE_K,  # noqa: F401
                   P2MError, header_symbols, load)


def __getattr__(name):
    # lazy: torch is imported only when the binding is used
    if name in ("ops", "autograd"):
        import importlib

        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
