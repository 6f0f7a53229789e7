"""MI355X-native (gfx950) implementation of the Variable Basis Mapping fine-tuning path.

The compute lives in ``libvbm.so`` (hand-written HIP kernels behind a C ABI declared in
``include/vbm.h``); this package only marshals torch tensors into it.  Importing the package does
not load the library; the first call does, and fails loudly if it has not been built.
"""
from ._lib import EXPORTS, LIB_PATH, VBMError, load  # noqa: F401

__all__ = ["EXPORTS", "LIB_PATH", "VBMError", "load", "api", "trainer"]


def __getattr__(name):
    if name in ("api", "trainer"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
