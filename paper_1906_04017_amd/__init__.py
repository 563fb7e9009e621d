"""dgsn: MI355X-native DGFEM S_n transport sweep (Tano & Ragusa, arXiv 1906.04017).

The compute path lives in the HIP library libdgsn.so (C ABI in
include/dgsn.h); this package is its Python binding.  Importing the package
does not load the library; the first call into ``api`` does, and fails loudly
if the library has not been built.
"""
import importlib

__all__ = ["api", "inputs", "ann_format"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
