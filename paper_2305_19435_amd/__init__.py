"""MI355X-native AdANNS-IVF / IVF-PQ search (HIP kernels for gfx950).

The library's compute lives in ``libadanns.so`` (HIP C++, C ABI declared in
include/adanns.h); this package only marshals arguments. Importing it fails
loudly when the shared library has not been built.
"""
from ._lib import AdannsError, check, last_error, lib, version  # noqa: F401
from .index import IvfIndex  # noqa: F401

__all__ = ["IvfIndex", "AdannsError", "version", "last_error", "lib"]
