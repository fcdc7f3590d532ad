"""MI355X-native AdANNS-IVF / IVF-PQ search (HIP kernels for gfx950).

The library's compute lives in ``libadanns.so`` (HIP C++, C ABI declared in
include/adanns.h); this package only marshals arguments. Importing it fails
loudly when the shared library has not been built.
"""
from ._lib import (AdannsError, check, filtered_stats, last_error, lib, selection_stats,  # noqa: F401
                   set_search_scratch_cap, timing_enable, timing_read, timing_reset, version)
from .index import IvfIndex, polar_factor  # noqa: F401
from .batch import Batch, autotune_clear  # noqa: F401

__all__ = ["IvfIndex", "Batch", "AdannsError", "version", "last_error", "lib"]
