"""The C ABI library loads without a GPU, exports every declared symbol, and
rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(adanns_[a-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    import paper_2305_19435_amd as p
    return p


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "adanns_search" in names and "adanns_ivf_import" in names
    for n in sorted(names):
        assert hasattr(lib.lib, n), f"{n} not exported"


def test_version_and_error_text(lib):
    assert "gfx950" in lib.version()
    assert isinstance(lib.last_error(), str)


def test_validation_before_device_work(lib):
    L = lib.lib
    out = C.c_void_p()
    # NULL outputs / pointers and out-of-range sizes are rejected with EINVAL
    assert L.adanns_ivf_import(None, 10, 4, 4, None, 2, 2, None, None, None) == -1
    assert L.adanns_ivf_import(1, 0, 4, 4, 1, 2, 2, 1, None, C.byref(out)) == -1
    assert "n must be" in lib.last_error()
    assert L.adanns_ivf_import(1, 10, 4, 3, 1, 2, 2, 1, None, C.byref(out)) == -1
    assert L.adanns_ivf_import(1, 10, 4, 4, 1, 0, 2, 1, None, C.byref(out)) == -1
    assert L.adanns_ivf_import(1, 10, 4, 4, 1, 2, 5, 1, None, C.byref(out)) == -1
    assert L.adanns_search(None, None, 0, 4, 1, 1, 1, 1, None, None, None, None) == -1
    assert "index is NULL" in lib.last_error()
    assert L.adanns_index_info(None, None, None, None, None) == -1
    assert L.adanns_index_device_bytes(None) == 0
    L.adanns_index_free(None)
