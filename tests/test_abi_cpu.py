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
    assert L.adanns_ivf_import(None, 10, 4, 4, 0, None, 2, 2, None, None, None) == -1
    assert L.adanns_ivf_import(1, 0, 4, 4, 0, 1, 2, 2, 1, None, C.byref(out)) == -1
    assert "n must be" in lib.last_error()
    assert L.adanns_ivf_import(1, 10, 4, 3, 0, 1, 2, 2, 1, None, C.byref(out)) == -1
    assert L.adanns_ivf_import(1, 10, 4, 4, 2, 1, 2, 2, 1, None, C.byref(out)) == -1
    assert "dtype" in lib.last_error()
    assert L.adanns_ivf_import(1, 10, 4, 4, 0, 1, 0, 2, 1, None, C.byref(out)) == -1
    assert L.adanns_ivf_import(1, 10, 4, 4, 0, 1, 2, 5, 1, None, C.byref(out)) == -1
    assert L.adanns_search(None, None, 0, 4, 1, 1, 1, 1, None, None, None, None) == -1
    assert "index is NULL" in lib.last_error()
    assert L.adanns_index_info(None, None, None, None, None) == -1
    assert L.adanns_index_device_bytes(None) == 0
    L.adanns_index_free(None)


def test_index_file_checked_before_device_work(lib, tmp_path):
    """A file that is not an index is refused (ADANNS_EIO) from its host part
    alone; NULL arguments are EINVAL."""
    L = lib.lib
    out = C.c_void_p()
    assert L.adanns_index_load(None, None, C.byref(out)) == -1
    assert L.adanns_index_save(None, b"/nonexistent/x") == -1
    missing = tmp_path / "missing.adanns"
    assert L.adanns_index_load(str(missing).encode(), None, C.byref(out)) == -6
    assert "cannot open" in lib.last_error()
    junk = tmp_path / "junk.adanns"
    junk.write_bytes(b"NOTANIDX" + b"\0" * 64)
    assert L.adanns_index_load(str(junk).encode(), None, C.byref(out)) == -6
    assert "magic" in lib.last_error()
    # right magic, wrong version; then a truncated header
    junk.write_bytes(b"ADANNSIX" + (99).to_bytes(4, "little") + b"\0" * 4)
    assert L.adanns_index_load(str(junk).encode(), None, C.byref(out)) == -6
    assert "version" in lib.last_error()
    junk.write_bytes(b"ADANNSIX" + (1).to_bytes(4, "little") + b"\0" * 4 + b"\1\0")
    assert L.adanns_index_load(str(junk).encode(), None, C.byref(out)) == -6
    assert "header" in lib.last_error()
    assert out.value is None
