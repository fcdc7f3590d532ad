"""ctypes binding of libadanns.so: argument marshalling only.

Every function here forwards to the C ABI declared in include/adanns.h with
the same name; device buffers are torch tensors on the current HIP device
and the stream is torch's current stream. No search arithmetic happens in
Python, and there is no fallback: if the shared library is missing or fails
to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libadanns.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python -c 'import __graft_entry__ as g; g.build()')")
lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, EBUDGET, EIO = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSUPPORTED", -5: "EBUDGET",
                -6: "EIO"}

vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
PIX = C.POINTER(vp)

_SIGS = {
    "adanns_last_error": (C.c_char_p, []),
    "adanns_version": (C.c_char_p, []),
    "adanns_ivf_import": (C.c_int, [vp, i64, i32, i64, i32, vp, i32, i32, vp, vp, PIX]),
    "adanns_build_ivf": (C.c_int, [vp, i64, i32, i64, i32, i32, i32, i32, vp, vp, i64, vp, vp,
                                   PIX]),
    "adanns_pq_import": (C.c_int, [vp, i32, i32, vp, vp, vp, vp]),
    "adanns_pq_codec": (C.c_int, [vp, i32, vp, vp, vp]),
    "adanns_pq_train": (C.c_int, [vp, vp, i64, i32, i32, i32, vp, i32, vp, vp, i64, vp]),
    "adanns_opq_train": (C.c_int, [vp, vp, i64, i32, i32, i32, vp, i32, i32, vp, vp, i64, vp,
                                   vp]),
    "adanns_polar_factor": (C.c_int, [vp, i32, vp, vp, vp]),
    "adanns_search_pq": (C.c_int, [vp, vp, i64, i64, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp]),
    "adanns_set_precision": (C.c_int, [vp, i32, vp]),
    "adanns_index_add_row_copy": (C.c_int, [vp, vp]),
    "adanns_index_quantized": (C.c_int, [vp, i32, vp, vp]),
    "adanns_search_precision": (C.c_int, [vp, vp, i64, i64, i32, i32, i32, i32, i32, i32, i32,
                                          vp, vp, vp, vp]),
    "adanns_search_filtered": (C.c_int, [vp, vp, i64, i64, i32, i32, i32, i32, i32, vp, vp, vp,
                                         vp]),
    "adanns_batch_create": (C.c_int, [vp, i32, i64, i64, vp, PIX]),
    "adanns_batch_run": (C.c_int, [vp, vp, vp, vp, vp, vp]),
    "adanns_batch_run_graph": (C.c_int, [vp, vp, vp, vp, vp]),
    "adanns_batch_set_shape": (C.c_int, [vp, i32, i32, i32]),
    "adanns_batch_autotune": (C.c_int, [vp, vp, vp, vp, i32, vp, vp, vp, vp]),
    "adanns_batch_info": (C.c_int, [vp, vp, vp, vp, vp, vp]),
    "adanns_batch_free": (None, [vp]),
    "adanns_autotune_clear": (C.c_int, []),
    "adanns_serve": (C.c_int, [vp, vp, i64, i64, vp, vp, vp, vp, i32, i32, i32, i32, i32,
                               C.c_size_t, vp, vp, vp, vp]),
    "adanns_timing_enable": (C.c_int, [i32]),
    "adanns_timing_reset": (C.c_int, []),
    "adanns_timing_read": (C.c_int, [C.c_char_p, vp, vp]),
    "adanns_selection_stats": (C.c_int, [vp, vp, i32]),
    "adanns_filtered_stats": (C.c_int, [vp, vp, i32]),
    "adanns_stream_read": (C.c_int, [vp, C.c_size_t, vp, i32, vp]),
    "adanns_search": (C.c_int, [vp, vp, i64, i64, i32, i32, i32, i32, vp, vp, vp, vp]),
    "adanns_search_noalloc": (C.c_int, [vp, vp, i64, i64, i32, i32, i32, i32, vp, vp, vp, vp]),
    "adanns_search_noalloc_max_bytes": (C.c_size_t, []),
    "adanns_search_probes": (C.c_int, [vp, vp, i64, i64, i32, i32, vp, i32, vp, vp, vp]),
    "adanns_index_info": (C.c_int, [vp, vp, vp, vp, vp]),
    "adanns_index_lists": (C.c_int, [vp, vp, vp]),
    "adanns_index_centroids": (C.c_int, [vp, vp]),
    "adanns_index_device_bytes": (C.c_size_t, [vp]),
    "adanns_index_free": (None, [vp]),
    "adanns_index_save": (C.c_int, [vp, C.c_char_p]),
    "adanns_set_search_scratch_cap": (C.c_int, [C.c_size_t]),
    "adanns_index_load": (C.c_int, [C.c_char_p, vp, vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BatchConfig(C.Structure):
    """adanns_batch_config."""
    _fields_ = [("index", vp), ("nq", i64), ("d_c", i32), ("d_s", i32), ("nprobe", i32),
                ("k", i32)]


class ServeStats(C.Structure):
    """adanns_serve_stats."""
    _fields_ = [("wall_s", C.c_double), ("steps", i64), ("mean_batch", C.c_double),
                ("max_inflight_bytes", C.c_size_t), ("max_streams_busy", i32),
                ("rejected", i64)]


class AdannsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != OK:
        raise AdannsError(status, lib.adanns_last_error().decode())


def last_error() -> str:
    return lib.adanns_last_error().decode()


def version() -> str:
    return lib.adanns_version().decode()


def timing_enable(on: bool = True):
    check(lib.adanns_timing_enable(1 if on else 0))


def timing_reset():
    check(lib.adanns_timing_reset())


def timing_read(kernel: str):
    """(launches, total_ms) of a kernel group since the last reset."""
    n = C.c_int64()
    ms = C.c_double()
    check(lib.adanns_timing_read(kernel.encode(), C.addressof(n), C.addressof(ms)))
    return n.value, ms.value


def selection_stats(reset: bool = False):
    """adanns_selection_stats: (queries re-selected with a wider shortlist,
    queries left uncertified) since the last reset, current device."""
    a = C.c_int64()
    b = C.c_int64()
    check(lib.adanns_selection_stats(C.addressof(a), C.addressof(b), 1 if reset else 0))
    return a.value, b.value


def filtered_stats(reset: bool = False):
    """adanns_filtered_stats: (candidates measured exactly, queries taken in
    several windows) by adanns_search_filtered since the last reset."""
    a = C.c_int64()
    b = C.c_int64()
    check(lib.adanns_filtered_stats(C.addressof(a), C.addressof(b), 1 if reset else 0))
    return a.value, b.value


def set_search_scratch_cap(nbytes: int = 0):
    """adanns_set_search_scratch_cap: split larger searches into query chunks."""
    check(lib.adanns_set_search_scratch_cap(int(nbytes)))
