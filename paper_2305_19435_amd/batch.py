"""Python face of the batching form (adanns_batch_*): argument marshalling."""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import BatchConfig, check, lib
from .index import _stream


class Batch:
    """Many search configurations run as one set of persistent launches.

    ``configs``: list of (IvfIndex, nq, d_c, d_s, nprobe, k). Queries are
    passed as one [sum nq, ldq] CUDA tensor in configuration order.
    """

    def __init__(self, configs, ldq: int, ldk: int | None = None, stream=None):
        self.configs = list(configs)
        self.ldq = ldq
        self.ldk = ldk or max(c[5] for c in self.configs)
        arr = (BatchConfig * len(self.configs))()
        for i, (ix, nq, d_c, d_s, nprobe, k) in enumerate(self.configs):
            arr[i] = BatchConfig(ix.handle.value, nq, d_c, d_s, nprobe, k)
        self._keep = [c[0] for c in self.configs]
        h = C.c_void_p()
        check(lib.adanns_batch_create(C.addressof(arr), len(self.configs), ldq, self.ldk,
                                      _stream(stream), C.byref(h)))
        self._h = h
        self.nq = sum(c[1] for c in self.configs)
        self.npairs = sum(c[1] * c[4] for c in self.configs)

    def outputs(self, device="cuda"):
        return (torch.empty((self.nq, self.ldk), dtype=torch.float32, device=device),
                torch.empty((self.nq, self.ldk), dtype=torch.int64, device=device))

    def run(self, Q, out=None, probes=None, stream=None, graph=False):
        dist, ids = out if out is not None else self.outputs(Q.device)
        if graph:
            check(lib.adanns_batch_run_graph(self._h, Q.data_ptr(), dist.data_ptr(), ids.data_ptr(),
                                             _stream(stream)))
        else:
            check(lib.adanns_batch_run(self._h, Q.data_ptr(), dist.data_ptr(), ids.data_ptr(),
                                       None if probes is None else probes.data_ptr(),
                                       _stream(stream)))
        return dist, ids

    def set_shape(self, tq: int, grid: int, tv: int = 64):
        check(lib.adanns_batch_set_shape(self._h, tq, tv, grid))

    def autotune(self, Q, out=None, reps: int = 2, stream=None):
        """Returns the chosen (tq, tv, grid)."""
        dist, ids = out if out is not None else self.outputs(Q.device)
        tq, tv, grid = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib.adanns_batch_autotune(self._h, Q.data_ptr(), dist.data_ptr(), ids.data_ptr(),
                                        reps, C.byref(tq), C.byref(tv), C.byref(grid),
                                        _stream(stream)))
        return tq.value, tv.value, grid.value

    def info(self):
        q, tq, tv, grid, sb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_size_t()
        check(lib.adanns_batch_info(self._h, C.byref(q), C.byref(tq), C.byref(tv), C.byref(grid),
                                    C.byref(sb)))
        return {"queries": q.value, "tq": tq.value, "tv": tv.value, "grid": grid.value,
                "scratch_bytes": sb.value}

    def free(self):
        if self._h is not None and self._h.value:
            lib.adanns_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def autotune_clear():
    check(lib.adanns_autotune_clear())
