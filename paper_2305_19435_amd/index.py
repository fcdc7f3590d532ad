"""Python face of the index object: thin wrappers over the C ABI."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev_f32(x, dev):
    t = x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device=dev, dtype=torch.float32).contiguous()


def _dev_x(X, dev="cuda"):
    """A database matrix as the library takes it: a CUDA tensor with unit
    column stride, FP32 or FP16 (kept as given), anything else as FP32.
    Returns (tensor, adanns_dtype code)."""
    if (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype in (torch.float32, torch.float16)
            and X.dim() == 2 and X.stride(1) == 1):
        return X, (1 if X.dtype == torch.float16 else 0)
    if isinstance(X, np.ndarray) and X.dtype == np.float16:
        return torch.from_numpy(np.ascontiguousarray(X)).to(dev), 1
    if isinstance(X, torch.Tensor) and X.dtype == torch.float16:
        return X.to(dev).contiguous(), 1
    return _dev_f32(X, dev), 0


def _dev_i32(x, dev):
    t = x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device=dev, dtype=torch.int32).contiguous()


class IvfIndex:
    """An IVF index resident in HBM (owns a library ``adanns_index``)."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)
        n, d, nl, dcb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib.adanns_index_info(self._h, C.byref(n), C.byref(d), C.byref(nl), C.byref(dcb)))
        self.n, self.d, self.nlist, self.d_c_build = n.value, d.value, nl.value, dcb.value

    # ---- construction -------------------------------------------------------
    @classmethod
    def import_ivf(cls, X, centroids, assign, device="cuda", stream=None) -> "IvfIndex":
        """adanns_ivf_import: X [n, d] FP32 or FP16, centroids [nlist, d_c_build],
        assign [n]."""
        dev = torch.device(device)
        Xd, xt = _dev_x(X, dev)
        Cd = _dev_f32(centroids, dev)
        Ad = _dev_i32(assign, dev)
        out = C.c_void_p()
        check(lib.adanns_ivf_import(Xd.data_ptr(), Xd.shape[0], Xd.shape[1], Xd.stride(0), xt,
                                    Cd.data_ptr(), Cd.shape[0], Cd.shape[1], Ad.data_ptr(),
                                    _stream(stream), C.byref(out)))
        return cls(out.value)

    @classmethod
    def build_ivf(cls, X, nlist: int, d_c: int, iters: int, init_rows, train_rows=None,
                  stream=None, return_objective=False):
        """adanns_build_ivf: GPU Lloyd k-means on X[:, :d_c] (X FP32 or FP16)."""
        Xd, xt = _dev_x(X)
        init = np.ascontiguousarray(init_rows, dtype=np.int32)
        tr = None if train_rows is None else np.ascontiguousarray(train_rows, dtype=np.int64)
        obj = np.zeros(iters + 1, dtype=np.float64)
        out = C.c_void_p()
        check(lib.adanns_build_ivf(Xd.data_ptr(), Xd.shape[0], Xd.shape[1], Xd.stride(0), xt,
                                   nlist,
                                   d_c, iters, init.ctypes.data,
                                   None if tr is None else tr.ctypes.data,
                                   0 if tr is None else len(tr), obj.ctypes.data,
                                   _stream(stream), C.byref(out)))
        ix = cls(out.value)
        return (ix, obj) if return_objective else ix

    @classmethod
    def load(cls, path, stream=None) -> "IvfIndex":
        """adanns_index_load: an index written by save(), onto the current device."""
        out = C.c_void_p()
        check(lib.adanns_index_load(str(path).encode(), _stream(stream), C.byref(out)))
        return cls(out.value)

    def save(self, path):
        """adanns_index_save: centroids, lists, vectors and PQ codecs to ``path``."""
        check(lib.adanns_index_save(self._h, str(path).encode()))

    # ---- search ---------------------------------------------------------------
    def search(self, Q, d_c: int, d_s: int, nprobe: int, k: int, return_probes=False,
               stream=None, out=None):
        """adanns_search. Returns (dist [nq,k] f32, ids [nq,k] i64[, probes])."""
        Qd = Q if (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dtype == torch.float32
                   and Q.stride(1) == 1) else _dev_f32(Q, "cuda")
        nq = Qd.shape[0]
        if out is None:
            dist = torch.empty((nq, k), dtype=torch.float32, device=Qd.device)
            ids = torch.empty((nq, k), dtype=torch.int64, device=Qd.device)
        else:
            dist, ids = out
        probes = torch.empty((nq, nprobe), dtype=torch.int32, device=Qd.device) if return_probes else None
        check(lib.adanns_search(self._h, Qd.data_ptr(), nq, Qd.stride(0) if nq else Qd.shape[1],
                                d_c, d_s, nprobe, k, dist.data_ptr(), ids.data_ptr(),
                                _ptr(probes), _stream(stream)))
        return (dist, ids, probes) if return_probes else (dist, ids)

    def search_probes(self, Q, probes, d_s: int, k: int, stream=None):
        """adanns_search_probes: scan the given probe lists [nq, nprobe]."""
        Qd = _dev_f32(Q, "cuda") if not isinstance(Q, torch.Tensor) or not Q.is_cuda else Q
        Pd = _dev_i32(probes, Qd.device)
        nq, nprobe = Pd.shape
        dist = torch.empty((nq, k), dtype=torch.float32, device=Qd.device)
        ids = torch.empty((nq, k), dtype=torch.int64, device=Qd.device)
        check(lib.adanns_search_probes(self._h, Qd.data_ptr(), nq, Qd.stride(0) if nq else Qd.shape[1],
                                       d_s, nprobe, Pd.data_ptr(), k, dist.data_ptr(),
                                       ids.data_ptr(), _stream(stream)))
        return dist, ids

    # ---- IVF-PQ -------------------------------------------------------------------
    def pq_import(self, M: int, d_s: int, R, codebooks, codes, stream=None):
        """adanns_pq_import: R [d_s, d_s] or None, codebooks [M, 256, d_s/M], codes [n, M]."""
        dev = torch.device("cuda")
        Rd = None if R is None else _dev_f32(R, dev)
        Cd = _dev_f32(codebooks, dev)
        codes_t = codes if isinstance(codes, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(codes, dtype=np.uint8))
        Kd = codes_t.to(device=dev, dtype=torch.uint8).contiguous()
        check(lib.adanns_pq_import(self._h, M, d_s, _ptr(Rd), Cd.data_ptr(), Kd.data_ptr(),
                                   _stream(stream)))

    def pq_train(self, X, M: int, d_s: int, iters: int, init_rows, train_rows=None, R=None,
                 stream=None):
        """adanns_pq_train: GPU-trained PQ codec on X (the index's rows, FP32 or
        FP16) for rotation R."""
        Xd, xt = _dev_x(X)
        init = np.ascontiguousarray(init_rows, dtype=np.int32)
        tr = None if train_rows is None else np.ascontiguousarray(train_rows, dtype=np.int64)
        Rd = None if R is None else _dev_f32(R, Xd.device)
        check(lib.adanns_pq_train(self._h, Xd.data_ptr(), Xd.stride(0), xt, M, d_s, _ptr(Rd), iters,
                                  init.ctypes.data, None if tr is None else tr.ctypes.data,
                                  0 if tr is None else len(tr), _stream(stream)))

    def opq_train(self, X, M: int, d_s: int, outer: int, pq_iters: int, init_rows,
                  train_rows=None, R_init=None, stream=None):
        """adanns_opq_train: GPU-trained OPQ codec (rotation learned from R_init,
        default the identity). Returns the distortion after each PQ training
        [outer + 1]."""
        Xd, xt = _dev_x(X)
        init = np.ascontiguousarray(init_rows, dtype=np.int32)
        tr = None if train_rows is None else np.ascontiguousarray(train_rows, dtype=np.int64)
        Rd = None if R_init is None else _dev_f32(R_init, Xd.device)
        dist = np.zeros(outer + 1, dtype=np.float64)
        check(lib.adanns_opq_train(self._h, Xd.data_ptr(), Xd.stride(0), xt, M, d_s, _ptr(Rd),
                                   outer, pq_iters, init.ctypes.data,
                                   None if tr is None else tr.ctypes.data,
                                   0 if tr is None else len(tr), dist.ctypes.data,
                                   _stream(stream)))
        return dist

    def pq_codec(self, M: int, d_s: int):
        """(R [d_s, d_s], codebooks [M, 256, d_s/M], codes [n, M]) as stored."""
        R = np.empty((d_s, d_s), dtype=np.float32)
        cb = np.empty((M, 256, d_s // M), dtype=np.float32)
        codes = np.empty((self.n, M), dtype=np.uint8)
        check(lib.adanns_pq_codec(self._h, M, R.ctypes.data, cb.ctypes.data, codes.ctypes.data))
        return R, cb, codes

    def search_pq(self, Q, d_c: int, nprobe: int, M: int, k: int, rerank_k: int = 0,
                  d_rerank: int = 0, return_probes=False, stream=None, out=None):
        """adanns_search_pq. Returns (dist, ids[, probes])."""
        Qd = Q if (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dtype == torch.float32
                   and Q.stride(1) == 1) else _dev_f32(Q, "cuda")
        nq = Qd.shape[0]
        if out is None:
            dist = torch.empty((nq, k), dtype=torch.float32, device=Qd.device)
            ids = torch.empty((nq, k), dtype=torch.int64, device=Qd.device)
        else:
            dist, ids = out
        probes = torch.empty((nq, nprobe), dtype=torch.int32, device=Qd.device) if return_probes else None
        check(lib.adanns_search_pq(self._h, Qd.data_ptr(), nq, Qd.stride(0) if nq else Qd.shape[1],
                                   d_c, nprobe, M, k, rerank_k, d_rerank, dist.data_ptr(),
                                   ids.data_ptr(), _ptr(probes), _stream(stream)))
        return (dist, ids, probes) if return_probes else (dist, ids)

    # ---- precision form -----------------------------------------------------------
    FORMATS = {"bf16": 1, "fp8": 2}

    def add_row_copy(self, stream=None):
        """adanns_index_add_row_copy: row-major FP32 copy read by the exact
        re-measurements (results unchanged)."""
        check(lib.adanns_index_add_row_copy(self._h, _stream(stream)))

    def set_precision(self, fmt: str, stream=None):
        """adanns_set_precision: build the BF16 or FP8-e4m3 copy."""
        check(lib.adanns_set_precision(self._h, self.FORMATS[fmt], _stream(stream)))

    def search_precision(self, Q, d_c: int, d_s: int, nprobe: int, k: int, fmt: str,
                         rerank_k: int, coarse_margin: int = 8, return_probes=False,
                         stream=None, out=None):
        """adanns_search_precision. Returns (dist, ids[, probes])."""
        Qd = Q if (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dtype == torch.float32
                   and Q.stride(1) == 1) else _dev_f32(Q, "cuda")
        nq = Qd.shape[0]
        if out is None:
            dist = torch.empty((nq, k), dtype=torch.float32, device=Qd.device)
            ids = torch.empty((nq, k), dtype=torch.int64, device=Qd.device)
        else:
            dist, ids = out
        probes = torch.empty((nq, nprobe), dtype=torch.int32, device=Qd.device) if return_probes else None
        check(lib.adanns_search_precision(self._h, Qd.data_ptr(), nq,
                                          Qd.stride(0) if nq else Qd.shape[1], d_c, d_s, nprobe,
                                          k, self.FORMATS[fmt], rerank_k, coarse_margin,
                                          dist.data_ptr(), ids.data_ptr(), _ptr(probes),
                                          _stream(stream)))
        return (dist, ids, probes) if return_probes else (dist, ids)

    def search_filtered(self, Q, d_c: int, d_s: int, nprobe: int, k: int, fmt: str,
                        return_probes=False, stream=None, out=None):
        """adanns_search_filtered: adanns_search's result from a quantised first
        pass. Returns (dist, ids[, probes])."""
        Qd = Q if (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dtype == torch.float32
                   and Q.stride(1) == 1) else _dev_f32(Q, "cuda")
        nq = Qd.shape[0]
        if out is None:
            dist = torch.empty((nq, k), dtype=torch.float32, device=Qd.device)
            ids = torch.empty((nq, k), dtype=torch.int64, device=Qd.device)
        else:
            dist, ids = out
        probes = torch.empty((nq, nprobe), dtype=torch.int32, device=Qd.device) if return_probes else None
        check(lib.adanns_search_filtered(self._h, Qd.data_ptr(), nq,
                                         Qd.stride(0) if nq else Qd.shape[1], d_c, d_s, nprobe,
                                         k, self.FORMATS[fmt], dist.data_ptr(), ids.data_ptr(),
                                         _ptr(probes), _stream(stream)))
        return (dist, ids, probes) if return_probes else (dist, ids)

    def quantized(self, fmt: str):
        """The low-precision copy in id order: (values [n, d], scales [n])."""
        dt = np.uint16 if fmt == "bf16" else np.uint8
        vals = np.empty((self.n, self.d), dtype=dt)
        sc = np.empty(self.n, dtype=np.float32)
        check(lib.adanns_index_quantized(self._h, self.FORMATS[fmt], vals.ctypes.data,
                                         sc.ctypes.data))
        return vals, sc

    # ---- serving form -------------------------------------------------------------
    def serve(self, Q, arrival_s, d_c, nprobe, M, k: int, rerank_k: int = 0, d_rerank: int = 0,
              nstreams: int = 4, max_batch: int = 1024, hbm_budget: int = 8 << 30):
        """adanns_serve: open-loop request loop. Returns (dist, ids, latency_s, stats)."""
        from ._lib import ServeStats
        Qd = Q if (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dtype == torch.float32
                   and Q.stride(1) == 1) else _dev_f32(Q, "cuda")
        n = Qd.shape[0]
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        dc = np.ascontiguousarray(d_c, dtype=np.int32)
        npb = np.ascontiguousarray(nprobe, dtype=np.int32)
        mm = np.ascontiguousarray(M, dtype=np.int32)
        dist = torch.empty((n, k), dtype=torch.float32, device=Qd.device)
        ids = torch.empty((n, k), dtype=torch.int64, device=Qd.device)
        lat = np.empty(n, dtype=np.float64)
        st = ServeStats()
        torch.cuda.synchronize()
        check(lib.adanns_serve(self._h, Qd.data_ptr(), Qd.stride(0), n, arr.ctypes.data,
                               dc.ctypes.data, npb.ctypes.data, mm.ctypes.data, k, rerank_k,
                               d_rerank, nstreams, max_batch, hbm_budget, dist.data_ptr(),
                               ids.data_ptr(), lat.ctypes.data, C.byref(st)))
        stats = {f: getattr(st, f) for f, _ in ServeStats._fields_}
        return dist, ids, lat, stats

    # ---- introspection ----------------------------------------------------------
    def lists(self):
        off = np.empty(self.nlist + 1, dtype=np.int64)
        ids = np.empty(self.n, dtype=np.int64)
        check(lib.adanns_index_lists(self._h, off.ctypes.data, ids.ctypes.data))
        return off, ids

    def centroids(self):
        c = np.empty((self.nlist, self.d_c_build), dtype=np.float32)
        check(lib.adanns_index_centroids(self._h, c.ctypes.data))
        return c

    def device_bytes(self) -> int:
        return int(lib.adanns_index_device_bytes(self._h))

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            lib.adanns_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def polar_factor(A, stream=None):
    """adanns_polar_factor of a square FP64 matrix (a CUDA tensor or an array).
    Returns (R as a CUDA FP64 tensor, Newton-Schulz steps taken)."""
    Ad = A if isinstance(A, torch.Tensor) and A.is_cuda else torch.from_numpy(np.asarray(A))
    Ad = Ad.to(device="cuda", dtype=torch.float64).contiguous()
    d = Ad.shape[0]
    R = torch.empty_like(Ad)
    it = C.c_int32()
    check(lib.adanns_polar_factor(Ad.data_ptr(), d, R.data_ptr(), C.byref(it), _stream(stream)))
    return R, it.value
