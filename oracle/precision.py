"""Low-precision storage formats and the shortlist-then-rerank form
(test infrastructure).

Section 4.3 describes shortlist generation with cheap, approximate distances
followed by re-ranking of the shortlist with the high-dimensional full-
precision representation. The precision form stores the database (and the
centroids) in BF16, or in FP8-e4m3 with one FP32 scale per vector, computes
first-pass distances on those values, keeps a shortlist, and re-ranks it with
exact distances on the FP32 vectors at the full d_s.

The storage formats are fixed by their definitions, and both sides must take
every rounding decision in the same precision, so these quantisers work on
float32 inputs and reproduce the formats bit for bit:

* BF16: the upper 16 bits of the float32 encoding after round-to-nearest,
  ties-to-even on the dropped 16 bits;
* FP8-e4m3 (OCP "fn" variant): 1 sign, 4 exponent bits with bias 7, 3
  mantissa bits, subnormal quantum 2^-9, largest finite value 448, no
  infinities; per-vector scale s = amax / 448 and codes of x * (448 / amax),
  both quotients rounded to float32, the product rounded to float32, then
  round-to-nearest-even to e4m3 with saturation at +-448. A zero vector has
  scale 0 and all-zero codes.

Everything after quantisation runs in float64 on the dequantised values.

Pins (tests/test_oracle_precision.py): every e4m3 byte decodes to the value
the definition gives and re-encodes to itself; values exactly representable
pass through unchanged; rounding picks the nearest neighbour with ties to the
even code; BF16 agrees with a pure-Python bit rounding; with the shortlist as
long as the candidate list, the form reduces exactly to IVF search; on a
hand-built four-centroid layout whose BF16 / e4m3 rounding swaps the two
nearest centroids, the coarse step's probes for nprobe 1..3 and margins 0
and 1 are the ones worked out by hand from the definition.
"""
from __future__ import annotations

import numpy as np

from .exact import sqdist64, topk_by_dist_then_id
from .ivf import coarse64, probe_order

FP8_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 value (RNE), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).reshape(x.shape)


def bf16_bits(x) -> np.ndarray:
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def e4m3_value(code) -> np.ndarray:
    """Decode e4m3 bytes to float64 (0x7F / 0xFF are NaN)."""
    code = np.asarray(code, dtype=np.uint8).astype(np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 0xF
    f = code & 0x7
    val = np.where(e == 0, f * 2.0 ** -9, (1.0 + f / 8.0) * np.exp2(e - 7.0))
    val = np.where((e == 15) & (f == 7), np.nan, val)
    return s * val


def e4m3_round(y) -> np.ndarray:
    """Round float32 values to the nearest e4m3 value (ties to even code),
    saturating at +-448. Returns float64 values."""
    y = np.asarray(y, dtype=np.float32).astype(np.float64)
    a = np.abs(y)
    _, ex = np.frexp(a)                     # a = m * 2^ex, m in [0.5, 1)
    e = ex - 1                              # floor(log2 a) for a > 0
    quantum = np.where(a < 2.0 ** -6, 2.0 ** -9, np.exp2(e - 3.0))
    r = np.round(a / quantum) * quantum      # numpy rounds half to even
    r = np.minimum(r, FP8_MAX)
    return np.copysign(r, y)


def e4m3_encode_value(v) -> np.ndarray:
    """Exact e4m3 byte for values already on the e4m3 grid."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    sign = (np.signbit(v) & (a > 0)).astype(np.int64) << 7
    _, ex = np.frexp(np.where(a > 0, a, 1.0))
    e = ex - 1
    normal = a >= 2.0 ** -6
    E = np.where(normal, e + 7, 0)
    F = np.where(normal, np.round((a / np.exp2(e) - 1.0) * 8.0), np.round(a / 2.0 ** -9))
    return (sign | (E << 3) | F.astype(np.int64)).astype(np.uint8)


def fp8_quantize_rows(X):
    """Per-row e4m3 quantisation. Returns (codes uint8 [n,d], scale float32 [n])."""
    X = np.asarray(X, dtype=np.float32)
    amax = np.max(np.abs(X), axis=1).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(amax > 0, np.float32(FP8_MAX) / amax, np.float32(0)).astype(np.float32)
    scale = (amax / np.float32(FP8_MAX)).astype(np.float32)
    y = (X * inv[:, None]).astype(np.float32)
    vals = e4m3_round(y)
    return e4m3_encode_value(vals), scale


def fp8_dequantize_rows(codes, scale) -> np.ndarray:
    return e4m3_value(codes) * np.asarray(scale, dtype=np.float64)[:, None]


def dequantized(X, fmt: str) -> np.ndarray:
    """The float64 values a first pass in ``fmt`` works on."""
    if fmt == "fp32":
        return np.asarray(X, dtype=np.float32).astype(np.float64)
    if fmt == "bf16":
        return bf16_round(X).astype(np.float64)
    if fmt == "fp8":
        codes, scale = fp8_quantize_rows(X)
        return fp8_dequantize_rows(codes, scale)
    raise ValueError(fmt)


def precision_search64(X, Q, centroids, offsets, list_ids, d_c: int, d_s: int, nprobe: int,
                       k: int, fmt: str, rerank: int, coarse_margin: int,
                       forced_probes=None, return_shortlist=False):
    """Shortlist-then-rerank IVF search with a ``fmt`` first pass.

    Coarse: first-pass scores on quantised query and centroid prefixes, the
    best nprobe + coarse_margin by (score, h), then exact distances decide
    the nprobe probes. Scan: first-pass distances on quantised query and
    vectors, the best ``rerank`` by (distance, id), then exact distances at
    d_s on the float32 vectors give the top-k.

    Quantisation is per vector over the prefix that is multiplied: for FP8
    the scale of a database vector covers its full stored length d, the
    query's and centroid's scale covers their full stored length too.
    """
    X = np.asarray(X)
    Q = np.asarray(Q)
    Cq = dequantized(np.asarray(centroids, dtype=np.float32), fmt)
    Qq = dequantized(Q, fmt)
    nq = Q.shape[0]
    D = np.empty((nq, k))
    I = np.empty((nq, k), dtype=np.int64)
    P = np.empty((nq, nprobe), dtype=np.int64)
    shortlists = []
    xq_cache = {}
    for qi in range(nq):
        q = np.asarray(Q[qi], dtype=np.float64)
        if forced_probes is None:
            approx = sqdist64(Qq[qi, :d_c], Cq[:, :d_c])
            short = probe_order(approx)[: nprobe + coarse_margin]
            exact = coarse64(q, np.asarray(centroids)[short], d_c)
            order = np.lexsort((short, exact))
            probes = short[order][:nprobe]
        else:
            probes = np.asarray(forced_probes[qi], dtype=np.int64)
        P[qi] = probes
        members = np.concatenate([list_ids[offsets[h]:offsets[h + 1]] for h in probes])
        members = np.asarray(members, dtype=np.int64)
        if len(members) == 0:
            D[qi], I[qi] = topk_by_dist_then_id(np.zeros(0), members, k)
            shortlists.append(members)
            continue
        need = [h for h in probes if h not in xq_cache]
        for h in need:
            rows = list_ids[offsets[h]:offsets[h + 1]]
            xq_cache[h] = dequantized(X[rows], fmt)
        xq = np.concatenate([xq_cache[h] for h in probes])
        first = sqdist64(Qq[qi, :d_s], xq[:, :d_s])
        _, sl = topk_by_dist_then_id(first, members, rerank)
        sl = sl[sl >= 0]
        shortlists.append(sl)
        exact = sqdist64(q[:d_s], X[sl, :d_s])
        D[qi], I[qi] = topk_by_dist_then_id(exact, sl, k)
    if return_shortlist:
        return D, I, P, shortlists
    return D, I, P
