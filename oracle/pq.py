"""Product quantisation, OPQ and ADC search in float64 (test infrastructure).

PQ (Section 3, "Optimized Product Quantization"; Section 4.2): split a
vector into M contiguous sub-vectors and quantise each with its own codebook
of 2^b = 256 centroids learned by k-means, so a vector becomes M bytes; a
distance then needs only M codebook look-ups. OPQ learns an orthonormal
rotation R applied before PQ (Section 3; Appendix D). AdANNS-OPQ runs this
on the first d_s coordinates with d_s/M-dimensional blocks (Section 4.2).
AdANNS-IVFOPQ clusters with full-precision prefixes and scans the probed
lists with the compressed vectors, optionally re-ranking a shortlist with
the high-dimensional vectors (Section 4.3).

Readings:

* OPQ is the non-parametric alternation of Ge et al. (named in Section 3):
  R = R0 (a given orthonormal start, the identity by default); repeat { PQ
  on Y = X R (warm-started k-means), then
  R = U V^T from the SVD of X^T Y_hat (orthogonal Procrustes) };
* the scan compares the *unquantised* rotated query with the codes
  (asymmetric distance): LUT_m[c] = |q'_m - C_m[c]|^2 and
  D(x) = sum_m LUT_m[code_m(x)];
* inside IVF the codes encode the rotated vectors themselves (not residuals
  to the centroid), so one table per query serves every probed list;
* results ordered by (distance, id), padded with -1 / +inf.

Pins (tests/test_oracle_pq.py): the table decomposition equals the distance
to the decoded vector; with at most 256 training rows and init on all rows
the codebooks reproduce the data and ADC equals exact search; R^T R = I;
distances are invariant under R; OPQ distortion never increases across
alternations; with a random orthonormal R and every row its own codeword in
the rotated space, IVF-OPQ over one list equals exact search (rotation
invariance), while the same codes searched with R^T do not.
"""
from __future__ import annotations

import numpy as np

from .exact import sqdist64, topk_by_dist_then_id
from .kmeans import assign64, kmeans64
from .ivf import coarse64, probe_order

KSUB = 256


def split(d: int, M: int):
    if d % M:
        raise ValueError("M must divide d")
    return d // M


def pq_train64(Y, M: int, iters: int, init_rows=None, init_codebooks=None):
    """Codebooks [M, 256, d/M] by k-means in every sub-space."""
    Y = np.asarray(Y, dtype=np.float64)
    dsub = split(Y.shape[1], M)
    cbs = np.empty((M, KSUB, dsub))
    for m in range(M):
        ym = Y[:, m * dsub:(m + 1) * dsub]
        if init_codebooks is not None:
            C, _, _ = kmeans64(ym, KSUB, iters, init_centroids=init_codebooks[m])
        else:
            C, _, _ = kmeans64(ym, KSUB, iters, init_rows=init_rows)
        cbs[m] = C
    return cbs


def pq_encode64(Y, codebooks) -> np.ndarray:
    """codes[j, m] = argmin_c |y_{j,m} - C_m[c]|^2 (ties to the smaller c)."""
    Y = np.asarray(Y, dtype=np.float64)
    M, _, dsub = codebooks.shape
    codes = np.empty((Y.shape[0], M), dtype=np.uint8)
    for m in range(M):
        codes[:, m] = assign64(Y[:, m * dsub:(m + 1) * dsub], codebooks[m]).astype(np.uint8)
    return codes


def pq_decode64(codes, codebooks) -> np.ndarray:
    M, _, dsub = codebooks.shape
    out = np.empty((codes.shape[0], M * dsub))
    for m in range(M):
        out[:, m * dsub:(m + 1) * dsub] = codebooks[m][codes[:, m]]
    return out


def distortion64(Y, codes, codebooks) -> float:
    diff = np.asarray(Y, dtype=np.float64) - pq_decode64(codes, codebooks)
    return float(np.einsum("ij,ij->", diff, diff))


def procrustes64(X, Yhat) -> np.ndarray:
    """argmin over orthonormal R of |X R - Yhat|_F: R = U V^T, X^T Yhat = U S V^T."""
    U, _, Vt = np.linalg.svd(np.asarray(X, dtype=np.float64).T @ Yhat)
    return U @ Vt


def opq_train64(X, M: int, outer: int, pq_iters: int, init_rows, R0=None):
    """Returns (R [d,d], codebooks [M,256,d/M], distortion after each PQ step).
    The alternation starts from the orthonormal R0 (identity if None)."""
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    R = np.eye(d) if R0 is None else np.asarray(R0, dtype=np.float64)
    cbs = None
    hist = []
    for _ in range(outer):
        Y = X @ R
        cbs = pq_train64(Y, M, pq_iters, init_rows=init_rows, init_codebooks=cbs)
        codes = pq_encode64(Y, cbs)
        hist.append(distortion64(Y, codes, cbs))
        R = procrustes64(X, pq_decode64(codes, cbs))
    Y = X @ R
    cbs = pq_train64(Y, M, pq_iters, init_codebooks=cbs)
    codes = pq_encode64(Y, cbs)
    hist.append(distortion64(Y, codes, cbs))
    return R, cbs, np.array(hist)


def adc_lut64(q_rot, codebooks) -> np.ndarray:
    """LUT[m, c] = |q'_m - C_m[c]|^2 for one rotated query."""
    q_rot = np.asarray(q_rot, dtype=np.float64)
    M, _, dsub = codebooks.shape
    lut = np.empty((M, KSUB))
    for m in range(M):
        lut[m] = sqdist64(q_rot[m * dsub:(m + 1) * dsub], codebooks[m])
    return lut


def adc_dist64(lut, codes) -> np.ndarray:
    """D(x_j) = sum_m LUT[m, code_{j,m}]."""
    codes = np.asarray(codes)
    M = lut.shape[0]
    return lut[np.arange(M)[None, :], codes.astype(np.int64)].sum(axis=1)


def ivfpq_search64(Q, centroids, offsets, list_ids, codes, R, codebooks, d_c: int,
                   nprobe: int, k: int, rerank_k: int = 0, X=None, d_rerank=None,
                   forced_probes=None, return_candidates=False):
    """AdANNS-IVFOPQ: coarse on the unrotated d_c prefix, ADC scan of the probed
    lists, optional exact re-rank of the best ``rerank_k`` on X[:, :d_rerank].

    ``codes`` are indexed by database id. R is [d_s, d_s] (identity for plain
    PQ); the query's first d_s = R.shape[0] coordinates are rotated.
    Returns (dist, ids, probes); with re-ranking the distances are exact.
    With ``return_candidates`` also the ids each query's final order was
    chosen from (the probed members, or the re-ranked shortlist) and the
    query's table.
    """
    cands = []
    luts = []
    Q = np.asarray(Q)
    nq = Q.shape[0]
    d_s = R.shape[0]
    D = np.empty((nq, k))
    I = np.empty((nq, k), dtype=np.int64)
    P = np.empty((nq, nprobe), dtype=np.int64)
    for qi in range(nq):
        q = np.asarray(Q[qi], dtype=np.float64)
        if forced_probes is None:
            probes = probe_order(coarse64(q, centroids, d_c))[:nprobe]
        else:
            probes = np.asarray(forced_probes[qi], dtype=np.int64)
        P[qi] = probes
        members = np.concatenate([list_ids[offsets[h]:offsets[h + 1]] for h in probes])
        members = np.asarray(members, dtype=np.int64)
        lut = adc_lut64(q[:d_s] @ R, codebooks)
        luts.append(lut)
        approx = adc_dist64(lut, codes[members]) if len(members) else np.zeros(0)
        if rerank_k:
            sd, si = topk_by_dist_then_id(approx, members, rerank_k)
            si = si[si >= 0]
            dr = d_rerank if d_rerank is not None else X.shape[1]
            exact = sqdist64(q[:dr], np.asarray(X)[si, :dr]) if len(si) else np.zeros(0)
            D[qi], I[qi] = topk_by_dist_then_id(exact, si, k)
            cands.append(si)
        else:
            D[qi], I[qi] = topk_by_dist_then_id(approx, members, k)
            cands.append(members)
    if return_candidates:
        return D, I, P, cands, luts
    return D, I, P
