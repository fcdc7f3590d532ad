"""Exact nearest-neighbour search in float64 (test infrastructure).

The paper's problem statement (Section 3) retrieves the nearest database
points to a query under the L2 distance (Section 3, "Inverted File Index":
"L2 or cosine"; the retrieval formulas in Appendix A use the norm of the
difference). Exact search is the brute-force O(dN) scan (Section 2) and its
k nearest neighbours are the ground truth of k-Recall@N (Appendix C).

Reading used throughout: distances are *squared* L2 over the first ``d_s``
coordinates (a Matryoshka prefix, Section 3), which has the same arg-min as
the norm. Ties are broken by the smaller database id; missing results are
padded with id -1 and distance +inf.

Pins (tests/test_oracle_exact.py): a pure-Python triple loop on tiny inputs,
k = N gives a full sort of all distances, a query that is itself in the
database is returned first at distance 0, and the blocked path agrees with the
direct path.
"""
from __future__ import annotations

import numpy as np


def sqdist64(q: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """sum_i (q_i - x_i)^2 for every row, difference form, float64."""
    diff = np.asarray(rows, dtype=np.float64) - np.asarray(q, dtype=np.float64)[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def topk_by_dist_then_id(dist: np.ndarray, ids: np.ndarray, k: int):
    """The k smallest (distance, id) pairs in lexicographic order, padded."""
    order = np.lexsort((ids, dist))[:k]
    out_d = np.full(k, np.inf)
    out_i = np.full(k, -1, dtype=np.int64)
    out_d[: len(order)] = dist[order]
    out_i[: len(order)] = ids[order]
    return out_d, out_i


def exact_knn_direct64(X, Q, k: int, d_s: int | None = None):
    """Difference-form distances from every query to every row (small inputs)."""
    X = np.asarray(X)
    Q = np.asarray(Q)
    d_s = X.shape[1] if d_s is None else d_s
    n = X.shape[0]
    ids = np.arange(n, dtype=np.int64)
    D = np.empty((Q.shape[0], k))
    I = np.empty((Q.shape[0], k), dtype=np.int64)
    for qi in range(Q.shape[0]):
        dist = sqdist64(Q[qi, :d_s], X[:, :d_s])
        D[qi], I[qi] = topk_by_dist_then_id(dist, ids, k)
    return D, I


def exact_knn64(X, Q, k: int, d_s: int | None = None, chunk: int = 65536,
                margin: int = 16):
    """Exact k-NN over all rows of X at prefix d_s.

    For large inputs the candidates are first narrowed with the expanded
    identity |q - x|^2 = |q|^2 + |x|^2 - 2 q.x evaluated in float64 with a
    matrix product (keeping k + margin per query per pass), then every
    surviving candidate's distance is recomputed in the difference form and
    the final order is (distance, id). In float64 the identity's rounding
    error (~1e-15 relative) is far below any gap the margin has to cover.
    """
    X = np.asarray(X)
    Q = np.asarray(Q)
    n, d = X.shape
    d_s = d if d_s is None else d_s
    nq = Q.shape[0]
    if n * d_s <= 4_000_000 or nq == 0:
        return exact_knn_direct64(X, Q, k, d_s)
    keep = min(n, k + margin)
    q64 = np.asarray(Q[:, :d_s], dtype=np.float64)
    qn = np.einsum("ij,ij->i", q64, q64)
    cand_d = np.full((nq, 0), np.inf)
    cand_i = np.zeros((nq, 0), dtype=np.int64)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        xb = np.asarray(X[a:b, :d_s], dtype=np.float64)
        xn = np.einsum("ij,ij->i", xb, xb)
        approx = qn[:, None] + xn[None, :] - 2.0 * (q64 @ xb.T)
        kk = min(keep, b - a)
        part = np.argpartition(approx, kk - 1, axis=1)[:, :kk]
        pd = np.take_along_axis(approx, part, axis=1)
        cand_d = np.concatenate([cand_d, pd], axis=1)
        cand_i = np.concatenate([cand_i, part + a], axis=1)
        if cand_d.shape[1] > keep:
            sel = np.argpartition(cand_d, keep - 1, axis=1)[:, :keep]
            cand_d = np.take_along_axis(cand_d, sel, axis=1)
            cand_i = np.take_along_axis(cand_i, sel, axis=1)
    D = np.empty((nq, k))
    I = np.empty((nq, k), dtype=np.int64)
    for qi in range(nq):
        ids = np.unique(cand_i[qi])
        dist = sqdist64(q64[qi], X[ids, :d_s])
        D[qi], I[qi] = topk_by_dist_then_id(dist, ids, k)
    return D, I
