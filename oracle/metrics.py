"""Retrieval metrics and the compute cost model (test infrastructure).

* k-Recall@N (Section 3 "Metrics"; Appendix C): the overlap between the k
  exact nearest neighbours and the N retrieved items, averaged over queries.
  Ground truth is exact search; here it is exact search at the full d
  unless a prefix is given (reading: the paper's centroid study takes the
  highest dimensionality as ground truth, Appendix E.2).
* Compute cost per query (Appendix B.1). The printed formula multiplies the
  scan dimensionality into the coarse term and reuses k for two things; it is
  read here as C = d_c * nlist + nprobe * d_s * N / nlist multiply-adds,
  which is the only form in which a number of clusters near sqrt(N) is the
  FLOP-optimal choice for d_c = d_s, as Section 5.3 states.
* Relative contrast (Appendix H.2): C_r = E_q[D_mean] / E_q[D_min].
* Centroid k-Recall@N (Appendix E.2): centroids ranked with a low-d prefix
  scored against the ranking at the highest d.

Pins: tests/test_oracle_metrics.py (hand-built overlaps, the cost optimum at
sqrt(nprobe * d_s * N / d_c), C_r of a hand-built set, centroid recall of a
hand-built layout for k < N and k = N).
"""
from __future__ import annotations

import numpy as np

from .exact import sqdist64


def k_recall_at_n(retrieved_ids, true_ids, k: int) -> float:
    """mean over queries of |top-k true  intersect  retrieved| / k."""
    retrieved_ids = np.asarray(retrieved_ids)
    true_ids = np.asarray(true_ids)[:, :k]
    hits = 0
    for r, t in zip(retrieved_ids, true_ids):
        hits += len(set(int(v) for v in r if v >= 0) & set(int(v) for v in t if v >= 0))
    return hits / (k * len(true_ids)) if len(true_ids) else 0.0


def cost_macs(d_c: int, d_s: int, nlist: int, nprobe: int, n: int) -> float:
    """Multiply-adds per query of AdANNS-IVF (reading of Appendix B.1)."""
    return d_c * nlist + nprobe * d_s * n / nlist


def relative_contrast(X, Q, d: int | None = None) -> float:
    """E_q[mean_x D(q,x)] / E_q[min_x D(q,x)] with D the L2 distance."""
    X = np.asarray(X)
    Q = np.asarray(Q)
    d = X.shape[1] if d is None else d
    dmean = []
    dmin = []
    for q in Q:
        dist = np.sqrt(sqdist64(q[:d], X[:, :d]))
        dmean.append(dist.mean())
        dmin.append(dist.min())
    return float(np.mean(dmean) / np.mean(dmin))


def centroid_recall(Q, centroids, d_low: int, k: int, n: int) -> float:
    """k-Recall@N of centroids ranked at prefix d_low against the full width."""
    Q = np.asarray(Q)
    C = np.asarray(centroids)
    hits = 0
    for q in Q:
        full = np.lexsort((np.arange(len(C)), sqdist64(q, C)))[:k]
        low = np.lexsort((np.arange(len(C)), sqdist64(q[:d_low], C[:, :d_low])))[:n]
        hits += len(set(full.tolist()) & set(low.tolist()))
    return hits / (k * len(Q))
