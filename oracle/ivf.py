"""AdANNS-IVF search in float64 (test infrastructure).

Follows Algorithm 1 (inference) and the AdANNS-IVF row of the retrieval
formulas (Appendix A, Table "formula"): per query,

1. distance from the query's first ``d_c`` coordinates to every centroid's
   first ``d_c`` coordinates;
2. order the clusters by that distance and keep the ``nprobe`` nearest;
3. gather the members of those clusters;
4. linear scan of the members with the first ``d_s`` coordinates, keeping
   the k nearest.

Readings of points the paper leaves open or prints ambiguously:

* the pseudocode slices rows (``database[:d_cluster]``) where the method
  means coordinates; here every slice is a column prefix ``[:, :m]``;
* ``sortAscending(distances)[:num_probes]`` is read as an arg-sort; equal
  distances go to the smaller cluster index;
* the formula table probes a single cluster h(q); nprobe > 1 probes the union
  of the nprobe nearest lists, and nprobe = 1 is the formula;
* centroids may be wider than the search's d_c (built on d_c_build >= d_c):
  the search uses their first d_c coordinates (the AdANNS-IVF-D row);
* distances are squared L2, top-k ordered by (distance, id), padded with
  -1 / +inf when fewer than k members were scanned.

``forced_probes`` replaces step 2 with a given probe set, so a candidate
result whose probes differ only inside a tie band can be re-checked.

Pins (tests/test_oracle_ivf.py): nprobe = nlist with d_s = d reproduces exact
search for any d_c; probe sets are nested in nprobe, so the k-th distance never
grows with nprobe; a pure-Python loop agrees on tiny inputs.
"""
from __future__ import annotations

import numpy as np

from .exact import sqdist64, topk_by_dist_then_id


def coarse64(q, centroids, d_c: int):
    """c_h = sum_{i<d_c} (q_i - mu_{h,i})^2 for every cluster h."""
    return sqdist64(np.asarray(q)[:d_c], np.asarray(centroids)[:, :d_c])


def probe_order(c: np.ndarray) -> np.ndarray:
    """Clusters sorted by (c_h, h)."""
    return np.lexsort((np.arange(len(c)), c))


def ivf_search64(X, Q, centroids, offsets, list_ids, d_c: int, d_s: int,
                 nprobe: int, k: int, forced_probes=None, return_candidates=False):
    """Returns (dist [nq,k] f64, ids [nq,k] i64, probes [nq,nprobe] i64)."""
    X = np.asarray(X)
    Q = np.asarray(Q)
    centroids = np.asarray(centroids)
    nq = Q.shape[0]
    D = np.empty((nq, k))
    I = np.empty((nq, k), dtype=np.int64)
    P = np.empty((nq, nprobe), dtype=np.int64)
    cands = []
    for qi in range(nq):
        q = Q[qi]
        if forced_probes is None:
            c = coarse64(q, centroids, d_c)
            probes = probe_order(c)[:nprobe]
        else:
            probes = np.asarray(forced_probes[qi], dtype=np.int64)
        P[qi] = probes
        members = np.concatenate([list_ids[offsets[h]:offsets[h + 1]] for h in probes])
        members = np.asarray(members, dtype=np.int64)
        if return_candidates:
            cands.append(members)
        if len(members):
            dist = sqdist64(q[:d_s], X[members, :d_s])
        else:
            dist = np.zeros(0)
        D[qi], I[qi] = topk_by_dist_then_id(dist, members, k)
    if return_candidates:
        return D, I, P, cands
    return D, I, P
