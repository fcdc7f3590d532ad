"""Lloyd's k-means and the inverted file, float64 (test infrastructure).

IVF construction clusters the database with k-means (Lloyd's algorithm) and
keeps, per cluster, the list of its members (Section 3, "Inverted File
Index"; Appendix E). AdANNS-IVF runs the clustering on the first ``d_c``
coordinates of the Matryoshka representation (Section 4.1; Algorithm 1,
construction).

Details the paper leaves open, and the readings taken here:

* initial centroids are given rows of the data (the caller draws them from a
  seeded permutation);
* one iteration = assign every point to its nearest centroid (ties to the
  smaller centroid index), record the objective, move every centroid to the
  mean of its members; a centroid with no members stays where it is;
* after the last update, one final assignment against the final centroids
  defines the inverted lists;
* each inverted list holds its member ids in ascending order.

Pins (tests/test_oracle_kmeans.py): the objective never increases (Lloyd's
guarantee), one cluster converges to the global mean, N clusters seeded on
all N points give objective 0, a fixed point has every centroid equal to the
mean of its members, and assignment agrees with a pure-Python loop.
"""
from __future__ import annotations

import numpy as np

from .exact import sqdist64


def _nearest_two_expanded(xb: np.ndarray, C: np.ndarray, cn: np.ndarray):
    """Indices of the two smallest |x - c|^2 per row via the expanded identity."""
    approx = cn[None, :] - 2.0 * (xb @ C.T)
    m = C.shape[0]
    if m == 1:
        return np.zeros((xb.shape[0], 1), dtype=np.int64)
    return np.argpartition(approx, 1, axis=1)[:, :2]


def assign64(X, C, chunk: int = 32768) -> np.ndarray:
    """argmin_h |x - mu_h|^2 for every row, ties to the smaller h.

    The expanded identity in float64 shortlists the two nearest centroids;
    both are then re-measured in the difference form, which decides.
    """
    X = np.asarray(X)
    C = np.asarray(C, dtype=np.float64)
    n = X.shape[0]
    out = np.empty(n, dtype=np.int64)
    cn = np.einsum("ij,ij->i", C, C)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        xb = np.asarray(X[a:b], dtype=np.float64)
        two = _nearest_two_expanded(xb, C, cn)
        if two.shape[1] == 1:
            out[a:b] = 0
            continue
        d0 = np.einsum("ij,ij->i", xb - C[two[:, 0]], xb - C[two[:, 0]])
        d1 = np.einsum("ij,ij->i", xb - C[two[:, 1]], xb - C[two[:, 1]])
        pick1 = (d1 < d0) | ((d1 == d0) & (two[:, 1] < two[:, 0]))
        out[a:b] = np.where(pick1, two[:, 1], two[:, 0])
    return out


def objective64(X, C, assign) -> float:
    """J = sum_j |x_j - mu_{a(j)}|^2 (difference form)."""
    X = np.asarray(X, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    diff = X - C[np.asarray(assign)]
    return float(np.einsum("ij,ij->", diff, diff))


def update64(X, assign, C_prev) -> np.ndarray:
    """Each centroid becomes the mean of its members; empty ones stay."""
    X = np.asarray(X, dtype=np.float64)
    nlist = C_prev.shape[0]
    sums = np.zeros((nlist, X.shape[1]))
    np.add.at(sums, np.asarray(assign), X)
    counts = np.bincount(assign, minlength=nlist).astype(np.float64)
    C = np.array(C_prev, dtype=np.float64, copy=True)
    nz = counts > 0
    C[nz] = sums[nz] / counts[nz, None]
    return C


def kmeans64(X, nlist: int, iters: int, init_rows=None, init_centroids=None):
    """Lloyd's k-means on the rows of X (already sliced to the d_c prefix).

    Starts from the given rows of X, or from given centroids (a warm start).
    Returns (centroids [nlist, d] f64, final assignment [n] i64,
    objectives J_0..J_{iters} where J_t is measured right after the t-th
    assignment, the last one being the final assignment).
    """
    X = np.asarray(X)
    if init_centroids is not None:
        C = np.array(init_centroids, dtype=np.float64, copy=True)
    else:
        init_rows = np.asarray(init_rows, dtype=np.int64)
        if len(init_rows) != nlist:
            raise ValueError("need nlist initial rows")
        C = np.asarray(X[init_rows], dtype=np.float64).copy()
    if C.shape[0] != nlist:
        raise ValueError("need nlist initial centroids")
    history = []
    for _ in range(iters):
        a = assign64(X, C)
        history.append(objective64(X, C, a))
        C = update64(X, a, C)
    a = assign64(X, C)
    history.append(objective64(X, C, a))
    return C, a, np.array(history)


def build_lists(assign, nlist: int):
    """Inverted lists: offsets [nlist+1] and member ids grouped by list,
    ascending within each list."""
    assign = np.asarray(assign, dtype=np.int64)
    counts = np.bincount(assign, minlength=nlist)
    offsets = np.zeros(nlist + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    ids = np.argsort(assign, kind="stable").astype(np.int64)
    return offsets, ids
