"""Tie-aware comparison of a candidate search result with the oracle
(test infrastructure).

Several answers are correct when distances tie, so the comparison checks
what is unique and checks the rest for validity:

* probes: with c* the oracle's nprobe-th smallest coarse distance, a probe
  set is valid iff each member has c_h <= c*(1 + tol) and every cluster with
  c_h < c*(1 - tol) is a member;
* ids: equal position by position, except where the two ids' float64
  distances differ by at most ``tol`` relative; every returned id must be a
  scanned candidate, no candidate left out may be nearer than the returned
  k-th by more than ``tol``, and no id may repeat;
* distances: |d_gpu - d64| <= dist_tol * d64, with an absolute floor of
  dist_tol * |q[:d_s]|^2 for d64 near 0;
* padding: -1 / +inf in the same positions.

These rules compare float64 distances the oracle computes itself; nothing in
them is taken from the candidate other than its ids, distances and probes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .exact import sqdist64


@dataclass
class Report:
    ok: bool = True
    problems: list = field(default_factory=list)
    max_rel_dist_err: float = 0.0
    id_mismatch_ties: int = 0

    def fail(self, msg):
        self.ok = False
        if len(self.problems) < 20:
            self.problems.append(msg)


def probes_valid(c: np.ndarray, probes, nprobe: int, tol: float = 1e-6) -> bool:
    order = np.lexsort((np.arange(len(c)), c))
    cstar = c[order[nprobe - 1]]
    probes = np.asarray(probes)
    if len(set(probes.tolist())) != nprobe:
        return False
    if np.any(c[probes] > cstar * (1 + tol) + 1e-300):
        return False
    must = np.nonzero(c < cstar * (1 - tol))[0]
    return set(must.tolist()) <= set(probes.tolist())


def compare_knn(q, X, cand_ids, got_d, got_i, ref_d, ref_i, d_s: int,
                tol: float = 1e-6, dist_tol: float = 1e-5, report: Report | None = None,
                tag: str = "", dist64=None) -> Report:
    """Compare one query's result (got) with the oracle's (ref).

    ``cand_ids`` are the ids the method ranked (union of probed lists, or the
    shortlist that was re-ranked), ``X`` the database (any float dtype), ``q``
    the query. ``dist64`` maps an id array to the oracle's float64 distances
    of the method being checked (default: squared L2 on the first d_s
    coordinates of X).
    """
    rep = report or Report()
    q = np.asarray(q, dtype=np.float64)
    if dist64 is None:
        def dist64(idx):
            return sqdist64(q[:d_s], np.asarray(X)[np.asarray(idx), :d_s])
    got_i = np.asarray(got_i, dtype=np.int64)
    ref_i = np.asarray(ref_i, dtype=np.int64)
    k = len(ref_i)
    valid_g = got_i >= 0
    valid_r = ref_i >= 0
    if not np.array_equal(valid_g, valid_r):
        rep.fail(f"{tag} padding differs: got {got_i.tolist()} ref {ref_i.tolist()}")
        return rep
    if np.any(np.isfinite(np.asarray(got_d)[~valid_g])):
        rep.fail(f"{tag} padded slots must hold +inf")
    gi = got_i[valid_g]
    if len(set(gi.tolist())) != len(gi):
        rep.fail(f"{tag} repeated ids {gi.tolist()}")
        return rep
    cand = set(np.asarray(cand_ids).tolist())
    if not set(gi.tolist()) <= cand:
        rep.fail(f"{tag} ids outside the probed lists: {sorted(set(gi.tolist()) - cand)[:5]}")
        return rep
    if len(gi) == 0:
        return rep
    d64_got = dist64(gi)
    d64_ref = np.asarray(ref_d)[valid_r]
    # positions
    for pos in range(len(gi)):
        if gi[pos] != ref_i[pos]:
            a, b = d64_got[pos], d64_ref[pos]
            if abs(a - b) > tol * max(a, b, 1e-300):
                rep.fail(f"{tag} id mismatch at {pos}: got {gi[pos]} ({a!r}) ref {ref_i[pos]} ({b!r})")
                return rep
            rep.id_mismatch_ties += 1
    # nothing better was left out
    kth = d64_got.max()
    if len(cand) > len(gi):
        rest = np.array(sorted(cand - set(gi.tolist())), dtype=np.int64)
        if len(rest) and len(gi) == k:
            dr = dist64(rest)
            if np.any(dr < kth * (1 - tol)):
                j = rest[np.argmin(dr)]
                rep.fail(f"{tag} left out a nearer candidate {j} ({dr.min()!r} < {kth!r})")
                return rep
    # distances
    gd = np.asarray(got_d, dtype=np.float64)[valid_g]
    floor = dist_tol * float(q[:d_s] @ q[:d_s]) if X is not None else 0.0
    err = np.abs(gd - d64_got)
    rel = err / np.maximum(d64_got, 1e-300)
    bad = err > np.maximum(dist_tol * d64_got, floor)
    if np.any(bad):
        p = int(np.argmax(bad))
        rep.fail(f"{tag} distance error at {p}: got {gd[p]!r} exact {d64_got[p]!r}")
    small = d64_got > floor / dist_tol * 1e-3
    if np.any(small):
        rep.max_rel_dist_err = max(rep.max_rel_dist_err, float(rel[small].max()))
    return rep
