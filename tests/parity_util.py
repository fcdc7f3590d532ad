"""Helpers shared by the GPU parity tests: build an oracle index, run the
library, compare with the oracle under the tie-aware rules."""
from __future__ import annotations

import numpy as np

import synth
from oracle import check, ivf, kmeans, pq


def oracle_index(X, nlist, d_c, iters, seed, n_train=None):
    """Oracle k-means on X[:, :d_c] (optionally on a seeded training subset,
    then one assignment of every row). Returns (C32, assign, offsets, ids)."""
    if n_train is not None and n_train < len(X):
        rows = synth.subsample_rows(len(X), n_train, seed)
        Xt = X[rows, :d_c]
    else:
        Xt = X[:, :d_c]
    init = synth.init_rows(len(Xt), nlist, seed)
    C64, a, _ = kmeans.kmeans64(Xt, nlist, iters, init)
    C32 = C64.astype(np.float32)
    if n_train is not None and n_train < len(X):
        a = kmeans.assign64(X[:, :d_c], C32.astype(np.float64))
    else:
        # lists are defined by the centroids the library will hold (FP32)
        a = kmeans.assign64(X[:, :d_c], C32.astype(np.float64))
    off, ids = kmeans.build_lists(a, nlist)
    return C32, a.astype(np.int32), off, ids


def check_search(X, Q, C32, off, ids, d_c, d_s, nprobe, k, got_d, got_i, got_p=None,
                 forced=None, queries=None, dist_tol=1e-5):
    """Tie-aware parity of a search result against the FP64 oracle.

    With ``got_p`` the probe sets are first checked for validity, then the
    oracle result is recomputed on the library's probes; with ``forced`` the
    given probes were used by both sides.
    """
    Cf = C32.astype(np.float64)
    rep = check.Report()
    qsel = range(len(Q)) if queries is None else queries
    qsel = list(qsel)
    if got_p is not None:
        probes = got_p
        own_diff = 0
        for qi in qsel:
            c = ivf.coarse64(Q[qi], Cf, d_c)
            if not check.probes_valid(c, got_p[qi], nprobe):
                rep.fail(f"q{qi}: probe set outside the tie band")
            if not np.array_equal(ivf.probe_order(c)[:nprobe], got_p[qi]):
                own_diff += 1
        rep.probe_diffs = own_diff
    else:
        probes = forced
    sub = np.asarray(qsel)
    rd, ri, _, cands = ivf.ivf_search64(X, Q[sub], Cf, off, ids, d_c, d_s, nprobe, k,
                                        forced_probes=np.asarray(probes)[sub],
                                        return_candidates=True)
    for j, qi in enumerate(qsel):
        check.compare_knn(Q[qi], X, cands[j], got_d[qi], got_i[qi], rd[j], ri[j], d_s,
                          report=rep, tag=f"q{qi}", dist_tol=dist_tol)
    return rep


def make_codec(X, M, d_s, opq, seed):
    """Oracle-trained PQ (or OPQ) codec on X[:, :d_s], rounded to the FP32
    values the library holds. Returns (R32, codebooks32, codes)."""
    X64 = X[:, :d_s].astype(np.float64)
    init = synth.init_rows(len(X), 256, seed, synth.STREAM_PQ)
    if opq:
        R, cbs, _ = pq.opq_train64(X64[:4000], M, 3, 3, synth.init_rows(4000, 256, seed, synth.STREAM_PQ))
    else:
        R, cbs = np.eye(d_s), pq.pq_train64(X64, M, 4, init_rows=init)
    R32, cb32 = R.astype(np.float32), cbs.astype(np.float32)
    codes = pq.pq_encode64(X64 @ R32.astype(np.float64), cb32.astype(np.float64))
    return R32, cb32, codes
