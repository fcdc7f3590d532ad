"""Pins for oracle.ivf: exhaustive probing reproduces exact search, probe sets
are nested, d_c = d_s is plain IVF, a pure-Python loop agrees."""
import numpy as np
import pytest

import synth
from oracle import exact, ivf, kmeans


@pytest.fixture(scope="module")
def index(small_data):
    w, X, Q = small_data
    init = synth.init_rows(w.n, w.nlist, w.seed)
    C, a, _ = kmeans.kmeans64(X[:, : w.d_c], w.nlist, 10, init)
    off, ids = kmeans.build_lists(a, w.nlist)
    return C, a, off, ids


@pytest.mark.parametrize("d_c", [4, 16])
def test_all_probes_is_exact(small_data, index, d_c):
    w, X, Q = small_data
    C, _, off, ids = index
    D, I, _ = ivf.ivf_search64(X, Q, C, off, ids, d_c, w.d, w.nlist, w.k)
    De, Ie = exact.exact_knn64(X, Q, w.k)
    assert np.array_equal(I, Ie)
    np.testing.assert_allclose(D, De, rtol=1e-12)


def test_nested_probes_monotone(small_data, index):
    w, X, Q = small_data
    C, _, off, ids = index
    prev_kth = None
    prev_probes = None
    _, Ie = exact.exact_knn64(X, Q, w.k)
    prev_rec = -1
    from oracle.metrics import k_recall_at_n
    for p in (1, 2, 4, 8, 16, 32):
        D, I, P = ivf.ivf_search64(X, Q, C, off, ids, w.d_c, w.d, p, w.k)
        if prev_probes is not None:
            for a, b in zip(prev_probes, P):
                assert set(a.tolist()) <= set(b.tolist())
            assert np.all(D[:, -1] <= prev_kth)
        rec = k_recall_at_n(I, Ie, w.k)
        assert rec >= prev_rec
        prev_rec, prev_kth, prev_probes = rec, D[:, -1], P
    assert prev_rec == 1.0


def test_probe_order_and_python_loop(small_data, index):
    w, X, Q = small_data
    C, a, off, ids = index
    q = Q[3]
    D, I, P = ivf.ivf_search64(X, Q[3:4], C, off, ids, w.d_c, w.d_s, w.nprobe, w.k)
    # centroid distances by hand
    cd = [(sum((float(q[i]) - C[h, i]) ** 2 for i in range(w.d_c)), h) for h in range(w.nlist)]
    cd.sort()
    probes = [h for _, h in cd[: w.nprobe]]
    assert P[0].tolist() == probes
    cand = [j for j in range(w.n) if a[j] in probes]
    dd = sorted((sum((float(q[i]) - float(X[j, i])) ** 2 for i in range(w.d_s)), j) for j in cand)
    assert I[0].tolist() == [j for _, j in dd[: w.k]]
    np.testing.assert_allclose(D[0], [s for s, _ in dd[: w.k]], rtol=1e-12)


def test_plain_ivf_is_dc_equals_ds(small_data):
    w, X, Q = small_data
    init = synth.init_rows(w.n, w.nlist, w.seed)
    C, a, _ = kmeans.kmeans64(X, w.nlist, 5, init)          # clustered on full d
    off, ids = kmeans.build_lists(a, w.nlist)
    D, I, P = ivf.ivf_search64(X, Q, C, off, ids, w.d, w.d, 1, w.k)
    # formula row for IVF with one probe: argmin within C_{h(q)}
    for qi in range(len(Q)):
        h = int(np.argmin(((C - Q[qi]) ** 2).sum(1)))
        assert P[qi, 0] == h
        mem = ids[off[h]:off[h + 1]]
        assert I[qi, 0] == mem[np.argmin(((X[mem] - Q[qi]) ** 2).sum(1))]


def test_forced_probes_and_padding(small_data, index):
    w, X, Q = small_data
    C, a, off, ids = index
    # a one-element list to force padding
    sizes = np.diff(off)
    h_small = int(np.argmin(sizes))
    forced = np.full((2, 1), h_small)
    D, I, P = ivf.ivf_search64(X, Q[:2], C, off, ids, w.d_c, w.d_s, 1, sizes[h_small] + 3,
                               forced_probes=forced)
    assert np.all(I[:, -3:] == -1) and np.all(np.isinf(D[:, -3:]))
    assert np.all(P == h_small)
