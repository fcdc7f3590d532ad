"""Pins for oracle.exact: brute force, full sort, self-query, blocked path."""
import numpy as np

import synth
from oracle import exact


def triple_loop(X, Q, k, d_s):
    out = []
    for q in Q:
        ds = []
        for j, x in enumerate(X):
            s = 0.0
            for i in range(d_s):
                t = float(q[i]) - float(x[i])
                s += t * t
            ds.append((s, j))
        ds.sort()
        out.append(ds[:k])
    return out


def test_matches_triple_loop():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, 7)).astype(np.float32)
    Q = rng.standard_normal((5, 7)).astype(np.float32)
    for d_s in (3, 7):
        D, I = exact.exact_knn_direct64(X, Q, 6, d_s)
        ref = triple_loop(X, Q, 6, d_s)
        for qi in range(5):
            assert I[qi].tolist() == [j for _, j in ref[qi]]
            np.testing.assert_allclose(D[qi], [s for s, _ in ref[qi]], rtol=1e-13)


def test_k_equals_n_is_full_sort():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((30, 5))
    Q = rng.standard_normal((3, 5))
    D, I = exact.exact_knn_direct64(X, Q, 30)
    for qi in range(3):
        full = ((X - Q[qi]) ** 2).sum(1)
        assert sorted(I[qi].tolist()) == list(range(30))
        assert np.all(np.diff(D[qi]) >= 0)
        np.testing.assert_allclose(np.sort(full), D[qi], rtol=1e-13)


def test_padding_and_ties():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    Q = np.array([[0.0, 0.0]])
    D, I = exact.exact_knn_direct64(X, Q, 5)
    assert I[0].tolist() == [0, 1, 2, -1, -1]     # tie between 1 and 2 -> smaller id
    assert np.isinf(D[0, 3:]).all()


def test_self_query_first_at_zero():
    m = synth.Mixture(32, 10, seed=5)
    X = m.database(2000)
    picks = [0, 17, 1999]
    D, I = exact.exact_knn64(X, X[picks], 3)
    assert I[:, 0].tolist() == picks
    assert np.all(D[:, 0] == 0.0)


def test_blocked_equals_direct():
    m = synth.Mixture(96, 20, seed=6)
    X = m.database(50_000)
    Q = m.queries(12)
    Db, Ib = exact.exact_knn64(X, Q, 10, d_s=96, chunk=7000)
    Dd, Id = exact.exact_knn_direct64(X, Q, 10, 96)
    assert np.array_equal(Ib, Id)
    np.testing.assert_array_equal(Db, Dd)
