"""Pins for oracle.kmeans: Lloyd's monotone objective, closed forms,
fixed points, a pure-Python assignment."""
import numpy as np

import synth
from oracle import kmeans


def test_objective_never_increases(small_data):
    w, X, _ = small_data
    init = synth.init_rows(w.n, w.nlist, w.seed)
    C, a, hist = kmeans.kmeans64(X[:, : w.d_c], w.nlist, 10, init)
    assert len(hist) == 11
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-12))
    assert hist[-1] < hist[0]
    # final assignment is the nearest centroid of every point
    assert np.array_equal(a, kmeans.assign64(X[:, : w.d_c], C))


def test_one_cluster_is_global_mean():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 6))
    C, a, hist = kmeans.kmeans64(X, 1, 3, [7])
    np.testing.assert_allclose(C[0], X.mean(0), rtol=0, atol=1e-14)
    assert np.all(a == 0)
    np.testing.assert_allclose(hist[-1], ((X - X.mean(0)) ** 2).sum(), rtol=1e-12)


def test_n_clusters_on_all_points_is_zero():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((64, 5))
    C, a, hist = kmeans.kmeans64(X, 64, 4, np.arange(64)[::-1].copy())
    assert hist[-1] == 0.0
    assert np.array_equal(np.sort(a), np.arange(64))


def test_fixed_point_centroids_are_member_means(small_data):
    w, X, _ = small_data
    Xs = X[:3000, :8]
    init = synth.init_rows(3000, 8, w.seed, tag=1)
    C, a, hist = kmeans.kmeans64(Xs, 8, 5, init)
    for _ in range(1000):                      # Lloyd until the assignment is stable
        C = kmeans.update64(Xs, a, C)
        a_next = kmeans.assign64(Xs, C)
        if np.array_equal(a_next, a):
            break
        a = a_next
    else:
        raise AssertionError("no fixed point within 1000 iterations")
    # at the fixed point one more update does not move anything
    C2 = kmeans.update64(Xs, a, C)
    np.testing.assert_allclose(C2, C, atol=1e-12)
    for h in range(8):
        if np.any(a == h):
            np.testing.assert_allclose(C[h], Xs[a == h].astype(np.float64).mean(0), atol=1e-12)


def test_assign_matches_python_loop():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((200, 4)).astype(np.float32)
    C = rng.standard_normal((9, 4))
    C[5] = C[2]                       # an exact tie: index 2 must win
    ref = []
    for x in X:
        best = None
        for h, c in enumerate(C):
            d = sum((float(x[i]) - c[i]) ** 2 for i in range(4))
            if best is None or d < best[0]:
                best = (d, h)
        ref.append(best[1])
    got = kmeans.assign64(X, C)
    assert got.tolist() == ref
    assert not np.any(got == 5)


def test_empty_cluster_keeps_centroid():
    X = np.array([[0.0], [0.1], [0.2]])
    C0 = np.array([[0.1], [100.0]])
    C1 = kmeans.update64(X, kmeans.assign64(X, C0), C0)
    assert C1[1, 0] == 100.0
    np.testing.assert_allclose(C1[0, 0], 0.1)


def test_lists_are_grouped_and_ascending():
    a = np.array([2, 0, 2, 1, 0, 2])
    off, ids = kmeans.build_lists(a, 4)
    assert off.tolist() == [0, 2, 3, 6, 6]
    assert ids.tolist() == [1, 4, 3, 0, 2, 5]
