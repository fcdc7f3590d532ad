"""Pins for oracle.pq: LUT identity, exactness with <= 256 rows, R orthonormal,
rotation invariance, monotone OPQ distortion, pure-Python ADC."""
import numpy as np
import pytest

import synth
from oracle import exact, ivf, kmeans, pq


@pytest.fixture(scope="module")
def opq_small():
    m = synth.Mixture(32, 20, seed=9)
    X = m.database(3000).astype(np.float64)
    init = synth.init_rows(3000, 256, 9, synth.STREAM_PQ)
    R, cbs, hist = pq.opq_train64(X, 8, 4, 4, init)
    return X, R, cbs, hist


def test_rotation_is_orthonormal(opq_small):
    _, R, _, _ = opq_small
    np.testing.assert_allclose(R.T @ R, np.eye(R.shape[0]), atol=1e-10)
    np.testing.assert_allclose(R @ R.T, np.eye(R.shape[0]), atol=1e-10)


def test_distortion_never_increases(opq_small):
    _, _, _, hist = opq_small
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-10))


def test_rotation_preserves_distances(opq_small):
    X, R, _, _ = opq_small
    a = ((X[:50, None, :] - X[None, 50:80, :]) ** 2).sum(-1)
    Y = X @ R
    b = ((Y[:50, None, :] - Y[None, 50:80, :]) ** 2).sum(-1)
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12)


def test_lut_identity(opq_small):
    X, R, cbs, _ = opq_small
    codes = pq.pq_encode64(X @ R, cbs)
    q = X[5] + 0.01
    lut = pq.adc_lut64(q @ R, cbs)
    d_lut = pq.adc_dist64(lut, codes)
    d_dec = ((pq.pq_decode64(codes, cbs) - (q @ R)[None, :]) ** 2).sum(1)
    np.testing.assert_allclose(d_lut, d_dec, rtol=1e-12, atol=1e-14)
    # pure-Python ADC for a few rows
    for j in (0, 7, 2999):
        s = sum(lut[m, codes[j, m]] for m in range(codes.shape[1]))
        assert abs(s - d_lut[j]) <= 1e-12 * max(1.0, s)


def test_small_database_adc_is_exact():
    m = synth.Mixture(16, 5, seed=11)
    X = m.database(256).astype(np.float64)
    Q = m.queries(6).astype(np.float64)
    cbs = pq.pq_train64(X, 4, 3, init_rows=np.arange(256))    # every row its own centroid
    codes = pq.pq_encode64(X, cbs)
    np.testing.assert_array_equal(pq.pq_decode64(codes, cbs), X)
    off = np.array([0, 256])
    ids = np.arange(256)
    D, I, _ = pq.ivfpq_search64(Q, np.zeros((1, 16)), off, ids, codes, np.eye(16), cbs, 4, 1, 10)
    De, Ie = exact.exact_knn64(X, Q, 10)
    assert np.array_equal(I, Ie)
    np.testing.assert_allclose(D, De, rtol=1e-12)


def test_ivfpq_rerank_full_is_ivf(small_data):
    w, X, Q = small_data
    init = synth.init_rows(w.n, w.nlist, w.seed)
    C, a, _ = kmeans.kmeans64(X[:, : w.d_c], w.nlist, 3, init)
    off, ids = kmeans.build_lists(a, w.nlist)
    pinit = synth.init_rows(w.n, 256, w.seed, synth.STREAM_PQ)
    cbs = pq.pq_train64(X, 8, 2, init_rows=pinit)
    codes = pq.pq_encode64(X, cbs)
    # a re-rank depth larger than any candidate set reduces to plain IVF search
    D, I, P = pq.ivfpq_search64(Q[:20], C, off, ids, codes, np.eye(w.d), cbs, w.d_c, w.nprobe,
                                w.k, rerank_k=w.n, X=X, d_rerank=w.d_s)
    D2, I2, P2 = ivf.ivf_search64(X, Q[:20], C, off, ids, w.d_c, w.d_s, w.nprobe, w.k)
    assert np.array_equal(P, P2) and np.array_equal(I, I2)
    np.testing.assert_allclose(D, D2, rtol=1e-13)


def test_rotated_adc_is_exact_under_rotation_invariance():
    """Every row its own codeword in the rotated space: the decoded rotated
    rows equal X R, and |q R - x R| = |q - x| for orthonormal R (Section 3,
    OPQ; Appendix D), so IVF-OPQ over one list equals exact search. The same
    codes searched with R^T (a transposed rotation of the query) do not."""
    d, M, n = 16, 4, 256
    m = synth.Mixture(d, 7, seed=23)
    X = m.database(n).astype(np.float64)
    Q = m.queries(12).astype(np.float64)
    # the float32 draw re-orthonormalised in float64 (QR, signs fixed)
    R, r = np.linalg.qr(synth.random_rotation(d, seed=23).astype(np.float64))
    R = R * np.sign(np.diag(r))[None, :]
    np.testing.assert_allclose(R.T @ R, np.eye(d), atol=1e-13)
    assert not np.allclose(R, R.T)
    Y = X @ R
    cbs = pq.pq_train64(Y, M, 2, init_rows=np.arange(n))
    codes = pq.pq_encode64(Y, cbs)
    np.testing.assert_allclose(pq.pq_decode64(codes, cbs), Y, rtol=0, atol=1e-12)
    off = np.array([0, n])
    ids = np.arange(n)
    D, I, _ = pq.ivfpq_search64(Q, np.zeros((1, d)), off, ids, codes, R, cbs, 4, 1, 10)
    De, Ie = exact.exact_knn64(X, Q, 10)
    assert np.array_equal(I, Ie)
    np.testing.assert_allclose(D, De, rtol=1e-10, atol=1e-12)
    # a query rotated by R^T instead of R misses neighbours
    Dt, It, _ = pq.ivfpq_search64(Q, np.zeros((1, d)), off, ids, codes, R.T.copy(), cbs, 4, 1, 10)
    assert not np.array_equal(It, Ie)


def test_opq_from_a_given_rotation():
    """Started from an orthonormal R0, the alternation's first PQ step is PQ
    on X R0, the distortion never increases, and R stays orthonormal."""
    m = synth.Mixture(16, 6, seed=31)
    X = m.database(1500).astype(np.float64)
    init = synth.init_rows(1500, 256, 31, synth.STREAM_PQ)
    R0 = synth.random_rotation(16, seed=31).astype(np.float64)
    R0, r = np.linalg.qr(R0)
    R0 = R0 * np.sign(np.diag(r))[None, :]
    R, cbs, hist = pq.opq_train64(X, 4, 3, 2, init, R0=R0)
    first = pq.pq_train64(X @ R0, 4, 2, init_rows=init)
    codes = pq.pq_encode64(X @ R0, first)
    assert hist[0] == pytest.approx(pq.distortion64(X @ R0, codes, first), rel=1e-12)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-10))
    np.testing.assert_allclose(R.T @ R, np.eye(16), atol=1e-10)
