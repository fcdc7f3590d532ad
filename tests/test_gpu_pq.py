"""GPU parity of AdANNS-IVF-PQ search (adanns_search_pq) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import check, ivf, pq
from parity_util import make_codec, oracle_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as p
    return p


@pytest.fixture(scope="module")
def pq_small(lib, small_data):
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 10, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    codecs = {}
    for M, opq in ((16, True), (8, False), (32, False), (64, False)):
        R32, cb32, codes = make_codec(X, M, w.d, opq, w.seed + M)
        index.pq_import(M, w.d, R32 if opq else None, cb32, codes)
        codecs[M] = (R32, cb32, codes)
    yield w, X, Q, C32, off, ids, index, codecs
    index.free()


@pytest.mark.parametrize("M,nprobe,k,rerank", [(16, 4, 10, 0), (8, 4, 10, 0), (16, 4, 10, 40),
                                               (16, 32, 5, 0), (8, 2, 50, 60), (32, 4, 10, 0),
                                               (64, 8, 10, 0), (64, 4, 10, 40)])
def test_pq_parity(pq_small, M, nprobe, k, rerank):
    w, X, Q, C32, off, ids, index, codecs = pq_small
    R32, cb32, codes = codecs[M]
    d_c = w.d_c
    dist, gid, probes = index.search_pq(torch.from_numpy(Q).cuda(), d_c, nprobe, M, k,
                                        rerank_k=rerank, d_rerank=w.d, return_probes=True)
    torch.cuda.synchronize()
    dist, gid, probes = dist.cpu().numpy(), gid.cpu().numpy(), probes.cpu().numpy()
    Cf = C32.astype(np.float64)
    for qi in range(len(Q)):
        assert check.probes_valid(ivf.coarse64(Q[qi], Cf, d_c), probes[qi], nprobe)
    rd, ri, _, cands, luts = pq.ivfpq_search64(
        Q, Cf, off, ids, codes, R32.astype(np.float64), cb32.astype(np.float64), d_c, nprobe, k,
        rerank_k=rerank, X=X, d_rerank=w.d, forced_probes=probes, return_candidates=True)
    rep = check.Report()
    for qi in range(len(Q)):
        if rerank:
            fn = None
        else:
            lut = luts[qi]
            fn = (lambda lut: (lambda idx: pq.adc_dist64(lut, codes[np.asarray(idx)])))(lut)
        check.compare_knn(Q[qi], X, cands[qi], dist[qi], gid[qi], rd[qi], ri[qi], w.d,
                          report=rep, tag=f"q{qi}", dist64=fn)
    assert rep.ok, rep.problems


def test_pq_invalid(pq_small, lib):
    w, X, Q, C32, off, ids, index, codecs = pq_small
    Qd = torch.from_numpy(Q).cuda()
    with pytest.raises(lib.AdannsError):
        index.search_pq(Qd, w.d_c, 4, 12, 10)           # no codec with M = 12
    with pytest.raises(lib.AdannsError):
        index.search_pq(Qd, w.d_c, 4, 16, 10, rerank_k=5, d_rerank=w.d)   # rerank_k < k
    with pytest.raises(lib.AdannsError):
        index.pq_import(16, w.d, None, codecs[16][1], codecs[16][2])      # duplicate M


def test_pq_train_matches_oracle(lib, small_data):
    """GPU-trained plain PQ (adanns_pq_train) against the oracle's PQ k-means."""
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 5, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    M, iters = 8, 6
    init = synth.init_rows(w.n, 256, w.seed, synth.STREAM_PQ, tag=3)
    index.pq_train(torch.from_numpy(X).cuda(), M, w.d, iters, init)
    R, cb, codes = index.pq_codec(M, w.d)
    assert np.array_equal(R, np.eye(w.d, dtype=np.float32))
    ref_cb = pq.pq_train64(X, M, iters, init_rows=init)
    # after several rounds a near-tie assignment (FP32 vs FP64) may have
    # moved codewords apart; the training objective must agree regardless
    # (the exact one-round comparison is test_pq_train_one_round_traced)
    Xf = X.astype(np.float64)
    got_j = pq.distortion64(Xf, pq.pq_encode64(Xf, cb.astype(np.float64)), cb.astype(np.float64))
    ref_j = pq.distortion64(Xf, pq.pq_encode64(Xf, ref_cb), ref_cb)
    assert abs(got_j - ref_j) <= 1e-3 * ref_j, (got_j, ref_j)
    ref_codes = pq.pq_encode64(X, cb.astype(np.float64))
    diff = np.argwhere(codes != ref_codes)
    dsub = w.d // M
    for j, m in diff:       # only near-ties may differ
        y = X[j, m * dsub:(m + 1) * dsub].astype(np.float64)
        dg = ((y - cb[m, codes[j, m]]) ** 2).sum()
        dr = ((y - cb[m, ref_codes[j, m]]) ** 2).sum()
        assert abs(dg - dr) <= 1e-5 * max(dr, 1e-12)
    assert len(diff) <= 0.001 * codes.size
    # the trained codec searches like an imported one
    dist, gid = index.search_pq(torch.from_numpy(Q).cuda(), w.d_c, 4, M, 10)
    torch.cuda.synchronize()
    assert np.all(gid.cpu().numpy() >= 0)
    index.free()


def test_pq_train_with_rotation(lib, small_data):
    """A given rotation: training and encoding happen on the rotated rows."""
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 5, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    M, iters = 16, 5
    R = synth.random_rotation(w.d, w.seed, tag=1)
    np.testing.assert_allclose(R.T.astype(np.float64) @ R, np.eye(w.d), atol=1e-5)
    rows = synth.subsample_rows(w.n, 4000, w.seed, tag=2)
    init = synth.init_rows(len(rows), 256, w.seed, synth.STREAM_PQ, tag=4)
    index.pq_train(torch.from_numpy(X).cuda(), M, w.d, iters, init, train_rows=rows, R=R)
    R2, cb, codes = index.pq_codec(M, w.d)
    assert np.array_equal(R2, R)
    Y = X.astype(np.float64) @ R.astype(np.float64)
    ref_cb = pq.pq_train64(Y[rows], M, iters, init_rows=init)
    got_j = pq.distortion64(Y[rows], pq.pq_encode64(Y[rows], cb.astype(np.float64)),
                            cb.astype(np.float64))
    ref_j = pq.distortion64(Y[rows], pq.pq_encode64(Y[rows], ref_cb), ref_cb)
    assert abs(got_j - ref_j) <= 1e-3 * ref_j, (got_j, ref_j)
    ref_codes = pq.pq_encode64(Y, cb.astype(np.float64))
    diff = np.argwhere(codes != ref_codes)
    dsub = w.d // M
    for j, m in diff:
        y = Y[j, m * dsub:(m + 1) * dsub]
        dg = ((y - cb[m, codes[j, m]]) ** 2).sum()
        dr = ((y - cb[m, ref_codes[j, m]]) ** 2).sum()
        assert abs(dg - dr) <= 1e-5 * max(dr, 1e-12)
    assert len(diff) <= 0.001 * codes.size
    index.free()


@pytest.mark.parametrize("rotate", [False, True])
def test_pq_train_one_round_traced(lib, small_data, rotate):
    """One Lloyd round per block from the same initial codewords (the
    training rows' sub-vectors given by init_rows): every GPU codeword equals
    the oracle's mean to FP32 rounding, except the codewords of clusters that
    a near-tie row (best two squared distances within 1e-5 relative, where
    FP32 and FP64 may choose differently) joins or leaves."""
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 5, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    M = 8
    dsub = w.d // M
    R = synth.random_rotation(w.d, w.seed, tag=5) if rotate else None
    rows = synth.subsample_rows(w.n, 5000, w.seed, tag=6)
    init = synth.init_rows(len(rows), 256, w.seed, synth.STREAM_PQ, tag=7)
    index.pq_train(torch.from_numpy(X).cuda(), M, w.d, 1, init, train_rows=rows, R=R)
    _, cb, _ = index.pq_codec(M, w.d)
    Y = X[rows].astype(np.float64)
    if rotate:
        Y = Y @ R.astype(np.float64)
    ref_cb = pq.pq_train64(Y, M, 1, init_rows=init)
    traced = 0
    for m in range(M):
        ym = Y[:, m * dsub:(m + 1) * dsub]
        c0 = ym[init]                                   # the common initial codewords
        dd = ((ym[:, None, :] - c0[None, :, :]) ** 2).sum(-1)
        two = np.sort(dd, axis=1)[:, :2]
        near = (two[:, 1] - two[:, 0]) <= 1e-5 * np.maximum(two[:, 1], 1e-30)
        touched = set()
        for j in np.flatnonzero(near):                  # codewords a near-tie row may choose
            touched |= set(np.flatnonzero(dd[j] <= two[j, 0] * (1 + 1e-5) + 1e-30).tolist())
        bad = np.flatnonzero(np.any(np.abs(cb[m] - ref_cb[m]) > 2e-6, axis=1))
        assert set(bad.tolist()) <= touched, (m, sorted(set(bad.tolist()) - touched))
        traced += len(bad)
    assert traced <= 0.01 * M * 256
    index.free()


@pytest.mark.parametrize("d_s,M", [(64, 16), (32, 8)])
def test_exhaustive_opq_prefix(lib, small_data, d_s, M):
    """AdANNS-OPQ without clustering (Section 4.2): one list holding every
    vector, ADC over the d_s prefix with d_s/M-dimensional blocks. Both sides
    scan all N codes; the oracle is ivfpq_search64 with a single list."""
    w, X, Q = small_data
    C1 = X.astype(np.float64).mean(axis=0, keepdims=True).astype(np.float32)
    a = np.zeros(len(X), dtype=np.int32)
    index = lib.IvfIndex.import_ivf(X, C1, a)
    R32, cb32, codes = make_codec(X, M, d_s, True, w.seed + 100 + d_s)
    index.pq_import(M, d_s, R32, cb32, codes)
    k = 10
    dist, gid = index.search_pq(torch.from_numpy(Q).cuda(), w.d, 1, M, k)
    torch.cuda.synchronize()
    dist, gid = dist.cpu().numpy(), gid.cpu().numpy()
    off = np.array([0, len(X)], dtype=np.int64)
    ids = np.arange(len(X), dtype=np.int64)
    rd, ri, _, cands, luts = pq.ivfpq_search64(
        Q, C1.astype(np.float64), off, ids, codes, R32.astype(np.float64),
        cb32.astype(np.float64), w.d, 1, k, return_candidates=True)
    rep = check.Report()
    for qi in range(len(Q)):
        fn = (lambda lut: (lambda idx: pq.adc_dist64(lut, codes[np.asarray(idx)])))(luts[qi])
        check.compare_knn(Q[qi], X, cands[qi], dist[qi], gid[qi], rd[qi], ri[qi], d_s,
                          report=rep, tag=f"q{qi}", dist64=fn)
    assert rep.ok, rep.problems
    index.free()


def test_pq_chunked_equals_whole(pq_small, lib):
    w, X, Q, C32, off, ids, index, codecs = pq_small
    Qd = torch.from_numpy(Q).cuda()
    whole = index.search_pq(Qd, w.d_c, 4, 16, 10, rerank_k=40, d_rerank=w.d, return_probes=True)
    torch.cuda.synchronize()
    try:
        lib.set_search_scratch_cap(64 * 1024)
        parts = index.search_pq(Qd, w.d_c, 4, 16, 10, rerank_k=40, d_rerank=w.d,
                                return_probes=True)
        torch.cuda.synchronize()
    finally:
        lib.set_search_scratch_cap(0)
    for x, y in zip(whole, parts):
        assert torch.equal(x, y)
