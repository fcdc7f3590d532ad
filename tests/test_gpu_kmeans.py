"""GPU Lloyd k-means (adanns_build_ivf) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import kmeans

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as p
    return p


def _assign_agrees(X, C64, a_gpu, a_ref, tol=1e-5):
    """Assignments equal except at near-ties under the oracle's centroids."""
    diff = np.nonzero(a_gpu != a_ref)[0]
    for j in diff:
        dg = ((X[j].astype(np.float64) - C64[a_gpu[j]]) ** 2).sum()
        dr = ((X[j].astype(np.float64) - C64[a_ref[j]]) ** 2).sum()
        assert abs(dg - dr) <= tol * max(dr, 1e-30), (j, dg, dr)
    return len(diff)


@pytest.mark.parametrize("use_train", [False, True])
def test_build_ivf_matches_oracle(lib, small_data, use_train):
    w, X, _ = small_data
    if use_train:
        rows = synth.subsample_rows(w.n, 3000, w.seed)
        Xt = X[rows, : w.d_c]
    else:
        rows = None
        Xt = X[:, : w.d_c]
    init = synth.init_rows(len(Xt), w.nlist, w.seed)
    Xd = torch.from_numpy(X).cuda()
    index, obj = lib.IvfIndex.build_ivf(Xd, w.nlist, w.d_c, 10, init, train_rows=rows,
                                         return_objective=True)
    C64, a_t, hist = kmeans.kmeans64(Xt, w.nlist, 10, init)
    # Lloyd's objective never increases on the GPU either
    assert np.all(obj[1:] <= obj[:-1] * (1 + 1e-6)), obj
    np.testing.assert_allclose(obj, hist, rtol=1e-5)
    Cg = index.centroids().astype(np.float64)
    np.testing.assert_allclose(Cg, C64, atol=1e-5 * np.abs(C64).max())
    a_ref = kmeans.assign64(X[:, : w.d_c], C64)
    off, ids = index.lists()
    a_gpu = np.empty(w.n, dtype=np.int64)
    for h in range(w.nlist):
        a_gpu[ids[off[h]:off[h + 1]]] = h
        assert np.all(np.diff(ids[off[h]:off[h + 1]]) > 0)
    nd = _assign_agrees(X[:, : w.d_c], C64, a_gpu, a_ref)
    assert nd <= 2
    index.free()


def test_build_then_search_exhaustive_is_exact(lib, small_data):
    from oracle import exact
    w, X, Q = small_data
    init = synth.init_rows(w.n, w.nlist, w.seed)
    index = lib.IvfIndex.build_ivf(torch.from_numpy(X).cuda(), w.nlist, w.d_c, 3, init)
    dist, ids = index.search(torch.from_numpy(Q).cuda(), w.d_c, w.d, w.nlist, w.k)
    torch.cuda.synchronize()
    De, Ie = exact.exact_knn64(X, Q, w.k)
    assert np.array_equal(ids.cpu().numpy(), Ie)
    np.testing.assert_allclose(dist.cpu().numpy(), De, rtol=1e-5)
    index.free()


def test_build_ivf_invalid(lib, small_data):
    w, X, _ = small_data
    Xd = torch.from_numpy(X).cuda()
    with pytest.raises(lib.AdannsError):
        lib.IvfIndex.build_ivf(Xd, w.nlist, w.d + 1, 3, synth.init_rows(w.n, w.nlist))
    with pytest.raises(lib.AdannsError):
        bad = synth.init_rows(w.n, w.nlist)
        bad[0] = w.n
        lib.IvfIndex.build_ivf(Xd, w.nlist, w.d_c, 3, bad)


def test_fp16_database_equals_fp32_of_the_same_values(lib, small_data):
    """An FP16 database (ADANNS_DTYPE_F16) builds, imports and trains exactly
    like the FP32 matrix holding the same (half-representable) values."""
    w, X, Q = small_data
    X16 = X.astype(np.float16)
    X32 = X16.astype(np.float32)
    init = synth.init_rows(w.n, w.nlist, w.seed)
    a16, o16 = lib.IvfIndex.build_ivf(torch.from_numpy(X16).cuda(), w.nlist, w.d_c, 5, init,
                                      return_objective=True)
    a32, o32 = lib.IvfIndex.build_ivf(torch.from_numpy(X32).cuda(), w.nlist, w.d_c, 5, init,
                                      return_objective=True)
    assert np.array_equal(o16, o32)
    assert np.array_equal(a16.centroids(), a32.centroids())
    for x, y in zip(a16.lists(), a32.lists()):
        assert np.array_equal(x, y)
    Qd = torch.from_numpy(Q).cuda()
    r16 = a16.search(Qd, w.d_c, w.d_s, w.nprobe, w.k)
    r32 = a32.search(Qd, w.d_c, w.d_s, w.nprobe, w.k)
    torch.cuda.synchronize()
    assert torch.equal(r16[0], r32[0]) and torch.equal(r16[1], r32[1])
    pinit = synth.init_rows(w.n, 256, w.seed, synth.STREAM_PQ)
    a16.pq_train(torch.from_numpy(X16).cuda(), 8, w.d, 3, pinit)
    a32.pq_train(torch.from_numpy(X32).cuda(), 8, w.d, 3, pinit)
    for x, y in zip(a16.pq_codec(8, w.d), a32.pq_codec(8, w.d)):
        assert np.array_equal(x, y)
    C = a32.centroids()
    off, ids = a32.lists()
    assign = np.empty(w.n, dtype=np.int32)
    for h in range(w.nlist):
        assign[ids[off[h]:off[h + 1]]] = h
    i16 = lib.IvfIndex.import_ivf(X16, C, assign)
    s16 = i16.search(Qd, w.d_c, w.d_s, w.nprobe, w.k)
    torch.cuda.synchronize()
    assert torch.equal(s16[0], r32[0]) and torch.equal(s16[1], r32[1])
    for ix in (a16, a32, i16):
        ix.free()
