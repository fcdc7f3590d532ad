"""GPU edge cases against the FP64 oracle: empty inverted lists (IVF, IVF-PQ
and the precision form), one list probed by every query (many query tiles
on one list), and a batch holding a configuration without queries."""
import numpy as np
import pytest

from oracle import check, kmeans, pq, precision
from parity_util import check_search, oracle_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as p
    return p


@pytest.fixture(scope="module")
def holes(lib, small_data):
    """The small index with lists 3 and 7 emptied (their members moved to 4
    and 8); the centroids stay, so queries still probe the empty lists."""
    w, X, Q = small_data
    C32, a, _, _ = oracle_index(X, w.nlist, w.d_c, 10, w.seed)
    a = a.copy()
    a[a == 3] = 4
    a[a == 7] = 8
    off, ids = kmeans.build_lists(a.astype(np.int64), w.nlist)
    assert off[4] == off[3] and off[8] == off[7]
    index = lib.IvfIndex.import_ivf(X, C32, a)
    yield w, X, Q, C32, off, ids, a, index
    index.free()


@pytest.mark.parametrize("nprobe,k", [(8, 10), (32, 20), (2, 300)])
def test_empty_lists_ivf(holes, nprobe, k):
    w, X, Q, C32, off, ids, a, index = holes
    dist, gid, probes = index.search(torch.from_numpy(Q).cuda(), w.d_c, w.d_s, nprobe, k,
                                     return_probes=True)
    torch.cuda.synchronize()
    rep = check_search(X, Q, C32, off, ids, w.d_c, w.d_s, nprobe, k, dist.cpu().numpy(),
                       gid.cpu().numpy(), got_p=probes.cpu().numpy())
    assert rep.ok, rep.problems


def test_empty_lists_pq(holes):
    w, X, Q, C32, off, ids, a, index = holes
    M = 8
    rng = np.random.default_rng(11)
    cb = (rng.standard_normal((M, 256, w.d // M)) * 0.1).astype(np.float32)
    codes = pq.pq_encode64(X.astype(np.float64), cb.astype(np.float64))
    index.pq_import(M, w.d, None, cb, codes)
    nprobe, k = 8, 10
    dist, gid, probes = index.search_pq(torch.from_numpy(Q).cuda(), w.d_c, nprobe, M, k,
                                        return_probes=True)
    torch.cuda.synchronize()
    dist, gid, probes = dist.cpu().numpy(), gid.cpu().numpy(), probes.cpu().numpy()
    rd, ri, _, cands, luts = pq.ivfpq_search64(
        Q, C32.astype(np.float64), off, ids, codes, np.eye(w.d), cb.astype(np.float64), w.d_c,
        nprobe, k, forced_probes=probes, return_candidates=True)
    rep = check.Report()
    for qi in range(len(Q)):
        fn = (lambda lut: (lambda idx: pq.adc_dist64(lut, codes[np.asarray(idx)])))(luts[qi])
        check.compare_knn(Q[qi], X, cands[qi], dist[qi], gid[qi], rd[qi], ri[qi], w.d,
                          report=rep, tag=f"q{qi}", dist64=fn)
    assert rep.ok, rep.problems


def test_empty_lists_precision(holes):
    w, X, Q, C32, off, ids, a, index = holes
    index.set_precision("bf16")
    d_c, d_s, nprobe, k, rerank, margin = w.d_c, w.d_s, 8, 10, 24, 8
    dist, gid, probes = index.search_precision(torch.from_numpy(Q).cuda(), d_c, d_s, nprobe, k,
                                               "bf16", rerank, margin, return_probes=True)
    torch.cuda.synchronize()
    dist, gid, probes = dist.cpu().numpy(), gid.cpu().numpy(), probes.cpu().numpy()
    rd, ri, rp, shortlists = precision.precision_search64(
        X, Q, C32.astype(np.float64), off, ids, d_c, d_s, nprobe, k, "bf16", rerank, margin,
        return_shortlist=True)
    assert np.array_equal(probes, rp)
    rep = check.Report()
    for qi in range(len(Q)):
        check.compare_knn(Q[qi], X, shortlists[qi], dist[qi], gid[qi], rd[qi], ri[qi], d_s,
                          report=rep, tag=f"q{qi}")
    assert rep.ok, rep.problems


def test_one_hot_list(lib, small_data):
    """1,000 copies of three queries: every list they probe is met by ~330
    query rows (several query tiles of every height)."""
    w, X, Qs = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 10, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    Q = np.repeat(Qs[:3], 333, axis=0)
    dist, gid, probes = index.search(torch.from_numpy(Q).cuda(), w.d_c, w.d_s, w.nprobe, w.k,
                                     return_probes=True)
    torch.cuda.synchronize()
    dist, gid, probes = dist.cpu().numpy(), gid.cpu().numpy(), probes.cpu().numpy()
    # identical queries get identical answers, and those are the oracle's
    for r in range(len(Q)):
        assert np.array_equal(gid[r], gid[(r // 333) * 333])
    rep = check_search(X, Q, C32, off, ids, w.d_c, w.d_s, w.nprobe, w.k, dist, gid,
                       got_p=probes, queries=[0, 333, 666])
    assert rep.ok, rep.problems
    index.free()


def test_batch_with_empty_configuration(lib, small_data):
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 10, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    Qd = torch.from_numpy(Q).cuda()
    batch = lib.Batch([(index, 0, w.d_c, w.d_s, 4, 10), (index, len(Q), w.d_c, w.d_s, 4, 10),
                       (index, 0, 8, 32, 2, 5)], ldq=w.d, ldk=10)
    dist, gid = batch.run(Qd)
    torch.cuda.synchronize()
    d1, g1 = index.search(Qd, w.d_c, w.d_s, 4, 10)
    torch.cuda.synchronize()
    assert torch.equal(dist[:len(Q)], d1) and torch.equal(gid[:len(Q)], g1)
    batch.free()
    index.free()
