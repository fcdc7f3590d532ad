"""Parity at the full width of the image-retrieval workload (d = d_s = 2048)
with enough queries (2,500) to take the launch shapes of a full batch: the
64x128 and 128x128 scan tiles (and the others), the one-wave scan selection
for batches past 2048 queries (two passes of 1024 coordinates per
re-measure), and the precision and IVF-PQ selections' many-query wave
branch (precision re-ranks of 32 and 256, PQ re-rank at d_rerank 2048).
Queries spread over the whole batch are compared with the FP64 oracle
(Algorithm 1; Section 4.3 for the shortlist-then-re-rank forms)."""
import numpy as np
import pytest

import synth
from oracle import check, pq, precision
from parity_util import check_search, oracle_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D, N, NQ, NLIST, D_C, NPROBE, K = 2048, 20_000, 2500, 32, 64, 4, 10
SAMPLE = list(range(0, NQ, 40)) + [NQ - 1]
SAMPLE_PREC = list(range(0, NQ, 125)) + [NQ - 1]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as p
    return p


@pytest.fixture(scope="module")
def wide(lib):
    m = synth.Mixture(D, 200, seed=2048)
    X = m.database(N)
    Q = m.queries(NQ)
    C32, a, off, ids = oracle_index(X, NLIST, D_C, 6, 2048)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    yield X, Q, C32, off, ids, index
    index.free()


def test_fullwidth_search(wide, lib):
    """adanns_search as the bench calls it (untuned: 64x128 tiles here)."""
    X, Q, C32, off, ids, index = wide
    lib.selection_stats(reset=True)
    dist, gid, probes = index.search(torch.from_numpy(Q).cuda(), D_C, D, NPROBE, K,
                                     return_probes=True)
    torch.cuda.synchronize()
    _, uncert = lib.selection_stats(reset=True)
    rep = check_search(X, Q, C32, off, ids, D_C, D, NPROBE, K, dist.cpu().numpy(),
                       gid.cpu().numpy(), got_p=probes.cpu().numpy(), queries=SAMPLE)
    assert rep.ok, rep.problems
    assert uncert == 0


@pytest.mark.parametrize("tq,tv", [(64, 128), (128, 128), (64, 64), (32, 128), (128, 64)])
def test_fullwidth_tile_shapes(wide, lib, tq, tv):
    X, Q, C32, off, ids, index = wide
    b = lib.Batch([(index, NQ, D_C, D, NPROBE, K)], ldq=D)
    try:
        b.set_shape(tq, 2048, tv)
        probes = torch.empty(NQ * NPROBE, dtype=torch.int32, device="cuda")
        dist, gid = b.run(torch.from_numpy(Q).cuda(), probes=probes)
        torch.cuda.synchronize()
        rep = check_search(X, Q, C32, off, ids, D_C, D, NPROBE, K, dist.cpu().numpy(),
                           gid.cpu().numpy(), got_p=probes.view(NQ, NPROBE).cpu().numpy(),
                           queries=SAMPLE)
        assert rep.ok, rep.problems
    finally:
        b.free()


@pytest.mark.parametrize("fmt,rerank", [("bf16", 32), ("fp8", 32), ("bf16", 256), ("fp8", 256)])
def test_fullwidth_precision(wide, lib, fmt, rerank):
    X, Q, C32, off, ids, index = wide
    index.set_precision(fmt)
    dist, gid, probes = index.search_precision(torch.from_numpy(Q).cuda(), D_C, D, NPROBE, K, fmt,
                                               rerank, 8, return_probes=True)
    torch.cuda.synchronize()
    dist, gid, probes = dist.cpu().numpy(), gid.cpu().numpy(), probes.cpu().numpy()
    rd, ri, rp, shortlists = precision.precision_search64(
        X, Q[SAMPLE_PREC], C32.astype(np.float64), off, ids, D_C, D, NPROBE, K, fmt, rerank, 8,
        return_shortlist=True)
    assert np.array_equal(probes[SAMPLE_PREC], rp)
    rep = check.Report()
    for j, qi in enumerate(SAMPLE_PREC):
        check.compare_knn(Q[qi], X, shortlists[j], dist[qi], gid[qi], rd[j], ri[j], D,
                          report=rep, tag=f"q{qi}")
    assert rep.ok, rep.problems


def test_fullwidth_pq_rerank(wide, lib):
    """PQ on the 256-coordinate prefix (M = 32), re-rank of 48 at d_rerank
    2048: the many-query one-wave selection."""
    X, Q, C32, off, ids, index = wide
    M, d_s, rerank = 32, 256, 48
    # codebooks from a 4,000-row training subset, every row encoded
    X64 = X[:, :d_s].astype(np.float64)
    cb32 = pq.pq_train64(X64[:4000], M, 4, init_rows=synth.init_rows(4000, 256, 2049,
                                                                      synth.STREAM_PQ))
    cb32 = cb32.astype(np.float32)
    R32 = np.eye(d_s, dtype=np.float32)
    codes = pq.pq_encode64(X64, cb32.astype(np.float64))
    index.pq_import(M, d_s, None, cb32, codes)
    dist, gid, probes = index.search_pq(torch.from_numpy(Q).cuda(), D_C, NPROBE, M, K,
                                        rerank_k=rerank, d_rerank=D, return_probes=True)
    torch.cuda.synchronize()
    dist, gid, probes = dist.cpu().numpy(), gid.cpu().numpy(), probes.cpu().numpy()
    rd, ri, _, cands, _ = pq.ivfpq_search64(
        Q[SAMPLE], C32.astype(np.float64), off, ids, codes, R32.astype(np.float64),
        cb32.astype(np.float64), D_C, NPROBE, K, rerank_k=rerank, X=X, d_rerank=D,
        forced_probes=probes[SAMPLE], return_candidates=True)
    rep = check.Report()
    for j, qi in enumerate(SAMPLE):
        check.compare_knn(Q[qi], X, cands[j], dist[qi], gid[qi], rd[j], ri[j], D, report=rep,
                          tag=f"q{qi}")
    assert rep.ok, rep.problems


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_fullwidth_filtered_equals_search(wide, lib, fmt):
    """The FP32 search's result from a quantised first pass: bit for bit the
    plain search's at the full width (every query of the batch)."""
    X, Q, C32, off, ids, index = wide
    index.set_precision(fmt)
    Qd = torch.from_numpy(Q).cuda()
    a = index.search(Qd, D_C, D, NPROBE, K, return_probes=True)
    b = index.search_filtered(Qd, D_C, D, NPROBE, K, fmt, return_probes=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
