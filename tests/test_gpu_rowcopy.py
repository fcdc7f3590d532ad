"""The optional row-major copy of an index's vectors changes where the exact
re-measurements read each candidate, not what they compute: every search
form returns the same bits with and without it, and stays at parity with the
FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import pq
from parity_util import check_search, oracle_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as lib
    m = synth.Mixture(160, 300, seed=91)
    X = m.database(30_000)
    Q = m.queries(400)
    C32, a, off, ids = oracle_index(X, 48, 24, 6, 91)
    plain = lib.IvfIndex.import_ivf(X, C32, a)
    rowed = lib.IvfIndex.import_ivf(X, C32, a)
    b0 = rowed.device_bytes()
    rowed.add_row_copy()
    rowed.add_row_copy()  # idempotent
    grown = rowed.device_bytes() - b0
    yield lib, X, Q, C32, off, ids, plain, rowed, grown
    plain.free()
    rowed.free()


def _np(*ts):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("d_c,d_s,nprobe,k", [(24, 160, 4, 10), (16, 97, 8, 60), (8, 33, 2, 100)])
def test_ivf_same_bits(pair, d_c, d_s, nprobe, k):
    lib, X, Q, C32, off, ids, plain, rowed, grown = pair
    Qd = torch.from_numpy(Q).cuda()
    a = _np(*plain.search(Qd, d_c, d_s, nprobe, k, return_probes=True))
    b = _np(*rowed.search(Qd, d_c, d_s, nprobe, k, return_probes=True))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    rep = check_search(X, Q, C32, off, ids, d_c, d_s, nprobe, k, b[0], b[1], got_p=b[2],
                       queries=range(0, len(Q), 9))
    assert rep.ok, rep.problems


def test_memory_accounted(pair):
    lib, X, Q, C32, off, ids, plain, rowed, grown = pair
    assert grown >= X.shape[0] * X.shape[1] * 4


def test_batch_same_bits(pair):
    lib, X, Q, C32, off, ids, plain, rowed, grown = pair
    Qd = torch.from_numpy(Q).cuda()
    cfg = [(200, 24, 160, 4, 10), (200, 16, 64, 8, 20)]
    outs = []
    for ix in (plain, rowed):
        b = lib.Batch([(ix, *c) for c in cfg], ldq=X.shape[1])
        outs.append(_np(*b.run(Qd)))
        b.free()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_pq_rerank_same_bits(pair):
    lib, X, Q, C32, off, ids, plain, rowed, grown = pair
    M, d = 8, X.shape[1]
    rng = np.random.default_rng(3)
    cb = (rng.standard_normal((M, 256, d // M)) * 0.1).astype(np.float32)
    codes = pq.pq_encode64(X.astype(np.float64), cb.astype(np.float64))
    Qd = torch.from_numpy(Q).cuda()
    res = []
    for ix in (plain, rowed):
        ix.pq_import(M, d, None, cb, codes)
        res.append(_np(*ix.search_pq(Qd, 24, 6, M, 10, rerank_k=40, d_rerank=120)))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_precision_same_bits(pair, fmt):
    lib, X, Q, C32, off, ids, plain, rowed, grown = pair
    Qd = torch.from_numpy(Q).cuda()
    res = []
    for ix in (plain, rowed):
        ix.set_precision(fmt)
        res.append(_np(*ix.search_precision(Qd, 24, 160, 4, 10, fmt, 48)))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
