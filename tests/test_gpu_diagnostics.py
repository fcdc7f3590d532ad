"""Data diagnostics computed through the library, against the oracle's
definitions: centroid k-Recall@N of the coarse step at a prefix d_low
against the full-width ranking (Appendix E.2, the highest width as ground
truth), from the library's probes on full-width centroids; and the relative
contrast E_q[mean_x D] / E_q[min_x D] (Appendix H.2) from the library's
exhaustive search distances."""
import numpy as np
import pytest

import synth
from oracle import check, ivf, metrics
from parity_util import oracle_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as p
    return p


@pytest.fixture(scope="module")
def full_width(lib, small_data):
    """IVF on every coordinate (d_c_build = d): its centroids rank at any
    prefix d_low <= d."""
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d, 8, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    yield w, X, Q, C32, index
    index.free()


def _probes(index, Q, d_c, nprobe):
    _, _, p = index.search(torch.from_numpy(Q).cuda(), d_c, 1, nprobe, 1, return_probes=True)
    torch.cuda.synchronize()
    return p.cpu().numpy()


@pytest.mark.parametrize("d_low", [2, 4, 8, 16, 33, 64])
def test_centroid_recall_from_library_probes(full_width, d_low):
    w, X, Q, C32, index = full_width
    Cf = C32.astype(np.float64)
    truth = _probes(index, Q, w.d, 4)         # the full-width ranking's first 4
    low = _probes(index, Q, d_low, 16)         # the prefix ranking's first 16
    for qi in range(len(Q)):                   # both are the coarse step's own probes
        assert check.probes_valid(ivf.coarse64(Q[qi], Cf, w.d), truth[qi], 4)
        assert check.probes_valid(ivf.coarse64(Q[qi], Cf, d_low), low[qi], 16)
    for k, N in ((1, 1), (1, 4), (1, 16), (4, 4), (4, 16)):
        got = np.mean([len(set(truth[q, :k]) & set(low[q, :N])) / k for q in range(len(Q))])
        ref = metrics.centroid_recall(Q, Cf, d_low, k, N)
        assert got == pytest.approx(ref, abs=1e-12), (k, N)


@pytest.mark.parametrize("d", [8, 32, 64])
def test_relative_contrast_from_library_distances(lib, small_data, d):
    """Exhaustive search (one list, every row returned) gives every squared
    distance; the contrast computed from them matches the oracle's."""
    w, X0, Q = small_data
    X = X0[:1000]
    C1 = X.astype(np.float64).mean(axis=0, keepdims=True).astype(np.float32)
    index = lib.IvfIndex.import_ivf(X, C1, np.zeros(len(X), dtype=np.int32))
    try:
        dist, gid = index.search(torch.from_numpy(Q).cuda(), 1, d, 1, len(X))
        torch.cuda.synchronize()
        dist, gid = dist.cpu().numpy().astype(np.float64), gid.cpu().numpy()
        assert np.all(gid >= 0) and np.all(np.sort(gid, axis=1) == np.arange(len(X)))
        dl = np.sqrt(np.maximum(dist, 0.0))
        got = float(np.mean(dl.mean(axis=1)) / np.mean(dl.min(axis=1)))
        ref = metrics.relative_contrast(X, Q, d)
        assert got == pytest.approx(ref, rel=1e-5)
    finally:
        index.free()
