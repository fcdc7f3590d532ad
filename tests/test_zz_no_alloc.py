"""The allocation-free search entry point (adanns_search_noalloc), called
through the C ABI: its results equal adanns_search's bit for bit on two calls
in a row (the second with fewer queries, so that stale contents of the fixed
scratch array from the first call cannot leak into it), and a batch beyond
the array is rejected with ADANNS_EBUDGET, outputs untouched."""
import ctypes as C

import numpy as np
import pytest

from parity_util import check_search, oracle_index

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EBUDGET = -5


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_19435_amd as p
    return p


@pytest.fixture(scope="module")
def setup(lib, small_data):
    w, X, Q = small_data
    C32, a, off, ids = oracle_index(X, w.nlist, w.d_c, 10, w.seed)
    index = lib.IvfIndex.import_ivf(X, C32, a)
    yield w, X, Q, C32, off, ids, index
    index.free()


def _call(lib, fn, index, Qd, d_c, d_s, nprobe, k):
    nq = Qd.shape[0]
    dist = torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda")
    ids = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    probes = torch.full((nq, nprobe), -7, dtype=torch.int32, device="cuda")
    st = fn(index.handle, Qd.data_ptr(), nq, Qd.stride(0), d_c, d_s, nprobe, k, dist.data_ptr(),
            ids.data_ptr(), probes.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return st, dist.cpu().numpy(), ids.cpu().numpy(), probes.cpu().numpy()


@pytest.mark.parametrize("nq_first,nq_second,d_c,d_s,nprobe,k", [
    (100, 37, 16, 64, 4, 10),
    (100, 1, 12, 40, 32, 100),     # every list, k past a list (padding), ragged prefixes
])
def test_noalloc_equals_search(lib, setup, nq_first, nq_second, d_c, d_s, nprobe, k):
    w, X, Q, C32, off, ids, index = setup
    L = lib.lib
    for nq in (nq_first, nq_second):
        Qd = torch.from_numpy(Q[:nq]).cuda()
        st_a, da, ia, pa = _call(lib, L.adanns_search, index, Qd, d_c, d_s, nprobe, k)
        st_b, db, ib, pb = _call(lib, L.adanns_search_noalloc, index, Qd, d_c, d_s, nprobe, k)
        assert st_a == 0 and st_b == 0, lib.last_error()
        assert np.array_equal(da, db) and np.array_equal(ia, ib) and np.array_equal(pa, pb)
        rep = check_search(X, Q[:nq], C32, off, ids, d_c, d_s, nprobe, k, db, ib, got_p=pb)
        assert rep.ok, rep.problems


def test_noalloc_rejects_oversized_batch(lib, setup):
    w, X, Q, C32, off, ids, index = setup
    L = lib.lib
    cap = L.adanns_search_noalloc_max_bytes()
    assert cap == 64 << 20
    # every list probed: each query needs about n * 4 bytes of first-pass values
    nq = cap // (4 * len(X)) + 64
    Qd = torch.from_numpy(np.resize(Q, (nq, Q.shape[1]))).cuda()
    st, d, i, p = _call(lib, L.adanns_search_noalloc, index, Qd, w.d_c, w.d_s, w.nlist, w.k)
    assert st == EBUDGET
    assert "scratch" in lib.last_error()
    assert np.all(d == -7.0) and np.all(i == -7) and np.all(p == -7)
    # a call after the rejection works again
    Qs = torch.from_numpy(Q[:5]).cuda()
    st_a, da, ia, _ = _call(lib, L.adanns_search, index, Qs, w.d_c, w.d_s, w.nprobe, w.k)
    st_b, db, ib, _ = _call(lib, L.adanns_search_noalloc, index, Qs, w.d_c, w.d_s, w.nprobe, w.k)
    assert st_a == 0 and st_b == 0
    assert np.array_equal(da, db) and np.array_equal(ia, ib)
