"""Batching form: one batched (and graph-captured) launch over many search
configurations equals each configuration searched alone, bit for bit, for
every tile shape; and matches the FP64 oracle."""
import numpy as np
import pytest

import synth
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
def setup(lib):
    m = synth.Mixture(128, 200, seed=31)
    X = m.database(40_000)
    indices = {}
    for d_c in (16, 32, 64):
        C32, a, off, ids = oracle_index(X, 64, d_c, 5, 31 + d_c)
        indices[d_c] = (lib.IvfIndex.import_ivf(X, C32, a), C32, off, ids)
    rng = np.random.default_rng(5)
    configs = []
    for _ in range(12):
        d_c = int(rng.choice([16, 32, 64]))
        d_s = int(rng.choice([32, 64, 128]))
        nprobe = int(rng.choice([2, 4, 8]))
        nq = int(np.round(np.exp(rng.uniform(0, np.log(300)))))
        configs.append((d_c, d_s, nprobe, nq))
    Qall = m.queries(sum(c[3] for c in configs))
    yield X, indices, configs, Qall
    for ix, *_ in indices.values():
        ix.free()


def _alone(indices, configs, Qall, k):
    out = []
    r = 0
    for d_c, d_s, nprobe, nq in configs:
        ix = indices[d_c][0]
        d, i = ix.search(torch.from_numpy(Qall[r:r + nq]).cuda(), d_c, d_s, nprobe, k)
        torch.cuda.synchronize()
        out.append((d.cpu().numpy(), i.cpu().numpy()))
        r += nq
    return out


def _split(dist, ids, configs, k):
    res, r = [], 0
    for c in configs:
        res.append((dist[r:r + c[3], :k], ids[r:r + c[3], :k]))
        r += c[3]
    return res


def test_batch_equals_alone_all_shapes(lib, setup):
    X, indices, configs, Qall = setup
    k = 10
    alone = _alone(indices, configs, Qall, k)
    batch = lib.Batch([(indices[c[0]][0], c[3], c[0], c[1], c[2], k) for c in configs], ldq=128)
    Qd = torch.from_numpy(Qall).cuda()
    for tq in (32, 64, 128):
        for tv in (64, 128):
            for grid in (8, 1024):
                batch.set_shape(tq, grid, tv)
                dist, ids = batch.run(Qd)
                torch.cuda.synchronize()
                got = _split(dist.cpu().numpy(), ids.cpu().numpy(), configs, k)
                for (gd, gi), (ad, ai) in zip(got, alone):
                    assert np.array_equal(gi, ai) and np.array_equal(gd, ad), (tq, tv, grid)
    batch.free()


def test_many_configurations_beyond_lds_histogram(lib, setup):
    """136 configurations of 64 lists each: more virtual lists (8704) than the
    bucketing's LDS histogram holds, so it takes its per-pair atomic path;
    every configuration still equals its search alone, bit for bit."""
    X, indices, _, _ = setup
    k = 10
    rng = np.random.default_rng(9)
    many = []
    for _ in range(136):
        many.append((int(rng.choice([16, 32, 64])), int(rng.choice([32, 64, 128])),
                     int(rng.choice([2, 4, 8])), int(rng.integers(1, 6))))
    Q = rng.standard_normal((sum(c[3] for c in many), 128)).astype(np.float32)
    alone = _alone(indices, many, Q, k)
    batch = lib.Batch([(indices[c[0]][0], c[3], c[0], c[1], c[2], k) for c in many], ldq=128)
    dist, ids = batch.run(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    got = _split(dist.cpu().numpy(), ids.cpu().numpy(), many, k)
    for (gd, gi), (ad, ai) in zip(got, alone):
        assert np.array_equal(gi, ai) and np.array_equal(gd, ad)
    batch.free()


def test_graph_replays_equal_eager(lib, setup):
    X, indices, configs, Qall = setup
    k = 10
    batch = lib.Batch([(indices[c[0]][0], c[3], c[0], c[1], c[2], k) for c in configs], ldq=128)
    Qd = torch.from_numpy(Qall).cuda()
    ed, ei = batch.run(Qd)
    torch.cuda.synchronize()
    ed, ei = ed.cpu().numpy(), ei.cpu().numpy()
    out = batch.outputs()
    for rep in range(3):
        out[0].fill_(-1.0)
        out[1].fill_(-7)
        batch.run(Qd, out=out, graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out[1].cpu().numpy(), ei), rep
        assert np.array_equal(out[0].cpu().numpy(), ed), rep
        # eager work of the program's own between replays
        batch.run(Qd)
        torch.cuda.synchronize()
    batch.free()


def test_autotune_keeps_results_and_parity(lib, setup):
    X, indices, configs, Qall = setup
    k = 10
    alone = _alone(indices, configs, Qall, k)
    batch = lib.Batch([(indices[c[0]][0], c[3], c[0], c[1], c[2], k) for c in configs], ldq=128)
    Qd = torch.from_numpy(Qall).cuda()
    tq, tv, grid = batch.autotune(Qd, reps=1)
    assert tq in (32, 64, 128) and tv in (64, 128) and grid in (1024, 2048, 4096)
    dist, ids = batch.run(Qd)
    torch.cuda.synchronize()
    got = _split(dist.cpu().numpy(), ids.cpu().numpy(), configs, k)
    for (gd, gi), (ad, ai) in zip(got, alone):
        assert np.array_equal(gi, ai) and np.array_equal(gd, ad)
    # oracle parity of two configurations
    r = 0
    for ci, (d_c, d_s, nprobe, nq) in enumerate(configs[:4]):
        _, C32, off, ids_ = indices[d_c]
        Qc = Qall[r:r + nq]
        gd, gi = got[ci]
        ix = indices[d_c][0]
        _, _, probes = ix.search(torch.from_numpy(Qc).cuda(), d_c, d_s, nprobe, k,
                                 return_probes=True)
        torch.cuda.synchronize()
        rep = check_search(X, Qc, C32, off, ids_, d_c, d_s, nprobe, k, gd, gi,
                           got_p=probes.cpu().numpy())
        assert rep.ok, rep.problems
        r += nq
    batch.free()
    lib.autotune_clear()


def test_batch_invalid(lib, setup):
    X, indices, configs, Qall = setup
    ix = indices[16][0]
    with pytest.raises(lib.AdannsError):
        lib.Batch([(ix, 5, 17, 64, 4, 10)], ldq=128)       # d_c above d_c_build
    with pytest.raises(lib.AdannsError):
        lib.Batch([(ix, 5, 16, 64, 4, 10)], ldq=32)        # ldq too small
    b = lib.Batch([(ix, 5, 16, 64, 4, 10)], ldq=128)
    for tq, tv in ((8, 64), (48, 64), (64, 256), (64, 32)):  # no such tile
        with pytest.raises(lib.AdannsError):
            b.set_shape(tq, 1024, tv)
    with pytest.raises(lib.AdannsError):
        b.set_shape(64, 4, 64)                             # grid below 8
    b.free()


def test_all_shapes_ragged_prefixes_parity(lib, setup):
    """Every tile shape on prefixes that end inside a 32-coordinate slab
    (coarse and scan), against the FP64 oracle on the library's probes; one
    list is probed by enough queries to fill several 128-row query tiles."""
    X, indices, configs, Qall = setup
    k = 10
    _, C32, off, ids_ = indices[16]
    ix = indices[16][0]
    cfgs = [(12, 40, 4, 300), (16, 33, 8, 57), (9, 97, 2, 1)]
    batch = lib.Batch([(ix, nq, d_c, d_s, nprobe, k) for d_c, d_s, nprobe, nq in cfgs], ldq=128)
    # the first configuration repeats three queries 100 times each, so that
    # its probed lists hold one to three full 128-row query tiles
    Q = np.concatenate([np.repeat(Qall[:3], 100, axis=0), Qall[3:3 + 58]])
    Qd = torch.from_numpy(Q).cuda()
    for tq in (32, 64, 128):
        for tv in (64, 128):
            batch.set_shape(tq, 1024, tv)
            dist, ids = batch.run(Qd)
            torch.cuda.synchronize()
            dist, ids = dist.cpu().numpy(), ids.cpu().numpy()
            r = 0
            for d_c, d_s, nprobe, nq in cfgs:
                Qc = Q[r:r + nq]
                _, _, probes = ix.search(torch.from_numpy(Qc).cuda(), d_c, d_s, nprobe, k,
                                         return_probes=True)
                torch.cuda.synchronize()
                rep = check_search(X, Qc, C32, off, ids_, d_c, d_s, nprobe, k,
                                   dist[r:r + nq, :k], ids[r:r + nq, :k],
                                   got_p=probes.cpu().numpy(), queries=range(0, nq, 7))
                assert rep.ok, ((tq, tv), (d_c, d_s), rep.problems)
                r += nq
    batch.free()
