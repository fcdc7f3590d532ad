"""The generator is seeded, chunk-deterministic and normalised."""
import numpy as np

import synth


def test_deterministic_and_thread_independent():
    m = synth.Mixture(48, 30, seed=123)
    a = m.rows(synth.STREAM_DB, 140_000, threads=1)
    b = synth.Mixture(48, 30, seed=123).rows(synth.STREAM_DB, 140_000, threads=4)
    assert np.array_equal(a, b)
    # a prefix of the rows is the same whatever n is asked for
    c = m.rows(synth.STREAM_DB, 70_000, threads=2)
    assert np.array_equal(a[:65536], c[:65536])


def test_unit_norm_and_decaying_energy():
    m = synth.Mixture(256, 50, seed=7)
    X = m.database(5000)
    np.testing.assert_allclose((X.astype(np.float64) ** 2).sum(1), 1.0, rtol=1e-5)
    e = (X.astype(np.float64) ** 2).mean(0)
    # the first quarter of the coordinates carries most of the energy
    assert e[:64].sum() > 0.7 * e.sum()


def test_streams_differ_and_init_rows():
    m = synth.Mixture(16, 4, seed=1)
    assert not np.array_equal(m.database(100), m.queries(100))
    r = synth.init_rows(1000, 32, 5)
    assert len(set(r.tolist())) == 32 and r.min() >= 0 and r.max() < 1000
    assert np.array_equal(r, synth.init_rows(1000, 32, 5))
