"""Pins for oracle.precision: the e4m3 and bf16 formats from their
definitions, round-to-nearest-even with saturation, and the reduction of the
shortlist-then-rerank form to plain IVF search."""
import json
import os

import numpy as np

import synth
from oracle import ivf, kmeans, precision

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_e4m3_golden_values():
    # byte -> value pairs of the OCP 8-bit floating point specification (E4M3)
    with open(os.path.join(GOLDEN, "e4m3_values.json")) as f:
        g = json.load(f)
    for hexcode, val in g["pairs"]:
        code = int(hexcode, 16)
        assert precision.e4m3_value(np.uint8(code)) == val
        assert int(precision.e4m3_encode_value(np.float64(val))) == code or val == 0.0


def test_e4m3_roundtrip_all_codes():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    vals = precision.e4m3_value(codes)
    back = precision.e4m3_encode_value(vals)
    nz = vals != 0
    assert np.array_equal(back[nz], codes[nz])
    # values on the grid are fixed points of rounding
    assert np.array_equal(precision.e4m3_round(vals.astype(np.float32)), vals)
    # the finite positive grid is strictly increasing in the code
    pos = precision.e4m3_value(np.arange(0, 127, dtype=np.uint8))
    assert np.all(np.diff(pos) > 0) and pos[-1] == 448.0


def test_e4m3_nearest_and_ties_to_even():
    grid = precision.e4m3_value(np.arange(0, 127, dtype=np.uint8))
    rng = np.random.default_rng(0)
    y = rng.uniform(0, 460, 20000).astype(np.float32)
    r = precision.e4m3_round(y)
    # nearest grid point (saturating)
    idx = np.searchsorted(grid, y.astype(np.float64))
    lo = grid[np.clip(idx - 1, 0, len(grid) - 1)]
    hi = grid[np.clip(idx, 0, len(grid) - 1)]
    best = np.where(np.abs(y - lo) <= np.abs(hi - y), lo, hi)
    tie = np.abs(y - lo) == np.abs(hi - y)
    assert np.array_equal(r[~tie], best[~tie])
    # exact midpoints go to the even code
    mids = ((grid[1:] + grid[:-1]) / 2).astype(np.float32)
    rm = precision.e4m3_round(mids)
    codes = precision.e4m3_encode_value(rm)
    assert np.all(codes % 2 == 0)
    assert precision.e4m3_round(np.float32(1000.0)) == 448.0
    assert precision.e4m3_round(np.float32(-1000.0)) == -448.0


def test_bf16_matches_python_bit_rounding():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(5000).astype(np.float32)
    x[:4] = [1.0, -2.5, np.float32(1.00390625), np.float32(1.01171875)]   # exact and tie cases
    got = precision.bf16_round(x)
    for v, g in zip(x.tolist()[:300], got.tolist()[:300]):
        b = int(np.float32(v).view(np.uint32))
        low = b & 0xFFFF
        top = b >> 16
        if low > 0x8000 or (low == 0x8000 and (top & 1)):
            top += 1
        assert np.uint32(top << 16).view(np.float32) == np.float32(g)
    assert got[2] == np.float32(1.0)              # tie, even stays
    assert got[3] == np.float32(1.015625)         # tie, odd rounds up


def test_fp8_rows_scale_and_codes():
    x = np.array([[0.0, 1.0, -2.0, 0.5], [0, 0, 0, 0]], dtype=np.float32)
    codes, scale = precision.fp8_quantize_rows(x)
    assert scale[0] == np.float32(2.0) / np.float32(448.0)
    assert scale[1] == 0 and np.all(codes[1] == 0)
    deq = precision.fp8_dequantize_rows(codes, scale)
    np.testing.assert_allclose(deq[0], [0.0, 1.0, -2.0, 0.5], rtol=2 ** -4)
    assert precision.e4m3_value(codes[0, 2]) == -448.0


def test_full_rerank_reduces_to_ivf(small_data):
    w, X, Q = small_data
    init = synth.init_rows(w.n, w.nlist, w.seed)
    C, a, _ = kmeans.kmeans64(X[:, : w.d_c], w.nlist, 3, init)
    off, ids = kmeans.build_lists(a, w.nlist)
    ref = ivf.ivf_search64(X, Q[:25], C, off, ids, w.d_c, w.d_s, w.nprobe, w.k)
    for fmt in ("bf16", "fp8"):
        got = precision.precision_search64(X, Q[:25], C, off, ids, w.d_c, w.d_s, w.nprobe, w.k,
                                           fmt, rerank=w.n, coarse_margin=w.nlist)
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[1], ref[1])
        np.testing.assert_allclose(got[0], ref[0], rtol=1e-13)


def _two_list_index(C):
    """Two database rows per centroid (lists 0..3), d = 2."""
    X = np.repeat(np.asarray(C, dtype=np.float32), 2, axis=0) + np.float32(0.01)
    a = np.repeat(np.arange(len(C)), 2)
    off, ids = kmeans.build_lists(a, len(C))
    return X, off, ids


def test_coarse_first_pass_reorders_by_hand():
    """Coarse step of the precision form with a small margin: the quantised
    first pass picks the nprobe + coarse_margin best by quantised distance,
    exact FP64 distances order that shortlist. Centroids are built so that
    rounding swaps the two nearest (values worked out by hand; d_c = 1)."""
    q = np.array([[1.0, 0.0]], dtype=np.float32)
    # BF16: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 and rounds to the even
    # 1.0 (quantised distance 0, exact 2^-16); 0.997 rounds to 1 - 2^-8
    # (quantised distance 2^-16, exact 9e-6 < 2^-16)
    cb = [[1.0 + 2.0 ** -8, 1.75], [0.997, 1.75], [3.0, 1.75], [-2.0, 1.75]]
    # e4m3: the 1.75 sets the scale 1/256, so a coordinate a becomes
    # round_e4m3(256 a) / 256; 1.06 -> 256/256 = 1 (exact distance 0.0036),
    # 0.96 -> 240/256 = 0.9375 (exact 0.0016 < 0.0036, quantised 0.0039 > 0)
    cf = [[1.06, 1.75], [0.96, 1.75], [3.0, 1.75], [-2.0, 1.75]]
    for fmt, C in (("bf16", cb), ("fp8", cf)):
        C = np.asarray(C, dtype=np.float32)
        X, off, ids = _two_list_index(C)
        deq = precision.dequantized(C, fmt)[:, 0]
        # the construction does what the comments say
        assert abs(deq[0] - 1.0) < 1e-6 and deq[1] < 0.9999
        assert abs(C[1, 0] - 1.0) < abs(C[0, 0] - 1.0)

        def probes(nprobe, margin):
            return precision.precision_search64(X, q, C, off, ids, 1, 2, nprobe, 1, fmt,
                                                rerank=4, coarse_margin=margin)[2][0].tolist()

        assert probes(1, 0) == [0]        # quantised pass keeps only centroid 0
        assert probes(1, 1) == [1]        # margin 1 lets the exact step pick 1
        assert probes(2, 0) == [1, 0]     # both shortlisted, exact order
        assert probes(3, 0) == [1, 0, 2]
