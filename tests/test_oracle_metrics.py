"""Pins for oracle.metrics and oracle.check."""
import json
import math
import os

import numpy as np

from oracle import check, metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_k_recall_hand_built():
    true = np.array([[1, 2, 3], [4, 5, 6]])
    got = np.array([[3, 9, 1], [-1, 6, 7]])
    assert metrics.k_recall_at_n(got, true, 3) == (2 + 1) / 6


def test_cost_model_optimum_is_sqrt_n():
    # Section 5.3: nlist = sqrt(N) is FLOP-optimal (d_c = d_s); Appendix B.1 defaults
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["cost_model_defaults"]
    n = g["N"]
    d = 64
    grid = np.arange(64, 8192)
    cost = [metrics.cost_macs(d, d, int(L), g["nprobe"], n) for L in grid]
    best = grid[int(np.argmin(cost))]
    assert abs(best - math.sqrt(n)) <= 1
    # the general optimum moves to sqrt(nprobe * d_s * N / d_c)
    cost2 = [metrics.cost_macs(16, 256, int(L), 1, n) for L in grid]
    assert abs(grid[int(np.argmin(cost2))] - math.sqrt(1 * 256 * n / 16)) <= 1
    # the default setting's scan term dominates the coarse term when d_c << d_s
    assert 2048 * n / 1024 > 100 * 16 * 1024


def test_relative_contrast_hand_built():
    X = np.array([[0.0], [1.0], [3.0]])
    Q = np.array([[0.0], [3.0]])
    # q=0: D=[0,1,3] mean 4/3 min 0; q=3: D=[3,2,0] mean 5/3 min 0 -> use shifted queries
    Q = np.array([[0.5], [2.0]])
    dmean = np.mean([(0.5 + 0.5 + 2.5) / 3, (2 + 1 + 1) / 3])
    dmin = np.mean([0.5, 1.0])
    assert abs(metrics.relative_contrast(X, Q) - dmean / dmin) < 1e-12


def test_centroid_recall_full_width_is_one():
    rng = np.random.default_rng(0)
    C = rng.standard_normal((50, 8))
    Q = rng.standard_normal((10, 8))
    assert metrics.centroid_recall(Q, C, 8, 1, 1) == 1.0
    assert metrics.centroid_recall(Q, C, 2, 1, 50) == 1.0


def test_checker_accepts_ties_rejects_mistakes():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [2.0, 2.0], [3.0, 0.0]])
    q = np.array([0.0, 0.0])
    cand = [0, 1, 2, 3, 4]
    ref_i = np.array([0, 1, 2])
    ref_d = np.array([0.0, 1.0, 1.0])
    # ids 1 and 2 tie: swapped order is fine
    r = check.compare_knn(q, X, cand, [0.0, 1.0, 1.0], [0, 2, 1], ref_d, ref_i, 2)
    assert r.ok and r.id_mismatch_ties == 2
    # a wrong neighbour is caught
    r = check.compare_knn(q, X, cand, [0.0, 1.0, 8.0], [0, 1, 3], ref_d, ref_i, 2)
    assert not r.ok
    # a distance off by more than the tolerance is caught
    r = check.compare_knn(q, X, cand, [0.0, 1.0, 1.001], [0, 1, 2], ref_d, ref_i, 2)
    assert not r.ok
    # an id outside the scanned candidates is caught
    r = check.compare_knn(q, X, [0, 1, 3], [0.0, 1.0, 1.0], [0, 1, 2], ref_d, ref_i, 2)
    assert not r.ok
    # padding must match
    r = check.compare_knn(q, X, cand, [0.0, 1.0, np.inf], [0, 1, -1], ref_d, ref_i, 2)
    assert not r.ok


def test_probe_validity_band():
    c = np.array([1.0, 2.0, 2.0 * (1 + 1e-7), 3.0])
    assert check.probes_valid(c, [0, 1], 2)
    assert check.probes_valid(c, [0, 2], 2)        # inside the tie band
    assert not check.probes_valid(c, [0, 3], 2)
    assert not check.probes_valid(c, [1, 2], 2)    # left out a strictly nearer one


def test_centroid_recall_hand_built():
    """k-Recall@N of centroids ranked on a one-coordinate prefix against the
    full width (Appendix E.2), distances worked out by hand."""
    C = np.array([[0.1, 5.0], [1.0, 0.0], [2.0, 0.0], [-3.0, 0.0]])
    # q = (0, 0): full 25.01, 1, 4, 9 -> order 1, 2, 3, 0; prefix 0.01, 1, 4, 9 -> 0, 1, 2, 3
    q0 = np.array([[0.0, 0.0]])
    assert metrics.centroid_recall(q0, C, 1, 1, 1) == 0.0
    assert metrics.centroid_recall(q0, C, 1, 1, 2) == 1.0
    assert metrics.centroid_recall(q0, C, 1, 2, 2) == 0.5
    assert metrics.centroid_recall(q0, C, 1, 2, 3) == 1.0
    # q = (3, 0): full 33.41, 4, 1, 36 -> 2, 1, 0, 3; prefix 8.41, 4, 1, 36 -> 2, 1, 0, 3
    Q = np.array([[0.0, 0.0], [3.0, 0.0]])
    assert metrics.centroid_recall(Q, C, 1, 2, 2) == (1 + 2) / 4
    assert metrics.centroid_recall(Q, C, 2, 2, 2) == 1.0
