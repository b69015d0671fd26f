"""Pins of the oracle's load-balancing arithmetic (Sec. 2.2, Eq. 1).

The efficiency and threshold are checked on the paper's Fig. 1 example; the
space-filling-curve partition against brute force over every cut set; the
knapsack mapping against hand-derived tie-break results, Graham's LPT bound
and brute-force optima; box counts against a direct floor-and-compare.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import picsynth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fig1():
    with open(os.path.join(GOLD, "fig1_domain.json")) as f:
        return json.load(f)


def test_fig1_efficiency_and_heuristic():
    g = _fig1()
    parts = np.array(g["particles"], dtype=float)
    rank = np.array(g["fig1b_rank_of_box"])
    assert oracle.efficiency(parts, rank, 2) == g["derived"]["E_particles_only_fig1b"]
    # 2D boxes of 2x2 cells -> treat as 2x2x1 boxes
    boxes = np.array([[0, 2, 0, 2, 4, 1], [2, 2, 0, 4, 4, 1], [0, 0, 0, 2, 2, 1], [2, 0, 0, 4, 2, 1]])
    counts = np.array(g["particles"], dtype=np.int64)[:, None]
    w = g["heuristic_weights_sec3_3_footnote"]
    costs = oracle.heuristic(boxes, counts, w["particle"], w["cell"])
    np.testing.assert_array_equal(costs, g["derived"]["heuristic_costs"])
    assert abs(oracle.efficiency(costs, rank, 2) - g["derived"]["E_heuristic_fig1b"]) < 1e-15
    best = oracle.knapsack(costs, 2)
    assert abs(oracle.efficiency(costs, best, 2) - g["derived"]["E_heuristic_optimal_two_ranks"]) < 1e-15


def test_efficiency_edge_cases():
    # all-zero costs -> 1; empty ranks count in the average
    assert oracle.efficiency(np.zeros(3), [0, 1, 2], 3) == 1.0
    assert oracle.efficiency(np.array([1.0, 1.0]), [0, 0], 4) == 0.25
    e = oracle.efficiency(np.random.default_rng(1).uniform(0, 1, 40), np.arange(40) % 7, 7)
    assert 0.0 <= e <= 1.0


def test_threshold_met_or_exceeded():
    assert oracle.should_adopt(0.5, 0.55, 0.10)       # exactly 10% better: met
    assert oracle.should_adopt(0.5, 0.56, 0.10)
    assert not oracle.should_adopt(0.5, 0.54, 0.10)
    assert not oracle.should_adopt(0.91, 1.0, 0.10)   # 9.9% (the paper's rounded example)
    assert oracle.should_adopt(0.90, 1.0, 0.10)


def test_morton_keys_by_hand():
    assert oracle.morton3(0, 0, 0) == 0
    assert oracle.morton3(1, 0, 0) == 1
    assert oracle.morton3(0, 1, 0) == 2
    assert oracle.morton3(0, 0, 1) == 4
    assert oracle.morton3(1, 1, 1) == 7
    assert oracle.morton3(2, 0, 0) == 8
    # (3,5,6): x=011 y=101 z=110 -> bits (z y x) per level: l0: 0 1 1, l1: 1 0 1, l2: 1 1 0
    assert oracle.morton3(3, 5, 6) == (0b011) | (0b101 << 3) | (0b110 << 6)


def test_sfc_c1_split():
    wl = picsynth.config("c1")
    rank, B = oracle.sfc(wl.boxes, np.ones(8), 4)
    np.testing.assert_array_equal(rank, [0, 0, 1, 1, 2, 2, 3, 3])
    assert B == 2.0


def _morton_order(boxes):
    g = 0
    for b in boxes:
        for d in range(3):
            g = math.gcd(g, int(b[3 + d] - b[d]))
    keys = [oracle.morton3(b[0] // g, b[1] // g, b[2] // g) for b in boxes]
    return np.argsort(keys, kind="stable")


def _brute_bstar(c, R):
    nb = len(c)
    best = math.inf
    for k in range(1, min(R, nb) + 1):
        for cuts in itertools.combinations(range(1, nb), k - 1):
            edges = (0,) + cuts + (nb,)
            m = 0.0
            for a, b in zip(edges[:-1], edges[1:]):
                acc = 0.0
                for v in c[a:b]:
                    acc += v
                m = max(m, acc)
            best = min(best, m)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_sfc_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = (64, 32, 32)
    boxes = picsynth.uniform_boxes(n, 16)[: rng.integers(5, 13)]
    rng.shuffle(boxes)
    nb = len(boxes)
    R = int(rng.integers(2, 5))
    costs = rng.uniform(0, 10, nb)
    if seed % 3 == 0:
        costs = np.round(costs)          # ties
    rank, B = oracle.sfc(boxes, costs, R)
    order = _morton_order(boxes)
    c_ord = costs[order]
    assert B == _brute_bstar(list(c_ord), R)
    r_ord = rank[order]
    assert np.all(np.diff(r_ord) >= 0)               # contiguous along the curve
    assert set(r_ord) == set(range(R))               # every rank used (nb >= R)
    for r in range(R):
        acc = 0.0
        for v in c_ord[r_ord == r]:
            acc += v
        assert acc <= B


def test_sfc_fewer_boxes_than_ranks():
    boxes = picsynth.uniform_boxes((32, 16, 16), 16)
    rank, _ = oracle.sfc(boxes, np.array([3.0, 1.0]), 5)
    np.testing.assert_array_equal(rank, [0, 1])


def test_knapsack_tie_breaks_and_cap():
    # equal costs: each box goes to the least-loaded, lowest-index rank -> round robin
    rank = oracle.knapsack(np.ones(12), 4)
    np.testing.assert_array_equal(rank, np.arange(12) % 4)
    # one heavy box on rank 0; the light ones go round-robin over ranks 1..3
    rank = oracle.knapsack(np.array([100.0] + [1.0] * 9), 4)
    np.testing.assert_array_equal(rank, [0, 1, 2, 3, 1, 2, 3, 1, 2, 3])
    # 9 boxes on 2 ranks: cap = ceil(1.5 * 9 / 2) = 7.  Rank 1 takes seven light
    # boxes (load 7 < 100), then the cap, not the load, sends the last to rank 0.
    rank = oracle.knapsack(np.array([100.0] + [1.0] * 8), 2)
    np.testing.assert_array_equal(rank, [0, 1, 1, 1, 1, 1, 1, 1, 0])


@pytest.mark.parametrize("seed", range(10))
def test_knapsack_lpt_bound_and_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    nb = int(rng.integers(4, 9))
    R = int(rng.integers(2, 4))
    costs = rng.uniform(1, 10, nb)
    rank = oracle.knapsack(costs, R)
    loads = np.bincount(rank, weights=costs, minlength=R)
    opt = min(max(np.bincount(np.array(a), weights=costs, minlength=R))
              for a in itertools.product(range(R), repeat=nb))
    cap = (3 * nb + 2 * R - 1) // (2 * R)
    assert np.bincount(rank, minlength=R).max() <= cap
    if np.bincount(rank, minlength=R).max() < cap:
        assert loads.max() <= (4.0 / 3.0 - 1.0 / (3 * R)) * opt + 1e-12
    # the best contiguous (SFC) efficiency cannot beat the best unconstrained one
    boxes = picsynth.uniform_boxes((128, 16, 16), 16)[:nb]
    srank, B = oracle.sfc(boxes, costs, R)
    e_sfc_opt = (costs.sum() / R) / B
    e_any_opt = (costs.sum() / R) / opt
    assert e_sfc_opt <= e_any_opt + 1e-15


def test_box_counts_and_face_tie():
    wl = picsynth.config("c1")
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 32, (5000, 3))
    x[0] = [16.0, 0.0, 0.0]          # exactly on a face: belongs to the upper box
    sp = np.zeros(len(x), np.int32)
    counts = oracle.box_counts(wl.boxes, x, sp, 1)
    assert counts.sum() == len(x)
    c = np.floor(x).astype(int)
    b = (c[:, 0] // 16) + 2 * (c[:, 1] // 16) + 4 * (c[:, 2] // 16)
    np.testing.assert_array_equal(counts[:, 0], np.bincount(b, minlength=8))
    one = oracle.box_counts(wl.boxes, x[:1], sp[:1], 1)
    assert one[1, 0] == 1


def test_heuristic_no_fma_order():
    # cost = fl(fl(wp*N) + fl(wc*cells)); with values whose fused form differs
    boxes = np.array([[0, 0, 0, 3, 1, 1]])
    counts = np.array([[123456789]], dtype=np.int64)
    c = oracle.heuristic(boxes, counts, 0.1, 0.7)
    a = np.float64(0.1) * np.float64(123456789)
    b = np.float64(0.7) * np.float64(3)
    assert c[0] == a + b


def test_comm_volume_by_hand():
    # two 16^3 boxes side by side in a periodic 32x16x16 domain on two ranks:
    # they share the x = 16 plane and, through the periodic wrap, x = 0:
    # 2 x 256 faces, each counted for both ranks
    boxes = picsynth.uniform_boxes((32, 16, 16), 16)
    per = oracle.comm_volume((32, 16, 16), boxes, [0, 1], 2)
    np.testing.assert_array_equal(per, [512.0, 512.0])
    assert oracle.comm_volume((32, 16, 16), boxes, [0, 0], 2).sum() == 0.0
    # c1's eight boxes: rank of box b = b: every box has 6 neighbouring faces
    # of 16^2 cells (two per axis, one of them through the wrap)
    wl = picsynth.config("c1")
    per = oracle.comm_volume(wl.n, wl.boxes, np.arange(8), 8, 2.0)
    np.testing.assert_array_equal(per, np.full(8, 6 * 256 * 2.0))
