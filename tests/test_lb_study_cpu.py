"""The balancing study's bookkeeping, on hand-made cost records (no GPU).

A mapping decided at interval boundary t_i governs interval i and is judged
by the cycles measured in interval i; the timer strategy can only use the
interval that just ended (i-1), the heuristic and the learned model use the
state at t_i."""
import numpy as np

import picsynth
from paper_2104_11385_amd import lb_study as S
from paper_2104_11385_amd import picbal as pb


def _rec(timer, heur, learned=None):
    nint = len(timer)
    rec = {"timer": np.array(timer, dtype=float), "heuristic": np.array(heur, dtype=float),
           "feat": np.zeros((nint + 1, len(timer[0]), 16), np.float32),
           "counts": np.zeros((nint + 1, len(timer[0]))), "learned": np.array(learned if learned else []),
           "learned_used": np.array([])}
    return rec


def test_timer_strategy_lags_one_interval():
    boxes = picsynth.uniform_boxes((64, 16, 16), 16)      # 4 boxes in a row
    # the load moves from box 0 to box 3 between intervals
    timer = [[8, 1, 1, 1], [1, 1, 1, 8], [1, 1, 1, 8]]
    heur = [[8, 1, 1, 1], [1, 1, 1, 8], [1, 1, 1, 8], [1, 1, 1, 8]]
    E = S.evaluate(_rec(timer, heur), boxes, 2)
    # decisions at t_1, t_2 (two rebalances)
    assert len(E["timer"]["knapsack"]) == 2
    # heuristic sees the new state at t_1: {8} | {1,1,1} -> E = 5.5/8
    np.testing.assert_allclose(E["heuristic"]["knapsack"], [5.5 / 8, 5.5 / 8])
    # timer at t_1 uses interval 0 (load on box 0): box 0 alone, boxes 1..3 together;
    # judged on interval 1 -> loads {1} | {1+1+8}
    rank, _ = pb.lb_distribute(np.array([8.0, 1, 1, 1]), boxes, 2, pb.LB_KNAPSACK)
    want = pb.lb_efficiency(np.array([1.0, 1, 1, 8]), rank, 2)
    assert E["timer"]["knapsack"][0] == want
    assert E["timer"]["knapsack"][1] == 5.5 / 8


def test_training_pairs_state_with_following_interval():
    rec = _rec([[3, 0], [5, 7]], [[0, 0]] * 3)
    rec["feat"][:, :, 0] = np.array([[10, 11], [20, 21], [30, 31]])
    X, y = S.training_set([rec])
    np.testing.assert_array_equal(X[:, 0], [10, 11, 20, 21])
    np.testing.assert_allclose(y, np.log1p([3, 0, 5, 7]), rtol=1e-6)


def test_identical_costs_give_identical_efficiency():
    boxes = picsynth.uniform_boxes((64, 64, 16), 16)
    rng = np.random.default_rng(1)
    timer = rng.uniform(1, 5, (4, len(boxes)))
    heur = np.vstack([timer[:1], timer])            # heuristic at t_i equals timer[i-1]
    E = S.evaluate(_rec(timer, heur), boxes, 3)
    for p in ("sfc", "knapsack"):
        np.testing.assert_array_equal(E["heuristic"][p], E["timer"][p])
        assert ((E["timer"][p] > 0) & (E["timer"][p] <= 1)).all()


def test_replay_modes():
    boxes = picsynth.uniform_boxes((64, 16, 16), 16)
    # load sits on box 0, then moves to box 3 and stays
    timer = [[9, 1, 1, 1], [9, 1, 1, 1], [1, 1, 1, 9], [1, 1, 1, 9], [1, 1, 1, 9]]
    rec = _rec(timer, [[0] * 4] * 6)
    # initial SFC of equal costs on 2 ranks: {0,1} | {2,3}
    En, an = S.replay(rec, boxes, 2, pb.LB_KNAPSACK, mode="none")
    np.testing.assert_allclose(En, [6 / 10] * 5)
    assert an == 0
    Es, as_ = S.replay(rec, boxes, 2, pb.LB_KNAPSACK, mode="static")
    assert as_ == 1
    # static adopts {0} | {1,2,3} from interval 0 at t_1 and keeps it
    np.testing.assert_allclose(Es, [6 / 10, 6 / 9, 6 / 11, 6 / 11, 6 / 11])
    Ed, ad = S.replay(rec, boxes, 2, pb.LB_KNAPSACK, mode="dynamic")
    # dynamic follows the move one interval late (timer costs)
    np.testing.assert_allclose(Ed, [6 / 10, 6 / 9, 6 / 11, 6 / 9, 6 / 9])
    assert ad == 2
    # a 100% threshold never adopts
    Ek, ak = S.replay(rec, boxes, 2, pb.LB_KNAPSACK, mode="dynamic", threshold=1.0)
    assert ak == 0 and np.allclose(Ek, En)


def test_replay_sums_timer_since_last_balance():
    boxes = picsynth.uniform_boxes((64, 16, 16), 16)
    # per-step cycles: box 0 is heavy on even steps, box 3 on odd steps; the
    # two-step sums are uniform, so every-2 balancing sees no imbalance
    timer = [[5, 1, 1, 1], [1, 1, 1, 5]] * 3
    rec = _rec(timer, [[0] * 4] * 7)
    E2, a2 = S.replay(rec, boxes, 2, pb.LB_KNAPSACK, mode="dynamic", every=2, threshold=0.01)
    assert a2 == 0
    # every-1 balancing chases last step's heavy box and always lands wrong
    E1, a1 = S.replay(rec, boxes, 2, pb.LB_KNAPSACK, mode="dynamic", every=1, threshold=0.01)
    assert a1 >= 1
    assert E1[1:].mean() < E2[1:].mean()


def test_sweep_keys_and_bounds():
    boxes = picsynth.uniform_boxes((64, 64, 16), 16)
    rng = np.random.default_rng(2)
    ts = rng.uniform(1, 3, (12, len(boxes)))
    out = S.sweep(ts, boxes, 3, intervals=(1, 3, 30), thresholds=(0.05, 0.15))
    assert set(out) == {"sfc/none", "knapsack/none", "sfc/every1/thr5", "sfc/every1/thr15", "sfc/every3/thr5",
                        "sfc/every3/thr15", "knapsack/every1/thr5", "knapsack/every1/thr15",
                        "knapsack/every3/thr5", "knapsack/every3/thr15"}
    for k, v in out.items():
        e = v if isinstance(v, float) else v["E_mean"]
        assert 0 < e <= 1


def test_heuristic_from_counts_and_extra_strategy():
    boxes = picsynth.uniform_boxes((64, 16, 16), 16)
    timer = [[8, 1, 1, 1], [1, 1, 1, 8]]
    rec = _rec(timer, [[0] * 4] * 3)
    rec["counts"] = np.array([[10, 0, 0, 0], [0, 0, 0, 10], [0, 0, 0, 10]], dtype=float)
    h = S.heuristic_from_counts(rec, boxes, 0.5, 0.001)
    np.testing.assert_allclose(h[0], [5 + 4.096, 4.096, 4.096, 4.096])
    E = S.evaluate(rec, boxes, 2, extra={"mine": h})
    assert {k for k, v in E.items() if v} == {"heuristic", "timer", "mine"}
    # the extra strategy sees the load on box 3 at t_1: {3} | {0,1,2}
    np.testing.assert_allclose(E["mine"]["knapsack"], [5.5 / 8])
