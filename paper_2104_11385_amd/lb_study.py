"""Dynamic load-balancing study on virtual ranks (Sec. 2.2 and Sec. 3.3).

One simulation run on one GPU supplies every cost strategy's per-box costs
at each load-balancing step, because a mapping onto virtual ranks does not
change how the single GPU executes the boxes:

* at every interval boundary t_i the study records the heuristic costs and
  the box features (state at t_i) and, if a model is loaded, the learned
  costs (with the library's 15% fallback rule);
* over the following interval it records the device-timer cycles.

A mapping chosen at t_i from a strategy's costs is then judged by the
efficiency E = c_avg / c_max (Eq. 1) of the cycles actually measured during
the interval it would govern.  The timer strategy at t_i can only use the
interval that just ended, as in the paper's loop.

The learned model predicts ln(1 + cycles) from the 16 box features; boxes
whose features show no particles are predicted as the model says (the
network learns that empty boxes cost nothing).
"""
from __future__ import annotations

import numpy as np

from . import picbal as pb

STRATS = ("heuristic", "timer", "learned")
POLICIES = {"sfc": pb.LB_SFC, "knapsack": pb.LB_KNAPSACK}


def collect(ctx, steps: int, interval: int, learned: bool = False, per_step: bool = False):
    """Runs `steps` steps, recording costs every `interval` steps.  With
    `per_step` the device-timer cycles are also read after every step
    (`timer_step`, one row per step; the interval rows are their sums)."""
    nint = steps // interval
    rec = {"heuristic": [], "feat": [], "timer": [], "learned": [], "learned_used": [], "counts": [],
           "timer_step": []}
    ctx.reset_costs()
    for i in range(nint + 1):
        h, _ = ctx.box_costs(pb.PIC_COST_HEURISTIC)
        rec["heuristic"].append(h)
        rec["feat"].append(ctx.box_features())
        rec["counts"].append(ctx.box_counts().sum(axis=1))
        if learned:
            c, used = ctx.box_costs(pb.PIC_COST_LEARNED)
            rec["learned"].append(c)
            rec["learned_used"].append(used)
        if i == nint:
            break
        ctx.reset_costs()
        if per_step:
            # the counters keep running over the interval, so the library's
            # last timer reading (which its learned-cost fallback compares
            # with) is still the whole interval's; steps are differences
            prev = 0.0
            for _ in range(interval):
                ctx.step(1)
                t, _ = ctx.box_costs(pb.PIC_COST_DEVICE_TIMER)
                rec["timer_step"].append(t - prev)
                prev = t
            rec["timer"].append(prev)
            continue
        ctx.step(interval)
        t, _ = ctx.box_costs(pb.PIC_COST_DEVICE_TIMER)
        rec["timer"].append(t)
    return {k: np.array(v) for k, v in rec.items()}


def training_set(recs):
    """(features at t_i, ln(1 + cycles measured over interval i)) pairs."""
    X, y = [], []
    for r in recs:
        for i in range(len(r["timer"])):
            X.append(r["feat"][i])
            y.append(np.log1p(r["timer"][i]))
    return np.concatenate(X).astype(np.float32), np.concatenate(y).astype(np.float32)


def heuristic_from_counts(rec, boxes, w_particle: float, w_cell: float):
    """Heuristic costs w_p * N + w_c * cells at every t_i from the recorded
    particle counts (for weights other than the run's own)."""
    b = np.asarray(boxes, dtype=np.int64)
    cells = ((b[:, 3] - b[:, 0]) * (b[:, 4] - b[:, 1]) * (b[:, 5] - b[:, 2])).astype(float)
    return w_particle * np.asarray(rec["counts"], dtype=float) + w_cell * cells[None, :]


def evaluate(rec, boxes, n_ranks: int, predictions=None, extra=None):
    """Efficiency of each (strategy, policy) per load-balancing step.

    Decision at t_i (i >= 1) governs interval i, judged by timer[i]:
    heuristic and learned use the state at t_i, the timer uses timer[i-1].
    `extra` maps further strategy names to costs at every t_i."""
    extra = extra or {}
    out = {s: {p: [] for p in POLICIES} for s in (*STRATS, *extra)}
    nint = len(rec["timer"])
    for i in range(1, nint):
        judge = rec["timer"][i]
        costs = {"heuristic": rec["heuristic"][i], "timer": rec["timer"][i - 1]}
        if predictions is not None:
            costs["learned"] = predictions[i]
        elif len(rec["learned"]):
            costs["learned"] = rec["learned"][i]
        for name, c in extra.items():
            costs[name] = c[i]
        for s, c in costs.items():
            for pname, pol in POLICIES.items():
                rank, _ = pb.lb_distribute(np.maximum(c, 0.0), boxes, n_ranks, pol)
                out[s][pname].append(pb.lb_efficiency(judge, rank, n_ranks))
    return {s: {p: np.array(v) for p, v in d.items() if len(v)} for s, d in out.items()}


def comm_per_policy(rec, boxes, n_cells, n_ranks: int, strategy="timer", bytes_per_face_cell=1.0):
    """Mean over rebalances of the total and the largest per-rank halo traffic
    of each policy's mappings (the communication SFC is meant to save)."""
    out = {}
    for pname, pol in POLICIES.items():
        tots, mx = [], []
        for i in range(1, len(rec["timer"])):
            c = rec["timer"][i - 1] if strategy == "timer" else rec[strategy][i]
            rank, _ = pb.lb_distribute(np.maximum(c, 0.0), boxes, n_ranks, pol)
            per, tot = pb.lb_comm_volume(boxes, n_cells, rank, n_ranks, bytes_per_face_cell)
            tots.append(tot)
            mx.append(per.max())
        out[pname] = {"total": float(np.mean(tots)), "max_rank": float(np.mean(mx))}
    return out


def replay(rec, boxes, n_ranks: int, policy: int, strategy="timer", mode="dynamic", every=1, threshold=0.10):
    """The balancing loop replayed on recorded costs (Sec. 2.2 and Sec. 3.2).

    The initial mapping is the space-filling curve with equal box costs (no
    load information).  mode "none" keeps it; "static" adopts the strategy's
    mapping once, at the first balancing step; "dynamic" proposes a mapping
    every `every` intervals and adopts it when its efficiency, estimated
    from the same costs, improves on the current mapping's by the relative
    threshold.  Returns (E of each interval under the mapping in force, the
    number of adoptions)."""
    nint = len(rec["timer"])
    nb = len(boxes)
    mapping, _ = pb.lb_distribute(np.ones(nb), boxes, n_ranks, pb.LB_SFC)
    E, adopted = [], 0
    for i in range(nint):
        if i >= 1 and mode != "none" and (mode == "dynamic" and i % every == 0 or mode == "static" and i == 1):
            if strategy == "timer":
                c = np.sum(rec["timer"][max(0, i - every) if mode == "dynamic" else 0:i], axis=0)
            else:
                c = rec[strategy][i]
            c = np.maximum(c, 0.0)
            proposed, e_new = pb.lb_distribute(c, boxes, n_ranks, policy)
            e_cur = pb.lb_efficiency(c, mapping, n_ranks)
            if mode == "static" or pb.lb_should_adopt(e_cur, e_new, threshold):
                mapping = proposed
                adopted += 1
        E.append(pb.lb_efficiency(rec["timer"][i], mapping, n_ranks))
    return np.array(E), adopted


def sweep(timer_step, boxes, n_ranks: int, intervals=(1, 3, 10, 30, 100, 300), thresholds=(0.05, 0.10, 0.15)):
    """Mean step efficiency of dynamic balancing on per-step timer records,
    for each policy, balancing interval (steps) and adoption threshold, next
    to no balancing (Sec. 3.3's parameter study, on virtual ranks)."""
    rec = {"timer": np.asarray(timer_step, dtype=float)}
    T = len(rec["timer"])
    out = {}
    for pname, pol in POLICIES.items():
        out[f"{pname}/none"] = float(replay(rec, boxes, n_ranks, pol, mode="none")[0].mean())
        for k in intervals:
            if k >= T:
                continue
            for thr in thresholds:
                E, a = replay(rec, boxes, n_ranks, pol, mode="dynamic", every=k, threshold=thr)
                out[f"{pname}/every{k}/thr{int(round(thr * 100))}"] = {"E_mean": float(E.mean()), "adoptions": a}
    return out


def summary(E):
    return {s: {p: float(v.mean()) for p, v in d.items()} for s, d in E.items() if d}
