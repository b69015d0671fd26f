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


def collect(ctx, steps: int, interval: int, learned: bool = False):
    """Runs `steps` steps, recording costs every `interval` steps."""
    nint = steps // interval
    rec = {"heuristic": [], "feat": [], "timer": [], "learned": [], "learned_used": [], "counts": []}
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


def evaluate(rec, boxes, n_ranks: int, predictions=None):
    """Efficiency of each (strategy, policy) per load-balancing step.

    Decision at t_i (i >= 1) governs interval i, judged by timer[i]:
    heuristic and learned use the state at t_i, the timer uses timer[i-1]."""
    out = {s: {p: [] for p in POLICIES} for s in STRATS}
    nint = len(rec["timer"])
    for i in range(1, nint):
        judge = rec["timer"][i]
        costs = {"heuristic": rec["heuristic"][i], "timer": rec["timer"][i - 1]}
        if predictions is not None:
            costs["learned"] = predictions[i]
        elif len(rec["learned"]):
            costs["learned"] = rec["learned"][i]
        for s, c in costs.items():
            for pname, pol in POLICIES.items():
                rank, _ = pb.lb_distribute(np.maximum(c, 0.0), boxes, n_ranks, pol)
                out[s][pname].append(pb.lb_efficiency(judge, rank, n_ranks))
    return {s: {p: np.array(v) for p, v in d.items() if len(v)} for s, d in out.items()}


def summary(E):
    return {s: {p: float(v.mean()) for p, v in d.items()} for s, d in E.items() if d}
