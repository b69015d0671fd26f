"""Calibration of the heuristic cost's particle and cell weights (Sec. 3.3).

The paper derives the weights from two benchmark runs on the target machine:
one with many particles per cell (27) spread uniformly over the domain, and
one with no particles at all.  The run without particles prices a cell, the
difference between the two prices the particles:

    t_cell     = T_empty / N_cells
    t_particle = (T_full - T_empty) / N_particles

and the weights are those per-unit times normalised to sum to one, so that
w_p * N + w_c * C ranks boxes as t_particle * N + t_cell * C does.
"""
from __future__ import annotations

import time

import numpy as np

from . import picbal as pb


def heuristic_weights(t_full: float, t_empty: float, n_particles: int, n_cells: int):
    """(w_particle, w_cell, t_particle, t_cell) from the two runs' step times."""
    if n_particles <= 0 or n_cells <= 0:
        raise ValueError("both runs need a positive particle and cell count")
    if not (t_full > t_empty > 0.0):
        raise ValueError("the run with particles must take longer than the run without")
    t_cell = t_empty / n_cells
    t_particle = (t_full - t_empty) / n_particles
    s = t_particle + t_cell
    return t_particle / s, t_cell / s, t_particle, t_cell


def _time_steps(ctx, steps: int, warmup: int) -> float:
    ctx.step(warmup)
    ctx.sync()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    return (time.perf_counter() - t0) / steps


def run(n=(256, 256, 256), box_edge=64, ppc=27, order=2, precision=4, u_th=0.01, dt=0.5,
        steps=20, warmup=5, seed=11):
    """Times the two calibration runs on the GPU and returns the weights.

    Full run: electrons at `ppc` per cell over the whole periodic domain with
    thermal momenta `u_th` (the paper's electron spread), sorted and stepped
    with the persistent kernel and graph replay; empty run: the same grid and
    boxes with no particles.  Step times are wall-clock seconds per step."""
    n = tuple(int(v) for v in n)
    boxes = []
    for bz in range(n[2] // box_edge):
        for by in range(n[1] // box_edge):
            for bx in range(n[0] // box_edge):
                lo = (bx * box_edge, by * box_edge, bz * box_edge)
                boxes.append([*lo, *(v + box_edge for v in lo)])
    boxes = np.array(boxes, dtype=np.int32)
    n_cells = int(np.prod(n))
    out = {}
    for name, sp in (("full", pb.Species(-1.0, 1.0, 0.274 ** 2, load_mode=1, ppc=ppc, region_hi=n,
                                         u_th=(u_th,) * 3)),
                     ("empty", pb.Species(-1.0, 1.0, 0.274 ** 2, load_mode=0))):
        ctx = pb.pic_init(n, boxes, [sp], dt, order, precision, seed)
        try:
            ctx.set_launch_mode(pb.PIC_LAUNCH_PERSISTENT, True)
            out[name] = _time_steps(ctx, steps, warmup)
        finally:
            ctx.finalize()
    n_p = n_cells * ppc
    wp, wc, tp, tc = heuristic_weights(out["full"], out["empty"], n_p, n_cells)
    return {"w_particle": wp, "w_cell": wc, "ns_per_particle": tp * 1e9, "ns_per_cell": tc * 1e9,
            "ms_step_full": out["full"] * 1e3, "ms_step_empty": out["empty"] * 1e3,
            "particles": n_p, "cells": n_cells, "boxes": int(len(boxes)), "order": order,
            "precision": precision, "ppc": ppc}
