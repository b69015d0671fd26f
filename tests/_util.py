"""Shared test helpers: build a library context or an oracle run from a
seeded workload, and compare states with explicit tolerances."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import picsynth  # noqa: E402


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def species_for_library(wl, load=True):
    from paper_2104_11385_amd import picbal as pb
    out = []
    for s in wl.species:
        if s.box_ppc is not None:
            mode, ppc = 2, 0
        else:
            mode, ppc = 1, s.ppc
        out.append(pb.Species(s.charge, s.mass, s.density, load_mode=mode if load else 0, ppc=ppc,
                              box_ppc=s.box_ppc, region_lo=s.region_lo,
                              region_hi=s.region_hi if s.region_hi is not None else wl.n,
                              u_th=s.u_th, u_drift=s.u_drift,
                              capacity=picsynth.species_count(wl, wl.species.index(s))))
    return out


def make_ctx(wl, precision=None, load=True, stream=None):
    from paper_2104_11385_amd import picbal as pb
    prec = wl.precision if precision is None else precision
    return pb.pic_init(wl.n, wl.boxes, species_for_library(wl, load), wl.dt, wl.order, prec, wl.seed,
                       b_ext=wl.b_ext, stream=stream)


def set_state(ctx, wl, F=None):
    """Loads picsynth's host particles (and fields F, default initial) into ctx.
    Returns the host copies (x, u, w, ids, sp, F) for the oracle."""
    x, u, w, ids, sp = picsynth.all_particles(wl)
    for s in range(len(wl.species)):
        m = sp == s
        ctx.set_particles(s, x[m], u[m], w[m], ids[m])
    if F is None:
        F = picsynth.initial_fields(wl)
    ctx.set_fields(F)
    return x.copy(), u.copy(), w.copy(), ids.copy(), sp.copy(), F.copy()


def oracle_steps(wl, x, u, w, sp, F, nsteps):
    import oracle
    q = np.array([s.charge for s in wl.species])
    m = np.array([s.mass for s in wl.species])
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    F = np.ascontiguousarray(F, dtype=np.float64).copy()
    oracle.pic_step(wl.order, np.array(wl.n), wl.dt, x, u, w, sp, q, m, F, nsteps)
    return x, u, F


def gpu_particles(ctx, wl):
    """All species' particles from the library, ordered by (species, id)."""
    xs, us, ids, sps = [], [], [], []
    for s in range(len(wl.species)):
        x, u, w, i = ctx.get_particles(s)
        o = np.argsort(i, kind="stable")
        xs.append(x[o]); us.append(u[o]); ids.append(i[o]); sps.append(np.full(len(i), s, np.int32))
    return np.concatenate(xs), np.concatenate(us), np.concatenate(ids), np.concatenate(sps)


def order_by_species_id(x, u, ids, sp):
    o = np.lexsort((ids, sp))
    return x[o], u[o], ids[o], sp[o]


def min_image(d, n):
    n = np.asarray(n, dtype=np.float64)[None, :]
    return d - n * np.round(d / n)


def normwise(a, b):
    """max |a - b| / max |b| (0 if both vanish)."""
    den = np.abs(b).max()
    num = np.abs(a - b).max()
    return 0.0 if den == 0 and num == 0 else num / max(den, 1e-300)


def u_floor(wl, e_max, nsteps):
    """Per species: |q| dt nsteps max|E| / m, the momentum the strongest
    electric field of the run can give a particle of that species over the
    run.  A particle near rest has a momentum made of such impulses, each
    carrying the rounding of the field it came from, so its momentum error
    is measured against this scale rather than against its own |u|."""
    return np.array([abs(s.charge) * wl.dt * nsteps * e_max / s.mass for s in wl.species])


def check_u_per_particle(gu, ou, sp, ids, floors, tol, what=""):
    """|u_gpu - u_oracle| <= tol * max(|u_oracle|, floor of its species), for
    every particle (vector norms); names the worst particle on failure."""
    du = np.linalg.norm(np.asarray(gu) - np.asarray(ou), axis=1)
    uu = np.linalg.norm(np.asarray(ou), axis=1)
    ref = np.maximum(uu, np.maximum(np.asarray(floors)[np.asarray(sp)], 1e-300))
    rel = du / ref
    k = int(np.argmax(rel)) if len(rel) else 0
    assert len(rel) == 0 or rel[k] <= tol, (
        f"{what}particle id {int(ids[k])} of species {int(sp[k])}: |du| = {du[k]:.3e}, |u| = {uu[k]:.3e}, "
        f"floor {np.asarray(floors)[int(sp[k])]:.3e}: {rel[k]:.3e} > {tol:g}; "
        f"{int((rel > tol).sum())} particles over the bar")
    return float(rel.max()) if len(rel) else 0.0


def box_face_planes(boxes, n):
    """Per dimension, the sorted coordinates of every box face (0 and n
    included)."""
    b = np.asarray(boxes)
    return [np.unique(np.concatenate([b[:, d], b[:, 3 + d], [0, n[d]]])) for d in range(3)]


def near_box_face(x, boxes, n, eps):
    """Particles within eps of a box face plane in some dimension."""
    near = np.zeros(len(x), bool)
    for d, planes in enumerate(box_face_planes(boxes, n)):
        dist = np.abs(x[:, d][:, None] - planes[None, :]).min(axis=1)
        near |= dist < eps
    return near


def box_of(x, boxes):
    """Index of the box holding each position's cell floor(x)."""
    c = np.floor(x).astype(np.int64)
    b = np.asarray(boxes, dtype=np.int64)
    out = np.full(len(x), -1, np.int64)
    for i, bb in enumerate(b):
        m = np.all((c >= bb[:3]) & (c < bb[3:]), axis=1)
        out[m] = i
    return out
