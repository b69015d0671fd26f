"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds none of the PIC or load-balancing arithmetic.  It provides

* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11) -- a counter-based generator, written here from its
  published definition in vectorised numpy;
* the particle-loading recipe (which random word becomes which coordinate);
* the box layouts and species of the benchmark workloads;
* small field initialisers for tests.

The HIP library's on-device loader implements the same published generator
and the same recipe independently, so large workloads can be created on the
GPU while any sampled particle can be regenerated here.

Loading recipe (per species s with 64-bit seed S, particle index p):
  key  = (lo32(S), hi32(S) xor s)
  blkA = philox(ctr=(lo32(p), hi32(p), 0, 0), key) -> r0 r1 r2 r3
  blkB = philox(ctr=(lo32(p), hi32(p), 1, 0), key) -> r4 r5 r6 r7
  position offset in its cell, per dimension d: U_d = (r_d >> 8) * 2^-24
  Gaussians (Box-Muller): a = ((r3 >> 8) + 1) 2^-24, b = (r4 >> 8) 2^-24,
      n0 = sqrt(-2 ln a) cos(2 pi b), n1 = sqrt(-2 ln a) sin(2 pi b);
      c = ((r5 >> 8) + 1) 2^-24, e = (r6 >> 8) 2^-24,
      n2 = sqrt(-2 ln c) cos(2 pi e)
  u = (u_th_x n0, u_th_y n1, u_th_z n2) + u_drift,   w = density / ppc
Particle p of a fixed-ppc region lives in region cell p // ppc, cells counted
x fastest over the region; with a per-box ppc table, boxes are visited in
order and each box's cells x fastest within the box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

# normalised plasma density: omega_pe * dx / c = 0.274 (the paper's resolution)
N0_DEFAULT = 0.274 ** 2


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x32 with 10 rounds.  Counters are uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = c0 * M0
        p1 = c2 * M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32), c3.astype(np.uint32))


def species_key(seed: int, s: int):
    return seed & 0xFFFFFFFF, ((seed >> 32) & 0xFFFFFFFF) ^ (s & 0xFFFFFFFF)


def draws(seed: int, s: int, p: np.ndarray):
    """The 8 random words r0..r7 of particles with indices p."""
    p = np.asarray(p, dtype=np.uint64)
    lo = p & MASK32
    hi = p >> np.uint64(32)
    k0, k1 = species_key(seed, s)
    a = philox4x32_10(lo, hi, 0, 0, k0, k1)
    b = philox4x32_10(lo, hi, 1, 0, k0, k1)
    return a + b


def _unit(r):
    return (np.asarray(r, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * (2.0 ** -24)


def _unit_open(r):
    return ((np.asarray(r, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) + 1.0) * (2.0 ** -24)


def offsets_and_normals(seed: int, s: int, p: np.ndarray):
    r = draws(seed, s, p)
    U = np.stack([_unit(r[0]), _unit(r[1]), _unit(r[2])], axis=1)
    a, b = _unit_open(r[3]), _unit(r[4])
    c, e = _unit_open(r[5]), _unit(r[6])
    ra = np.sqrt(-2.0 * np.log(a))
    rc = np.sqrt(-2.0 * np.log(c))
    N = np.stack([ra * np.cos(2.0 * np.pi * b), ra * np.sin(2.0 * np.pi * b),
                  rc * np.cos(2.0 * np.pi * e)], axis=1)
    return U, N


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------

@dataclass
class Species:
    name: str
    charge: float
    mass: float
    density: float
    ppc: int = 0                      # fixed ppc in region (load mode 1)
    region_lo: Sequence[int] = (0, 0, 0)
    region_hi: Optional[Sequence[int]] = None   # None = whole domain
    box_ppc: Optional[np.ndarray] = None        # per-box ppc (load mode 2)
    u_th: Sequence[float] = (0.0, 0.0, 0.0)
    u_drift: Sequence[float] = (0.0, 0.0, 0.0)


@dataclass
class Workload:
    name: str
    n: Sequence[int]
    boxes: np.ndarray                 # [nb, 6] lo_x lo_y lo_z hi_x hi_y hi_z
    species: List[Species]
    dt: float = 0.5
    order: int = 2
    precision: int = 4                # bytes per float
    seed: int = 1
    b_ext: Sequence[float] = (0.0, 0.0, 0.0)
    steps: int = 10
    extra: dict = field(default_factory=dict)


def uniform_boxes(n, edge):
    """Boxes of edge^3 (or per-dim edges), box index x fastest."""
    ex, ey, ez = (edge, edge, edge) if np.isscalar(edge) else edge
    out = []
    for bz in range(n[2] // ez):
        for by in range(n[1] // ey):
            for bx in range(n[0] // ex):
                out.append([bx * ex, by * ey, bz * ez, (bx + 1) * ex, (by + 1) * ey, (bz + 1) * ez])
    return np.array(out, dtype=np.int32)


def mixed_boxes_512():
    """512^3 in 8^3 regions of 64^3: regions with I+J+K even stay one 64^3
    box; odd regions split into eight 32^3 octants whose lowest-corner octant
    splits again into eight 16^3 boxes.  256 + 1792 + 2048 = 4096 boxes."""
    out = []
    for K in range(8):
        for J in range(8):
            for I in range(8):
                o = np.array([I, J, K]) * 64
                if (I + J + K) % 2 == 0:
                    out.append([*o, *(o + 64)])
                    continue
                for oz in range(2):
                    for oy in range(2):
                        for ox in range(2):
                            q = o + np.array([ox, oy, oz]) * 32
                            if ox == oy == oz == 0:
                                for sz in range(2):
                                    for sy in range(2):
                                        for sx in range(2):
                                            r = q + np.array([sx, sy, sz]) * 16
                                            out.append([*r, *(r + 16)])
                            else:
                                out.append([*q, *(q + 32)])
    return np.array(out, dtype=np.int32)


def lognormal_box_ppc(nb: int, seed: int, mu=1.5, sigma=1.2, cap=64):
    """Per-box ppc = min(cap, floor(exp(mu + sigma n) + 1/2)), n from Philox
    (species slot 0x7fffffff of the seed, counter = box index)."""
    U, N = offsets_and_normals(seed, 0x7FFFFFFF, np.arange(nb))
    X = np.exp(mu + sigma * N[:, 0])
    return np.minimum(cap, np.floor(X + 0.5)).astype(np.int32)


def config(name: str) -> Workload:
    """The benchmark workloads (c1..c4) as plain data."""
    if name == "c1":
        n = (32, 32, 32)
        return Workload(
            "c1", n, uniform_boxes(n, 16),
            [Species("electrons", -1.0, 1.0, N0_DEFAULT, ppc=2, u_th=(0.01, 0.01, 0.01))],
            dt=0.5, order=1, precision=8, seed=1, b_ext=(0.0, 0.0, 1.0), steps=10)
    if name == "c2":
        n = (256, 256, 256)
        slab_lo, slab_hi = (0, 0, 115), (256, 256, 141)
        return Workload(
            "c2", n, uniform_boxes(n, 64),
            [Species("electrons", -1.0, 1.0, N0_DEFAULT, ppc=8, region_lo=slab_lo, region_hi=slab_hi,
                     u_th=(0.005, 0.005, 0.005)),
             Species("protons", 1.0, 1836.0, N0_DEFAULT, ppc=8, region_lo=slab_lo, region_hi=slab_hi)],
            dt=0.5, order=2, precision=4, seed=2, steps=100)
    if name == "c3":
        n = (512, 512, 512)
        boxes = mixed_boxes_512()
        return Workload(
            "c3", n, boxes,
            [Species("electrons", -1.0, 1.0, N0_DEFAULT, box_ppc=lognormal_box_ppc(len(boxes), 3),
                     u_th=(0.005, 0.005, 0.005))],
            dt=0.5, order=2, precision=4, seed=3, steps=20)
    if name == "c4":
        n = (384, 384, 768)
        slab_lo, slab_hi = (0, 0, 374), (384, 384, 394)
        return Workload(
            "c4", n, uniform_boxes(n, 32),
            [Species("electrons", -1.0, 1.0, N0_DEFAULT, ppc=16, region_lo=slab_lo, region_hi=slab_hi,
                     u_th=(0.005, 0.005, 0.005), u_drift=(0.0, 0.0, 0.05)),
             Species("protons", 1.0, 1836.0, N0_DEFAULT, ppc=16, region_lo=slab_lo, region_hi=slab_hi,
                     u_drift=(0.0, 0.0, 0.05))],
            dt=0.5, order=2, precision=4, seed=4, steps=300)
    raise KeyError(name)


# --------------------------------------------------------------------------
# Particle generation on the host
# --------------------------------------------------------------------------

def species_count(wl: Workload, s: int) -> int:
    sp = wl.species[s]
    if sp.box_ppc is not None:
        b = wl.boxes
        cells = (b[:, 3] - b[:, 0]).astype(np.int64) * (b[:, 4] - b[:, 1]) * (b[:, 5] - b[:, 2])
        return int((cells * sp.box_ppc).sum())
    lo = np.array(sp.region_lo)
    hi = np.array(sp.region_hi if sp.region_hi is not None else wl.n)
    return int(np.prod(hi - lo)) * sp.ppc


def cell_of_index(wl: Workload, s: int, p: np.ndarray) -> np.ndarray:
    """Integer cell [len(p), 3] that particle index p is loaded into."""
    sp = wl.species[s]
    p = np.asarray(p, dtype=np.int64)
    if sp.box_ppc is not None:
        b = wl.boxes.astype(np.int64)
        ext = b[:, 3:] - b[:, :3]
        cells = ext[:, 0] * ext[:, 1] * ext[:, 2]
        base = np.concatenate([[0], np.cumsum(cells * sp.box_ppc)])
        bi = np.searchsorted(base, p, side="right") - 1
        ppc = sp.box_ppc[bi].astype(np.int64)
        local = (p - base[bi]) // ppc
        ex, ey = ext[bi, 0], ext[bi, 1]
        cx = local % ex
        cy = (local // ex) % ey
        cz = local // (ex * ey)
        return np.stack([b[bi, 0] + cx, b[bi, 1] + cy, b[bi, 2] + cz], axis=1)
    lo = np.array(sp.region_lo, dtype=np.int64)
    hi = np.array(sp.region_hi if sp.region_hi is not None else wl.n, dtype=np.int64)
    ext = hi - lo
    local = p // sp.ppc
    cx = local % ext[0]
    cy = (local // ext[0]) % ext[1]
    cz = local // (ext[0] * ext[1])
    return np.stack([lo[0] + cx, lo[1] + cy, lo[2] + cz], axis=1)


def weight_of_index(wl: Workload, s: int, p: np.ndarray) -> np.ndarray:
    sp = wl.species[s]
    p = np.asarray(p, dtype=np.int64)
    if sp.box_ppc is not None:
        b = wl.boxes.astype(np.int64)
        ext = b[:, 3:] - b[:, :3]
        cells = ext[:, 0] * ext[:, 1] * ext[:, 2]
        base = np.concatenate([[0], np.cumsum(cells * sp.box_ppc)])
        bi = np.searchsorted(base, p, side="right") - 1
        return sp.density / sp.box_ppc[bi].astype(np.float64)
    return np.full(p.shape, sp.density / sp.ppc)


def particles(wl: Workload, s: int, p: Optional[np.ndarray] = None):
    """Host copy of species s's initial particles (all, or indices p):
    returns x [n,3] (global cell units), u [n,3], w [n], id [n] (int64)."""
    if p is None:
        p = np.arange(species_count(wl, s), dtype=np.int64)
    p = np.asarray(p, dtype=np.int64)
    sp = wl.species[s]
    cell = cell_of_index(wl, s, p)
    U, N = offsets_and_normals(wl.seed, s, p)
    x = cell.astype(np.float64) + U
    u = N * np.asarray(sp.u_th, dtype=np.float64)[None, :] + np.asarray(sp.u_drift, dtype=np.float64)[None, :]
    w = weight_of_index(wl, s, p)
    return x, u, w, p.copy()


def all_particles(wl: Workload):
    """Concatenated particles of every species plus a species index array."""
    xs, us, ws, ids, sps = [], [], [], [], []
    for s in range(len(wl.species)):
        x, u, w, i = particles(wl, s)
        xs.append(x); us.append(u); ws.append(w); ids.append(i)
        sps.append(np.full(len(w), s, dtype=np.int32))
    return (np.concatenate(xs), np.concatenate(us), np.concatenate(ws),
            np.concatenate(ids), np.concatenate(sps))


def initial_fields(wl: Workload) -> np.ndarray:
    """F[9, nz, ny, nx]: uniform external B, zero E and J."""
    nx, ny, nz = wl.n
    F = np.zeros((9, nz, ny, nx))
    for d in range(3):
        F[3 + d] = wl.b_ext[d]
    return F


def small_workload(n=(16, 16, 16), box=8, order=2, ppc=2, seed=11, dt=0.5,
                   species=("electrons",), u_th=0.05, precision=8, b_ext=(0.0, 0.0, 0.0),
                   region_lo=(0, 0, 0), region_hi=None, u_drift=(0.0, 0.0, 0.0)) -> Workload:
    """A small periodic workload for parity tests."""
    sp = []
    for name in species:
        if name == "electrons":
            sp.append(Species(name, -1.0, 1.0, N0_DEFAULT, ppc=ppc, region_lo=region_lo,
                              region_hi=region_hi, u_th=(u_th,) * 3, u_drift=u_drift))
        else:
            sp.append(Species(name, 1.0, 1836.0, N0_DEFAULT, ppc=ppc, region_lo=region_lo,
                              region_hi=region_hi, u_th=(u_th / 43.0,) * 3, u_drift=u_drift))
    return Workload("small", tuple(n), uniform_boxes(n, box), sp, dt=dt, order=order,
                    precision=precision, seed=seed, b_ext=b_ext)


def random_fields(n, seed, amp=0.05):
    """Smooth-ish random E and B (zero J) for gather/push parity: a sum of a
    few periodic modes with Philox-drawn amplitudes and phases."""
    nx, ny, nz = n
    k = np.arange(24, dtype=np.int64)
    r = philox4x32_10(k, 0, 0, 0, seed & 0xFFFFFFFF, 0x5EED)
    vals = np.stack([_unit(x) for x in r], axis=1).reshape(-1)
    F = np.zeros((9, nz, ny, nx))
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    q = 0
    for c in range(6):
        for mode in range(2):
            kx, ky, kz = 1 + mode, 1 + (c % 2), 1 + ((c + mode) % 3)
            a = amp * (2 * vals[q] - 1); ph = 2 * np.pi * vals[q + 1]; q += 2
            F[c] += a * np.cos(2 * np.pi * (kx * xx / nx + ky * yy / ny + kz * zz / nz) + ph)
    return F
