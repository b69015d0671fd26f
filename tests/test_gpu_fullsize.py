"""Parity at the benchmark's full size, in the launch configuration the
benchmark times (256^3 cells, 64 boxes of 64^3, 27,262,976 particles, FP32,
quadratic shapes, persistent kernel with graph replay).

The oracle cannot step 27 M particles in a test, so it is checked on samples
it can compute one by one:
  * 4,000 particles drawn across both species: position and momentum after
    one step (their gather, push and move only need the fields at step n);
  * 24 cells, including periodic and box faces and the slab's edges: J, E and
    B after one step.  J at a cell needs only the particles that start within
    a few cells of it, so the oracle steps exactly those (plus the sampled
    particles) over the full field arrays; E^{n+1} and B^{n+1} at the cell
    need J at the cell and its +x, +y, +z neighbours, which the neighbourhood
    covers.
The oracle's particles come from the host generator (the library loads the
same particles on the device; the loader itself is checked bit for bit in
test_gpu_parity).  Tolerance: the FP32 bar, 1e-5 (positions absolute in
cells, momenta and fields relative to the largest sampled magnitude).
"""
import numpy as np
import pytest

import picsynth

pytestmark = pytest.mark.gpu

TOL = 1e-5
REACH = 4  # cells: deposit window of a particle that moves at most one cell, plus one


def _neighbourhood_ids(wl, s, cells):
    """Ids of species s whose initial cell lies within REACH of any cell."""
    sp = wl.species[s]
    lo = np.array(sp.region_lo)
    hi = np.array(sp.region_hi)
    ext = hi - lo
    n = np.array(wl.n)
    ids = []
    r = np.arange(-REACH, REACH + 1)
    for c in cells:
        gx, gy, gz = np.meshgrid((c[0] + r) % n[0], (c[1] + r) % n[1], (c[2] + r) % n[2], indexing="ij")
        g = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        inside = np.all((g >= lo) & (g < hi), axis=1)
        g = g[inside] - lo
        rank = g[:, 0] + ext[0] * (g[:, 1] + ext[1] * g[:, 2])
        ids.append((rank[:, None] * sp.ppc + np.arange(sp.ppc)[None, :]).ravel())
    return np.unique(np.concatenate(ids)) if ids else np.zeros(0, np.int64)


def test_c2_one_step_sampled_against_oracle():
    import bench
    import oracle
    from paper_2104_11385_amd import picbal as pb

    wl = bench.workload()
    n = tuple(wl.n)
    print("full-size parity: c2, persistent + graph, 1 step", flush=True)
    F0 = picsynth.random_fields(n, 7, amp=0.03)
    ctx = bench.make_ctx(wl)
    try:
        ctx.set_launch_mode(pb.PIC_LAUNCH_PERSISTENT, True)
        ctx.set_fields(F0)
        ctx.step(1)
        ctx.sync()
        G = ctx.get_fields()
        gpu = [ctx.get_particles(s) for s in range(len(wl.species))]
    finally:
        ctx.finalize()

    rng = np.random.default_rng(2)
    lo = np.array(wl.species[0].region_lo)
    hi = np.array(wl.species[0].region_hi)
    cells = [tuple(int(v) for v in rng.integers(lo, hi)) for _ in range(14)]
    cells += [(0, 17, 120), (255, 40, 121), (63, 9, 130), (64, 200, 118), (100, 63, 127), (31, 64, 128),
              (12, 12, lo[2]), (200, 90, hi[2] - 1), (5, 250, hi[2]), (77, 3, lo[2] - 1)]

    xs, us, ws, sps, idlist = [], [], [], [], []
    samples = []
    for s in range(len(wl.species)):
        N = picsynth.species_count(wl, s)
        smp = np.sort(rng.choice(N, 2000, replace=False))
        ids = np.union1d(smp, _neighbourhood_ids(wl, s, cells))
        x, u, w, i = picsynth.particles(wl, s, ids)
        xs.append(x); us.append(u); ws.append(w); sps.append(np.full(len(w), s, np.int32)); idlist.append(i)
        samples.append(smp)
    x = np.ascontiguousarray(np.concatenate(xs)); u = np.ascontiguousarray(np.concatenate(us))
    w = np.concatenate(ws); sp = np.concatenate(sps)
    q = np.array([s.charge for s in wl.species]); mass = np.array([s.mass for s in wl.species])
    F = np.ascontiguousarray(F0.copy())
    oracle.pic_step(wl.order, n, wl.dt, x, u, w, sp, q, mass, F, 1)

    # sampled particles
    off = 0
    for s in range(len(wl.species)):
        gx, gu, _, gids = gpu[s]
        where = np.empty(len(gids), np.int64)
        where[gids] = np.arange(len(gids))
        ids = idlist[s]
        k = np.searchsorted(ids, samples[s])
        ox, ou = x[off + k], u[off + k]
        px, pu = gx[where[samples[s]]], gu[where[samples[s]]]
        d = np.abs(px - ox)
        d = np.minimum(d, np.array(n) - d)             # periodic images
        assert d.max() <= TOL, f"species {s}: max |dx| = {d.max():.3e}"
        scale = max(np.abs(ou).max(), 1e-30)
        assert np.abs(pu - ou).max() <= TOL * scale, f"species {s}: max |du| = {np.abs(pu - ou).max():.3e}"
        off += len(ids)

    # sampled cells
    cz = np.array([c[2] for c in cells]); cy = np.array([c[1] for c in cells]); cx = np.array([c[0] for c in cells])
    for comp in range(9):
        want = F[comp, cz, cy, cx]
        got = G[comp, cz, cy, cx]
        scale = max(np.abs(want).max(), np.abs(F0[comp]).max(), 1e-30)
        err = np.abs(got - want).max()
        assert err <= TOL * scale, f"component {comp}: max error {err:.3e} against scale {scale:.3e}"
