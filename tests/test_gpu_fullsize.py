"""Parity at full size, in the launch configuration the benchmark times
(persistent kernel with graph replay): the benchmark workload (256^3 cells,
64 boxes of 64^3, 27,262,976 particles, FP32, quadratic shapes), and the
uneven-box (512^3, 4096 mixed boxes, 1.13e9 particles) and balancing-study
(384x384x768, 3456 boxes, 94,371,840 particles) workloads from their own
initial state.

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
cells; momenta per particle relative to max(|u|, u_floor), u_floor the
momentum the strongest field can impart in the step; fields relative to the
largest sampled magnitude).
"""
import numpy as np
import pytest

import picsynth
from tests._util import check_u_per_particle, u_floor

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


@pytest.mark.parametrize("precision,order", [(4, 2), (8, 2), (4, 3)])
def test_c2_one_step_sampled_against_oracle(precision, order):
    # FP32 (the benchmark) at the workload's bar; FP64 (the same kernel
    # compiled in double, two waves per SIMD) at the FP64 bar, 1e-12; and
    # the paper's cubic shapes in FP32 (a particle's deposit reaches two
    # nodes below and three above its cell, inside REACH)
    import bench
    import oracle
    from paper_2104_11385_amd import picbal as pb

    wl = bench.workload()
    wl.precision = precision
    wl.order = order
    tol = TOL if precision == 4 else 1e-12
    n = tuple(wl.n)
    print(f"full-size parity: c2, precision {precision}, order {order}, persistent + graph, 1 step", flush=True)
    F0 = picsynth.random_fields(n, 7, amp=0.03)
    ctx = bench.ctx_for(wl)
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
        assert d.max() <= tol, f"species {s}: max |dx| = {d.max():.3e}"
        e_max = max(np.abs(F0[0:3]).max(), np.abs(F[0:3]).max())
        check_u_per_particle(pu, ou, np.full(len(ou), s), samples[s], u_floor(wl, e_max, 1), tol)
        off += len(ids)

    # sampled cells
    cz = np.array([c[2] for c in cells]); cy = np.array([c[1] for c in cells]); cx = np.array([c[0] for c in cells])
    for comp in range(9):
        want = F[comp, cz, cy, cx]
        got = G[comp, cz, cy, cx]
        scale = max(np.abs(want).max(), np.abs(F0[comp]).max(), 1e-30)
        err = np.abs(got - want).max()
        assert err <= tol * scale, f"component {comp}: max error {err:.3e} against scale {scale:.3e}"


def test_c2_sampled_step_at_the_end_of_a_sort_interval():
    # The 20th step after a sort (the last before the next one): over 19
    # steps ~7% of the particles a step have changed node while keeping
    # their slots, so the node runs of the lane sums are at their most cut up
    # (a node's run broken by particles of other nodes, one node in several
    # runs of a row).  The oracle steps the library's own state after step 19
    # once: every particle within reach of the sampled cells, and sampled
    # particles of both species.
    import bench
    import oracle
    from paper_2104_11385_amd import picbal as pb

    wl = bench.workload()
    n = np.array(wl.n)
    print("full-size parity: c2, persistent + graph, step 20 after a sort", flush=True)
    rng = np.random.default_rng(12)
    lo = np.array(wl.species[0].region_lo)
    hi = np.array(wl.species[0].region_hi)
    cells = [tuple(int(v) for v in rng.integers(lo, hi)) for _ in range(10)]
    cells += [(0, 17, 121), (255, 40, 122), (63, 9, 130), (64, 200, 119), (100, 63, 127), (31, 64, 128)]
    cz = np.array([c[2] for c in cells]); cy = np.array([c[1] for c in cells]); cx = np.array([c[0] for c in cells])
    ctx = bench.make_ctx(wl)
    try:
        ctx.set_launch_mode(pb.PIC_LAUNCH_PERSISTENT, True)
        ctx.set_fields(picsynth.random_fields(tuple(n), 7, amp=0.03))
        ctx.step(19)
        ctx.sync()
        F = np.ascontiguousarray(ctx.get_fields())
        xs, us, ws, sps, samples = [], [], [], [], []
        for s in range(len(wl.species)):
            x, u, w, ids = ctx.get_particles(s)
            c = np.floor(x).astype(np.int64)
            near = np.zeros(len(w), bool)
            for cell in cells:
                d = np.abs(c - np.array(cell))
                near |= np.all(np.minimum(d, n - d) <= REACH, axis=1)
            smp = np.sort(rng.choice(len(w), 2000, replace=False))
            keep = np.union1d(np.nonzero(near)[0], smp)
            xs.append(x[keep]); us.append(u[keep]); ws.append(w[keep]); sps.append(np.full(len(keep), s, np.int32))
            samples.append((ids[smp], np.searchsorted(keep, smp)))
            del x, u, w, ids, c, near
        ctx.step(1)
        ctx.sync()
        got_cells = np.stack([ctx.get_field(c)[cz, cy, cx] for c in range(9)])
        got = [ctx.get_particles_by_id(s, samples[s][0]) for s in range(len(wl.species))]
    finally:
        ctx.finalize()

    off = np.cumsum([0] + [len(w) for w in ws])
    x = np.ascontiguousarray(np.concatenate(xs)); u = np.ascontiguousarray(np.concatenate(us))
    w = np.concatenate(ws); sp = np.concatenate(sps)
    u0 = u.copy()
    q = np.array([s.charge for s in wl.species]); mass = np.array([s.mass for s in wl.species])
    F0 = F.copy()
    oracle.pic_step(wl.order, tuple(n), wl.dt, x, u, w, sp, q, mass, F, 1)
    e_max = max(np.abs(F0[0:3]).max(), np.abs(F[0:3]).max())
    for s in range(len(wl.species)):
        gx, gu, found = got[s]
        assert found.all()
        k = off[s] + samples[s][1]
        d = np.abs(gx - x[k])
        d = np.minimum(d, n - d)
        assert d.max() <= TOL, f"species {s}: max |dx| = {d.max():.3e}"
        # momenta against the step's own impulse scale (the particles start
        # from the library's state, so one step's rounding is what differs)
        check_u_per_particle(gu, u[k], np.full(len(k), s), samples[s][0], u_floor(wl, e_max, 1), TOL)
        assert np.abs(u[k] - u0[k]).max() > 0
    want = F[:, cz, cy, cx]
    for comp in range(9):
        scale = max(np.abs(want[comp]).max(), np.abs(F0[comp]).max(), 1e-30)
        err = np.abs(got_cells[comp] - want[comp]).max()
        assert err <= TOL * scale, f"component {comp}: max error {err:.3e} against scale {scale:.3e}"
    assert np.abs(want[6:9]).max() > 0


def _ids_of_cells(wl, s, cells):
    """Ids of species s whose initial cell is one of `cells` ([k, 3])."""
    sp = wl.species[s]
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    if sp.box_ppc is None:
        lo = np.array(sp.region_lo)
        hi = np.array(sp.region_hi if sp.region_hi is not None else wl.n)
        ext = hi - lo
        inside = np.all((cells >= lo) & (cells < hi), axis=1)
        g = cells[inside] - lo
        rank = g[:, 0] + ext[0] * (g[:, 1] + ext[1] * g[:, 2])
        return (rank[:, None] * sp.ppc + np.arange(sp.ppc)[None, :]).ravel()
    b = wl.boxes.astype(np.int64)
    ext = b[:, 3:] - b[:, :3]
    base = np.concatenate([[0], np.cumsum(ext.prod(axis=1) * sp.box_ppc)])
    out = []
    for c in cells:
        bi = int(np.nonzero(np.all((c >= b[:, :3]) & (c < b[:, 3:]), axis=1))[0][0])
        ppc = int(sp.box_ppc[bi])
        if ppc == 0:
            continue
        l = c - b[bi, :3]
        local = l[0] + ext[bi, 0] * (l[1] + ext[bi, 1] * l[2])
        out.append(base[bi] + local * ppc + np.arange(ppc))
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def _neighbourhood(wl, s, cells):
    n = np.array(wl.n)
    r = np.arange(-REACH, REACH + 1)
    allc = []
    for c in cells:
        gx, gy, gz = np.meshgrid((c[0] + r) % n[0], (c[1] + r) % n[1], (c[2] + r) % n[2], indexing="ij")
        allc.append(np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1))
    return np.unique(_ids_of_cells(wl, s, np.concatenate(allc)))


def _sampled_one_step(name, cells, nsample=2000, seed=5):
    """One step of workload `name` from its initial state on the device,
    checked on sampled particles (looked up by id) and at sampled cells."""
    import bench
    import oracle
    from paper_2104_11385_amd import picbal as pb

    wl = picsynth.config(name)
    n = tuple(wl.n)
    print(f"full-size parity: {name}, persistent + graph, 1 step", flush=True)
    rng = np.random.default_rng(seed)
    samples = [np.sort(rng.choice(picsynth.species_count(wl, s), nsample, replace=False))
               for s in range(len(wl.species))]
    ctx = bench.ctx_for(wl)
    try:
        ctx.set_launch_mode(pb.PIC_LAUNCH_PERSISTENT, True)
        ctx.step(1)
        ctx.sync()
        cz = np.array([c[2] for c in cells]); cy = np.array([c[1] for c in cells]); cx = np.array([c[0] for c in cells])
        got_cells = np.stack([ctx.get_field(c)[cz, cy, cx] for c in range(9)])
        got = [ctx.get_particles_by_id(s, samples[s]) for s in range(len(wl.species))]
    finally:
        ctx.finalize()

    xs, us, ws, sps, idl = [], [], [], [], []
    for s in range(len(wl.species)):
        ids = np.union1d(samples[s], _neighbourhood(wl, s, cells))
        x, u, w, i = picsynth.particles(wl, s, ids)
        xs.append(x); us.append(u); ws.append(w); sps.append(np.full(len(w), s, np.int32)); idl.append(i)
    x = np.ascontiguousarray(np.concatenate(xs)); u = np.ascontiguousarray(np.concatenate(us))
    w = np.concatenate(ws); sp = np.concatenate(sps)
    q = np.array([s.charge for s in wl.species]); mass = np.array([s.mass for s in wl.species])
    F0 = np.ascontiguousarray(picsynth.initial_fields(wl))
    F = F0.copy()
    oracle.pic_step(wl.order, n, wl.dt, x, u, w, sp, q, mass, F, 1)

    off = 0
    for s in range(len(wl.species)):
        gx, gu, found = got[s]
        assert found.all(), f"species {s}: {int((~found).sum())} sampled ids not found"
        k = np.searchsorted(idl[s], samples[s])
        ox, ou = x[off + k], u[off + k]
        d = np.abs(gx - ox)
        d = np.minimum(d, np.array(n) - d)
        assert d.max() <= TOL, f"species {s}: max |dx| = {d.max():.3e}"
        e_max = max(np.abs(F0[0:3]).max(), np.abs(F[0:3]).max())
        check_u_per_particle(gu, ou, np.full(len(ou), s), samples[s], u_floor(wl, e_max, 1), TOL)
        off += len(idl[s])
    want_cells = F[:, cz, cy, cx]
    for comp in range(9):
        scale = max(np.abs(want_cells[comp]).max(), 1e-30)
        err = np.abs(got_cells[comp] - want_cells[comp]).max()
        assert err <= TOL * scale, f"component {comp}: max error {err:.3e} against scale {scale:.3e}"
    # the sampled cells carry current: the check is not vacuous
    assert np.abs(want_cells[6:9]).max() > 0


def test_mixed_boxes_one_step_sampled_against_oracle():
    # 512^3, 4096 boxes of 64^3 / 32^3 / 16^3 with lognormal ppc up to 64
    rng = np.random.default_rng(8)
    cells = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(12)]
    # faces of boxes of each size and of the domain
    cells += [(64, 10, 20), (63, 10, 20), (96, 64, 32), (80, 80, 79), (16, 16, 16), (511, 0, 255),
              (0, 511, 128), (255, 256, 511), (128, 130, 64), (47, 48, 49)]
    _sampled_one_step("c3", cells)


def test_balancing_study_one_step_sampled_against_oracle():
    # 384 x 384 x 768, 3456 boxes of 32^3, two drifting species in z [374, 394)
    rng = np.random.default_rng(9)
    cells = [(int(rng.integers(0, 384)), int(rng.integers(0, 384)), int(rng.integers(374, 394))) for _ in range(14)]
    cells += [(0, 0, 384), (383, 100, 383), (31, 32, 374), (32, 31, 393), (200, 383, 373), (5, 6, 394),
              (160, 160, 384), (64, 95, 375)]
    _sampled_one_step("c4", cells)


def _div_e(F):
    # divergence at the nodes of the edge-centred E (F[0:3], arrays [z][y][x])
    return (F[0] - np.roll(F[0], 1, axis=2)) + (F[1] - np.roll(F[1], 1, axis=1)) + (F[2] - np.roll(F[2], 1, axis=0))


@pytest.mark.parametrize("name,steps", [("c2", 200), ("c2-cubic", 25), ("c4", 25)])
def test_gauss_law_holds_over_steps_and_sorts(name, steps):
    # A property of the whole step at full size: with a charge-conserving
    # deposit on E's stagger, div E - rho keeps its initial value at every
    # node.  25 or 200 steps in the benchmark's configuration (persistent
    # kernel, graph replay, particle sort every 20 steps) cover the staged windows,
    # the queued node-changing particles, the flush, the global-memory path
    # and the Yee passes at every node, not only sampled ones: the benchmark
    # workload (256^3, random initial fields) and the balancing-study
    # workload (384x384x768, 9.4e7 particles drifting at u_z = 0.05, so that
    # ~2.5% of them change node each step), from its own initial state; and
    # the benchmark workload with cubic shapes.
    import bench
    import oracle
    from paper_2104_11385_amd import picbal as pb

    wl = bench.workload() if name.startswith("c2") else picsynth.config(name)
    if name == "c2-cubic":
        wl.order = 3
    n = tuple(wl.n)
    q = np.array([s.charge for s in wl.species])
    print(f"full-size Gauss law: {name}, persistent + graph, {steps} steps", flush=True)

    def particles(ctx):
        xs, ws, sps = [], [], []
        for s in range(len(wl.species)):
            x, _, w, _ = ctx.get_particles(s)
            xs.append(x); ws.append(w); sps.append(np.full(len(w), s, np.int32))
        return np.ascontiguousarray(np.concatenate(xs)), np.concatenate(ws), np.concatenate(sps)

    def residual(ctx):
        x, w, sp = particles(ctx)
        rho = oracle.rho(wl.order, n, x, w, sp, q)
        return _div_e(ctx.get_fields()) - rho, rho

    ctx = bench.make_ctx(wl) if name.startswith("c2") else bench.ctx_for(wl)
    try:
        ctx.set_launch_mode(pb.PIC_LAUNCH_PERSISTENT, True)
        if name.startswith("c2"):
            ctx.set_fields(picsynth.random_fields(n, 7, amp=0.03))
        x, w, sp = particles(ctx)
        e = sp == 0
        scale = np.abs(oracle.rho(wl.order, n, x[e], w[e], sp[e], q)).max()
        del x, w, sp, e
        g0, rho0 = residual(ctx)
        ctx.step(steps)
        ctx.sync()
        g1, rho1 = residual(ctx)
    finally:
        ctx.finalize()
    drift = np.abs(g1 - g0).max()
    moved = np.abs(rho1 - rho0).max()
    print(f"max |d(div E - rho)| {drift:.3e}, max |d rho| {moved:.3e}, electron density scale {scale:.3e}", flush=True)
    # one particle's current left out of one step moves the residual by about
    # 2.5e-3 of its charge, 3e-4 of the electron density scale; FP32 rounding
    # over 200 steps stays near 1e-6 of it
    assert drift <= 3e-5 * scale, f"max |d(div E - rho)| = {drift:.3e}, density scale {scale:.3e}"
    assert moved > 30 * 3e-5 * scale, f"charge barely moved ({moved:.3e}): the check would be vacuous"
