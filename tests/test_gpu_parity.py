"""GPU parity: the HIP path against the FP64 oracle on identical seeded inputs.

Tolerances (derived from the arithmetic of each precision):
  FP64 library vs FP64 oracle: 1e-12; FP32 library vs FP64 oracle after 10
  steps: 1e-5.  Per particle: |dx| (minimal image) <= tol max(1, |x|) and
  |du| <= tol max(|u|, u_floor), with u_floor = |q| dt steps max|E| / m per
  species (the momentum the strongest field of the run can impart; a
  particle near rest is held to the rounding of the impulses its momentum is
  made of).  Fields norm-wise per component (J vanishes at many nodes).
Every case spans several tiles and boxes; particle orders are matched by id.
"""
import numpy as np
import pytest

import oracle
import picsynth
from tests._util import (box_of, check_u_per_particle, gpu_particles, make_ctx, min_image, near_box_face, normwise,
                         oracle_steps, order_by_species_id, set_state, u_floor)

pytestmark = pytest.mark.gpu

TOL = {8: 1e-12, 4: 1e-5}


def _pb():
    from paper_2104_11385_amd import picbal as pb
    return pb


def compare(ctx, wl, x, u, w, sp, ids, F, nsteps, tol, check_fields=True):
    gx, gu, gids, gsp = gpu_particles(ctx, wl)
    ox, ou, OF = oracle_steps(wl, x, u, w, sp, F, nsteps)
    ox, ou, oids, osp = order_by_species_id(ox, ou, ids, sp)
    np.testing.assert_array_equal(gids, oids)
    np.testing.assert_array_equal(gsp, osp)
    dx = np.abs(min_image(gx - ox, wl.n))
    assert (dx <= tol * np.maximum(1.0, np.abs(ox))).all(), f"max |dx| = {dx.max():.3e}"
    e_max = max(np.abs(F[0:3]).max(), np.abs(OF[0:3]).max())
    check_u_per_particle(gu, ou, gsp, gids, u_floor(wl, e_max, nsteps), tol)
    if check_fields:
        GF = ctx.get_fields()
        for c in range(9):
            if np.abs(OF[c]).max() == 0:
                assert np.abs(GF[c]).max() <= 1e-30
                continue
            err = normwise(GF[c], OF[c])
            assert err <= tol, f"field component {c}: error {err:.3e}"
    return gx, ox


def quad_workload(precision=8, n=(16, 16, 24), u_th=0.05, seed=21):
    return picsynth.small_workload(n=n, box=8, order=2, ppc=2, seed=seed, species=("electrons", "protons"),
                                   u_th=u_th, precision=precision, region_lo=(0, 0, 4), region_hi=(n[0], n[1], 20))


@pytest.mark.parametrize("precision", [8, 4])
def test_c1_ten_steps(precision):
    # 32^3, 8 boxes of 16^3, 65,536 electrons, B_z = 1, linear shapes, 10 steps
    wl = picsynth.config("c1")
    print(f"[parity] c1 precision={precision}", flush=True)
    ctx = make_ctx(wl, precision=precision, load=False)
    x, u, w, ids, sp, F = set_state(ctx, wl)
    ctx.step(wl.steps)
    compare(ctx, wl, x, u, w, sp, ids, F, wl.steps, TOL[precision])


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_random_fields_two_species(precision, order):
    wl = quad_workload(precision)
    wl.order = order
    print(f"[parity] two species order={order} precision={precision}", flush=True)
    ctx = make_ctx(wl, load=False)
    F0 = picsynth.random_fields(wl.n, 9, amp=0.05)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.step(10)
    compare(ctx, wl, x, u, w, sp, ids, F, 10, TOL[precision])


@pytest.mark.parametrize("mode,graph", [(0, False), (1, False), (2, False), (2, True), (0, True)])
def test_launch_modes_agree_with_oracle(mode, graph):
    wl = quad_workload(8, seed=5)
    print(f"[parity] launch mode={mode} graph={graph}", flush=True)
    ctx = make_ctx(wl, load=False)
    ctx.set_launch_mode(mode, graph)
    F0 = picsynth.random_fields(wl.n, 4, amp=0.03)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.step(7)
    compare(ctx, wl, x, u, w, sp, ids, F, 7, TOL[8])


@pytest.mark.parametrize("precision,mode", [(8, 2), (4, 2), (8, 0)])
def test_graph_replay_across_sorts(precision, mode):
    # every step one graph launch, with the particle sort and the work-queue
    # rebuild captured into the graphs of the steps that start with them:
    # sorts before steps 4, 7, 10 and 13; the graph of step 4 (field buffer
    # 1, particle buffer 0) is replayed at step 10, that of step 7 at step 13
    wl = quad_workload(precision, seed=9)
    print(f"[parity] graph replay across sorts, precision={precision} mode={mode}", flush=True)
    ctx = make_ctx(wl, load=False)
    ctx.set_tuning(sort_interval=3)
    ctx.set_launch_mode(mode, True)
    F0 = picsynth.random_fields(wl.n, 8, amp=0.03)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.step(14)
    compare(ctx, wl, x, u, w, sp, ids, F, 14, TOL[precision])


@pytest.mark.parametrize("precision,order,mode,graph", [(8, 2, 2, False), (8, 3, 2, True), (4, 2, 2, True),
                                                       (4, 2, 0, False), (8, 1, 1, True)])
def test_field_update_split_follows_a_drifting_slab(precision, order, mode, graph):
    # a thin electron slab drifting at 0.89c along z into planes that held no
    # current: each step the Yee update of the planes out of the deposit's
    # reach runs beside the particle kernel and the rest after it, and the
    # slab keeps entering planes of the first kind (within its tiles' windows
    # between sorts, beyond them on the global path); with and without the
    # split the step matches the oracle
    wl = picsynth.small_workload(n=(16, 16, 64), box=8, order=order, ppc=2, seed=31, species=("electrons",),
                                 u_th=0.05, precision=precision, region_lo=(0, 0, 8), region_hi=(16, 16, 12),
                                 u_drift=(0.0, 0.0, 2.0))
    nsteps = 30 if precision == 8 else 10
    for ov in (1, 0):
        print(f"[parity] drifting slab precision={precision} order={order} mode={mode} graph={graph} overlap={ov}",
              flush=True)
        ctx = make_ctx(wl, load=False)
        ctx.set_tuning(field_overlap=ov, sort_interval=7)
        ctx.set_launch_mode(mode, graph)
        F0 = picsynth.random_fields(wl.n, 23, amp=0.02)
        x, u, w, ids, sp, F = set_state(ctx, wl, F0)
        ctx.step(nsteps)
        compare(ctx, wl, x, u, w, sp, ids, F, nsteps, TOL[precision])


@pytest.mark.parametrize("precision,order", [(8, 2), (4, 2), (8, 3), (4, 1)])
def test_fast_particles_take_global_path(precision, order):
    # u_th = 0.6: particles drift several cells between sorts, beyond the
    # staged halo, and must still match through the global-memory path.
    wl = quad_workload(precision, u_th=0.6, seed=8)
    wl.order = order
    print(f"[parity] fast particles precision={precision}", flush=True)
    ctx = make_ctx(wl, load=False)
    ctx.set_tuning(sort_interval=1000)
    F0 = picsynth.random_fields(wl.n, 2, amp=0.02)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.slow_path_count()
    ctx.step(10)
    assert ctx.slow_path_count() > 0
    compare(ctx, wl, x, u, w, sp, ids, F, 10, TOL[precision])


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("run_sum", [0, 1])
def test_dense_nodes_both_particle_orders(precision, order, run_sum):
    # 24 particles per cell: a node's particles fill more than one 16-lane
    # row, so the lane sums of the node-major order span row boundaries; the
    # interleaved order deposits particle by particle.  Both match the oracle.
    wl = picsynth.small_workload(n=(16, 8, 16), box=8, order=order, ppc=24, seed=31, species=("electrons",),
                                 u_th=0.02, precision=precision, region_lo=(0, 0, 4), region_hi=(16, 8, 12))
    print(f"[parity] dense nodes order={order} precision={precision} run_sum={run_sum}", flush=True)
    ctx = make_ctx(wl, load=False)
    ctx.set_tuning(run_sum=run_sum, sort_interval=4)
    F0 = picsynth.random_fields(wl.n, 13, amp=0.04)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.step(10)
    compare(ctx, wl, x, u, w, sp, ids, F, 10, TOL[precision])


@pytest.mark.parametrize("mode,graph", [(0, False), (1, False), (2, True), (0, True)])
def test_global_path_in_every_launch_mode(mode, graph):
    # the particles the tile kernel leaves to the global-path kernel (its
    # list is filled by every launch of the tile kernel in the step and
    # emptied by the global kernel) match the oracle in every launch mode,
    # eager and replayed, across several steps
    wl = quad_workload(4, u_th=0.6, seed=9)
    print(f"[parity] global path mode={mode} graph={graph}", flush=True)
    ctx = make_ctx(wl, load=False)
    ctx.set_tuning(sort_interval=1000)
    ctx.set_launch_mode(mode, graph)
    F0 = picsynth.random_fields(wl.n, 3, amp=0.02)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.slow_path_count()
    ctx.step(8)
    n_slow = ctx.slow_path_count()
    assert 0 < n_slow < 8 * len(ids)
    compare(ctx, wl, x, u, w, sp, ids, F, 8, TOL[4])


@pytest.mark.parametrize("precision,order", [(8, 2), (4, 2), (8, 1), (4, 3)])
def test_unstaged_reference_path(precision, order):
    # no LDS windows: every particle gathers from and deposits into the
    # global arrays; the same oracle bar applies
    wl = quad_workload(precision, seed=17)
    wl.order = order
    print(f"[parity] unstaged precision={precision} order={order}", flush=True)
    ctx = make_ctx(wl, load=False)
    ctx.set_staging(False)
    F0 = picsynth.random_fields(wl.n, 5, amp=0.03)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.slow_path_count()
    ctx.step(6)
    assert ctx.slow_path_count() == 6 * len(ids)
    compare(ctx, wl, x, u, w, sp, ids, F, 6, TOL[precision])


@pytest.mark.parametrize("precision", [8, 4])
def test_four_species_in_shared_waves(precision):
    # four species with different charge-to-mass ratios: the particle loop
    # runs over a tile's species together, so waves hold particles of
    # several species and each lane takes its own q/m
    n = (16, 8, 16)
    N0 = picsynth.N0_DEFAULT
    sp = [picsynth.Species("electrons", -1.0, 1.0, N0, ppc=3, region_lo=(0, 0, 2), region_hi=(16, 8, 14),
                           u_th=(0.03,) * 3),
          picsynth.Species("positrons", 1.0, 1.0, N0, ppc=2, region_lo=(0, 0, 4), region_hi=(16, 8, 12),
                           u_th=(0.03,) * 3, u_drift=(0.0, 0.0, 0.02)),
          picsynth.Species("protons", 1.0, 1836.0, N0, ppc=2, region_lo=(0, 0, 2), region_hi=(16, 8, 14),
                           u_th=(0.001,) * 3),
          picsynth.Species("alphas", 2.0, 7294.0, N0, ppc=1, region_lo=(0, 0, 6), region_hi=(16, 8, 10),
                           u_th=(0.001,) * 3)]
    wl = picsynth.Workload("four", n, picsynth.uniform_boxes(n, 8), sp, dt=0.5, order=2, precision=precision,
                           seed=23)
    print(f"[parity] four species precision={precision}", flush=True)
    ctx = make_ctx(wl, load=False)
    F0 = picsynth.random_fields(wl.n, 19, amp=0.04)
    x, u, w, ids, sp_, F = set_state(ctx, wl, F0)
    ctx.step(8)
    compare(ctx, wl, x, u, w, sp_, ids, F, 8, TOL[precision])


def test_sort_interval_and_tiles_do_not_change_results():
    wl = quad_workload(8, seed=12)
    res = []
    for tile, si, blk, rs in (((8, 8, 4), 1, 256, 1), ((4, 4, 4), 3, 384, 0), ((8, 4, 4), 50, 512, 1),
                              ((8, 8, 4), 7, 384, 0)):
        print(f"[parity] tile={tile} sort_interval={si} block={blk} run_sum={rs}", flush=True)
        ctx = make_ctx(wl, load=False)
        ctx.set_tuning(tile=tile, sort_interval=si, block=blk, run_sum=rs)
        F0 = picsynth.random_fields(wl.n, 6, amp=0.03)
        x, u, w, ids, sp, F = set_state(ctx, wl, F0)
        ctx.step(6)
        gx, _ = compare(ctx, wl, x, u, w, sp, ids, F, 6, TOL[8], check_fields=False)
        res.append(gx)
    for r in res[1:]:
        assert np.abs(min_image(r - res[0], wl.n)).max() < 1e-12
    # an 8x8x8 tile of double-precision quadratic windows needs more LDS than a CU has
    ctx = make_ctx(wl, load=False)
    pb = _pb()
    with pytest.raises(pb.PicError) as e:
        ctx.set_tuning(tile=(8, 8, 8))
    assert e.value.code == pb.PIC_EUNSUPPORTED


def test_wrap_edges_and_empty_species():
    # particles sitting on the periodic faces, moving out of the domain; a
    # second species with no particles at all
    wl = picsynth.small_workload(n=(16, 16, 16), box=8, order=2, ppc=1, seed=3,
                                 species=("electrons", "protons"), precision=8)
    ctx = make_ctx(wl, load=False)
    n = 16.0
    x = np.array([[0.0, 0.0, 0.0], [n - 1e-13, 5.5, 7.25], [3.5, n - 1e-12, 0.0], [15.999, 15.999, 15.999]])
    u = np.array([[-0.3, -0.2, -0.1], [0.2, 0.0, 0.0], [0.0, 0.4, -0.3], [0.5, 0.5, 0.5]])
    w = np.full(4, 0.1)
    ids = np.arange(4)
    ctx.set_particles(0, x, u, w, ids)
    ctx.set_particles(1, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.int64))
    F = picsynth.initial_fields(wl)
    ctx.set_fields(F)
    ctx.step(5)
    sp = np.zeros(4, np.int32)
    compare(ctx, wl, x, u, w, sp, ids, F, 5, TOL[8])
    gx, _, _, _ = gpu_particles(ctx, wl)
    assert ((gx >= 0) & (gx < n)).all()


@pytest.mark.parametrize("precision", [8, 4])
def test_box_counts_after_steps(precision):
    wl = quad_workload(precision, u_th=0.2, seed=17)
    ctx = make_ctx(wl, load=False)
    x, u, w, ids, sp, F = set_state(ctx, wl)
    ctx.step(10)
    got = ctx.box_counts()
    ox, ou, _ = oracle_steps(wl, x, u, w, sp, F, 10)
    want = oracle.box_counts(wl.boxes, ox, sp, len(wl.species))
    assert got.sum() == len(x)
    # the library's counts are those of its own particles' cells, exactly
    gx, _, gids, gsp = gpu_particles(ctx, wl)
    np.testing.assert_array_equal(got, oracle.box_counts(wl.boxes, gx, gsp, len(wl.species)))
    if precision == 8:
        np.testing.assert_array_equal(got, want)
        return
    # FP32: a particle may sit in another box than the oracle's only if the
    # oracle places it within 1e-5 of a box face; those particles are listed
    ox_, _, oids, osp = order_by_species_id(ox, ou, ids, sp)
    np.testing.assert_array_equal(gids, oids)
    differ = box_of(gx, wl.boxes) != box_of(ox_, wl.boxes)
    near = near_box_face(ox_, wl.boxes, wl.n, 1e-5)
    listed = [(int(s_), int(i)) for s_, i in zip(osp[differ], oids[differ])]
    print(f"particles in another box than the oracle's: {listed}; within 1e-5 of a box face: "
          f"{int(near.sum())}", flush=True)
    assert not (differ & ~near).any(), f"box mismatches away from box faces: {listed}"
    # the counts then differ exactly by those particles
    moved = np.zeros_like(got)
    np.add.at(moved, (box_of(gx, wl.boxes)[differ], gsp[differ]), 1)
    np.add.at(moved, (box_of(ox_, wl.boxes)[differ], osp[differ]), -1)
    np.testing.assert_array_equal(got - want, moved)


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("per_box", [False, True])
def test_device_loader_matches_generator(precision, per_box):
    # pic_init's on-device Philox loader against the host generator: a
    # loading region at fixed ppc, or a ppc per box (mixed box sizes)
    wl = quad_workload(precision, seed=77)
    if per_box:
        n = (32, 32, 32)
        boxes = []
        for bz in range(2):
            for by in range(2):
                for bx in range(2):
                    o = np.array([bx, by, bz]) * 16
                    if (bx + by + bz) % 2:
                        boxes.append([*o, *(o + 16)])
                    else:
                        for k in range(8):
                            q = o + 8 * np.array([k & 1, (k >> 1) & 1, k >> 2])
                            boxes.append([*q, *(q + 8)])
        boxes = np.array(boxes, dtype=np.int32)
        ppc = picsynth.lognormal_box_ppc(len(boxes), 41, cap=6)
        sp = [picsynth.Species("electrons", -1.0, 1.0, picsynth.N0_DEFAULT, box_ppc=ppc, u_th=(0.01,) * 3),
              picsynth.Species("protons", 1.0, 1836.0, picsynth.N0_DEFAULT, box_ppc=ppc[::-1].copy(),
                               u_th=(0.001,) * 3)]
        wl = picsynth.Workload("per-box", n, boxes, sp, dt=0.5, order=2, precision=precision, seed=78)
    ctx = make_ctx(wl, load=True)
    for s in range(2):
        gx, gu, gw, gi = ctx.get_particles(s)
        o = np.argsort(gi)
        gx, gu, gw, gi = gx[o], gu[o], gw[o], gi[o]
        hx, hu, hw, hi = picsynth.particles(wl, s)
        np.testing.assert_array_equal(gi, hi)
        np.testing.assert_array_equal(gx, hx)          # 24-bit offsets: exact in both precisions
        tol = 1e-14 if precision == 8 else 1e-7
        assert np.abs(gu - hu).max() <= tol * max(1e-300, np.abs(hu).max()) + (0 if s == 0 else 1e-30)
        np.testing.assert_allclose(gw, hw, rtol=1e-7 if precision == 4 else 0)


@pytest.mark.parametrize("mode", [2, 0])
def test_autotune_keeps_state_and_picks_a_valid_tuning(mode):
    # the autotuner's trial steps must leave the simulation untouched: a run
    # with an autotune in the middle still matches the oracle step for step
    wl = quad_workload(8, seed=31)
    ctx = make_ctx(wl, load=False)
    ctx.set_launch_mode(mode, False)
    F0 = picsynth.random_fields(wl.n, 5, amp=0.03)
    x, u, w, ids, sp, F = set_state(ctx, wl, F0)
    ctx.step(3)
    t, ms = ctx.autotune(2)
    assert ms > 0
    assert tuple(t.tile) in {(8, 4, 4), (4, 4, 4), (8, 8, 4), (8, 8, 8)}
    got = ctx.get_tuning()
    assert tuple(got.tile) == tuple(t.tile) and got.block == t.block
    ctx.step(4)
    compare(ctx, wl, x, u, w, sp, ids, F, 7, TOL[8])
    # a second context of the same workload reuses the cached choice
    ctx2 = make_ctx(wl, load=False)
    ctx2.set_launch_mode(mode, False)
    set_state(ctx2, wl, F0)
    t2, ms2 = ctx2.autotune(2)
    assert ms2 == -1.0 and tuple(t2.tile) == tuple(t.tile)


def test_particles_by_id_match_full_copy():
    pb = _pb()
    wl = quad_workload(4, seed=29)
    ctx = make_ctx(wl, load=True)
    ctx.step(2)
    gx, gu, gw, gi = ctx.get_particles(1)
    rng = np.random.default_rng(3)
    pick = rng.choice(len(gi), 300, replace=False)
    ids = np.concatenate([gi[pick], [10 ** 12]])       # the last id does not exist
    x, u, found = ctx.get_particles_by_id(1, ids)
    assert found[:-1].all() and not found[-1]
    np.testing.assert_array_equal(x[:-1], gx[pick])
    np.testing.assert_array_equal(u[:-1], gu[pick])
    with pytest.raises(pb.PicError):
        ctx.get_particles_by_id(1, np.array([gi[0], gi[0]]))


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("axis", [0, 2])
def test_packed_cell_limits(precision, axis):
    # the largest domains the packed cell index holds along x (2048 cells,
    # 11 bits) and z (1024, 10 bits): particles on the last cells cross the
    # periodic face and back, under random fields, with quadratic shapes
    n = [8, 8, 8]
    n[axis] = 2048 if axis == 0 else 1024
    lo = [0, 0, 0]
    lo[axis] = n[axis] - 6
    wl = picsynth.small_workload(n=tuple(n), box=8, order=2, ppc=2, seed=41, u_th=0.3,
                                 species=("electrons", "protons"), precision=precision, region_lo=tuple(lo),
                                 region_hi=tuple(n))
    ctx = make_ctx(wl, load=False)
    F = picsynth.random_fields(wl.n, 5, amp=0.02)
    x, u, w, ids, sp, F = set_state(ctx, wl, F)
    ctx.step(10)
    gx, _ = compare(ctx, wl, x, u, w, sp, ids, F, 10, TOL[precision])
    # some particles wrapped through the face
    assert (gx[:, axis] < 8).any() and (gx[:, axis] >= n[axis] - 8).any()


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_degenerate_offsets_and_velocities(precision, order):
    # particles at rest, on cell faces (offset 0), on the half-cell points
    # where the quadratic reference node changes (offset 1/2) and a rounding
    # step below the next face (1 - 2^-40, which FP32 stores as the next
    # cell's face), starting with no momentum, less than a rounding step of
    # displacement, or enough to cross those points
    wl = picsynth.small_workload(n=(16, 16, 16), box=8, order=order, ppc=1, seed=5,
                                 species=("electrons", "protons"), precision=precision)
    ctx = make_ctx(wl, load=False)
    rng = np.random.default_rng(12)
    offs = np.array([0.0, 0.5, 0.25, 1.0 - 2.0 ** -40])
    speeds = np.array([0.0, 1e-17, -1e-17, 1e-6, -1e-6, 0.05, -0.05])
    cells = rng.integers(0, 16, size=(len(offs) * len(speeds) * 3, 3))
    x, u = [], []
    k = 0
    for o in offs:
        for v in speeds:
            for d in range(3):
                pos = cells[k] + 0.5
                pos[d] = cells[k][d] + o
                vel = np.zeros(3)
                vel[d] = v
                x.append(pos); u.append(vel)
                k += 1
    x = np.array(x); u = np.array(u)
    w = np.full(len(x), 0.05)
    ids = np.arange(len(x))
    ctx.set_particles(0, x, u, w, ids)
    ctx.set_particles(1, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.int64))
    # fields present, so that the gather at these points matters
    F = picsynth.random_fields(wl.n, 9, amp=0.02)
    ctx.set_fields(F)
    ctx.step(4)
    sp = np.zeros(len(x), np.int32)
    compare(ctx, wl, x, u, w, sp, ids, F, 4, TOL[precision])
