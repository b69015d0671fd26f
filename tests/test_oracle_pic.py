"""Pins of the FP64 oracle's PIC pieces against closed forms and invariants.

Nothing here compares the oracle with itself: each check is a property that
the published method fixes (B-spline moments, the Boris rotation angle, the
discrete continuity of Esirkepov's scheme, the Yee dispersion relation and
energy, Gauss's law), chosen so that a dropped term, a wrong sign, a wrong
stagger or a transposed index fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import picsynth


# --------------------------------------------------------------------------
# B-spline shapes
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 3])
def test_shape_moments(m):
    # For the centred B-spline of order m: sum_i S(x-i) = 1, sum_i i S(x-i) = x;
    # a spline of degree m reproduces polynomials up to degree m, so for m >= 2
    # sum_i (x-i)^2 S(x-i) is the constant (m+1)/12 (variance of m+1 unit
    # boxes), and for m = 3 the third moment vanishes.
    rng = np.random.default_rng(m)
    for x in rng.uniform(-3, 3, 200):
        g = oracle.first_node(m, x)
        nodes = np.arange(g, g + m + 1)
        s = np.array([oracle.shape(m, x - i) for i in nodes])
        assert abs(s.sum() - 1.0) < 1e-14
        assert abs((nodes * s).sum() - x) < 1e-13
        if m >= 2:
            assert abs((((x - nodes) ** 2) * s).sum() - (m + 1) / 12.0) < 1e-13
        if m == 3:
            assert abs((((x - nodes) ** 3) * s).sum()) < 1e-13
        if m == 1:
            f = x - g
            assert abs((((x - nodes) ** 2) * s).sum() - f * (1 - f)) < 1e-14
        # nodes outside the stencil carry no weight
        assert oracle.shape(m, x - (g - 1)) == 0.0
        assert oracle.shape(m, x - (g + m + 1)) == 0.0


def test_shape_values():
    assert oracle.shape(1, 0.25) == 0.75
    assert oracle.shape(2, 0.0) == 0.75
    assert oracle.shape(2, 0.5) == 0.5
    assert oracle.shape(2, 1.0) == 0.125
    assert abs(oracle.shape(3, 0.0) - 2.0 / 3.0) < 1e-16
    assert abs(oracle.shape(3, 1.0) - 1.0 / 6.0) < 1e-16
    assert oracle.shape(3, 2.0) == 0.0


# --------------------------------------------------------------------------
# Gather
# --------------------------------------------------------------------------

STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


@pytest.mark.parametrize("m", [1, 2, 3])
def test_gather_linear_field_at_stagger(m):
    # Component c stores a + (i+sx) + 10 (j+sy) + 100 (k+sz) at its Yee
    # location; splines of any order reproduce linear functions, so the gather
    # must return exactly a + x + 10 y + 100 z.  A wrong stagger shows as an
    # offset of 0.5, 5 or 50.
    n = np.array([16, 16, 16])
    k, j, i = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    F = np.zeros((9, 16, 16, 16))
    for c in range(6):
        F[c] = c + (i + STAG[c, 0]) + 10 * (j + STAG[c, 1]) + 100 * (k + STAG[c, 2])
    rng = np.random.default_rng(3)
    for x in rng.uniform(4, 11, (50, 3)):
        E, B = oracle.gather(m, n, F, x)
        want = x[0] + 10 * x[1] + 100 * x[2]
        np.testing.assert_allclose(np.r_[E, B], want + np.arange(6), rtol=0, atol=1e-11)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_gather_periodic_translation(m):
    # Gathering at x from F equals gathering at x + s (mod n) from F rolled by s.
    n = np.array([8, 10, 12])
    F = np.random.default_rng(5).normal(size=(9, 12, 10, 8))
    s = np.array([3, 7, 5])
    Fr = np.roll(F, shift=(s[2], s[1], s[0]), axis=(1, 2, 3))
    rng = np.random.default_rng(6)
    for x in rng.uniform(0, 1, (30, 3)) * n:
        E0, B0 = oracle.gather(m, n, F, x)
        E1, B1 = oracle.gather(m, n, Fr, (x + s) % n)
        np.testing.assert_allclose(np.r_[E0, B0], np.r_[E1, B1], rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# Boris push
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q,uperp,uz", [(-1.0, 0.01, 0.0), (1.0, 0.01, 0.003), (-1.0, 1.0, 0.5)])
def test_boris_gyration_closed_form(q, uperp, uz):
    # E = 0, B = B0 z: |u| and u_z are invariant and u_perp turns by
    # theta = 2 atan(q B0 dt / (2 m gamma)) per step, clockwise for q > 0.
    m, B0, dt = 1.0, 1.0, 0.5
    u = np.array([uperp, 0.0, uz])
    gam = math.sqrt(1 + u @ u)
    th = 2 * math.atan(q * B0 * dt / (2 * m * gam))
    for nstep in range(1, 1001):
        u = oracle.boris(q, m, dt, [0, 0, 0], [0, 0, B0], u)
    want = np.array([uperp * math.cos(nstep * th), -uperp * math.sin(nstep * th), uz])
    np.testing.assert_allclose(u, want, rtol=0, atol=1e-13 * max(1.0, uperp) * 10)


def test_boris_c1_angle():
    # electrons, B_z = 1, dt = 0.5, |u_perp| = 0.01: theta = 0.4899338 rad
    u = oracle.boris(-1.0, 1.0, 0.5, [0, 0, 0], [0, 0, 1.0], [0.01, 0, 0])
    th = math.atan2(u[1], u[0])
    assert abs(th - 0.4899338) < 1e-7


def test_boris_parallel_e_and_pure_e():
    # E parallel to B: u_z gains exactly q E dt / m per step.
    q, m, dt, E0 = -1.0, 2.0, 0.5, 0.03
    u = np.array([0.02, 0.01, 0.0])
    for _ in range(50):
        u = oracle.boris(q, m, dt, [0, 0, E0], [0, 0, 0.7], u)
    assert abs(u[2] - 50 * q * E0 * dt / m) < 1e-14
    # B = 0: u gains q E dt / m.
    u = oracle.boris(1.0, 1.0, 0.5, [0.1, -0.2, 0.3], [0, 0, 0], [0.0, 0.0, 0.0])
    np.testing.assert_allclose(u, [0.05, -0.1, 0.15], rtol=0, atol=1e-16)


def test_gyration_orbit_is_circle():
    # Single particle with zero weight in uniform B through the full step:
    # positions lie on a circle of radius R = (dt |u_perp| / gamma) / (2 sin(theta/2)).
    n = np.array([16, 16, 16])
    F = np.zeros((9, 16, 16, 16)); F[5] = 1.0
    x = np.array([[8.3, 7.9, 8.1]]); u = np.array([[0.3, 0.0, 0.0]])
    gam = math.sqrt(1 + 0.09)
    th = 2 * math.atan(0.5 / (2 * gam))
    R = (0.5 * 0.3 / gam) / (2 * math.sin(th / 2))
    pts = [x[0, :2].copy()]
    for _ in range(40):
        oracle.pic_step(1, n, 0.5, x, u, np.zeros(1), np.zeros(1, np.int32), [-1.0], [1.0], F, 1)
        pts.append(x[0, :2].copy())
    pts = np.array(pts)
    # centre from three points
    (x1, y1), (x2, y2), (x3, y3) = pts[0], pts[1], pts[2]
    d = 2 * (x1 * (y2 - y3) + x2 * (y3 - y1) + x3 * (y1 - y2))
    cx = ((x1**2 + y1**2) * (y2 - y3) + (x2**2 + y2**2) * (y3 - y1) + (x3**2 + y3**2) * (y1 - y2)) / d
    cy = ((x1**2 + y1**2) * (x3 - x2) + (x2**2 + y2**2) * (x1 - x3) + (x3**2 + y3**2) * (x2 - x1)) / d
    r = np.hypot(pts[:, 0] - cx, pts[:, 1] - cy)
    np.testing.assert_allclose(r, R, rtol=1e-10)
    assert np.all(F[6:] == 0.0)


# --------------------------------------------------------------------------
# Esirkepov deposition
# --------------------------------------------------------------------------

def _div_face(Jc, axis_np):
    # divergence contribution of a face-centred component: J[i] - J[i-1] along axis
    return Jc - np.roll(Jc, 1, axis=axis_np)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_esirkepov_continuity(m):
    # rho^{n+1} - rho^n + dt div J = 0 at every node, to 1e-12 of max |rho|,
    # including particles that cross the periodic boundary.
    n = np.array([10, 9, 8])
    rng = np.random.default_rng(10 + m)
    npart = 60
    x0 = rng.uniform(0, 1, (npart, 3)) * n
    x0[:10] = rng.uniform(-0.4, 0.4, (10, 3)) % n     # near the periodic faces
    dx = rng.uniform(-0.49, 0.49, (npart, 3))
    x1 = x0 + dx
    w = rng.uniform(0.5, 1.5, npart)
    sp = np.zeros(npart, np.int32)
    q = np.array([-1.3])
    dt = 0.45
    J = np.zeros((3, n[2], n[1], n[0]))
    for p in range(npart):
        oracle.deposit(m, n, q[0] * w[p], dt, x0[p], x1[p], J)
    r0 = oracle.rho(m, n, x0, w, sp, q)
    r1 = oracle.rho(m, n, x1 % n, w, sp, q)
    div = _div_face(J[0], 2) + _div_face(J[1], 1) + _div_face(J[2], 0)
    resid = np.abs(r1 - r0 + dt * div).max()
    assert resid <= 1e-12 * np.abs(r0).max()


@pytest.mark.parametrize("m", [1, 2, 3])
def test_esirkepov_total_current(m):
    # Summed over nodes, J_d dt / (q w) equals the displacement along d.
    n = np.array([12, 12, 12])
    rng = np.random.default_rng(20 + m)
    for _ in range(20):
        x0 = rng.uniform(2, 10, 3)
        x1 = x0 + rng.uniform(-0.49, 0.49, 3)
        qw, dt = -0.7, 0.5
        J = oracle.deposit(m, n, qw, dt, x0, x1)
        tot = J.reshape(3, -1).sum(axis=1) * dt / qw
        np.testing.assert_allclose(tot, x1 - x0, rtol=0, atol=1e-14)


def test_esirkepov_1d_motion_and_cic_face_current():
    # Motion along x only leaves Jy = Jz = 0 exactly; with CIC inside one cell
    # the x-face current is q w v times the transverse CIC weights.
    n = np.array([8, 8, 8])
    x0 = np.array([3.3, 4.25, 5.5]); x1 = np.array([3.45, 4.25, 5.5])
    qw, dt = 2.0, 0.5
    J = oracle.deposit(1, n, qw, dt, x0, x1)
    assert np.all(J[1] == 0.0) and np.all(J[2] == 0.0)
    v = (x1[0] - x0[0]) / dt
    # face between nodes 3 and 4 is Jx index 3; transverse weights at y=4.25, z=5.5
    wy = {4: 0.75, 5: 0.25}; wz = {5: 0.5, 6: 0.5}
    for j in range(8):
        for k in range(8):
            want = qw * v * wy.get(j, 0.0) * wz.get(k, 0.0)
            assert abs(J[0][k, j, 3] - want) < 1e-15
    assert np.abs(J[0]).sum() - abs(qw * v) < 1e-14


# --------------------------------------------------------------------------
# Yee solver
# --------------------------------------------------------------------------

@pytest.mark.parametrize("comp,axes", [(2, (0, 1)), (0, (1, 2)), (1, (2, 0))])
def test_yee_standing_mode_dispersion(comp, axes):
    # A standing TM mode E_c = cos(k_a i_a) cos(k_b i_b) (other fields 0) evolves
    # as E_c^n = E_c^0 cos(w n dt) with sin^2(w dt/2)/dt^2 = sum_d sin^2(k_d/2).
    n = np.array([16, 12, 10])
    dt = 0.5
    ka = 2 * math.pi * 2 / n[axes[0]]
    kb = 2 * math.pi * 1 / n[axes[1]]
    k_, j_, i_ = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    idx = [i_, j_, k_]
    # the field lives at integer positions along the two transverse axes (E_c is
    # staggered only along c), so cos(k i) samples the mode exactly
    F = np.zeros((9, n[2], n[1], n[0]))
    F[comp] = np.cos(ka * idx[axes[0]]) * np.cos(kb * idx[axes[1]])
    E0 = F[comp].copy()
    s2 = (math.sin(ka / 2) ** 2 + math.sin(kb / 2) ** 2) * dt * dt
    w = 2 * math.asin(math.sqrt(s2)) / dt
    nsteps = 57
    for _ in range(nsteps):
        oracle.yee(n, dt, F)
    np.testing.assert_allclose(F[comp], E0 * math.cos(w * nsteps * dt), rtol=0, atol=1e-12)


def _curlE(F):
    Ex, Ey, Ez = F[0], F[1], F[2]
    sh = lambda a, ax: np.roll(a, -1, axis=ax)  # a[i+1]
    cx = (sh(Ez, 1) - Ez) - (sh(Ey, 0) - Ey)
    cy = (sh(Ex, 0) - Ex) - (sh(Ez, 2) - Ez)
    cz = (sh(Ey, 2) - Ey) - (sh(Ex, 1) - Ex)
    return np.stack([cx, cy, cz])


def test_yee_energy_invariant():
    # In vacuum W = 1/2 sum(|E^n|^2 + |B^n|^2 - (dt/2)^2 |curl E^n|^2) is
    # conserved by the split-B leapfrog.
    n = np.array([10, 8, 6])
    dt = 0.5
    F = np.zeros((9, n[2], n[1], n[0]))
    F[:6] = np.random.default_rng(7).normal(size=(6, n[2], n[1], n[0]))

    def W(F):
        c = _curlE(F)
        return 0.5 * ((F[:6] ** 2).sum() - (dt / 2) ** 2 * (c ** 2).sum())

    W0 = W(F)
    for _ in range(200):
        oracle.yee(n, dt, F)
    assert abs(W(F) - W0) < 1e-11 * W0


def _div_node(F, off):
    # node divergence of a face-centred vector field F[off:off+3]
    return (F[off] - np.roll(F[off], 1, axis=2)) + (F[off + 1] - np.roll(F[off + 1], 1, axis=1)) + \
           (F[off + 2] - np.roll(F[off + 2], 1, axis=0))


def test_yee_div_b_preserved():
    # B lives on faces' duals; its discrete divergence at cell centres is
    # unchanged by B -= dt curl E.
    n = np.array([8, 8, 8])
    F = np.random.default_rng(8).normal(size=(9, 8, 8, 8))
    F[6:] = 0

    def divB(F):
        Bx, By, Bz = F[3], F[4], F[5]
        return (np.roll(Bx, -1, 2) - Bx) + (np.roll(By, -1, 1) - By) + (np.roll(Bz, -1, 0) - Bz)

    d0 = divB(F)
    for _ in range(30):
        oracle.yee(n, 0.5, F)
    np.testing.assert_allclose(divB(F), d0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_pic_step_gauss_law_preserved(m):
    # Full step: div E - rho stays at its initial value at every node, which
    # needs the deposit to conserve charge AND to sit on E's stagger.
    wl = picsynth.small_workload(n=(8, 8, 8), box=4, order=m, ppc=2, u_th=0.2, seed=31,
                                 species=("electrons", "protons"))
    x, u, w, ids, sp = picsynth.all_particles(wl)
    q = np.array([s.charge for s in wl.species]); mass = np.array([s.mass for s in wl.species])
    n = np.array(wl.n)
    F = picsynth.random_fields(wl.n, 3, amp=0.02)
    g0 = _div_node(F, 0) - oracle.rho(m, n, x, w, sp, q)
    for _ in range(5):
        oracle.pic_step(m, n, wl.dt, x, u, w, sp, q, mass, F, 1)
    g1 = _div_node(F, 0) - oracle.rho(m, n, x, w, sp, q)
    assert np.abs(g1 - g0).max() < 1e-12
    assert np.abs(F[6:]).max() > 0


def test_pic_step_wrap_rule():
    # A particle that ends a step a rounding distance below 0 lands at 0, not n.
    n = np.array([4, 4, 4])
    F = np.zeros((9, 4, 4, 4))
    x = np.array([[1e-17, 2.5, 2.5]]); u = np.array([[-0.01, 0.0, 0.0]])
    oracle.pic_step(1, n, 0.5, x, u, np.zeros(1), np.zeros(1, np.int32), [-1.0], [1.0], F, 1)
    assert 0.0 <= x[0, 0] < 4.0
    x = np.array([[0.0, 2.5, 2.5]]); u = np.array([[-1e-18, 0.0, 0.0]])
    oracle.pic_step(1, n, 0.5, x, u, np.zeros(1), np.zeros(1, np.int32), [-1.0], [1.0], F, 1)
    assert x[0, 0] == 0.0


# --------------------------------------------------------------------------
# Charge density (used as the reference in the Gauss-law checks)
# --------------------------------------------------------------------------

# 1D B-spline values at the nodes around a particle sitting exactly on node 0
_ON_NODE = {1: {0: 1.0}, 2: {-1: 0.125, 0: 0.75, 1: 0.125}, 3: {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}}


@pytest.mark.parametrize("m", [1, 2, 3])
def test_rho_of_a_particle_on_a_node(m):
    # the tensor product of the 1D node values, at the particle's node and
    # its neighbours, periodic through the domain's faces
    n = np.array([6, 6, 6])
    for node in ([2, 3, 4], [0, 5, 0]):
        x = np.array([node], dtype=float)
        r = oracle.rho(m, n, x, np.array([0.5]), np.array([0], np.int32), [-2.0])
        want = np.zeros((6, 6, 6))
        for dx, vx in _ON_NODE[m].items():
            for dy, vy in _ON_NODE[m].items():
                for dz, vz in _ON_NODE[m].items():
                    want[(node[2] + dz) % 6, (node[1] + dy) % 6, (node[0] + dx) % 6] += -1.0 * vx * vy * vz
        np.testing.assert_allclose(r, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_rho_total_charge_and_translation(m):
    # partition of unity: the nodes hold every particle's charge q w; moving
    # all particles by whole cells moves rho by the same cells
    rng = np.random.default_rng(7)
    n = np.array([8, 6, 10])
    x = rng.random((50, 3)) * n
    w = rng.random(50)
    sp = rng.integers(0, 2, 50).astype(np.int32)
    q = [-1.0, 3.0]
    r = oracle.rho(m, n, x, w, sp, q)
    assert abs(r.sum() - np.sum(np.array(q)[sp] * w)) < 1e-12
    shift = np.array([3, 1, 7])
    r2 = oracle.rho(m, n, (x + shift) % n, w, sp, q)
    np.testing.assert_allclose(r2, np.roll(r, (7, 1, 3), axis=(0, 1, 2)), rtol=0, atol=1e-13)
