"""The learned cost model on the GPU against the FP64 oracle's MLP in bf16
mirror mode (same roundings at the same points, double accumulation).

Tolerances: predictions 1e-2 and gradients 1e-3 relative to the largest
entry of each layer's parameter block (fp32 accumulation order and fp32 vs
double biases are the only differences left after mirroring).
"""
import numpy as np
import pytest

import oracle
import picsynth
from tests._util import make_ctx

pytestmark = pytest.mark.gpu

NP = oracle.NPARAM_MLP
BLOCKS = {"W1": (0, 1024), "b1": (1024, 1088), "W2": (1088, 5184), "b2": (5184, 5248), "W3": (5248, 5312),
          "b3": (5312, 5313)}


def _init(seed):
    rng = np.random.default_rng(seed)
    P = np.zeros(NP)
    o = 0
    for fi, fo in ((16, 64), (64, 64), (64, 1)):
        lim = np.sqrt(6.0 / fi)
        P[o:o + fi * fo] = rng.uniform(-lim, lim, fi * fo); o += fi * fo
        P[o:o + fo] = rng.uniform(-0.2, 0.2, fo); o += fo
    return P.astype(np.float32).astype(np.float64)


def _ctx():
    wl = picsynth.small_workload(n=(16, 16, 16), box=8, order=2, ppc=1, seed=2, species=("electrons",),
                                 precision=4)
    return make_ctx(wl, load=True)


def _identity_norm(P):
    return np.concatenate([P, np.zeros(16), np.ones(16)]).astype(np.float32)


@pytest.mark.parametrize("n", [16, 100, 1024])
def test_loss_and_gradient_match_mirror_oracle(n):
    ctx = _ctx()
    P = _init(n)
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 16)).astype(np.float32).astype(np.float64)
    y = rng.normal(size=n).astype(np.float32).astype(np.float64)
    ctx.mlp_set_weights(_identity_norm(P))
    loss, g = ctx.mlp_loss_grad(X, y)
    ol, og, _ = oracle.mlp_loss_grad(P, X, y, mirror=True)
    assert abs(loss - ol) <= 1e-3 * ol
    for name, (a, b) in BLOCKS.items():
        err = np.abs(g[a:b] - og[a:b]).max() / max(np.abs(og[a:b]).max(), 1e-30)
        assert err <= 1e-3, f"{name}: gradient error {err:.2e}"
    # the mirror roundings matter: the plain double model differs more
    _, pg, _ = oracle.mlp_loss_grad(P, X, y, mirror=False)
    assert np.abs(pg - og).max() > 0


def test_predictions_match_mirror_oracle():
    ctx = _ctx()
    P = _init(3)
    rng = np.random.default_rng(9)
    X = rng.normal(size=(333, 16))
    ctx.mlp_set_weights(_identity_norm(P))
    yh = ctx.mlp_predict(X)
    _, _, oy = oracle.mlp_loss_grad(P, X.astype(np.float32).astype(np.float64), np.zeros(333), mirror=True,
                                    want_grad=False)
    assert np.abs(yh - oy).max() <= 1e-2 * np.abs(oy).max()


def test_training_follows_oracle_adam_and_reduces_loss():
    ctx = _ctx()
    rng = np.random.default_rng(4)
    n, batch, epochs = 512, 128, 3
    X = rng.normal(size=(n, 16)).astype(np.float32)
    y = (np.log1p(3 * np.abs(X[:, 0])) + 0.5 * X[:, 1] ** 2).astype(np.float32)
    P0 = _init(5)
    perm = np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
    loss = ctx.mlp_train(X, y, epochs=epochs, batch=batch, perm=perm, init_w=P0.astype(np.float32))
    assert loss[-1] < loss[0]
    W = ctx.mlp_get_weights()
    mean, std = W[NP:NP + 16].astype(np.float64), W[NP + 16:NP + 32].astype(np.float64)
    rm, rs, rlo, rhi, flag = (float(v) for v in W[NP + 32:NP + 37])
    np.testing.assert_allclose(mean, X.astype(np.float64).mean(0), rtol=1e-5, atol=1e-6)
    # the network models the residual y - ln(1 + N), N from features 0 and 1
    base = np.log1p(np.maximum(0, np.expm1(X[:, 0].astype(np.float64))) +
                    np.maximum(0, np.expm1(X[:, 1].astype(np.float64))))
    res = y.astype(np.float64) - base
    assert flag == 1.0
    np.testing.assert_allclose([rm, rs, rlo, rhi], [res.mean(), res.std(), res.min(), res.max()], rtol=1e-5)
    # the oracle replays the same Adam steps on the standardised data and
    # standardised residuals
    Xs = ((X - mean.astype(np.float32)) * (1.0 / std.astype(np.float32))).astype(np.float32).astype(np.float64)
    Ys = ((res - rm) / rs).astype(np.float32).astype(np.float64)
    P = P0.copy(); m = np.zeros(NP); v = np.zeros(NP); t = 0
    for ep in range(epochs):
        for b0 in range(0, n, batch):
            idx = perm[ep, b0:b0 + batch]
            _, g, _ = oracle.mlp_loss_grad(P, Xs[idx], Ys[idx], mirror=True)
            t += 1
            oracle.adam(P, g, m, v, t)
    err = np.abs(W[:NP] - P).max() / np.abs(P).max()
    assert err < 2e-2, f"weights after training differ by {err:.2e}"
    # predictions come back in units of y
    _, _, oy = oracle.mlp_loss_grad(W[:NP].astype(np.float64), Xs[:64], np.zeros(64), mirror=True, want_grad=False)
    want = base[:64] + rm + rs * oy
    np.testing.assert_allclose(ctx.mlp_predict(X[:64]), want, rtol=0, atol=1e-2 * np.abs(want).max())


def test_constant_features_and_target_range():
    # trained where features 10 and 11 never vary, then shown boxes where
    # they do: those inputs enter as 0 (std 0), so predictions do not move,
    # and learned costs stay inside the training targets' range
    from paper_2104_11385_amd import picbal as pb
    ctx = _ctx()
    rng = np.random.default_rng(21)
    n = 2048
    X = rng.normal(size=(n, 16)).astype(np.float32)
    X[:, 10] = np.log(32.0 ** 3)
    X[:, 11] = 2.0
    y = (12.0 + 0.8 * X[:, 2] - 0.3 * X[:, 3]).astype(np.float32)
    ctx.mlp_train(X, y, epochs=5, batch=256, seed=3)
    W = ctx.mlp_get_weights()
    assert W[NP + 16 + 10] == 0.0 and W[NP + 16 + 11] == 0.0
    Xo = X[:100].copy()
    Xo[:, 10] = np.log(16.0 ** 3)
    Xo[:, 11] = 3.0
    np.testing.assert_array_equal(ctx.mlp_predict(Xo), ctx.mlp_predict(X[:100]))
    # the context's own boxes lie far outside these synthetic inputs: the
    # learned costs stay finite, the residual within its training range
    c, used = ctx.box_costs(pb.PIC_COST_LEARNED)
    assert used == pb.PIC_COST_LEARNED
    f = ctx.box_features().astype(np.float64)
    n_b = np.expm1(f[:, 0]) + np.expm1(f[:, 1])
    rlo, rhi = float(W[NP + 34]), float(W[NP + 35])
    assert np.isfinite(c).all() and (c >= 0).all()
    assert (c <= np.expm1(rhi + np.log1p(n_b)) * (1 + 1e-5)).all()
    assert (c >= np.expm1(rlo + np.log1p(n_b)) * (1 - 1e-5) - 1e-6).all()
    assert np.isfinite(ctx.mlp_predict(np.full((64, 16), 40.0, np.float32))).all()


def test_learned_costs_fall_back_when_error_exceeds_15_percent():
    from paper_2104_11385_amd import picbal as pb
    wl = picsynth.small_workload(n=(32, 32, 32), box=8, order=2, ppc=4, seed=6, species=("electrons",),
                                 precision=4, region_lo=(0, 0, 8), region_hi=(32, 32, 24), u_th=0.05)
    ctx = make_ctx(wl, load=True)
    # no model yet: heuristic
    c, used = ctx.box_costs(pb.PIC_COST_LEARNED)
    assert used == pb.PIC_COST_HEURISTIC
    # a deliberately wrong model: predicts ~e^20 cycles everywhere
    P = np.zeros(NP, np.float32); P[-1] = 20.0
    ctx.mlp_set_weights(np.concatenate([P, np.zeros(16, np.float32), np.ones(16, np.float32)]))
    ctx.step(5)
    ctx.box_costs(pb.PIC_COST_DEVICE_TIMER)            # measured interval 1
    c, used = ctx.box_costs(pb.PIC_COST_LEARNED)       # no prediction to judge yet
    assert used == pb.PIC_COST_LEARNED and np.allclose(c, np.exp(20.0), rtol=1e-5)
    ctx.reset_costs()
    ctx.step(5)
    ctx.box_costs(pb.PIC_COST_DEVICE_TIMER)            # measured interval 2
    c, used = ctx.box_costs(pb.PIC_COST_LEARNED)       # error >> 15%: fallback
    assert used == pb.PIC_COST_HEURISTIC
    h, _ = ctx.box_costs(pb.PIC_COST_HEURISTIC)
    np.testing.assert_array_equal(c, h)


@pytest.mark.parametrize("precision,box,ppc", [(8, 16, 3), (4, 8, 12), (4, 16, 1)])
def test_box_features_match_oracle(precision, box, ppc):
    # (4, 8, 12): 64 boxes, waves that lie in one box and waves that straddle
    # two; (4, 16, 1): more distinct cells per workgroup than its LDS table
    # of cell counts holds, so that the global-atomic path is taken too
    wl = picsynth.small_workload(n=(32, 32, 32), box=box, order=2, ppc=ppc, seed=8,
                                 species=("electrons", "protons"), precision=precision, region_lo=(0, 0, 10),
                                 region_hi=(32, 32, 20), u_th=0.1)
    ctx = make_ctx(wl, load=True)
    ctx.step(4)
    f = ctx.box_features()
    xs, us, sps = [], [], []
    for s in range(2):
        x, u, w, i = ctx.get_particles(s)
        xs.append(x); us.append(u); sps.append(np.full(len(w), s, np.int32))
    x = np.concatenate(xs); u = np.concatenate(us); sp = np.concatenate(sps)
    want = oracle.box_features(wl.n, wl.boxes, x, u, sp, 2, wl.order)
    np.testing.assert_allclose(f, want, rtol=2e-6, atol=1e-6)
