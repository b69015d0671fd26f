"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``picoracle.c`` -- a plain, slow, double-precision
implementation of the per-box PIC step (Yee-staggered B-spline gather,
relativistic Boris push, Esirkepov deposition, Yee update), the per-box
heuristic cost, Morton-curve and knapsack distribution mappings, the
load-balance efficiency of Eq. 1 and the learned cost model's MLP.  It shares
no code with the HIP library and never calls it.

Every function here is pinned by tests under ``tests/`` against closed forms,
invariants, brute force, hand-computed cases or the paper's worked example.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "picoracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NPARAM_MLP = 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def build(force: bool = False) -> str:
    """Compile picoracle.c with gcc (no FMA contraction) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_shape.restype = f64
        L.orc_shape.argtypes = [ctypes.c_int, f64]
        L.orc_first_node.restype = i64
        L.orc_first_node.argtypes = [ctypes.c_int, f64]
        L.orc_gather.argtypes = [ctypes.c_int, P, P, P, P]
        L.orc_boris.argtypes = [f64, f64, f64, P, P, P]
        L.orc_deposit.argtypes = [ctypes.c_int, P, f64, f64, P, P, P]
        L.orc_rho.argtypes = [ctypes.c_int, P, i64, P, P, P, P, P]
        L.orc_yee.argtypes = [P, f64, P]
        L.orc_pic_step.restype = ctypes.c_int
        L.orc_pic_step.argtypes = [ctypes.c_int, P, f64, i64, P, P, P, P, P, P, P, i32]
        L.orc_box_counts.restype = ctypes.c_int
        L.orc_box_counts.argtypes = [i32, P, i64, P, P, i32, P]
        L.orc_heuristic.argtypes = [i32, P, P, i32, f64, f64, P]
        L.orc_efficiency.restype = f64
        L.orc_efficiency.argtypes = [i32, P, P, i32]
        L.orc_should_adopt.restype = ctypes.c_int
        L.orc_should_adopt.argtypes = [f64, f64, f64]
        L.orc_morton3.restype = ctypes.c_uint64
        L.orc_morton3.argtypes = [ctypes.c_uint32] * 3
        L.orc_sfc.restype = ctypes.c_int
        L.orc_sfc.argtypes = [i32, P, P, i32, P, P]
        L.orc_knapsack.restype = ctypes.c_int
        L.orc_knapsack.argtypes = [i32, P, i32, P]
        L.orc_comm_volume.restype = ctypes.c_int
        L.orc_comm_volume.argtypes = [P, i32, P, P, i32, f64, P]
        L.orc_box_features.restype = ctypes.c_int
        L.orc_box_features.argtypes = [P, i32, P, i64, P, P, P, i32, i32, P]
        L.orc_mlp_nparam.restype = i32
        L.orc_bf16.restype = f64
        L.orc_bf16.argtypes = [f64]
        L.orc_mlp_loss_grad.restype = f64
        L.orc_mlp_loss_grad.argtypes = [P, P, P, i64, i32, P, P]
        L.orc_adam.argtypes = [P, P, P, P, i64, i64, f64, f64, f64, f64]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# --------------------------------------------------------------------------
# PIC pieces
# --------------------------------------------------------------------------

def shape(m: int, d: float) -> float:
    return lib().orc_shape(int(m), float(d))


def first_node(m: int, xi: float) -> int:
    return lib().orc_first_node(int(m), float(xi))


def gather(m, n, F, x):
    """Returns (E[3], B[3]) at position x from fields F[9, nz, ny, nx]."""
    n = _i64(n)
    F = _f64(F)
    x = _f64(x)
    out = np.zeros(6)
    lib().orc_gather(int(m), _p(n), _p(F), _p(x), _p(out))
    return out[:3].copy(), out[3:].copy()


def boris(q, mass, dt, E, B, u):
    u = _f64(u).copy()
    lib().orc_boris(float(q), float(mass), float(dt), _p(_f64(E)), _p(_f64(B)), _p(u))
    return u


def deposit(m, n, qw, dt, x0, x1, J=None):
    """Adds one particle's Esirkepov current into J[3, nz, ny, nx] (returned)."""
    n = _i64(n)
    if J is None:
        J = np.zeros((3, n[2], n[1], n[0]))
    else:
        J = _f64(J)
    lib().orc_deposit(int(m), _p(n), float(qw), float(dt), _p(_f64(x0)), _p(_f64(x1)), _p(J))
    return J


def rho(m, n, x, w, sp, q):
    n = _i64(n)
    x = _f64(x)
    out = np.zeros((n[2], n[1], n[0]))
    lib().orc_rho(int(m), _p(n), int(x.shape[0]), _p(x), _p(_f64(w)), _p(_i32(sp)), _p(_f64(q)), _p(out))
    return out


def yee(n, dt, F):
    """One Yee update of F[9, nz, ny, nx] in place (J read from F[6:9])."""
    n = _i64(n)
    assert F.dtype == np.float64 and F.flags.c_contiguous
    lib().orc_yee(_p(n), float(dt), _p(F))
    return F


def pic_step(m, n, dt, x, u, w, sp, q, mass, F, nsteps=1):
    """Advances particles (x, u modified in place) and fields F in place."""
    n = _i64(n)
    for a in (x, u, F):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    rc = lib().orc_pic_step(int(m), _p(n), float(dt), int(x.shape[0]), _p(x), _p(u),
                            _p(_f64(w)), _p(_i32(sp)), _p(_f64(q)), _p(_f64(mass)), _p(F),
                            int(nsteps))
    if rc != 0:
        raise ValueError("orc_pic_step rejected its arguments")


# --------------------------------------------------------------------------
# Load balancing
# --------------------------------------------------------------------------

def box_counts(boxes, x, sp, nsp):
    boxes = _i32(boxes).reshape(-1, 6)
    x = _f64(x)
    out = np.zeros((boxes.shape[0], nsp), dtype=np.int64)
    rc = lib().orc_box_counts(boxes.shape[0], _p(boxes), x.shape[0], _p(x), _p(_i32(sp)), int(nsp), _p(out))
    if rc != 0:
        raise ValueError("a particle lies in no box")
    return out


def heuristic(boxes, counts, wp=0.75, wc=0.25):
    boxes = _i32(boxes).reshape(-1, 6)
    counts = _i64(counts)
    out = np.zeros(boxes.shape[0])
    lib().orc_heuristic(boxes.shape[0], _p(boxes), _p(counts), counts.shape[1], float(wp), float(wc), _p(out))
    return out


def efficiency(costs, rank, R):
    costs = _f64(costs)
    return lib().orc_efficiency(costs.shape[0], _p(costs), _p(_i32(rank)), int(R))


def should_adopt(e_cur, e_new, thr=0.10):
    return bool(lib().orc_should_adopt(float(e_cur), float(e_new), float(thr)))


def morton3(X, Y, Z):
    return int(lib().orc_morton3(int(X), int(Y), int(Z)))


def sfc(boxes, costs, R):
    """Returns (rank_of_box, B*)."""
    boxes = _i32(boxes).reshape(-1, 6)
    costs = _f64(costs)
    rank = np.zeros(boxes.shape[0], dtype=np.int32)
    bstar = ctypes.c_double(0.0)
    rc = lib().orc_sfc(boxes.shape[0], _p(boxes), _p(costs), int(R), _p(rank), ctypes.byref(bstar))
    if rc != 0:
        raise ValueError("orc_sfc failed")
    return rank, bstar.value


def knapsack(costs, R):
    costs = _f64(costs)
    rank = np.zeros(costs.shape[0], dtype=np.int32)
    rc = lib().orc_knapsack(costs.shape[0], _p(costs), int(R), _p(rank))
    if rc != 0:
        raise ValueError("orc_knapsack failed")
    return rank


def comm_volume(n, boxes, rank, R, bytes_per_face_cell=1.0):
    """Per-rank halo bytes of a mapping (every cross-rank cell face)."""
    n = _i64(n)
    boxes = _i32(boxes).reshape(-1, 6)
    per = np.zeros(int(R))
    rc = lib().orc_comm_volume(_p(n), boxes.shape[0], _p(boxes), _p(_i32(rank)), int(R),
                               float(bytes_per_face_cell), _p(per))
    if rc != 0:
        raise ValueError("boxes do not cover the domain")
    return per


def box_features(n, boxes, x, u, sp, nsp, order):
    n = _i64(n)
    boxes = _i32(boxes).reshape(-1, 6)
    x = _f64(x)
    feat = np.zeros((boxes.shape[0], 16))
    rc = lib().orc_box_features(_p(n), boxes.shape[0], _p(boxes), x.shape[0], _p(x), _p(_f64(u)),
                                _p(_i32(sp)), int(nsp), int(order), _p(feat))
    if rc != 0:
        raise ValueError("a particle lies in no box")
    return feat


# --------------------------------------------------------------------------
# Learned cost model
# --------------------------------------------------------------------------

def bf16(v: float) -> float:
    return lib().orc_bf16(float(v))


def mlp_loss_grad(P, X, y, mirror=False, want_grad=True):
    """Returns (loss, grad or None, yhat)."""
    P = _f64(P)
    X = _f64(X)
    y = _f64(y)
    n = X.shape[0]
    grad = np.zeros(NPARAM_MLP) if want_grad else None
    yhat = np.zeros(n)
    loss = lib().orc_mlp_loss_grad(_p(P), _p(X), _p(y), n, 1 if mirror else 0, _p(grad), _p(yhat))
    return loss, grad, yhat


def adam(P, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    for a in (P, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(_p(P), _p(_f64(g)), _p(m), _p(v), P.shape[0], int(t), lr, beta1, beta2, eps)
