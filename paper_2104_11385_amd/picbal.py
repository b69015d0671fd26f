"""Thin ctypes binding of libpicbal.so (the C ABI in include/picbal.h).

Argument marshalling only: every step of the PIC path runs in the library's
HIP kernels.  The binding refuses to load anything else -- if the built
library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpicbal.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ECFL, PIC_ECAPACITY, PIC_ESTATE, PIC_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
PIC_FP32, PIC_FP64 = 4, 8
PIC_COST_HEURISTIC, PIC_COST_DEVICE_TIMER, PIC_COST_DEVICE_RTC, PIC_COST_LEARNED = 0, 1, 2, 3
LB_SFC, LB_KNAPSACK = 0, 1
PIC_LAUNCH_PER_BOX, PIC_LAUNCH_BATCHED, PIC_LAUNCH_PERSISTENT = 0, 1, 2

i32, i64, u64, f64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_float
P = ctypes.c_void_p


class pic_box(ctypes.Structure):
    _fields_ = [("lo", i32 * 3), ("hi", i32 * 3)]


class pic_grid_desc(ctypes.Structure):
    _fields_ = [("n_cells", i32 * 3), ("dt", f64), ("shape_order", i32), ("precision", i32),
                ("seed", u64), ("w_particle", f64), ("w_cell", f64), ("b_ext", f64 * 3)]


class pic_species_desc(ctypes.Structure):
    _fields_ = [("charge", f64), ("mass", f64), ("density", f64), ("load_mode", i32), ("ppc", i32),
                ("box_ppc", P), ("region_lo", i32 * 3), ("region_hi", i32 * 3),
                ("u_th", f64 * 3), ("u_drift", f64 * 3), ("capacity", i64)]


class pic_tuning(ctypes.Structure):
    _fields_ = [("tile", i32 * 3), ("halo", i32), ("block", i32), ("chunk", i32),
                ("sort_interval", i32), ("blocks_per_cu", i32), ("run_sum", i32), ("field_overlap", i32)]

    def as_dict(self):
        return {"tile": list(self.tile), "halo": self.halo, "block": self.block, "chunk": self.chunk,
                "sort_interval": self.sort_interval, "blocks_per_cu": self.blocks_per_cu,
                "run_sum": self.run_sum, "field_overlap": self.field_overlap}


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Loads the in-tree libpicbal.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2104_11385_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "pic_init": (ctypes.c_int, [P, P, i32, P, i32, P, P]),
            "pic_finalize": (None, [P]),
            "pic_step": (ctypes.c_int, [P, i32]),
            "pic_sync": (ctypes.c_int, [P]),
            "pic_set_launch_mode": (ctypes.c_int, [P, i32, i32]),
            "pic_get_tuning": (ctypes.c_int, [P, P]),
            "pic_set_tuning": (ctypes.c_int, [P, P]),
            "pic_autotune": (ctypes.c_int, [P, i32, P, P]),
            "pic_box_costs": (ctypes.c_int, [P, i32, P, P]),
            "pic_reset_costs": (ctypes.c_int, [P]),
            "pic_box_counts": (ctypes.c_int, [P, P]),
            "pic_get_particles": (ctypes.c_int, [P, i32, P, P, P, P, P]),
            "pic_set_particles": (ctypes.c_int, [P, i32, P, P, P, P, i64]),
            "pic_get_field": (ctypes.c_int, [P, i32, P]),
            "pic_set_field": (ctypes.c_int, [P, i32, P]),
            "lb_distribute": (ctypes.c_int, [P, P, i32, i32, i32, P, P]),
            "lb_efficiency": (f64, [P, P, i32, i32]),
            "lb_should_adopt": (ctypes.c_int, [f64, f64, f64]),
            "lb_morton_key": (u64, [ctypes.c_uint32] * 3),
            "lb_comm_volume": (ctypes.c_int, [P, i32, P, P, i32, f64, P, P]),
            "pic_box_features": (ctypes.c_int, [P, P]),
            "pic_mlp_nparam": (i32, []),
            "pic_mlp_train": (ctypes.c_int, [P, P, P, i64, i32, i32, P, P, u64, P]),
            "pic_mlp_predict": (ctypes.c_int, [P, P, i64, P]),
            "pic_mlp_loss_grad": (ctypes.c_int, [P, P, P, i64, P, P]),
            "pic_mlp_set_weights": (ctypes.c_int, [P, P, i64]),
            "pic_mlp_get_weights": (ctypes.c_int, [P, P, i64]),
            "pic_set_cost_timer": (ctypes.c_int, [P, i32]),
            "pic_set_staging": (ctypes.c_int, [P, i32]),
            "pic_get_particles_by_id": (ctypes.c_int, [P, i32, P, i64, P, P, P]),
            "pic_get_particles_by_id_noalloc": (ctypes.c_int, [P, i32, P, i64, P, P, P]),
            "pic_kernel_timing": (ctypes.c_int, [P, i32]),
            "pic_kernel_times": (ctypes.c_int, [P, P, P]),
            "pic_slow_path_count": (ctypes.c_int, [P, P]),
            "pic_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "pic_last_error": (ctypes.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return ["pic_init", "pic_finalize", "pic_step", "pic_sync", "pic_set_launch_mode", "pic_get_tuning",
            "pic_set_tuning", "pic_autotune", "pic_box_costs", "pic_reset_costs", "pic_box_counts",
            "pic_get_particles", "pic_set_particles", "pic_get_field", "pic_set_field", "lb_distribute",
            "lb_efficiency", "lb_should_adopt", "lb_morton_key", "lb_comm_volume", "pic_box_features", "pic_mlp_nparam",
            "pic_mlp_train", "pic_mlp_predict", "pic_mlp_loss_grad", "pic_mlp_set_weights",
            "pic_mlp_get_weights", "pic_set_cost_timer", "pic_set_staging", "pic_get_particles_by_id", "pic_get_particles_by_id_noalloc", "pic_kernel_timing", "pic_kernel_times", "pic_slow_path_count",
            "pic_strerror", "pic_last_error"]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(P)


def _check(rc, ctx=None):
    if rc != PIC_OK:
        L = lib()
        msg = L.pic_last_error(ctx)
        msg = msg.decode() if msg else ""
        raise PicError(rc, f"{L.pic_strerror(rc).decode()}: {msg}")
    return rc


def boxes_array(boxes) -> ctypes.Array:
    # pic_box is six int32 (lo[3], hi[3]): a C-contiguous [n, 6] int32 array
    # has the same layout, so the ctypes array is a view of a private copy
    boxes = np.array(boxes, dtype=np.int32, order="C", copy=True).reshape(-1, 6)
    assert ctypes.sizeof(pic_box) == 24
    return (pic_box * len(boxes)).from_buffer(boxes)


# ---------------------------------------------------------------------------
# load balancing (pure host functions)
# ---------------------------------------------------------------------------

def lb_distribute(costs, boxes, n_ranks: int, policy: int):
    """Returns (rank_of_box int32[n_boxes], efficiency)."""
    costs = np.ascontiguousarray(costs, dtype=np.float64)
    barr = boxes_array(boxes)
    rank = np.zeros(len(costs), dtype=np.int32)
    eff = f64(0.0)
    _check(lib().lb_distribute(_ptr(costs), ctypes.cast(barr, P), len(costs), int(n_ranks), int(policy),
                               _ptr(rank), ctypes.byref(eff)))
    return rank, eff.value


def lb_efficiency(costs, rank_of_box, n_ranks: int) -> float:
    costs = np.ascontiguousarray(costs, dtype=np.float64)
    rank = np.ascontiguousarray(rank_of_box, dtype=np.int32)
    return lib().lb_efficiency(_ptr(costs), _ptr(rank), len(costs), int(n_ranks))


def lb_should_adopt(e_current: float, e_proposed: float, threshold: float = 0.10) -> bool:
    return bool(lib().lb_should_adopt(float(e_current), float(e_proposed), float(threshold)))


def lb_morton_key(x: int, y: int, z: int) -> int:
    return int(lib().lb_morton_key(int(x), int(y), int(z)))


def lb_comm_volume(boxes, n_cells, rank_of_box, n_ranks: int, bytes_per_face_cell: float = 1.0):
    """Returns (per-rank halo bytes, total) of a mapping."""
    barr = boxes_array(boxes)
    n = np.ascontiguousarray(n_cells, dtype=np.int32)
    rank = np.ascontiguousarray(rank_of_box, dtype=np.int32)
    per = np.zeros(int(n_ranks))
    tot = f64(0.0)
    _check(lib().lb_comm_volume(ctypes.cast(barr, P), len(barr), _ptr(n), _ptr(rank), int(n_ranks),
                                float(bytes_per_face_cell), _ptr(per), ctypes.byref(tot)))
    return per, tot.value


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

class Species:
    """Host description of a species for pic_init (see pic_species_desc)."""

    def __init__(self, charge, mass, density, load_mode=1, ppc=0, box_ppc=None, region_lo=(0, 0, 0),
                 region_hi=None, u_th=(0.0, 0.0, 0.0), u_drift=(0.0, 0.0, 0.0), capacity=0):
        self.charge, self.mass, self.density = float(charge), float(mass), float(density)
        self.load_mode, self.ppc = int(load_mode), int(ppc)
        self.box_ppc = None if box_ppc is None else np.ascontiguousarray(box_ppc, dtype=np.int32)
        self.region_lo, self.region_hi = tuple(region_lo), region_hi
        self.u_th, self.u_drift, self.capacity = tuple(u_th), tuple(u_drift), int(capacity)


def pic_init(n_cells: Sequence[int], boxes, species: Sequence[Species], dt: float, shape_order: int,
             precision: int, seed: int, w_particle=0.75, w_cell=0.25, b_ext=(0.0, 0.0, 0.0),
             stream: Optional[int] = None) -> "PicContext":
    g = pic_grid_desc()
    g.n_cells[:] = [int(v) for v in n_cells]
    g.dt, g.shape_order, g.precision, g.seed = float(dt), int(shape_order), int(precision), int(seed)
    g.w_particle, g.w_cell = float(w_particle), float(w_cell)
    g.b_ext[:] = [float(v) for v in b_ext]
    barr = boxes_array(boxes)
    sarr = (pic_species_desc * len(species))()
    keep = []
    for s, sp in enumerate(species):
        d = sarr[s]
        d.charge, d.mass, d.density = sp.charge, sp.mass, sp.density
        d.load_mode, d.ppc = sp.load_mode, sp.ppc
        if sp.box_ppc is not None:
            keep.append(sp.box_ppc)
            d.box_ppc = sp.box_ppc.ctypes.data_as(P)
        d.region_lo[:] = [int(v) for v in sp.region_lo]
        d.region_hi[:] = [int(v) for v in (sp.region_hi if sp.region_hi is not None else n_cells)]
        d.u_th[:] = [float(v) for v in sp.u_th]
        d.u_drift[:] = [float(v) for v in sp.u_drift]
        d.capacity = sp.capacity
    out = P()
    rc = lib().pic_init(ctypes.byref(g), ctypes.cast(barr, P), len(barr), ctypes.cast(sarr, P), len(species),
                        P(stream) if stream else None, ctypes.byref(out))
    _check(rc, None)
    return PicContext(out, tuple(int(v) for v in n_cells), len(barr), len(species), precision)


class PicContext:
    def __init__(self, handle, n, n_boxes, n_species, precision):
        self.h = handle
        self.n = n
        self.n_boxes = n_boxes
        self.n_species = n_species
        self.precision = precision

    def __del__(self):
        self.finalize()

    def finalize(self):
        if getattr(self, "h", None):
            lib().pic_finalize(self.h)
            self.h = None

    def _c(self, rc):
        return _check(rc, self.h)

    def step(self, n=1):
        self._c(lib().pic_step(self.h, int(n)))

    def sync(self):
        self._c(lib().pic_sync(self.h))

    def set_launch_mode(self, mode, use_graph=False):
        self._c(lib().pic_set_launch_mode(self.h, int(mode), 1 if use_graph else 0))

    def get_tuning(self) -> pic_tuning:
        t = pic_tuning()
        self._c(lib().pic_get_tuning(self.h, ctypes.byref(t)))
        return t

    def set_tuning(self, t: pic_tuning = None, **kw):
        if t is None:
            t = self.get_tuning()
        for k, v in kw.items():
            if k == "tile":
                t.tile[:] = [int(x) for x in v]
            else:
                setattr(t, k, int(v))
        self._c(lib().pic_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, steps=3):
        t = pic_tuning()
        ms = f64(0.0)
        self._c(lib().pic_autotune(self.h, int(steps), ctypes.byref(t), ctypes.byref(ms)))
        return t, ms.value

    def box_costs(self, strategy):
        out = np.zeros(self.n_boxes)
        used = i32(-1)
        self._c(lib().pic_box_costs(self.h, int(strategy), _ptr(out), ctypes.byref(used)))
        return out, used.value

    def reset_costs(self):
        self._c(lib().pic_reset_costs(self.h))

    def box_counts(self):
        out = np.zeros((self.n_boxes, self.n_species), dtype=np.int64)
        self._c(lib().pic_box_counts(self.h, _ptr(out)))
        return out

    def get_particles(self, species):
        n = i64(0)
        rc = lib().pic_get_particles(self.h, int(species), None, None, None, None, ctypes.byref(n))
        if rc not in (PIC_OK, PIC_ECAPACITY):
            self._c(rc)
        m = n.value
        x = np.zeros((m, 3)); u = np.zeros((m, 3)); w = np.zeros(m); ids = np.zeros(m, dtype=np.int64)
        self._c(lib().pic_get_particles(self.h, int(species), _ptr(x), _ptr(u), _ptr(w), _ptr(ids),
                                        ctypes.byref(n)))
        return x, u, w, ids

    def set_particles(self, species, x, u, w, ids=None):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        w = np.ascontiguousarray(w, dtype=np.float64)
        ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
        self._c(lib().pic_set_particles(self.h, int(species), _ptr(x), _ptr(u), _ptr(w), _ptr(ids), len(w)))

    def get_field(self, comp):
        nx, ny, nz = self.n
        out = np.zeros((nz, ny, nx))
        self._c(lib().pic_get_field(self.h, int(comp), _ptr(out)))
        return out

    def get_fields(self):
        return np.stack([self.get_field(c) for c in range(9)])

    def set_field(self, comp, arr):
        nx, ny, nz = self.n
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(nz, ny, nx)
        self._c(lib().pic_set_field(self.h, int(comp), _ptr(a)))

    def set_fields(self, F):
        for c in range(9):
            self.set_field(c, F[c])

    def box_features(self):
        out = np.zeros((self.n_boxes, 16), dtype=np.float32)
        self._c(lib().pic_box_features(self.h, _ptr(out)))
        return out

    def set_cost_timer(self, enable=True):
        self._c(lib().pic_set_cost_timer(self.h, 1 if enable else 0))

    def get_particles_by_id(self, species, ids):
        """(x [n,3], u [n,3], found bool[n]) of the given ids of one species."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n = len(ids)
        x = np.zeros((n, 3)); u = np.zeros((n, 3)); found = np.zeros(n, dtype=np.int32)
        self._c(lib().pic_get_particles_by_id(self.h, int(species), _ptr(ids), n, _ptr(x), _ptr(u), _ptr(found)))
        return x, u, found.astype(bool)

    def get_particles_by_id_noalloc(self, species, ids):
        """As get_particles_by_id, through the entry point that allocates no
        device memory (at most 65,536 ids per call)."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n = len(ids)
        x = np.zeros((n, 3)); u = np.zeros((n, 3)); found = np.zeros(n, dtype=np.int32)
        self._c(lib().pic_get_particles_by_id_noalloc(self.h, int(species), _ptr(ids), n, _ptr(x), _ptr(u),
                                                      _ptr(found)))
        return x, u, found.astype(bool)

    def set_staging(self, enable=True):
        self._c(lib().pic_set_staging(self.h, 1 if enable else 0))

    def kernel_timing(self, enable=True):
        self._c(lib().pic_kernel_timing(self.h, 1 if enable else 0))

    def kernel_times(self):
        ms = np.zeros(4); n = np.zeros(4, dtype=np.int64)
        self._c(lib().pic_kernel_times(self.h, _ptr(ms), _ptr(n)))
        return ms, n

    def slow_path_count(self):
        c = i64(0)
        self._c(lib().pic_slow_path_count(self.h, ctypes.byref(c)))
        return c.value

    # learned cost model
    def mlp_train(self, X, y, epochs=30, batch=1024, perm=None, init_w=None, seed=0):
        X = np.ascontiguousarray(X, dtype=np.float32); y = np.ascontiguousarray(y, dtype=np.float32)
        perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        init_w = None if init_w is None else np.ascontiguousarray(init_w, dtype=np.float32)
        loss = np.zeros(epochs, dtype=np.float32)
        self._c(lib().pic_mlp_train(self.h, _ptr(X), _ptr(y), len(y), int(epochs), int(batch), _ptr(perm),
                                    _ptr(init_w), int(seed), _ptr(loss)))
        return loss

    def mlp_predict(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.zeros(len(X), dtype=np.float32)
        self._c(lib().pic_mlp_predict(self.h, _ptr(X), len(X), _ptr(out)))
        return out

    def mlp_loss_grad(self, X, y):
        X = np.ascontiguousarray(X, dtype=np.float32); y = np.ascontiguousarray(y, dtype=np.float32)
        loss = f32(0.0)
        grad = np.zeros(mlp_nparam(), dtype=np.float32)
        self._c(lib().pic_mlp_loss_grad(self.h, _ptr(X), _ptr(y), len(y), ctypes.byref(loss), _ptr(grad)))
        return loss.value, grad

    def mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._c(lib().pic_mlp_set_weights(self.h, _ptr(w), len(w)))

    def mlp_get_weights(self):
        w = np.zeros(mlp_nparam() + 37, dtype=np.float32)
        self._c(lib().pic_mlp_get_weights(self.h, _ptr(w), len(w)))
        return w


def mlp_nparam() -> int:
    return int(lib().pic_mlp_nparam())
