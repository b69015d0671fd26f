"""CPU-side checks of libpicbal: it loads, exports every symbol that
include/picbal.h declares, and its host load-balancing functions reproduce
the oracle's mappings bit for bit (no GPU needed)."""
import os
import re

import numpy as np
import pytest

import oracle
import picsynth
from paper_2104_11385_amd import picbal as pb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "picbal.h")).read()
    declared = set(re.findall(r"PIC_API\s+[\w\s\*]+?\b((?:pic|lb)_\w+)\s*\(", header))
    assert len(declared) >= 30
    L = pb.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(pb.exported_symbols())


def test_init_without_device_fails_cleanly():
    wl = picsynth.config("c1")
    from tests._util import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pb.PicError) as e:
        pb.pic_init(wl.n, wl.boxes, [pb.Species(-1, 1, 0.07, 1, 2)], 0.5, 1, pb.PIC_FP64, 1)
    assert e.value.code == pb.PIC_EDEVICE


def test_init_argument_errors():
    wl = picsynth.config("c1")
    sp = [pb.Species(-1, 1, 0.07, 1, 2)]
    with pytest.raises(pb.PicError) as e:
        pb.pic_init(wl.n, wl.boxes, sp, 0.6, 1, pb.PIC_FP64, 1)          # CFL
    assert e.value.code == pb.PIC_ECFL
    with pytest.raises(pb.PicError) as e:
        pb.pic_init(wl.n, wl.boxes, sp, 0.5, 4, pb.PIC_FP64, 1)          # no fourth-order shapes
    assert e.value.code == pb.PIC_EINVAL
    with pytest.raises(pb.PicError) as e:
        pb.pic_init(wl.n, wl.boxes, sp, 0.5, 1, 2, 1)                    # precision
    assert e.value.code == pb.PIC_EINVAL


def _tile16():
    return picsynth.uniform_boxes((32, 32, 32), 16)


def _sp(**kw):
    a = dict(charge=-1, mass=1, density=0.07, load_mode=1, ppc=2)
    a.update(kw)
    return pb.Species(**a)


_BAD_INIT = [
    # (description, n, boxes, species, expected code, message fragment)
    ("domain beyond the packed-cell x limit", (4096, 32, 32), [[0, 0, 0, 4096, 32, 32]], [_sp()],
     "EINVAL", "domain size"),
    ("domain beyond the packed-cell z limit", (32, 32, 2048), [[0, 0, 0, 32, 32, 2048]], [_sp()],
     "EINVAL", "domain size"),
    ("box past the domain", (32, 32, 32), [[0, 0, 0, 32, 32, 33]], [_sp()], "EINVAL", "outside"),
    ("empty box", (32, 32, 32), [[0, 0, 0, 32, 32, 32], [4, 4, 4, 4, 8, 8]], [_sp()], "EINVAL", "empty"),
    ("overlapping boxes", (32, 32, 32), [[0, 0, 0, 32, 32, 32], [0, 0, 0, 16, 16, 16]], [_sp()],
     "EINVAL", "overlap"),
    ("boxes with a gap", (32, 32, 32), None, [_sp()], "EINVAL", "gap"),
    ("five species", (32, 32, 32), "tile", [_sp()] * 5, "EINVAL", "species"),
    ("massless species", (32, 32, 32), "tile", [_sp(mass=0.0)], "EINVAL", "mass"),
    ("zero particles per cell", (32, 32, 32), "tile", [_sp(ppc=0)], "EINVAL", "ppc"),
    ("loading region past the domain", (32, 32, 32), "tile", [_sp(region_hi=(32, 32, 40))],
     "EINVAL", "loading region"),
    ("per-box counts missing", (32, 32, 32), "tile", [_sp(load_mode=2)], "EINVAL", "box_ppc"),
    ("negative per-box count", (32, 32, 32), "tile", [_sp(load_mode=2, box_ppc=[1, 1, -1, 1, 1, 1, 1, 1])],
     "EINVAL", "negative"),
    ("unknown load mode", (32, 32, 32), "tile", [_sp(load_mode=3)], "EINVAL", "load_mode"),
    ("more than 2^31-1 particles", (1024, 1024, 1024), [[0, 0, 0, 1024, 1024, 1024]], [_sp(ppc=3)],
     "EUNSUPPORTED", "2^31"),
]


@pytest.mark.parametrize("case", _BAD_INIT, ids=[c[0] for c in _BAD_INIT])
def test_init_rejects_bad_layouts_before_touching_a_device(case):
    # every one of these is refused on the host, so the status is the same
    # with or without a GPU
    _, n, boxes, species, code, frag = case
    if boxes == "tile":
        boxes = _tile16()
    elif boxes is None:
        boxes = _tile16()[1:]
    with pytest.raises(pb.PicError) as e:
        pb.pic_init(n, boxes, species, 0.5, 2, pb.PIC_FP32, 1)
    assert e.value.code == getattr(pb, "PIC_" + code), str(e.value)
    assert frag in str(e.value), str(e.value)


def test_lb_argument_errors():
    b = picsynth.uniform_boxes((32, 32, 32), 16)
    with pytest.raises(pb.PicError):
        pb.lb_distribute(np.array([1.0, -1.0] + [1.0] * 6), b, 4, pb.LB_KNAPSACK)
    with pytest.raises(pb.PicError):
        pb.lb_distribute(np.array([np.nan] + [1.0] * 7), b, 4, pb.LB_SFC)
    with pytest.raises(pb.PicError):
        pb.lb_distribute(np.ones(8), b, 0, pb.LB_SFC)
    assert pb.lb_efficiency(np.ones(8), np.zeros(8, np.int32), 0) == -1.0


def test_morton_matches_oracle():
    rng = np.random.default_rng(0)
    for X, Y, Z in rng.integers(0, 2 ** 21, (200, 3)):
        assert pb.lb_morton_key(X, Y, Z) == oracle.morton3(X, Y, Z)


@pytest.mark.parametrize("layout", ["c1", "c3", "c4"])
@pytest.mark.parametrize("R", [1, 3, 4, 96])
def test_lb_bit_exact_against_oracle(layout, R):
    wl = picsynth.config(layout) if layout != "c1" else picsynth.config("c1")
    boxes = wl.boxes
    rng = np.random.default_rng(R)
    for trial in range(3):
        if trial == 0:
            costs = rng.lognormal(1.0, 1.2, len(boxes))
        elif trial == 1:
            costs = np.round(rng.uniform(0, 5, len(boxes)))      # many ties
        else:
            costs = np.zeros(len(boxes)); costs[rng.integers(0, len(boxes), 5)] = 3.0
        for policy in (pb.LB_SFC, pb.LB_KNAPSACK):
            if policy == pb.LB_SFC and len(boxes) > 2000 and trial > 0:
                continue   # the oracle's O(n^2) candidate search is slow
            rank, e = pb.lb_distribute(costs, boxes, R, policy)
            if policy == pb.LB_SFC:
                want, _ = oracle.sfc(boxes, costs, R)
            else:
                want = oracle.knapsack(costs, R)
            np.testing.assert_array_equal(rank, want)
            assert e == oracle.efficiency(costs, want, R)


def test_threshold_matches_oracle():
    rng = np.random.default_rng(5)
    for a, b in rng.uniform(0, 1, (500, 2)):
        for t in (0.05, 0.10, 0.15):
            assert pb.lb_should_adopt(a, b, t) == oracle.should_adopt(a, b, t)
    assert pb.lb_should_adopt(0.5, 0.55, 0.10)


@pytest.mark.parametrize("layout,R", [("c1", 4), ("c1", 8), ("c4", 96)])
def test_comm_volume_matches_oracle(layout, R):
    wl = picsynth.config(layout)
    rng = np.random.default_rng(R)
    costs = rng.lognormal(0.0, 1.0, len(wl.boxes))
    for policy in (pb.LB_SFC, pb.LB_KNAPSACK):
        rank, _ = pb.lb_distribute(costs, wl.boxes, R, policy)
        per, tot = pb.lb_comm_volume(wl.boxes, wl.n, rank, R, 3.0)
        if np.prod(wl.n) <= 2 ** 20:
            want = oracle.comm_volume(wl.n, wl.boxes, rank, R, 3.0)
            np.testing.assert_array_equal(per, want)
        assert tot == per.sum()
    # everything on one rank: no traffic
    per, tot = pb.lb_comm_volume(wl.boxes, wl.n, np.zeros(len(wl.boxes), np.int32), R)
    assert tot == 0.0


def test_comm_volume_mixed_boxes_small():
    # mixed 8/16-cell boxes in a 32^3 domain against the oracle's cell walk
    boxes = []
    for K in range(2):
        for J in range(2):
            for I in range(2):
                o = np.array([I, J, K]) * 16
                if (I + J + K) % 2 == 0:
                    boxes.append([*o, *(o + 16)])
                else:
                    for dz in range(2):
                        for dy in range(2):
                            for dx in range(2):
                                q = o + np.array([dx, dy, dz]) * 8
                                boxes.append([*q, *(q + 8)])
    boxes = np.array(boxes, dtype=np.int32)
    rng = np.random.default_rng(3)
    rank = rng.integers(0, 5, len(boxes)).astype(np.int32)
    per, _ = pb.lb_comm_volume(boxes, (32, 32, 32), rank, 5, 2.0)
    np.testing.assert_array_equal(per, oracle.comm_volume((32, 32, 32), boxes, rank, 5, 2.0))


def _header_structs():
    """Field lists (type, name, count) of the header's typedef'd structs."""
    import re
    text = open(os.path.join(ROOT, "include", "picbal.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            m = re.match(r"((?:const )?[\w]+(?: \*)?)\s*(.*)", decl)
            ctype = m.group(1).replace(" *", "*")
            for item in m.group(2).split(","):
                item = item.strip()
                if item.startswith("*"):
                    ctype, item = ctype + "*", item[1:].strip()
                mm = re.match(r"(\w+)(?:\[(\d+)\])?", item)
                fields.append((ctype, mm.group(1), int(mm.group(2) or 1)))
        out[name] = fields
    return out


def test_binding_structs_match_the_header():
    # the ctypes structures of the binding list the header's fields in the
    # same order with the same widths, so the two agree on every offset
    import ctypes
    from paper_2104_11385_amd import picbal as pb
    width = {"int32_t": 4, "int64_t": 8, "uint64_t": 8, "double": 8, "float": 4}
    hs = _header_structs()
    for name in ("pic_box", "pic_grid_desc", "pic_species_desc", "pic_tuning"):
        cls = getattr(pb, name)
        got = [(f[0], ctypes.sizeof(f[1])) for f in cls._fields_]
        want = [(n, (8 if t.endswith("*") else width[t]) * k) for t, n, k in hs[name]]
        assert got == want, name
