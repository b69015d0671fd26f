"""The seeded input generator: Philox4x32-10 known answers and the loading
recipe's invariants."""
import numpy as np

import picsynth


def test_philox_known_answers():
    # Known-answer vectors of the published Philox4x32-10 definition.
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        out = picsynth.philox4x32_10(np.array([ctr[0]]), ctr[1], ctr[2], ctr[3], *key)
        assert tuple(int(o[0]) for o in out) == want


def test_loading_recipe_invariants():
    wl = picsynth.config("c1")
    x, u, w, ids = picsynth.particles(wl, 0)
    assert len(x) == 32 ** 3 * 2
    cell = np.floor(x).astype(int)
    # two particles per cell, every cell filled
    flat = cell[:, 0] + 32 * (cell[:, 1] + 32 * cell[:, 2])
    assert np.all(np.bincount(flat, minlength=32 ** 3) == 2)
    assert abs(u.std() - 0.01) < 2e-4 and abs(u.mean()) < 2e-4
    assert np.all(w == picsynth.N0_DEFAULT / 2)
    # sampling by index reproduces the full draw
    p = np.array([0, 17, 65535])
    xs, us, ws, _ = picsynth.particles(wl, 0, p)
    np.testing.assert_array_equal(xs, x[p]); np.testing.assert_array_equal(us, u[p])


def test_slab_and_box_table_layouts():
    wl = picsynth.config("c2")
    assert picsynth.species_count(wl, 0) == 256 * 256 * 26 * 8
    p = np.array([0, 256 * 256 * 26 * 8 - 1])
    c = picsynth.cell_of_index(wl, 0, p)
    np.testing.assert_array_equal(c, [[0, 0, 115], [255, 255, 140]])
    wl3 = picsynth.config("c3")
    b = wl3.boxes
    assert len(b) == 4096
    ext = b[:, 3:] - b[:, :3]
    assert (ext.prod(1)).sum() == 512 ** 3
    assert sorted(np.unique(ext[:, 0]).tolist()) == [16, 32, 64]
    ppc = wl3.species[0].box_ppc
    assert ppc.max() <= 64 and ppc.min() >= 0
