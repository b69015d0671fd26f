"""The id lookup that allocates nothing (pic_get_particles_by_id_noalloc)
against the allocating lookup (pic_get_particles_by_id), bit for bit, on two
calls in a row (the second with fewer ids, so that stale contents of the
shared scratch would show), in both precisions; and its limits."""
import numpy as np
import pytest

import picsynth
from tests._util import make_ctx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [4, 8])
def test_noalloc_lookup_matches_allocating_lookup(precision):
    from paper_2104_11385_amd import picbal as pb
    wl = picsynth.small_workload(n=(32, 32, 32), box=16, order=2, ppc=4, seed=41, species=("electrons", "protons"),
                                 precision=precision, u_th=0.05)
    print(f"[noalloc] precision={precision}", flush=True)
    ctx = make_ctx(wl, load=True)
    try:
        ctx.step(3)
        rng = np.random.default_rng(precision)
        n_e = picsynth.species_count(wl, 0)
        for n, s in ((5000, 0), (700, 1)):
            ids = rng.choice(picsynth.species_count(wl, s), n, replace=False).astype(np.int64)
            ids[::97] = 10 ** 12 + np.arange(len(ids[::97]))     # ids that do not exist
            want = ctx.get_particles_by_id(s, ids)
            got = ctx.get_particles_by_id_noalloc(s, ids)
            for a, b in zip(got, want):
                np.testing.assert_array_equal(a, b)
            assert want[2].sum() == n - len(ids[::97])
        # the largest lookup, then a repeated id
        ids = np.arange(65536, dtype=np.int64) % n_e
        ids[n_e:] += 10 ** 12
        np.testing.assert_array_equal(ctx.get_particles_by_id_noalloc(0, ids)[0],
                                      ctx.get_particles_by_id(0, ids)[0])
        with pytest.raises(pb.PicError) as e:
            ctx.get_particles_by_id_noalloc(0, np.arange(65537, dtype=np.int64))
        assert e.value.code == pb.PIC_EINVAL
        with pytest.raises(pb.PicError) as e:
            ctx.get_particles_by_id_noalloc(0, np.array([3, 5, 3], dtype=np.int64))
        assert e.value.code == pb.PIC_EINVAL
        x, u, f = ctx.get_particles_by_id_noalloc(0, np.zeros(0, dtype=np.int64))
        assert len(f) == 0
    finally:
        ctx.finalize()
