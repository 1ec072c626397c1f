"""npcf_accumulate_static (the entry point that allocates nothing) against
npcf_accumulate, through the C ABI: same estimator and pair counts on two
calls in a row (the second on a smaller catalogue, so stale contents of the
static workspace would show), with chunked primaries, and its rejections."""
import ctypes

import numpy as np
import pytest

from paper_2106_10278_amd import NPCF, binding, inputs
from npcf_testutil import condition_scale, conditioned_error, oracle_reported

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _both(plan, wl, static_first):
    pos, w = _dev(wl.pos), _dev(wl.w)
    out = {}
    order = ["static", "plain"] if static_first else ["plain", "static"]
    for kind in order:
        plan.reset()
        if kind == "static":
            plan.accumulate_static(pos, w)
        else:
            plan.accumulate(pos, w)
        out[kind] = (plan.finalize(), plan.pair_count()[0])
    return out


def test_static_matches_accumulate_on_two_calls():
    """Tiny 4PCF with mixed-sign weights, 300 points then 150: the static entry
    agrees with npcf_accumulate (pair counts bit for bit, per multipole within
    1e-6 of the sum of the magnitudes of the estimator's terms) and both agree
    with the FP64 oracle to the same bar."""
    plan = NPCF(3, 4, 3, inputs.tiny(3, 4, 3, 300, seed=2, box_side=16.0, rmax=4.5, nbins=4).edges,
                [16.0] * 3, max_points=400)
    for i, n in enumerate((300, 150)):
        wl = inputs.tiny(3, 4, 3, n, seed=2 + i, box_side=16.0, rmax=4.5, nbins=4)
        res = _both(plan, wl, static_first=(i == 0))
        ref, pairs, _ = oracle_reported(wl)
        sc = condition_scale(wl)
        zs, ps = res["static"]
        zp, pp = res["plain"]
        assert ps == pp == pairs
        err, _ = conditioned_error(zs, zp, sc)
        assert err <= 1e-6, (n, err)
        err_o, _ = conditioned_error(zs, ref, sc)
        assert err_o <= 1e-6, (n, err_o)
    plan.close()


def test_static_chunked_matches_accumulate():
    """60k then 30k uniform points (3PCF, lmax 4) with 4096-primary chunks on
    both entry points: the same kernels over the same chunks, so the outputs
    agree to rounding noise (the row hand-out order does not change any row)."""
    edges = np.linspace(2.0, 20.0, 9)
    plan = NPCF(3, 3, 4, edges, [100.0] * 3, max_points=60000)
    plan.set_tuning(chunk_rows=4096)
    rng = np.random.default_rng(7)
    for n in (60000, 30000):
        pos = inputs.to_lattice(rng.uniform(0, 100.0, size=(3, n)), [100.0] * 3)
        w = rng.uniform(0.5, 1.5, size=n)
        wl = type("W", (), {"pos": pos, "w": w})
        res = _both(plan, wl, static_first=True)
        zs, ps = res["static"]
        zp, pp = res["plain"]
        assert ps == pp > 0
        scale = np.max(np.abs(zp), axis=1, keepdims=True)
        assert np.max(np.abs(zs - zp) / scale) <= 1e-12, n
    plan.close()


def test_static_rejects_what_does_not_fit():
    """A catalogue beyond the 64 MiB workspace is refused before any launch,
    with the bytes it would need; the sphere geometry is refused."""
    n = 1_100_000
    plan = NPCF(3, 3, 2, [1.0, 2.0, 3.0], [1000.0] * 3, max_points=n)
    pos = _dev(np.zeros((3, n)))
    w = _dev(np.ones(n))
    with pytest.raises(binding.NPCFError) as e:
        plan.accumulate_static(pos, w)
    assert e.value.status == binding.NPCF_E_INVALID
    assert "static" in binding.load_library().npcf_last_error_detail().decode()
    plan.close()
    sph = NPCF(2, 3, 2, [0.2, 0.4, 0.6], [1.0, 1.0], max_points=100, sphere=True)
    with pytest.raises(binding.NPCFError) as e:
        sph.accumulate_static(_dev(np.tile(np.array([[0.0], [0.0], [1.0]]), (1, 10))), _dev(np.ones(10)))
    assert e.value.status == binding.NPCF_E_UNSUPPORTED
    sph.close()
