"""GPU parity of the estimator on the unit 2-sphere (section "Cosmic Microwave
Background"): the all-pairs sphere harmonic kernel (great-circle bins, D = 2
harmonics in a tangent frame) and the shared D = 2 coupling, against the FP64
oracle's sphere geometry on the same seeded points."""
import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import condition_scale, conditioned_error, gpu_run, oracle_reported, per_multipole_error

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-6, "mixed_fp16": 1e-5, "mixed_bf16x6": 1e-5, "mixed_bf16": 5e-5}


def _sphere_wl(N, lmax, n, seed, edges, weights="mixed"):
    rng = np.random.default_rng(seed)
    pos = inputs.sphere_points(rng, n)
    w = rng.uniform(-0.5, 1.5, size=n) if weights == "mixed" else np.ones(n)
    return inputs.Workload(f"s2-{N}-{lmax}-{n}", 2, N, lmax, np.asarray(edges, dtype=np.float64), [1.0, 1.0], pos, w, n,
                           sphere=True)


CASES = {
    "n4-l4": (4, 4, 600, np.arccos(np.linspace(0.5, -0.5, 6)), 0),
    "n4-l3-full": (4, 3, 400, np.array([0.2, 0.5, 0.9, 1.4]), 1),
    "n3-l5": (3, 5, 700, np.array([0.1, 0.3, 0.6, 1.0, 1.5, 2.2, 3.1]), 0),
    "n4-l1-nb11": (4, 1, 500, np.linspace(0.15, 2.9, 12), 0),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6", "mixed_fp16", "mixed_bf16"])
def test_sphere_parity(case, precision):
    N, lmax, n, edges, mode = CASES[case]
    wl = _sphere_wl(N, lmax, n, 200 + n, edges)
    print(f"[case] sphere {case} {precision}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl, btuple_mode=mode)
    got, pairs, plan = gpu_run(wl, precision=precision, btuple_mode=mode)
    assert np.array_equal(plan.lambda_labels, oracle.lambda_labels(2, N, lmax))
    assert pairs == pairs_ref
    scale = condition_scale(wl, mode)
    cerr, _ = conditioned_error(got, ref, scale)
    err, _ = per_multipole_error(got, ref)
    print(f"[err] sphere {case} {precision}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL[precision]


def test_sphere_alm_and_ranges():
    """The harmonic stage alone (npcf_alm on the sphere) against the oracle's
    a_l in the same tangent frame; primary ranges add up."""
    import torch
    from paper_2106_10278_amd import NPCF
    wl = _sphere_wl(4, 4, 500, 7, np.array([0.3, 0.8, 1.4, 2.0]))
    print("[case] sphere alm", flush=True)
    plan = NPCF(2, 4, 4, wl.edges, wl.box, max_points=wl.pos.shape[1], sphere=True)
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    got = plan.alm(pos, w, 20, 120)
    ref, _ = oracle.alm(2, 4, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(20, 120), sphere=True)
    olab = [int(r[0]) for r in oracle.state_labels(2, 4)]
    ref = ref[:, :, [olab.index(l) for l in range(5)]]
    assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))
    plan.close()
    whole, _, _ = gpu_run(wl)
    parts, _, _ = gpu_run(wl, ranges=[(0, 133), (133, 400), (400, 500)])
    scale = condition_scale(wl)
    cerr, _ = conditioned_error(parts, whole, scale)
    assert cerr <= 1e-6


def test_sphere_rejects():
    from paper_2106_10278_amd import NPCF, NPCFError
    e = np.array([0.2, 0.5, 1.0])
    with pytest.raises(NPCFError):
        NPCF(3, 3, 2, e, [1.0] * 3, max_points=50, sphere=True)       # the sphere takes D = 2
    with pytest.raises(NPCFError):
        NPCF(2, 4, 6, e, [1.0] * 2, max_points=50, sphere=True)       # lmax above 5
    with pytest.raises(NPCFError):
        NPCF(2, 3, 2, np.array([0.5, 3.5]), [1.0] * 2, max_points=50, sphere=True)   # beyond pi


_C9 = {}


@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6"])
def test_c9_full_sphere_sampled(precision):
    """The sphere workload at full size (100k points, the paper's CMB test
    bins): 32 primaries against every point, against the oracle on the same
    primaries."""
    if "wl" not in _C9:
        wl = inputs.c9_sphere_4pcf()
        prims = np.arange(0, 32)
        ref, pairs_ref, _ = oracle_reported(wl, prims=prims)
        _C9.update(wl=wl, ref=ref, pairs=pairs_ref, scale=condition_scale(wl, prims=prims))
    wl, ref = _C9["wl"], _C9["ref"]
    print(f"[case] c9 sampled {precision}", flush=True)
    got, pairs, _ = gpu_run(wl, ranges=[(0, 32)], precision=precision)
    assert pairs == _C9["pairs"]
    err, _ = per_multipole_error(got, ref)
    cerr, _ = conditioned_error(got, ref, _C9["scale"])
    print(f"[err] c9 {precision}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL[precision]
