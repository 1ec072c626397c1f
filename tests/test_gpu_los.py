"""GPU parity of the line-of-sight 3PCF basis P^{0L}_{l1 l2} (D = 3, N = 3;
section "Large-Scale Structure"): the term-list coupling kernel against the
FP64 oracle on the same seeded inputs, per multipole, with the conditioned
measure (weights of both signs) and the tolerances of the isotropic tests."""
import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import condition_scale, conditioned_error, gpu_run, oracle_reported, per_multipole_error

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-6, "mixed_fp16": 1e-5, "mixed_bf16x6": 1e-5, "mixed_bf16": 5e-5}


def _stretched(n, seed, lmax, box=12.0, rmax=4.0, nbins=4):
    """Tiny catalogue made anisotropic along the line of sight: half the
    points come in pairs displaced along axis 3, so L > 0 components are
    non-zero."""
    wl = inputs.tiny(3, 3, lmax, n, seed, box_side=box, rmax=rmax, nbins=nbins)
    rng = np.random.default_rng(seed + 1000)
    pos = wl.pos.copy()
    h = n // 2
    pos[:, h:] = pos[:, :n - h]
    pos[2, h:] = np.mod(pos[2, h:] + rng.uniform(1.2 * wl.edges[0], 0.8 * rmax, size=n - h), box)
    pos = inputs.to_lattice(pos, wl.box)
    return inputs.Workload(wl.name + "-los", 3, 3, lmax, wl.edges, wl.box, pos, wl.w, n)


@pytest.mark.parametrize("Lmax", [0, 3, 8])
@pytest.mark.parametrize("precision", ["plain", "mixed_fp16", "mixed_bf16x6", "mixed_bf16"])
@pytest.mark.parametrize("mode", [0, 1])
def test_los_parity(Lmax, precision, mode):
    wl = _stretched(400, 21 + Lmax, lmax=4)
    print(f"[case] los Lmax={Lmax} {precision} mode={mode}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl, btuple_mode=mode, Lmax=Lmax)
    got, pairs, plan = gpu_run(wl, precision=precision, btuple_mode=mode, Lmax=Lmax)
    assert np.array_equal(plan.lambda_labels, oracle.lambda_labels(3, 3, 4, Lmax))
    assert pairs == pairs_ref
    scale = condition_scale(wl, mode, Lmax=Lmax)
    cerr, _ = conditioned_error(got, ref, scale)
    err, _ = per_multipole_error(got, ref)
    print(f"[err] los Lmax={Lmax} {precision} mode={mode}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL[precision]


def test_los_l0_matches_isotropic_path():
    """L = 0 components from the term-list kernel equal the isotropic N = 3
    kernel's l components (two different GPU coupling kernels)."""
    wl = _stretched(400, 5, lmax=5)
    print("[case] los L=0 vs isotropic", flush=True)
    los, _, plan = gpu_run(wl, Lmax=0)
    iso, _, _ = gpu_run(wl)
    lab = plan.lambda_labels
    assert np.all(lab[:, 0] == lab[:, 1]) and np.all(lab[:, 2] == 0)
    scale = condition_scale(wl)
    cerr, _ = conditioned_error(los, iso[lab[:, 0]], scale[lab[:, 0]])
    assert cerr <= 2e-6


def test_los_rejects_other_dimensions():
    from paper_2106_10278_amd import NPCF, NPCFError
    wl = inputs.tiny(3, 4, 2, 50, 3, box_side=12.0, rmax=4.0, nbins=3)
    with pytest.raises(NPCFError):
        NPCF(3, 4, 2, wl.edges, wl.box, max_points=50, Lmax=2)
    with pytest.raises(NPCFError):
        NPCF(3, 3, 2, wl.edges, wl.box, max_points=50, Lmax=5)   # Lmax > 2 lmax


_C6 = {}


@pytest.mark.parametrize("precision", ["plain", "mixed_fp16", "mixed_bf16x6"])
def test_c6_full_catalogue_sampled(precision):
    """The line-of-sight workload at full size (800k points, L <= 6): 48 data
    and 48 random primaries against every secondary, in the benchmark's launch
    configuration, against the oracle on the same primaries."""
    if "wl" not in _C6:
        wl = inputs.c6_los_3pcf()
        prims = np.concatenate([np.arange(0, 48), np.arange(wl.n_data, wl.n_data + 48)])
        ref, pairs_ref, _ = oracle_reported(wl, prims=prims, Lmax=wl.Lmax)
        scale = condition_scale(wl, prims=prims, Lmax=wl.Lmax)
        _C6.update(wl=wl, ref=ref, pairs=pairs_ref, scale=scale)
    wl, ref = _C6["wl"], _C6["ref"]
    print(f"[case] c6 sampled {precision}", flush=True)
    got, pairs, _ = gpu_run(wl, ranges=[(0, 48), (wl.n_data, wl.n_data + 48)], precision=precision, Lmax=wl.Lmax)
    assert pairs == _C6["pairs"]
    err, _ = per_multipole_error(got, ref)
    cerr, _ = conditioned_error(got, ref, _C6["scale"])
    print(f"[err] c6 {precision}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL[precision]
