"""GPU parity of the estimator in hyperbolic space H^D (section
"Constant-Curvature Metric", curvature k = -1, chi(r) = sinh r) on the
hyperboloid of R^{D,1}: the all-pairs curved-space harmonic kernel with the
Minkowski product for the bins and the boost tangent frame, and the shared
D-dimensional coupling, against the FP64 oracle's hyperbolic geometry on the
same seeded points."""
import math

import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import (alm_error, condition_scale, conditioned_error, curved_plan, gpu_run, oracle_reported,
                           per_multipole_error, strict_where_well_conditioned)

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-6, "mixed_fp16": 1e-5, "mixed_bf16x6": 1e-5, "mixed_bf16": 5e-5}


def _ball_volume(D, R):
    return 2 * math.pi * (math.cosh(R) - 1) if D == 2 else math.pi * (math.sinh(2 * R) - 2 * R)


def _hyp_wl(D, N, lmax, n, seed, edges, R=1.5, weights="mixed"):
    rng = np.random.default_rng(seed)
    pos = inputs.hyperbolic_ball(rng, D, n, R)
    w = rng.uniform(-0.5, 1.5, size=n) if weights == "mixed" else np.ones(n)
    return inputs.Workload(f"h{D}-{N}-{lmax}-{n}", D, N, lmax, np.asarray(edges, dtype=np.float64),
                           [_ball_volume(D, R), 1.0, 1.0], pos, w, n, hyperbolic=True)


CASES = {
    "d3-n4-l5": (3, 4, 5, 500, np.linspace(0.2, 1.2, 6), 0),
    "d3-n4-l4-full": (3, 4, 4, 400, np.array([0.15, 0.45, 0.8, 1.3]), 1),
    "d3-n3-l3": (3, 3, 3, 600, np.array([0.1, 0.3, 0.6, 1.0, 1.5, 2.2, 2.9]), 0),
    "d2-n4-l4": (2, 4, 4, 500, np.linspace(0.15, 1.5, 6), 0),
    "d2-n3-l2-nb11": (2, 3, 2, 500, np.linspace(0.1, 2.6, 12), 1),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6", "mixed_fp16", "mixed_bf16"])
def test_hyp_parity(case, precision):
    D, N, lmax, n, edges, mode = CASES[case]
    wl = _hyp_wl(D, N, lmax, n, 500 + n + lmax + D, edges)
    print(f"[case] hyp {case} {precision}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl, btuple_mode=mode)
    got, pairs, plan = gpu_run(wl, precision=precision, btuple_mode=mode)
    assert np.array_equal(plan.lambda_labels, oracle.lambda_labels(D, N, lmax))
    assert pairs == pairs_ref
    scale = condition_scale(wl, mode)
    cerr, _ = conditioned_error(got, ref, scale)
    err, _ = per_multipole_error(got, ref)
    print(f"[err] hyp {case} {precision}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL[precision]


def _window_points(D, edges, rng):
    """Points at geodesic distance theta from the origin whose <origin, q> =
    cosh theta lies within 3e-7 and 1e-6 of cosh(edge), and the edge itself,
    in random directions (the FP64 product decides them)."""
    pts = []
    for e in edges:
        ce = math.cosh(e)
        for c in (ce, ce + 3e-7, ce - 3e-7, ce + 1e-6, ce - 1e-6, ce * (1 + 1e-12), ce * (1 - 1e-12)):
            th = math.acosh(max(c, 1.0))
            for _ in range(2):
                d = rng.normal(size=D)
                d /= np.linalg.norm(d)
                pts.append(np.concatenate([[math.cosh(th)], math.sinh(th) * d]))
    return np.array(pts).T


@pytest.mark.parametrize("width", ["wide", "narrow"])
@pytest.mark.parametrize("D", [2, 3])
def test_hyp_edge_windows(D, width):
    """Points planted at the bin edges' distances from the origin, within and
    beyond the FP32 guard band: pair counts exact and results as the
    oracle's.  11 bins take several passes, at both kernel widths (one bin
    per pass at the narrow one in H^3, which decides against the pass's two
    edges without the bucket table)."""
    rng = np.random.default_rng(91 + D)
    edges = np.linspace(0.2, 2.0, 12)
    planted = _window_points(D, edges, rng)
    origin = np.zeros((D + 1, 1))
    origin[0] = 1.0
    pos = np.concatenate([origin, planted, inputs.hyperbolic_ball(rng, D, 150, 1.5)], axis=1)
    n = pos.shape[1]
    wl = inputs.Workload(f"h{D}-windows", D, 4, 4 if D == 3 else 3, edges, [_ball_volume(D, 2.0), 1.0, 1.0], pos,
                         rng.uniform(0.5, 1.5, size=n), n, hyperbolic=True)
    print(f"[case] hyp edge windows D={D} n={n} {width}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl, plan=curved_plan(wl, width))
    assert pairs == pairs_ref
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    print(f"[err] hyp edge windows D={D} {width}: conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL["plain"]


def test_hyp_far_from_origin():
    """A catalogue about a point at distance 4 from the origin (x0 about 27,
    so the FP32 products carry errors 700 times those near the origin): the
    guard band grows with the largest x0 and the bins and pair counts stay
    exact."""
    rng = np.random.default_rng(93)
    local = inputs.hyperbolic_ball(rng, 3, 400, 1.2)
    c = np.array([math.cosh(4.0), math.sinh(4.0), 0.0, 0.0])
    pos = inputs._boost_to(c) @ local
    wl = inputs.Workload("h3-far", 3, 4, 3, np.linspace(0.2, 1.4, 6), [_ball_volume(3, 1.2), 1.0, 1.0], pos,
                         rng.uniform(-0.5, 1.5, size=400), 400, hyperbolic=True)
    print("[case] hyp far", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl)
    assert pairs == pairs_ref
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    print(f"[err] hyp far: conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL["plain"]


def test_hyp_alm_and_ranges():
    """The harmonic stage alone (npcf_alm in H^3) against the oracle's a^b_[l]
    in the same boost frame, value by value against its term-magnitude bound;
    primary ranges add up."""
    import torch
    from paper_2106_10278_amd import NPCF, stored_state_labels
    wl = _hyp_wl(3, 4, 5, 500, 9, np.array([0.2, 0.6, 1.1, 1.7]))
    print("[case] hyp alm", flush=True)
    plan = NPCF(3, 4, 5, wl.edges, wl.box, max_points=wl.pos.shape[1], hyperbolic=True)
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    got = plan.alm(pos, w, 20, 120)
    ref, _ = oracle.alm(3, 5, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(20, 120), hyperbolic=True)
    olab = [tuple(int(x) for x in r) for r in oracle.state_labels(3, 5)]
    ref = ref[:, :, [olab.index((int(s[0]), int(s[1]))) for s in stored_state_labels(3, 5)]]
    err = alm_error(got, ref, wl, np.arange(20, 120), 3, 5, hyperbolic=True)
    print(f"[err] hyp alm: {err:.3e} of each value's term-magnitude bound", flush=True)
    assert err <= 1e-6
    plan.close()
    whole, _, _ = gpu_run(wl)
    parts, _, _ = gpu_run(wl, ranges=[(0, 133), (133, 400), (400, 500)])
    cerr, _ = conditioned_error(parts, whole, condition_scale(wl))
    assert cerr <= 1e-6


def test_hyp_isometry_invariance():
    """A Lorentz transformation (rotation and boost, an isometry of H^3) of
    every point leaves the isotropic components unchanged: GPU results of the
    moved catalogue against the oracle's for the original one."""
    wl = _hyp_wl(3, 4, 3, 400, 31, np.array([0.3, 0.7, 1.2, 1.8]))
    rng = np.random.default_rng(32)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    Rt = np.eye(4)
    Rt[1:, 1:] = Q
    c = np.array([math.cosh(0.8), 0.0, math.sinh(0.8), 0.0])
    moved = inputs.Workload("h3-moved", 3, 4, 3, wl.edges, wl.box, inputs._boost_to(c) @ Rt @ wl.pos, wl.w,
                            wl.n_data, hyperbolic=True)
    print("[case] hyp isometry", flush=True)
    ref, _, _ = oracle_reported(wl)
    got, _, _ = gpu_run(moved)
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    print(f"[err] hyp moved vs original: conditioned {cerr:.3e}", flush=True)
    assert cerr <= 1e-5


def test_hyp_rejects():
    from paper_2106_10278_amd import NPCF, NPCFError
    e = np.array([0.2, 0.5, 1.0])
    with pytest.raises(NPCFError):
        NPCF(4, 3, 2, e, [1.0] * 4, max_points=50, hyperbolic=True)       # D = 2 or 3
    with pytest.raises(NPCFError):
        NPCF(3, 4, 6, e, [1.0] * 3, max_points=50, hyperbolic=True)       # lmax above 5
    with pytest.raises(NPCFError):
        NPCF(3, 3, 2, np.array([1e-6, 0.5]), [1.0] * 3, max_points=50, hyperbolic=True)   # cosh(e0) < 1 + 1e-9
    with pytest.raises(NPCFError):
        NPCF(3, 3, 2, e, [0.0, 1.0, 1.0], max_points=50, hyperbolic=True)  # V must be positive


@pytest.mark.parametrize("width", ["wide", "narrow"])
def test_h3_full_pair_count(width):
    """Every ordered pair of the 100k-point H^3 catalogue (1e10 visited), at
    both kernel widths: the number in the bins equals the FP64 oracle's count
    in tests/golden/h3_pairs.json, written by make_h3_pairs.py, exactly."""
    import json
    import os
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "h3_pairs.json")))
    wl = inputs.c11_h3_4pcf()
    assert gold["workload"] == wl.name and gold["n"] == wl.pos.shape[1]
    print(f"[case] h3 full pair count lmax=5 {width}", flush=True)
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).cuda()
    plan = curved_plan(wl, width)
    plan.accumulate(pos, w)
    assert plan.pair_count()[0] == gold["pairs"]


_C11 = {}


@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6", "plain-wide"])
def test_h3_full_sampled(precision):
    """The H^3 workload at full size (100k clustered points): 32 primaries
    against every point, against the oracle on the same primaries, per
    multipole: the conditioned measure on all of them, the strict one on
    every multipole whose terms cancel by at most a factor 3."""
    if "wl" not in _C11:
        wl = inputs.c11_h3_4pcf()
        prims = np.arange(0, 32)
        ref, pairs_ref, _ = oracle_reported(wl, prims=prims)
        _C11.update(wl=wl, ref=ref, pairs=pairs_ref, scale=condition_scale(wl, prims=prims))
    wl, ref, scale = _C11["wl"], _C11["ref"], _C11["scale"]
    print(f"[case] h3 full sampled {precision}", flush=True)
    if precision == "plain-wide":   # three bins per pass (the default is one)
        got, pairs, _ = gpu_run(wl, ranges=[(0, 32)], plan=curved_plan(wl, "wide"))
        precision = "plain"
    else:
        got, pairs, _ = gpu_run(wl, ranges=[(0, 32)], precision=precision)
    assert pairs == _C11["pairs"]
    err, _ = per_multipole_error(got, ref)
    cerr, _ = conditioned_error(got, ref, scale)
    serr, nwell, kappa = strict_where_well_conditioned(got, ref, scale, 3.0)
    print(f"[err] h3 full {precision}: strict {err:.3e} conditioned {cerr:.3e}; strict {serr:.3e} on {nwell} of "
          f"{len(kappa)} multipoles with kappa <= 3 (kappa max {kappa.max():.2f})", flush=True)
    assert cerr <= TOL[precision]
    assert nwell >= 1
    assert serr <= TOL[precision]
