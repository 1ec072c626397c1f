"""GPU parity of the estimator on the unit 3-sphere, the constant-curvature
space of section "Constant-Curvature Metric" with k = 1 (eq. metric,
chi(r) = sin r): the all-pairs sphere harmonic kernel at D = 3 (geodesic
bins, D = 3 harmonics of the tangent direction in the quaternion frame
p i, p j, p k) and the shared D = 3 coupling, against the FP64 oracle's
3-sphere geometry on the same seeded points."""
import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import (alm_error, condition_scale, conditioned_error, curved_plan, gpu_run, oracle_reported,
                           per_multipole_error, strict_where_well_conditioned)

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-6, "mixed_fp16": 1e-5, "mixed_bf16x6": 1e-5, "mixed_bf16": 5e-5}


def _s3_wl(N, lmax, n, seed, edges, weights="mixed"):
    rng = np.random.default_rng(seed)
    pos = inputs.s3_points(rng, n)
    w = rng.uniform(-0.5, 1.5, size=n) if weights == "mixed" else np.ones(n)
    return inputs.Workload(f"s3-{N}-{lmax}-{n}", 3, N, lmax, np.asarray(edges, dtype=np.float64), [1.0] * 3, pos, w,
                           n, sphere=True)


# at the default (narrow) width lmax 5 and 4 take one bin per pass, lmax 3 two,
# lmax 2 three and lmax 1 seven; test_gpu_curved_tuning.py covers the wide one
CASES = {
    "n4-l5": (4, 5, 500, np.linspace(0.3, 1.5, 6), 0),
    "n4-l4-full": (4, 4, 400, np.array([0.2, 0.6, 1.1, 1.7]), 1),
    "n3-l3": (3, 3, 600, np.array([0.1, 0.3, 0.6, 1.0, 1.5, 2.2, 3.1]), 0),
    "n4-l2-nb11": (4, 2, 400, np.linspace(0.15, 2.9, 12), 0),
    "n3-l1-nb11": (3, 1, 400, np.linspace(0.15, 3.1, 12), 1),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6", "mixed_fp16", "mixed_bf16"])
def test_s3_parity(case, precision):
    N, lmax, n, edges, mode = CASES[case]
    wl = _s3_wl(N, lmax, n, 300 + n + lmax, edges)
    print(f"[case] s3 {case} {precision}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl, btuple_mode=mode)
    got, pairs, plan = gpu_run(wl, precision=precision, btuple_mode=mode)
    assert np.array_equal(plan.lambda_labels, oracle.lambda_labels(3, N, lmax))
    assert pairs == pairs_ref
    scale = condition_scale(wl, mode)
    cerr, _ = conditioned_error(got, ref, scale)
    err, _ = per_multipole_error(got, ref)
    print(f"[err] s3 {case} {precision}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL[precision]


def _window_points(cos_edges, rng):
    """Points whose FP32 cosine to (1, 0, 0, 0) is the FP32 rounding of
    cos(edge) +- the guard, just beyond and just inside it, and points within
    3e-7 and 1e-6 of every edge cosine (decided by the FP64 dot product)."""
    g = np.float32(1e-6)
    zs = []
    for c in cos_edges:
        cf = np.float32(c)
        hi = np.float32(cf + g)
        if float(hi) - float(cf) > float(g):
            zs += [float(hi) - 1e-9, float(hi) - 5e-9]
        lo = np.float32(cf - g)
        if float(cf) - float(lo) > float(g):
            zs += [float(lo) + 1e-9, float(lo) + 5e-9]
        zs += [c + 1.0e-6, c - 1.0e-6, c + 3e-7, c - 3e-7, c]
    pts = []
    for z in zs:
        for _ in range(3):
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            r = np.sqrt(1.0 - z * z)
            pts.append((z, r * v[0], r * v[1], r * v[2]))
    return np.array(pts).T


@pytest.mark.parametrize("width", ["wide", "narrow"])
def test_s3_edge_rounding_windows(width):
    """Cosines within the FP32 guard of a bin edge are decided in FP64, and
    ones just beyond an outer edge of a pass are not admitted: pair counts and
    results match the oracle on points planted at every edge.  11 bins at
    lmax 4 take four passes of 3, 3, 3 and 2 bins at the wide width, eleven
    of one bin at the narrow one."""
    rng = np.random.default_rng(78)
    ce = np.array([0.5, 0.45, 0.4, 0.35, 0.3, 0.25, 0.2, 0.1, 0.0, -0.2, -0.4, -0.5])
    edges = np.arccos(ce)
    planted = _window_points(np.cos(edges), rng)
    pos = np.concatenate([np.array([[1.0], [0.0], [0.0], [0.0]]), planted, inputs.s3_points(rng, 150)], axis=1)
    n = pos.shape[1]
    wl = inputs.Workload("s3-windows", 3, 4, 4, edges, [1.0] * 3, pos, rng.uniform(0.5, 1.5, size=n), n, sphere=True)
    print(f"[case] s3 edge windows n={n} {width}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl, plan=curved_plan(wl, width))
    assert pairs == pairs_ref
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    print(f"[err] s3 edge windows plain {width}: conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL["plain"]


def test_s3_alm_and_ranges():
    """The harmonic stage alone (npcf_alm on the 3-sphere) against the
    oracle's a^b_[l] in the same quaternion frame, value by value against its
    term-magnitude bound; primary ranges add up."""
    import torch
    from paper_2106_10278_amd import NPCF, stored_state_labels
    wl = _s3_wl(4, 5, 500, 9, np.array([0.3, 0.8, 1.4, 2.0]))
    print("[case] s3 alm", flush=True)
    plan = NPCF(3, 4, 5, wl.edges, wl.box, max_points=wl.pos.shape[1], sphere=True)
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    got = plan.alm(pos, w, 20, 120)
    ref, _ = oracle.alm(3, 5, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(20, 120), sphere=True)
    olab = [tuple(int(x) for x in r) for r in oracle.state_labels(3, 5)]
    ref = ref[:, :, [olab.index((int(s[0]), int(s[1]))) for s in stored_state_labels(3, 5)]]
    err = alm_error(got, ref, wl, np.arange(20, 120), 3, 5, sphere=True)
    print(f"[err] s3 alm: {err:.3e} of each value's term-magnitude bound", flush=True)
    assert err <= 1e-6
    plan.close()
    whole, _, _ = gpu_run(wl)
    parts, _, _ = gpu_run(wl, ranges=[(0, 133), (133, 400), (400, 500)])
    cerr, _ = conditioned_error(parts, whole, condition_scale(wl))
    assert cerr <= 1e-6


def test_s3_rotation_invariance():
    """An SO(4) rotation of every point leaves the isotropic components
    unchanged (the frame turns with the points only up to a rotation of each
    tangent space): GPU results of the rotated catalogue against the oracle's
    for the original one."""
    wl = _s3_wl(4, 3, 400, 31, np.array([0.4, 0.9, 1.5, 2.2]))
    rng = np.random.default_rng(32)
    q, r = np.linalg.qr(rng.normal(size=(4, 4)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    rot = inputs.Workload("s3-rotated", 3, 4, 3, wl.edges, wl.box, q @ wl.pos, wl.w, wl.n_data, sphere=True)
    print("[case] s3 rotation", flush=True)
    ref, _, _ = oracle_reported(wl)
    got, _, _ = gpu_run(rot)
    # pair counts may differ where a rotated cosine crosses an edge by a rounding
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    print(f"[err] s3 rotated vs original: conditioned {cerr:.3e}", flush=True)
    assert cerr <= 1e-5


@pytest.mark.parametrize("width", ["wide", "narrow"])
def test_s3_full_pair_count(width):
    """Every ordered pair of the 100k-point 3-sphere catalogue (1e10 visited;
    four passes of up to three bins at lmax 5 at the wide width, ten of one
    at the narrow one, the autotuner's choice here): the number in the bins
    equals the FP64 oracle's count in tests/golden/s3_pairs.json, written by
    make_s3_pairs.py, exactly."""
    import json
    import os
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "s3_pairs.json")))
    wl = inputs.c10_s3_4pcf()
    assert gold["workload"] == wl.name and gold["n"] == wl.pos.shape[1]
    print(f"[case] s3 full pair count lmax=5 {width}", flush=True)
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).cuda()
    plan = curved_plan(wl, width)
    plan.accumulate(pos, w)
    assert plan.pair_count()[0] == gold["pairs"]


_C10 = {}


@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6", "plain-wide"])
def test_s3_full_sampled(precision):
    """The 3-sphere workload at full size (100k clustered points): 32
    primaries against every point, against the oracle on the same primaries,
    per multipole: the conditioned measure on all of them, the strict one on
    every multipole whose terms cancel by at most a factor 3
    (kappa = S / |zeta| <= 3; 30 of the 111 here: the isotropic 4PCF of
    increasing radial triples cancels strongly, kappa up to about 40)."""
    if "wl" not in _C10:
        wl = inputs.c10_s3_4pcf()
        prims = np.arange(0, 32)
        ref, pairs_ref, _ = oracle_reported(wl, prims=prims)
        _C10.update(wl=wl, ref=ref, pairs=pairs_ref, scale=condition_scale(wl, prims=prims))
    wl, ref, scale = _C10["wl"], _C10["ref"], _C10["scale"]
    print(f"[case] s3 full sampled {precision}", flush=True)
    if precision == "plain-wide":   # three bins per pass (the default is one)
        got, pairs, _ = gpu_run(wl, ranges=[(0, 32)], plan=curved_plan(wl, "wide"))
        precision = "plain"
    else:
        got, pairs, _ = gpu_run(wl, ranges=[(0, 32)], precision=precision)
    assert pairs == _C10["pairs"]
    err, _ = per_multipole_error(got, ref)
    cerr, _ = conditioned_error(got, ref, scale)
    serr, nwell, kappa = strict_where_well_conditioned(got, ref, scale, 3.0)
    print(f"[err] s3 full {precision}: strict {err:.3e} conditioned {cerr:.3e}; strict {serr:.3e} on {nwell} of "
          f"{len(kappa)} multipoles with kappa <= 3 (kappa max {kappa.max():.2f})", flush=True)
    assert cerr <= TOL[precision]
    assert nwell >= 25
    assert serr <= TOL[precision]
