"""GPU parity of the estimator on the unit 2-sphere (section "Cosmic Microwave
Background"): the all-pairs sphere harmonic kernel (great-circle bins, D = 2
harmonics in a tangent frame) and the shared D = 2 coupling, against the FP64
oracle's sphere geometry on the same seeded points."""
import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import (alm_error, condition_scale, conditioned_error, curved_plan, gpu_run, oracle_reported,
                           per_multipole_error)

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


def _window_points(cos_edges, rng):
    """Points whose FP32 cosine to (0, 0, 1) is the FP32 rounding of
    cos(edge) + 1e-6 where that lies beyond the guard of the edge (true cosine
    just beyond the edge), and mirror points just inside it."""
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
        zs += [c + 1.0e-6, c - 1.0e-6, c + 3e-7, c - 3e-7]
    pts = []
    for z in zs:
        for phi in rng.uniform(0.0, 2 * np.pi, 3):
            r = np.sqrt(1.0 - z * z)
            pts.append((r * np.cos(phi), r * np.sin(phi), z))
    return np.array(pts).T


@pytest.mark.parametrize("width", ["wide", "narrow"])
def test_sphere_edge_rounding_windows(width):
    """Cosines beyond an outer edge of a pass by more than the guard but no
    more than one FP32 rounding of (edge + guard): the FP32 range prefilter
    must not admit them without the FP64 decision (regression: such pairs
    were counted, twice at a boundary between passes).  11 bins at lmax 4
    take three passes of 5, 5 and 1 bins at the wide width, eleven of one
    at the narrow one."""
    rng = np.random.default_rng(77)
    ce = np.array([0.5, 0.45, 0.4, 0.35, 0.3, 0.25, 0.2, 0.1, 0.0, -0.2, -0.4, -0.5])
    edges = np.arccos(ce)
    planted = _window_points(np.cos(edges), rng)
    pos = np.concatenate([np.array([[0.0], [0.0], [1.0]]), planted, inputs.sphere_points(rng, 150)], axis=1)
    n = pos.shape[1]
    wl = inputs.Workload("s2-windows", 2, 4, 4, edges, [1.0, 1.0], pos, rng.uniform(0.5, 1.5, size=n), n, sphere=True)
    print(f"[case] sphere edge windows n={n} {width}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl, plan=curved_plan(wl, width))
    assert pairs == pairs_ref
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    print(f"[err] sphere edge windows plain {width}: conditioned {cerr:.3e}", flush=True)
    assert cerr <= TOL["plain"]


@pytest.mark.parametrize("width", ["wide", "narrow"])
@pytest.mark.parametrize("lmax", [1, 4, 5])
def test_c9_full_pair_count(lmax, width):
    """Every ordered pair of the 100k-point catalogue (1e10 visited): the
    number in the bins equals the FP64 oracle's count, stored in
    tests/golden/c9_sphere_pairs.json by make_c9_sphere_pairs.py, exactly.
    At the wide width lmax 1, 4 and 5 take the 10 bins in one, two and three
    passes; at the narrow one in five, ten and ten."""
    import json
    import os
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c9_sphere_pairs.json")))
    wl = inputs.c9_sphere_4pcf()
    assert gold["workload"] == wl.name and gold["n"] == wl.pos.shape[1]
    print(f"[case] c9 full pair count lmax={lmax} {width}", flush=True)
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).cuda()
    wl.lmax = lmax
    plan = curved_plan(wl, width)
    plan.accumulate(pos, w)
    assert plan.pair_count()[0] == gold["pairs"]


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
    err = alm_error(got, ref, wl, np.arange(20, 120), 2, 4, sphere=True)
    print(f"[err] sphere alm: {err:.3e} of each value's term-magnitude bound", flush=True)
    assert err <= 1e-6
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
        NPCF(4, 3, 2, e, [1.0] * 4, max_points=50, sphere=True)       # the sphere takes D = 2 or 3
    with pytest.raises(NPCFError):
        NPCF(2, 3, 2, np.array([1e-9, 0.5]), [1.0] * 2, max_points=50, sphere=True)   # cos(edges[0]) rounds to 1
    with pytest.raises(NPCFError):
        NPCF(2, 4, 6, e, [1.0] * 2, max_points=50, sphere=True)       # lmax above 5
    with pytest.raises(NPCFError):
        NPCF(2, 3, 2, np.array([0.5, 3.5]), [1.0] * 2, max_points=50, sphere=True)   # beyond pi


_C9 = {}


@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6"])
def test_c9_full_sphere_sampled(precision):
    """The sphere workload at full size (100k points, the paper's CMB test
    bins): 32 primaries against every point, against the oracle on the same
    primaries, per multipole on the strict measure (and the conditioned one)."""
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
    # every c9 multipole has S/|zeta| <= 3.2: the strict bar holds on all of them
    assert err <= TOL[precision]


@pytest.mark.parametrize("width", ["wide", "narrow"])
def test_sphere_cosine_not_fused(width):
    """The kernel's FP64 cosine rounds every product and sum as the definition
    (and the oracle) does: a planted pair whose rounded cosine lies above cos
    of the outer edge, and on it if the products were fused into FMAs, is
    counted (regression: the compiler's default contraction had fused them)."""
    from npcf_testutil import fused_dot_sphere_catalogue, sphere_pair_count_by_definition
    wl, c, cf, clo = fused_dot_sphere_catalogue()
    assert c > clo >= cf
    print(f"[case] fused sphere cosine {width} c {c!r} cos(e_last) {clo!r}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    assert pairs_ref == sphere_pair_count_by_definition(wl)
    got, pairs, _ = gpu_run(wl, plan=curved_plan(wl, width))
    assert pairs == pairs_ref
    cerr, _ = conditioned_error(got, ref, condition_scale(wl))
    assert cerr <= TOL["plain"]
