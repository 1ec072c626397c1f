"""GPU parity: the HIP path (called through the C ABI) against the FP64 oracle
on the same seeded inputs, per multipole.

Two error measures, both per multipole Lambda (max over b-tuples):
  strict       |got - ref| / max_b |ref|
  conditioned  |got - ref| / max_b S, with S the sum of the magnitudes of the
               estimator's terms (condition_scale); a sum evaluated with unit
               roundoff u has forward error below about u S.
The benchmark configurations are held to the strict targets: 1e-6 for the
plain FP32 path and 1e-5 for the split-precision coupling paths that carry
at least 22 significand bits (FP16 hi+lo with per-tile scaling, BF16
hi+mid+lo).  The tiny cases draw weights of both signs, so some multipoles
cancel to a small fraction of their terms (S / |zeta| up to ~270); there the
same tolerances apply to the conditioned measure.  BF16 hi+lo keeps 16
significand bits per operand (relative error up to 2^-16 each, about 3 x 2^-16
per product), so it is held to 5e-5 on the conditioned measure everywhere.
Bin assignment is exact on lattice inputs, so pair counts are compared bit
for bit.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import alm_error, condition_scale, conditioned_error, gpu_run, oracle_reported, per_multipole_error

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-6, "mixed_fp16": 1e-5, "mixed_bf16x6": 1e-5}
TOL_BF16X3 = 5e-5   # conditioned measure, from the 16-bit operand split


def _check(got, ref, precision, scale, label, strict=True):
    err, _ = per_multipole_error(got, ref)
    cerr, _ = conditioned_error(got, ref, scale) if scale is not None else (float("nan"), None)
    print(f"[err] {label} {precision}: strict {err:.3e} conditioned {cerr:.3e}", flush=True)
    if precision == "mixed_bf16":
        assert cerr <= TOL_BF16X3
    elif strict:
        assert err <= TOL[precision]
    else:
        assert cerr <= TOL[precision]


def _case(D, N, lmax, n, seed, box, rmax, nbins, weights="mixed"):
    return inputs.tiny(D, N, lmax, n, seed, box_side=box, rmax=rmax, nbins=nbins, weights=weights)


TINY = {
    "D3N3": (3, 3, 4, 400, 1, 20.0, 5.0, 4),
    "D3N4": (3, 4, 3, 300, 2, 16.0, 4.5, 4),
    "D3N4L6": (3, 4, 6, 200, 6, 16.0, 4.5, 3),   # lmax > 5: the term-by-term coupling kernel
    "D2N4": (2, 4, 4, 400, 3, 12.0, 3.0, 5),
    "D2N3": (2, 3, 5, 400, 4, 12.0, 3.0, 5),
    "D4N3": (4, 3, 3, 500, 5, 10.0, 3.5, 4),
}


@pytest.mark.parametrize("name", sorted(TINY))
@pytest.mark.parametrize("precision", ["plain", "mixed_fp16", "mixed_bf16x6", "mixed_bf16"])
@pytest.mark.parametrize("mode", [0, 1])
def test_tiny_parity(name, precision, mode):
    wl = _case(*TINY[name])
    print(f"[case] {name} {precision} mode={mode}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl, btuple_mode=mode)
    got, pairs, plan = gpu_run(wl, precision=precision, btuple_mode=mode)
    assert np.array_equal(plan.lambda_labels, oracle.lambda_labels(wl.D, wl.N, wl.lmax))
    assert np.array_equal(plan.btuples, oracle.btuple_labels(len(wl.edges) - 1, wl.N, mode))
    assert pairs == pairs_ref
    _check(got, ref, precision, condition_scale(wl, mode), f"{name} mode={mode}", strict=False)


@pytest.mark.parametrize("precision", ["plain", "mixed_fp16", "mixed_bf16x6", "mixed_bf16"])
def test_c1_full(precision):
    """D = 3, N = 3: 2000 uniform points, 8 bins in [2, 20], lmax = 4 (all primaries)."""
    wl = inputs.c1_small_3pcf()
    print(f"[case] c1 {precision}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl, precision=precision)
    assert pairs == pairs_ref
    _check(got, ref, precision, condition_scale(wl), "c1")


@pytest.mark.parametrize("D,lmax", [(2, 6), (3, 5), (4, 4)])
def test_alm_matches_oracle(D, lmax):
    """Harmonic stage alone (npcf_alm) against the oracle's a^b_[l]."""
    import torch
    from paper_2106_10278_amd import NPCF, stored_state_labels
    wl = _case(D, 3, lmax, 500, 11 + D, 12.0, 4.0, 3)
    print(f"[case] alm D={D}", flush=True)
    plan = NPCF(D, 3, lmax, wl.edges, wl.box, max_points=wl.pos.shape[1])
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    got = plan.alm(pos, w, 10, 70)
    ref, _ = oracle.alm(D, lmax, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(10, 70))
    olab = [tuple(r) for r in oracle.state_labels(D, lmax)]
    idx = []
    for s in stored_state_labels(D, lmax):
        key = (int(s[0]),) if D == 2 else ((int(s[0]), int(s[1])) if D == 3 else (int(s[0]), int(s[1]), int(s[2])))
        idx.append(olab.index(key))
    ref = ref[:, :, idx]
    err = alm_error(got, ref, wl, np.arange(10, 70), D, lmax)
    print(f"[err] alm D={D}: {err:.3e} of each value's term-magnitude bound", flush=True)
    assert err <= 1e-6


def test_additivity_and_pairs():
    """Disjoint primary ranges add up (eq. NPCF-estimator-discrete sums over primaries)."""
    wl = _case(3, 4, 3, 400, 21, 16.0, 4.5, 4)
    print("[case] additivity", flush=True)
    full, pf, _ = gpu_run(wl)
    split, ps, _ = gpu_run(wl, ranges=[(0, 123), (123, 250), (250, 400)])
    assert pf == ps
    # two FP32 evaluations in different orders, each within 1e-6 of the scale
    cerr, _ = conditioned_error(split, full, condition_scale(wl))
    print(f"[err] additivity conditioned {cerr:.3e}", flush=True)
    assert cerr <= 2e-6


def test_bin_edges_exact():
    """Separations exactly on a bin edge go to the upper bin, as in the definition
    e_b <= r < e_{b+1} (box 128: integer coordinates sit on the lattice)."""
    rng = np.random.default_rng(5)
    n = 300
    pos = rng.integers(0, 16, size=(3, n)).astype(np.float64) * 4.0   # many exact integer distances
    pos = pos + rng.integers(0, 2, size=(3, n)) * 1.0
    wl = inputs.Workload("edges", 3, 4, 2, np.array([1.0, 2.0, 4.0, 5.0, 8.0]), [128.0] * 3,
                         inputs.to_lattice(pos, [128.0] * 3), rng.uniform(0.5, 1.5, size=n), n)
    print("[case] bin edges", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl), "bin edges", strict=False)


def test_degenerate_inputs():
    import torch
    from paper_2106_10278_amd import NPCF, NPCFError
    wl = _case(3, 3, 2, 50, 31, 20.0, 1.0, 2)
    plan = NPCF(3, 3, 2, wl.edges, wl.box, max_points=50)
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    with pytest.raises(NPCFError):
        plan.accumulate(pos, w, 5, 5)           # empty range
    plan2 = NPCF(3, 3, 2, wl.edges, wl.box, max_points=10)
    with pytest.raises(NPCFError):
        plan2.accumulate(pos, w)                # n > max_points
    # a single point has no pairs: all zeros
    plan3 = NPCF(3, 3, 2, wl.edges, wl.box, max_points=50)
    plan3.accumulate(pos[:, :1].contiguous(), w[:1].contiguous())
    assert np.all(plan3.finalize() == 0.0)
    assert plan3.pair_count()[0] == 0
    # non-finite input is reported at finalize
    bad = pos.clone()
    bad[0, 3] = float("nan")
    plan4 = NPCF(3, 3, 2, wl.edges, wl.box, max_points=50)
    plan4.accumulate(bad, w)
    with pytest.raises(NPCFError):
        plan4.finalize()


def test_coincident_points():
    """Every point taken twice: pairs at zero separation lie outside every bin
    (the first edge is positive).  The doubled catalogue matches the oracle
    on it, and 2^N times the single catalogue's result (4x the pairs)."""
    base = _case(3, 4, 3, 150, 23, 16.0, 4.5, 4)
    wl = inputs.Workload("twins", 3, 4, 3, base.edges, base.box, np.concatenate([base.pos, base.pos], axis=1),
                         np.concatenate([base.w, base.w]), 300)
    print("[case] coincident points", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl)
    got1, pairs1, _ = gpu_run(base)
    assert pairs == pairs_ref == 4 * pairs1
    scale = condition_scale(wl)
    _check(got, ref, "plain", scale, "twins", strict=False)
    cerr, _ = conditioned_error(got, 16.0 * got1, scale)
    print(f"[err] twins vs 16 x single conditioned {cerr:.3e}", flush=True)
    assert cerr <= 2e-6


@pytest.mark.parametrize("D,N,lmax", [(3, 3, 4), (3, 4, 3), (2, 4, 4), (4, 3, 2)])
@pytest.mark.parametrize("mode", [0, 1])
def test_max_bins(D, N, lmax, mode):
    """The largest bin count the library takes (16): every bit plane of the
    in-batch bin sort and every bin row of the accumulators is used."""
    box, rmax = {2: (12.0, 3.0), 3: (14.0, 4.0), 4: (9.0, 3.0)}[D]
    wl = _case(D, N, lmax, 300, 70 + D + N, box, rmax, 16)
    print(f"[case] max bins D={D} N={N} lmax={lmax} mode={mode}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl, btuple_mode=mode)
    got, pairs, _ = gpu_run(wl, btuple_mode=mode)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl, mode), f"max bins D={D} N={N}", strict=False)


FULL = {
    # workload factory, sampled primary ranges (data part, randoms part)
    "c2": (inputs.c2_clustered_4pcf, [(0, 48), (200_000, 200_048)]),
    "c3": (inputs.c3_vorticity_4pcf, [(0, 24)]),
    "c5": (inputs.c5_hyper_3pcf, [(0, 24), (1_500_000, 1_500_024)]),
}


_FULL_CACHE = {}


@pytest.mark.parametrize("precision", ["plain", "mixed_fp16", "mixed_bf16x6", "mixed_bf16"])
@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_full_catalogue_sampled_primaries(name, precision):
    """Full-size catalogues of the benchmark configurations, in the launch
    configuration the benchmark uses, on a sample of primaries the oracle can
    afford (eq. NPCF-estimator-discrete is a sum over primaries)."""
    factory, ranges = FULL[name]
    if name not in _FULL_CACHE:   # the oracle's answer is shared by the precisions
        wl = factory()
        prims = np.concatenate([np.arange(a, b) for a, b in ranges])
        ref, pairs_ref, _ = oracle_reported(wl, prims=prims)
        _FULL_CACHE.clear()
        _FULL_CACHE[name] = (wl, prims, ref, pairs_ref, condition_scale(wl, prims=prims))
    wl, prims, ref, pairs_ref, scale = _FULL_CACHE[name]
    print(f"[case] {name} {precision} n={wl.pos.shape[1]} primaries={len(prims)}", flush=True)
    got, pairs, _ = gpu_run(wl, ranges=ranges, precision=precision)
    print(f"[pairs] {name}: {pairs} vs {pairs_ref}", flush=True)
    assert pairs == pairs_ref
    _check(got, ref, precision, scale, name)


def test_norm_by_randoms():
    """NPCF_NORM_BY_RANDOMS divides by the Lambda = 0 component of the randoms-only estimator."""
    import torch
    from paper_2106_10278_amd import NPCF
    data = _case(3, 4, 2, 300, 41, 16.0, 4.5, 3)
    rand = _case(3, 4, 2, 600, 42, 16.0, 4.5, 3, weights="ones")
    print("[case] by_randoms", flush=True)
    plan = NPCF(3, 4, 2, data.edges, data.box, norm="by_randoms", max_points=600)
    pd, wd = torch.from_numpy(data.pos).cuda(), torch.from_numpy(data.w).cuda()
    pr, wr = torch.from_numpy(rand.pos).cuda(), torch.from_numpy(rand.w).cuda()
    plan.accumulate(pd, wd, role="data")
    plan.accumulate(pr, wr, role="randoms")
    got = plan.finalize()
    zd, _, _ = oracle_reported(data)
    zr, _, _ = oracle_reported(rand)
    i0 = int(np.nonzero(np.all(oracle.lambda_labels(3, 4, 2) == 0, axis=1))[0][0])
    # the quotient's error is the data estimate's plus the (well conditioned,
    # positive-weight) randoms' Lambda = 0 term's: undo the division by the
    # oracle's denominator and assess the numerator on the conditioned measure
    cerr, _ = conditioned_error(got * zr[i0][None, :], zd, condition_scale(data))
    print(f"[err] by_randoms conditioned {cerr:.3e}", flush=True)
    assert cerr <= 2e-6


def test_autotune_keeps_results():
    """The autotuner only changes tile shapes: results after it match the
    oracle, and the chosen settings are in range."""
    import torch
    from paper_2106_10278_amd import NPCF
    wl = _case(3, 4, 3, 600, 51, 16.0, 4.5, 4)
    print("[case] autotune", flush=True)
    plan = NPCF(3, 4, 3, wl.edges, wl.box, max_points=600)
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    t = plan.autotune(pos, w, sample=256)
    assert 1 <= t["cell_subdiv"] <= 6 and t["couple_block"] in (0, 256, 512, 1024, 2048) and t["sample_ms"] > 0
    assert t["harmonic_blocks_per_cu"] in (2, 3, 4, 6, 8) and 1 <= t["chunk_rows"] <= 600
    got, pairs, _ = gpu_run(wl, plan=plan)
    ref, pairs_ref, _ = oracle_reported(wl)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl), f"autotuned {t}", strict=False)


def test_autotune_cache(tmp_path, monkeypatch):
    """NPCF_TUNE_CACHE: the first tuning is written to the JSON file under the
    problem's key; a second plan for the same problem applies it without
    timing; a different problem gets an entry of its own; results unchanged."""
    import json
    import torch
    from paper_2106_10278_amd import NPCF
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("NPCF_TUNE_CACHE", str(cache))
    wl = _case(3, 4, 3, 600, 52, 16.0, 4.5, 4)
    print("[case] autotune cache", flush=True)
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.w).cuda()
    first = NPCF(3, 4, 3, wl.edges, wl.box, max_points=600)
    t1 = first.autotune(pos, w, sample=256)
    entries = json.load(open(cache))["entries"]
    assert len(entries) == 1
    (key, ent), = entries.items()
    assert "D3-N4-L3-nb4-n600" in key
    assert {k: ent[k] for k in ("cell_subdiv", "couple_block", "chunk_rows", "harmonic_blocks_per_cu")} == \
        {k: t1[k] for k in ("cell_subdiv", "couple_block", "chunk_rows", "harmonic_blocks_per_cu")}
    # a planted entry is what a second plan applies (proof that no timing ran)
    ent.update(cell_subdiv=2, couple_block=512, harmonic_blocks_per_cu=3)
    json.dump({"npcf_tuning": 1, "entries": {key: ent}}, open(cache, "w"))
    second = NPCF(3, 4, 3, wl.edges, wl.box, max_points=600)
    t2 = second.autotune(pos, w, sample=256)
    assert (t2["cell_subdiv"], t2["couple_block"], t2["harmonic_blocks_per_cu"]) == (2, 512, 3)
    got, pairs, _ = gpu_run(wl, plan=second)
    ref, pairs_ref, _ = oracle_reported(wl)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl), "cached tuning", strict=False)
    other = NPCF(3, 4, 3, wl.edges, wl.box, precision="mixed_bf16x6", max_points=600)
    other.autotune(pos, w, sample=256)
    assert len(json.load(open(cache))["entries"]) == 2


@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6"])
def test_factorised_coupling_matches_terms(precision, monkeypatch):
    """D = 3, N = 4: the factorised coupling kernel (products shared by every l3
    of a pair) and the term-by-term kernel (NPCF_COUPLING=terms) agree with each
    other and with the oracle."""
    wl = _case(3, 4, 5, 300, 61, 16.0, 4.5, 4)
    print(f"[case] factorised vs terms {precision}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    scale = condition_scale(wl)
    fac, pf, _ = gpu_run(wl, precision=precision)
    monkeypatch.setenv("NPCF_COUPLING", "terms")
    trm, pt, _ = gpu_run(wl, precision=precision)
    assert pf == pt == pairs_ref
    _check(fac, ref, precision, scale, "factorised", strict=False)
    _check(trm, ref, precision, scale, "terms", strict=False)
    cerr, _ = conditioned_error(fac, trm, scale)
    assert cerr <= 2 * TOL[precision]


@pytest.mark.skip(reason="the per-bin queue harmonic kernel is switched off: its first GPU run "
                         "did not finish on the 300-point D=3 N=4 case; its source runs correctly "
                         "in a host emulation and its row loop compiles well formed, so no cause "
                         "is known; NPCF_HARMONIC=queue is rejected")
@pytest.mark.parametrize("name", ["D3N4", "D2N4", "D4N3", "D3N4L6"])
def test_harmonic_kernels_agree(name, monkeypatch):
    """The two harmonic-stage kernels (bin-sorted staging, NPCF_HARMONIC=stage;
    per-bin queues, NPCF_HARMONIC=queue) give the same pair counts and agree
    with each other and with the oracle."""
    wl = _case(*TINY[name])
    print(f"[case] harmonic kernels {name}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    scale = condition_scale(wl)
    monkeypatch.setenv("NPCF_HARMONIC", "stage")
    st, ps, _ = gpu_run(wl)
    monkeypatch.setenv("NPCF_HARMONIC", "queue")
    qu, pq, _ = gpu_run(wl)
    assert ps == pq == pairs_ref
    _check(st, ref, "plain", scale, f"{name} staging", strict=False)
    _check(qu, ref, "plain", scale, f"{name} queues", strict=False)
    cerr, _ = conditioned_error(st, qu, scale)
    assert cerr <= 2e-6


@pytest.mark.parametrize("name", ["D3N4", "D2N4", "D3N3", "D4N3", "D3N4L6", "D3N4dense"])
def test_harmonic_pass_and_stage_agree(name, monkeypatch):
    """The two flat harmonic-stage kernels (one pass per radial bin, the
    default; bin-sorted staging, NPCF_HARMONIC=stage) give the oracle's pair
    counts and agree with it and with each other, on the tiny cases and on a
    dense catalogue with many batches per bin."""
    wl = _case(*(TINY[name] if name in TINY else MANY_PAIRS["D3N4dense"]))
    print(f"[case] harmonic pass and stage {name}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    scale = condition_scale(wl)
    monkeypatch.setenv("NPCF_HARMONIC", "stage")
    st, ps, _ = gpu_run(wl)
    monkeypatch.setenv("NPCF_HARMONIC", "pass")
    pa, pp, _ = gpu_run(wl)
    assert ps == pp == pairs_ref
    _check(st, ref, "plain", scale, f"{name} staging", strict=False)
    _check(pa, ref, "plain", scale, f"{name} per-bin passes", strict=False)
    cerr, _ = conditioned_error(st, pa, scale)
    assert cerr <= 2e-6


MANY_PAIRS = {
    # about 900-1200 pairs per primary: many 64-pair batches per primary with
    # bursts of one bin, up to 16 bins
    "D3N4dense": (3, 4, 3, 4000, 12, 16.0, 6.0, 7),
    "D3N3dense16": (3, 3, 4, 4000, 13, 16.0, 6.0, 16),
    "D2N4dense": (2, 4, 5, 6000, 14, 12.0, 3.0, 11),
    "D3N3L7": (3, 3, 7, 300, 8, 16.0, 4.5, 3),
}


@pytest.mark.parametrize("name", sorted(MANY_PAIRS))
def test_dense_catalogues(name):
    """Catalogues with hundreds of pairs per primary (many batches per row of
    a, the persistent loop over rows run to its end by every wave): pair
    counts exact and the multipoles within the bar of the conditioned measure."""
    wl = _case(*MANY_PAIRS[name])
    print(f"[case] dense {name}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl), f"{name} dense", strict=False)


def test_harmonic_queue_kernel_rejected(monkeypatch):
    """NPCF_HARMONIC names a kernel that is switched off: plan creation fails
    with NPCF_E_UNSUPPORTED before anything is launched."""
    from paper_2106_10278_amd import NPCF, NPCFError
    wl = _case(*TINY["D3N4"])
    monkeypatch.setenv("NPCF_HARMONIC", "queue")
    with pytest.raises(NPCFError, match="NPCF_HARMONIC"):
        NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, max_points=wl.pos.shape[1])


@pytest.mark.parametrize("sdv", [1, 3, 6, 8])
def test_cell_subdivision_keeps_results(sdv):
    """Finer or coarser cell lists change only which candidates phase A sees:
    pair counts stay exact and the multipoles match the oracle."""
    import torch
    from paper_2106_10278_amd import NPCF
    wl = _case(3, 4, 3, 500, 71, 20.0, 4.5, 4)
    print(f"[case] cell subdivision {sdv}", flush=True)
    plan = NPCF(3, 4, 3, wl.edges, wl.box, max_points=wl.pos.shape[1])
    plan.set_tuning(cell_subdiv=sdv)
    got, pairs, _ = gpu_run(wl, plan=plan)
    ref, pairs_ref, _ = oracle_reported(wl)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl), f"subdivision {sdv}", strict=False)


@pytest.mark.parametrize("D,N,lmax,n,box,rmax", [(3, 4, 3, 400, 10.0, 4.0), (2, 4, 4, 400, 8.0, 3.0),
                                                  (4, 3, 3, 500, 8.0, 3.5), (3, 3, 4, 400, 10.0, 4.0)])
@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6"])
def test_open_box_parity(D, N, lmax, n, box, rmax, precision):
    """Open (non-periodic) box: separations without wrap-around, cell ranges
    clipped at the walls (the kernels' non-periodic instantiations)."""
    import torch
    from paper_2106_10278_amd import NPCF
    wl = _case(D, N, lmax, n, 80 + D + N, box, rmax, 4)
    print(f"[case] open box D={D} N={N} {precision}", flush=True)
    plan = NPCF(D, N, lmax, wl.edges, wl.box, periodic=False, precision=precision, max_points=n)
    plan.accumulate(torch.from_numpy(wl.pos).cuda(), torch.from_numpy(wl.w).cuda())
    got = plan.finalize()
    z, pairs_ref = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, periodic=False)
    ref = oracle.reported_part(z, oracle.lambda_labels(D, N, lmax), D, N)
    assert plan.pair_count()[0] == pairs_ref
    # the periodic box would have more pairs: the open path is really taken
    _, pairs_per = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, periodic=True)
    assert pairs_per > pairs_ref
    scale = condition_scale(wl, periodic=False)
    _check(got, ref, precision, scale, f"open D={D} N={N}", strict=False)



@pytest.mark.parametrize("D,N,lmax,nbins", [(3, 3, 10, 3), (2, 3, 16, 3), (4, 3, 6, 3), (2, 4, 16, 3), (3, 4, 8, 3)])
def test_largest_lmax(D, N, lmax, nbins):
    """The largest harmonic orders the library takes (D = 2: 16, D = 3: 10,
    D = 4: 6; for D = 3, N = 4 a high order with the term-by-term coupling):
    the instantiations with the most emitted values per pair and the most
    staging chunks."""
    box, rmax = {2: (10.0, 3.0), 3: (12.0, 4.0), 4: (9.0, 3.5)}[D]
    wl = _case(D, N, lmax, 250, 90 + D + lmax, box, rmax, nbins)
    print(f"[case] largest lmax D={D} N={N} lmax={lmax}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    got, pairs, _ = gpu_run(wl)
    assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl), f"D={D} N={N} lmax={lmax}", strict=False)


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (2, 4, 4), (3, 3, 4)])
def test_off_lattice_positions(D, N, lmax):
    """Positions that are not on the library's 2^-32 box lattice: the library
    rounds each coordinate to the nearest lattice point (a shift of at most
    box 2^-33 per axis) while the oracle uses the FP64 positions as given.
    What may differ: a pair whose distance lies within that shift of a bin
    edge can fall in the other bin, so the pair counts may differ by at most
    the number of such pairs (counted here on the CPU), and directions move by
    about 1e-10, far below FP32 rounding.  Everything else is asserted: the
    pair counts exactly when no pair is that close to an edge, and every
    multipole within the plain bar of the conditioned measure."""
    rng = np.random.default_rng(900 + D + N)
    box = {2: 12.0, 3: 16.0}[D]
    n = 400
    wl = _case(D, N, lmax, n, 31 + D, box, 4.5 if D == 3 else 3.0, 4)
    pos = rng.uniform(0.0, box, size=(D, n))          # FP64, generally off the lattice
    w = wl.w
    wl2 = type(wl)(wl.name, D, N, lmax, wl.edges, wl.box, pos, w, n)
    assert np.any(np.abs(pos * 2.0 ** 32 / box - np.rint(pos * 2.0 ** 32 / box)) > 0.1)
    # pairs within the lattice shift of an edge (|r - e| <= sqrt(D) box 2^-32)
    near = 0
    tol = np.sqrt(D) * box * 2.0 ** -32
    for j in range(n):
        d = pos - pos[:, j:j + 1]
        d -= box * np.round(d / box)
        r = np.sqrt(np.sum(d * d, axis=0))
        r[j] = -1.0
        near += int(np.sum(np.min(np.abs(r[:, None] - wl.edges[None, :]), axis=1) <= tol))
    print(f"[case] off-lattice D={D} N={N}: {near} pairs within the lattice shift of an edge", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl2)
    got, pairs, _ = gpu_run(wl2)
    assert abs(pairs - pairs_ref) <= near
    if near == 0:
        assert pairs == pairs_ref
    _check(got, ref, "plain", condition_scale(wl2), f"off-lattice D={D} N={N}", strict=False)


# periodic boxes with unequal sides: the flat kernels' general pre-test (a
# scale per axis), not the instance for cubes, and the x cells sized from the
# first side while the stencil rows run over the others
NON_CUBIC = {
    "D2": (2, 4, 4, [8.0, 11.0], 3.5, 5),
    "D3": (3, 4, 3, [10.0, 14.0, 12.0], 4.5, 4),
    "D3long": (3, 3, 4, [24.0, 10.0, 11.0], 4.5, 6),
    "D4": (4, 3, 3, [9.0, 10.0, 11.0, 12.0], 4.0, 3),
}


@pytest.mark.parametrize("name", sorted(NON_CUBIC))
def test_non_cubic_periodic_box(name, monkeypatch):
    """Pair counts equal the oracle's and the multipoles are within the plain
    bar, on both flat harmonic kernels (per-bin passes and bin-sorted
    staging)."""
    D, N, lmax, box, rmax, nbins = NON_CUBIC[name]
    rng = np.random.default_rng(500 + len(name) + D)
    n = 500
    pos = inputs.uniform(rng, n, box)
    w = rng.uniform(-0.5, 1.5, size=n)
    edges = np.linspace(rmax / (nbins + 1), rmax, nbins + 1)
    wl = inputs.Workload(f"noncubic-{name}", D, N, lmax, edges, box, pos, w, n)
    print(f"[case] non-cubic periodic box {name} {box}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    scale = condition_scale(wl)
    for kernel in ("pass", "stage"):
        monkeypatch.setenv("NPCF_HARMONIC", kernel)
        got, pairs, _ = gpu_run(wl)
        assert pairs == pairs_ref
        _check(got, ref, "plain", scale, f"non-cubic {name} {kernel}", strict=False)


def test_fp64_distance_not_fused(monkeypatch):
    """The kernels' FP64 squared distance rounds every product and sum as the
    definition (and the oracle) does: a planted pair one ulp inside the outer
    edge by that arithmetic, and on the edge if the products were fused into
    FMAs, is counted by both flat harmonic kernels (regression: the
    compiler's default contraction had fused them)."""
    from npcf_testutil import fused_distance_catalogue, pair_count_by_definition
    wl, r2, r2f, e2 = fused_distance_catalogue()
    assert r2 < e2 <= r2f
    print(f"[case] fused distance r2 {r2!r} edge^2 {e2!r}", flush=True)
    ref, pairs_ref, _ = oracle_reported(wl)
    assert pairs_ref == pair_count_by_definition(wl)
    scale = condition_scale(wl)
    for kernel in ("pass", "stage"):
        monkeypatch.setenv("NPCF_HARMONIC", kernel)
        got, pairs, _ = gpu_run(wl)
        assert pairs == pairs_ref
        _check(got, ref, "plain", scale, f"fused distance {kernel}", strict=False)
