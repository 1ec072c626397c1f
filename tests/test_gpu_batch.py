"""GPU tests of the batched path (npcf_accumulate_batch / npcf_finalize_batch):
many catalogues in one captured launch sequence, each checked against the FP64
oracle and against the single-catalogue path, graph replays against the first
run, and the batched benchmark workload against the single-catalogue path.

The tiny mixed-sign catalogues use the conditioned measure of the parity
tests (|got - ref| over the sum of the magnitudes of the estimator's terms,
per multipole); the batched benchmark workload uses the strict per-multipole
measure (|got - ref| over the multipole's largest |ref|)."""
import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import condition_scale, conditioned_error, gpu_run, oracle_reported, per_multipole_error

pytestmark = pytest.mark.gpu

CASES = {
    # D, N, lmax, box side, r_max, bins, catalogue sizes
    "D3N4": (3, 4, 3, 16.0, 4.5, 4, [150, 320, 90, 260, 200]),
    "D3N3": (3, 3, 4, 20.0, 5.0, 4, [300, 120, 410]),
    "D2N4": (2, 4, 4, 12.0, 3.0, 5, [220, 400, 130]),
    "D4N3": (4, 3, 3, 10.0, 3.5, 4, [350, 180, 500]),
}


def _catalogues(name):
    D, N, L, box, rmax, nb, sizes = CASES[name]
    return [inputs.tiny(D, N, L, n, 100 + i, box_side=box, rmax=rmax, nbins=nb) for i, n in enumerate(sizes)]


def _batch(plan, cats):
    import torch
    pos = [torch.from_numpy(np.ascontiguousarray(c.pos)).cuda() for c in cats]
    w = [torch.from_numpy(np.ascontiguousarray(c.w)).cuda() for c in cats]
    plan.accumulate_batch(pos, w)
    return pos, w


def _plan(wl, precision="plain", max_points=1000):
    from paper_2106_10278_amd import NPCF
    return NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, precision=precision, max_points=max_points)


@pytest.mark.parametrize("name", sorted(CASES))
def test_batch_matches_oracle_and_single(name):
    cats = _catalogues(name)
    print(f"[case] batch {name} sizes={[c.pos.shape[1] for c in cats]}", flush=True)
    plan = _plan(cats[0])
    plan.set_tuning(chunk_rows=128)   # several chunks; catalogues straddle chunk boundaries
    _keep = _batch(plan, cats)
    done = []
    for i, wl in enumerate(cats):
        got, done_ms, pairs = plan.finalize_batch(i)
        done.append(done_ms)
        ref, pairs_ref, _ = oracle_reported(wl)
        single, pairs_single, _ = gpu_run(wl)
        scale = condition_scale(wl)
        cerr, _ = conditioned_error(got, ref, scale)
        serr, _ = conditioned_error(got, single, scale)
        print(f"[err] batch {name} cat {i}: oracle {cerr:.3e} single {serr:.3e} done {done_ms:.3f} ms", flush=True)
        assert pairs == pairs_ref == pairs_single
        assert cerr <= 1e-6
        assert serr <= 1e-6
    # catalogues are taken smallest first: completion times rise along the
    # stable ascending-size order (equal within one chunk)
    order = np.argsort([c.pos.shape[1] for c in cats], kind="stable")
    times = np.array(done)[order]
    assert np.all(times >= 0.0) and np.all(np.diff(times) >= 0.0)


def test_batch_graph_replay():
    """The captured graph replayed three times, with eager work and
    synchronisation between the replays, gives the first run's results bit
    for bit; a replay after an in-place change of the inputs sees the new
    values (weights doubled: zeta scales by 2^N exactly)."""
    import torch
    cats = _catalogues("D3N4")
    plan = _plan(cats[0])
    plan.set_tuning(chunk_rows=256)
    pos, w = _batch(plan, cats)
    first = [plan.finalize_batch(i) for i in range(len(cats))]
    other = _plan(cats[0])
    for rep in range(3):
        print(f"[case] replay {rep}", flush=True)
        gpu_run(cats[rep], plan=None)          # eager work of the program between replays
        torch.cuda.synchronize()
        plan.accumulate_batch(pos, w)
        for i in range(len(cats)):
            got, _, pairs = plan.finalize_batch(i)
            assert pairs == first[i][2]
            assert np.array_equal(got, first[i][0])
    for t in w:
        t.mul_(2.0)
    plan.accumulate_batch(pos, w)
    for i, wl in enumerate(cats):
        got, _, _ = plan.finalize_batch(i)
        assert np.allclose(got, first[i][0] * 2.0 ** wl.N, rtol=1e-13, atol=0.0)
    other.close()


@pytest.mark.parametrize("precision", ["mixed_fp16", "mixed_bf16x6"])
def test_batch_mixed_precision(precision):
    cats = _catalogues("D3N4")
    plan = _plan(cats[0], precision=precision)
    _keep = _batch(plan, cats)
    for i, wl in enumerate(cats):
        got, _, pairs = plan.finalize_batch(i)
        ref, pairs_ref, _ = oracle_reported(wl)
        cerr, _ = conditioned_error(got, ref, condition_scale(wl))
        print(f"[err] batch {precision} cat {i}: {cerr:.3e}", flush=True)
        assert pairs == pairs_ref
        assert cerr <= 1e-5


def test_batch_rejects_bad_input():
    import torch
    from paper_2106_10278_amd import NPCFError
    cats = _catalogues("D3N3")
    plan = _plan(cats[0])
    with pytest.raises(NPCFError):
        plan.finalize_batch(0)                  # no batch yet
    _batch(plan, cats)
    with pytest.raises(NPCFError):
        plan.finalize_batch(len(cats))          # out of range
    rnd = _plan(cats[0])
    from paper_2106_10278_amd import NPCF
    byr = NPCF(3, 3, cats[0].lmax, cats[0].edges, cats[0].box, norm="by_randoms", max_points=1000)
    with pytest.raises(NPCFError):
        _batch(byr, cats)
    rnd.close()


@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6"])
def test_batched_workload_against_single_path_and_oracle(precision):
    """The batched benchmark workload (64 catalogues, data sizes log-uniform
    in [20k, 300k] plus 3x randoms; D = 3, N = 4, lmax 5, 10 bins in [20, 160])
    in one batch launch, in the launch configuration the benchmark uses.  For
    the 8 smallest and the 2 largest catalogues:
      - the batch equals the single-catalogue path on the full catalogue: pair
        counts exactly, every multipole within the strict per-multipole bar
        (1e-6 plain, 1e-5 mixed) of it;
      - the single-catalogue path on 64 data and 64 random primaries of the
        same catalogue matches the FP64 oracle on those primaries (eq.
        NPCF-estimator-discrete is a sum over primaries), pair counts exactly
        and every multipole within the same strict bar.
    Together these hold each catalogue of the batch to the oracle per
    multipole; the oracle alone would need minutes per full catalogue."""
    import torch
    from paper_2106_10278_amd import NPCF
    tol = 1e-6 if precision == "plain" else 1e-5
    sizes = inputs.c4_batch_sizes()
    order = np.argsort(sizes)
    check = [int(c) for c in order[:8]] + [int(order[-2]), int(order[-1])]
    pos, w, wls = [], [], {}
    for c, nd in enumerate(sizes):
        wl = inputs.c4_catalogue(c, nd)
        if c in check:
            wls[c] = wl
        pos.append(torch.from_numpy(np.ascontiguousarray(wl.pos)).cuda())
        w.append(torch.from_numpy(np.ascontiguousarray(wl.w)).cuda())
    ref = next(iter(wls.values()))
    print(f"[case] batched workload {precision}: {len(sizes)} catalogues, "
          f"{sum(int(p.shape[1]) for p in pos)} points", flush=True)
    nmax = max(int(p.shape[1]) for p in pos)
    plan = NPCF(3, 4, 5, ref.edges, ref.box, precision=precision, max_points=nmax)
    plan.accumulate_batch(pos, w)
    single_plan = NPCF(3, 4, 5, ref.edges, ref.box, precision=precision, max_points=nmax)
    for c in check:
        wl = wls[c]
        got, done_ms, pairs = plan.finalize_batch(c)
        single, pairs_single, _ = gpu_run(wl, plan=single_plan)
        single_plan.reset()
        err_s, _ = per_multipole_error(got, single)
        nd = wl.n_data
        ranges = [(0, 64), (nd, nd + 64)]
        prims = np.concatenate([np.arange(a, b) for a, b in ranges])
        sampled, pairs_sampled, _ = gpu_run(wl, ranges=ranges, plan=single_plan)
        single_plan.reset()
        oref, pairs_ref, _ = oracle_reported(wl, prims=prims)
        err_o, _ = per_multipole_error(sampled, oref)
        print(f"[err] batched workload {precision} cat {c} n={wl.pos.shape[1]}: batch vs single {err_s:.3e}, "
              f"sampled vs oracle {err_o:.3e}, pairs {pairs}, done {done_ms:.1f} ms", flush=True)
        assert pairs == pairs_single
        assert pairs_sampled == pairs_ref
        assert err_s <= tol
        assert err_o <= tol
    plan.close()
    single_plan.close()
