"""Shared helpers of the parity tests: run the GPU path through the C ABI and
compare with the FP64 oracle per multipole."""
import numpy as np

import oracle


def per_multipole_error(got, ref):
    """max over multipoles of max_b |got - ref| / max(max_b |ref|, 1e-12 max |ref|)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    floor = 1e-12 * np.max(np.abs(ref)) if ref.size else 0.0
    errs = []
    for i in range(ref.shape[0]):
        den = max(np.max(np.abs(ref[i])), floor)
        errs.append(np.max(np.abs(got[i] - ref[i])) / den if den > 0 else np.max(np.abs(got[i])))
    errs = np.array(errs)
    return float(errs.max()) if errs.size else 0.0, errs


def oracle_reported(wl, prims=None, btuple_mode=0):
    z, pairs = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w, prims=prims,
                           btuple_mode=btuple_mode)
    labels = oracle.lambda_labels(wl.D, wl.N, wl.lmax)
    return oracle.reported_part(z, labels, wl.D, wl.N), pairs, z


def gpu_run(wl, ranges=None, precision="plain", btuple_mode=0, device="cuda:0", plan=None):
    import torch
    from paper_2106_10278_amd import NPCF
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).to(device)
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).to(device)
    n = wl.pos.shape[1]
    if plan is None:
        plan = NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, btuple_mode=btuple_mode, precision=precision,
                    max_points=n)
    if ranges is None:
        ranges = [(0, n)]
    for a, b in ranges:
        plan.accumulate(pos, w, a, b)
    out = plan.finalize()
    pairs = plan.pair_count()[0]
    return out, pairs, plan
