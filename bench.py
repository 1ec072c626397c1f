"""Benchmark of the separable NPCF estimator on one MI355X.

Workload (default): isotropic 4PCF in D = 3 -- 200k clustered data points
(half in 2000 Gaussian blobs of sigma 5, half uniform, w = +1) plus 600k
uniform randoms (w = -1/3) in a periodic cube of side 1000, 10 linear radial
bins in [20, 160], lmax = 5 (111 Lambda x 120 radial tuples).  Synthetic,
seeded (see paper_2106_10278_amd/inputs.py).

A step is one pass of the whole path over the catalogue: quantise + cell list,
harmonic stage, coupling stage, FP64 reduction and finalisation
(npcf_reset + npcf_accumulate + npcf_finalize), inputs resident in HBM.
The mixed-precision path (BF16 hi+lo split coupling) is the headline value;
the plain FP32 path is timed on the same inputs and reported beside it, with
the per-multipole relative error of both against the FP64 oracle on a
sample of primaries.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12      # MI355X, FP32 vector (packed) FLOP/s
HBM_PEAK = 8.0e12
# algorithmic FLOPs per in-range pair of the harmonic stage (geometry,
# recurrences and weighted accumulation), by (D, lmax)
FLOPS_PER_PAIR = {(3, 5): 235.0, (3, 4): 175.0, (2, 8): 100.0, (4, 6): 870.0}


def make_workload(name: str):
    from paper_2106_10278_amd import inputs
    if name == "c2":
        return inputs.c2_clustered_4pcf()
    if name == "c1":
        return inputs.c1_small_3pcf()
    if name == "c3":
        return inputs.c3_vorticity_4pcf()
    if name == "c5":
        return inputs.c5_hyper_3pcf()
    raise SystemExit(f"unknown workload {name}")


def run_steps(plan, pos, w, steps):
    import torch
    ms = []
    pairs = 0
    stage = {"harmonic": 0.0, "coupling": 0.0, "cells": 0.0}
    launches = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.reset()
        ts = time.perf_counter()
        plan.accumulate(pos, w)
        out = plan.finalize()
        ms.append((time.perf_counter() - ts) * 1e3)
        pairs += plan.pair_count()[0]
        st = plan.stage_ms()
        for k in stage:
            stage[k] += st[k]
        launches += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return out, pairs, ms, stage, launches, wall


def rel_err(got, ref):
    floor = 1e-12 * np.max(np.abs(ref))
    errs = [np.max(np.abs(got[i] - ref[i])) / max(np.max(np.abs(ref[i])), floor) for i in range(ref.shape[0])]
    return float(np.max(errs)), int(np.argmax(errs))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("npcf_harmonic_impl.h",):
        h.update(open(os.path.join(ROOT, "paper_2106_10278_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(key: str):
    """HBM bytes per launch of the harmonic kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "harmonic_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash() or d.get("workload") != key:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(wl, plan_factory, pos, w, sample_per_role: int):
    """Time the FP64 oracle on a bounded sample of primaries (both roles)."""
    import oracle
    nd = wl.n_data
    ranges = [(0, sample_per_role)]
    if wl.pos.shape[1] > nd:
        ranges.append((nd, nd + sample_per_role))
    prims = np.concatenate([np.arange(a, b) for a, b in ranges])
    t0 = time.perf_counter()
    z, pairs = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w, prims=prims)
    dt = time.perf_counter() - t0
    ref = oracle.reported_part(z, oracle.lambda_labels(wl.D, wl.N, wl.lmax), wl.D, wl.N)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    errs = {}
    for prec in ("plain", "mixed_bf16"):
        plan = plan_factory(prec)
        for a, b in ranges:
            plan.accumulate(pos, w, a, b)
        got = plan.finalize()
        gp = plan.pair_count()[0]
        e, worst = rel_err(got, ref)
        errs[prec] = {"max_rel_err": e, "worst_lambda": [int(x) for x in oracle.lambda_labels(wl.D, wl.N, wl.lmax)[worst]],
                      "pairs_match": bool(gp == pairs)}
        plan.close()
    base = {"value": pairs / dt, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(prims)} primaries ({'+'.join(f'[{a},{b})' for a, b in ranges)}) against all "
                      f"{wl.pos.shape[1]} secondaries, {pairs} in-range pairs, {dt:.1f} s",
            "seconds": dt}
    return base, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--cpu-sample", type=int, default=128, help="oracle primaries per role for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="mixed_bf16,plain")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2106_10278_amd import NPCF

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    wl = make_workload(args.workload)
    n = wl.pos.shape[1]
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).to("cuda:0")
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).to("cuda:0")

    def factory(prec):
        return NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, precision=prec, max_points=n)

    results = {}
    for prec in args.precisions.split(","):
        plan = factory(prec)
        for _ in range(args.warmup):
            plan.reset()
            plan.accumulate(pos, w)
            plan.finalize()
        out, pairs, ms, stage, launches, wall = run_steps(plan, pos, w, args.steps)
        results[prec] = {"pairs_per_s": pairs / wall, "ms_per_step": 1e3 * wall / args.steps,
                         "ms_median": float(np.median(ms)), "pairs_per_step": pairs // args.steps,
                         "stage_ms_per_step": {k: v / args.steps for k, v in stage.items()},
                         "harmonic_ms_per_launch": stage["harmonic"] / launches}
        plan.close()

    head = "mixed_bf16" if "mixed_bf16" in results else list(results)[0]
    r = results[head]
    key = f"D{wl.D}-N{wl.N}-lmax{wl.lmax}-{wl.name}"
    fpp = FLOPS_PER_PAIR.get((wl.D, wl.lmax))
    achieved = fpp * r["pairs_per_step"] / (r["harmonic_ms_per_launch"] * 1e-3) if fpp else None
    roof = {"kernel": "k_harmonic", "bound": "alu", "achieved": achieved / 1e12 if achieved else None,
            "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": (achieved / FP32_VECTOR_PEAK) if achieved else None,
            "traffic": load_traffic(key),
            "flops_per_pair": fpp, "launch_ms": r["harmonic_ms_per_launch"]}

    cpu = None
    errs = None
    if not args.no_cpu:
        cpu, errs = cpu_baseline(wl, factory, pos, w, args.cpu_sample)

    line = {
        "metric": "pairs/s + 4PCF wall time, mixed vs plain on one GPU at rel err <=1e-5",
        "value": r["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 harmonics + bf16x3 coupling" if head == "mixed_bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": key, "n_points": n, "n_data": wl.n_data, "D": wl.D, "N": wl.N, "lmax": wl.lmax,
                   "nbins": len(wl.edges) - 1, "r_range": [float(wl.edges[0]), float(wl.edges[-1])],
                   "box": float(wl.box[0]), "parallelism": "single GPU"},
        "paths": results,
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity_vs_oracle": errs,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
