"""Benchmark of the separable NPCF estimator on one MI355X.

Workload (default): isotropic 4PCF in D = 3 -- 200k clustered data points
(half in 2000 Gaussian blobs of sigma 5, half uniform, w = +1) plus 600k
uniform randoms (w = -1/3) in a periodic cube of side 1000, 10 linear radial
bins in [20, 160], lmax = 5 (111 Lambda x 120 radial tuples).  Synthetic,
seeded (see paper_2106_10278_amd/inputs.py).

A step is one pass of the whole path over the catalogue: quantise + cell list,
harmonic stage, coupling stage, FP64 reduction and finalisation
(npcf_reset + npcf_accumulate + npcf_finalize), inputs resident in HBM.
Every coupling precision is timed on the same inputs: plain FP32, FP16 hi+lo
(per-tile power-of-two scaling), BF16 hi+mid+lo and BF16 hi+lo.  The headline
value is the fastest split-precision path whose per-multipole relative error
against the FP64 oracle (on a sample of primaries) is within 1e-5, with a 10%
margin for the sampling of primaries (at most 9e-6 on the sample); the plain
path and the others are reported beside it with their errors.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12      # MI355X, FP32 vector (packed) FLOP/s
MIXED = ("mixed_fp16", "mixed_bf16x6", "mixed_bf16")
DTYPE = {"plain": "f32", "mixed_fp16": "f32 harmonics + fp16 hi+lo coupling",
         "mixed_bf16x6": "f32 harmonics + bf16 hi+mid+lo coupling", "mixed_bf16": "f32 harmonics + bf16 hi+lo coupling"}


def flops_per_pair(D: int, L: int) -> float:
    """Algorithmic FP32 operations of the harmonic stage per in-range pair.

    Geometry: D converts, D scalings, D multiplies + (D-1) adds for r^2, one
    reciprocal square root, D scalings to the unit vector.  Harmonics: the
    azimuthal factor (x + iy)^m by complex multiplication (6 flops per step),
    each Gegenbauer recurrence step c_n = alpha t c_{n-1} - beta c_{n-2}
    (4 flops; D = 4 also scales by rho^2, 1 more), one multiply per real
    output and one add per output to accumulate it (2 flops per real output).
    """
    geo = D + D + (2 * D - 1) + 1 + D
    if D == 2:
        return geo + 6 * L + 2 * (2 * L + 1)
    if D == 3:
        states = (L + 1) * (L + 2) // 2
        outputs = 2 * states - (L + 1)              # m = 0 states are real
        rec = sum(L - m for m in range(L + 1))      # steps with n >= 1
        return geo + 6 * L + 4 * rec + 2 * outputs
    states = (L + 1) * (L + 2) * (L + 3) // 6
    outputs = 2 * states - (L + 1) * (L + 2) // 2   # l1 = 0 states are real
    rec = 2 * sum(L - k for k in range(L + 1))      # c- and g-tables
    pair_products = states                          # g * c per state
    return geo + 1 + 6 * L + 5 * rec + pair_products + 2 * outputs


def scope_flops_per_pair(D: int, L: int) -> float:
    """Per-pair FP32 operations of the harmonic stage in the cost model the
    roofline is quoted against: geometry (10, 25, 30 for D = 2, 3, 4) plus 10
    per stored harmonic state (its share of the recurrences and of the
    azimuthal factor, the weight, and the accumulation of both parts).  This
    gives 235 at D = 3, lmax 5; 175 at D = 3, lmax 4; 100 at D = 2, |m| <= 8
    and 870 at D = 4, lmax 6.  The instruction-level count of flops_per_pair
    (177 at D = 3, lmax 5) leaves out the imaginary parts that vanish for
    m = 0 and counts a real output as one multiply and one add."""
    states = {2: L + 1, 3: (L + 1) * (L + 2) // 2, 4: (L + 1) * (L + 2) * (L + 3) // 6}[D]
    return {2: 10, 3: 25, 4: 30}[D] + 10 * states


def multipole_errors(got, ref, labels):
    """Per-multipole errors against the oracle, one row per (Lambda, part):
    strict max_b |got - ref| / max_b |ref| and the L2 variant
    ||got - ref||_2 / ||ref||_2 over the radial tuples (rows whose reference
    is below 1e-12 of the largest are judged against that floor)."""
    got, ref = np.asarray(got), np.asarray(ref)
    big = np.max(np.abs(ref))
    strict, l2 = [], []
    for i in range(ref.shape[0]):
        d = np.abs(got[i] - ref[i])
        strict.append(np.max(d) / max(np.max(np.abs(ref[i])), 1e-12 * big))
        l2.append(np.sqrt(np.sum(d ** 2)) / max(np.sqrt(np.sum(np.abs(ref[i]) ** 2)), 1e-12 * big))
    strict, l2 = np.array(strict), np.array(l2)
    ws, wl2 = int(np.argmax(strict)), int(np.argmax(l2))
    return {"max_rel_err": float(strict[ws]), "worst_lambda": [int(x) for x in labels[ws]],
            "quantiles": {q: float(np.percentile(strict, v)) for q, v in (("p50", 50), ("p90", 90), ("p99", 99))},
            "l2_max": float(l2[wl2]), "worst_lambda_l2": [int(x) for x in labels[wl2]],
            "per_lambda": [float(f"{e:.3g}") for e in strict]}


def c1_one_core():
    """The oracle on the whole c1 catalogue (2000 points, every primary) with
    one OpenMP thread, in a child process so that the thread count applies."""
    import subprocess
    code = ("import time, sys; sys.path.insert(0, %r)\n"
            "import oracle\n"
            "from paper_2106_10278_amd import inputs\n"
            "wl = inputs.c1_small_3pcf()\n"
            "t = time.perf_counter()\n"
            "z, p = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w)\n"
            "print(time.perf_counter() - t, p)\n") % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return None
    dt, pairs = r.stdout.split()[-2:]
    return {"workload": "c1 (D3-N3-lmax4, 2000 uniform points, every primary)", "cores": 1,
            "seconds": float(dt), "pairs": int(pairs), "pairs_per_s": int(pairs) / float(dt)}


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
    if name == "c6":
        return inputs.c6_los_3pcf()
    if name == "c7":
        return inputs.c7_uniform_5pcf()
    if name == "c8":
        return inputs.c8_grid_4pcf()
    if name == "c9":
        return inputs.c9_sphere_4pcf()
    if name == "c10":
        return inputs.c10_s3_4pcf()
    if name == "c11":
        return inputs.c11_h3_4pcf()
    raise SystemExit(f"unknown workload {name}")


def run_steps(plan, pos, w, steps, field=None):
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
        if field is not None:
            plan.accumulate_grid(field)
        else:
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


def _code_only(text: str) -> str:
    """C++/HIP source without its comments and blank lines, so that the hashes
    below follow the code and not the wording of its comments."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def _sources_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(_code_only(open(os.path.join(ROOT, "paper_2106_10278_amd", "csrc", f)).read()).encode())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    return _sources_hash(("npcf_harmonic_impl.h", "npcf_harmonic_pass.h", "npcf_harmonic_scan.h", "npcf_harmonics.h",
                          "npcf_lanefold.h"))


def harmonic_kernel_name(D: int, lmax: int) -> str:
    """The flat harmonic-stage kernel a plan launches: one pass per radial
    bin by default for D = 2 and 3, the bin-sorted staging kernel for D = 4;
    NPCF_HARMONIC=stage or =pass overrides (the per-bin kernel exists up to
    128 slots per bin: D = 4 up to lmax 5)."""
    states = {2: lmax + 1, 3: (lmax + 1) * (lmax + 2) // 2, 4: (lmax + 1) * (lmax + 2) * (lmax + 3) // 6}[D]
    env = os.environ.get("NPCF_HARMONIC")
    per_bin = env == "pass" if env else D <= 3
    if not per_bin or 2 * states > 128:
        return "k_harmonic"
    return "k_harmonic_pass"


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


def coupling_source_hash() -> str:
    return _sources_hash(("npcf_couple.hip", "npcf_couple_common.h", "npcf_plan4.cpp"))


def coupling_useful_flops(wl, labels) -> float | None:
    """Algorithmic minimum of the factorised D = 3, N = 4 coupling per pass:
    per primary, every term (l1, l2, l3, m1, m2) of every Lambda formed for
    each radial pair b1 < b2 (a complex multiply-add, 8 flops), and every
    (Lambda, m3) group contracted against a_{l3 m3}[b3] for each radial
    triple (8 flops).  About 2.02e6 flops per primary at lmax 5 with 10 bins,
    1.6e12 for the 800k primaries of the 4PCF workload."""
    if wl.D != 3 or wl.N != 4 or wl.Lmax is not None:
        return None
    nb = len(wl.edges) - 1
    terms = groups = 0
    for l1, l2, l3 in (tuple(int(x) for x in r[:3]) for r in labels):
        groups += 2 * l3 + 1
        terms += sum(1 for m1 in range(-l1, l1 + 1) for m2 in range(-l2, l2 + 1) if abs(m1 + m2) <= l3)
    pairs = nb * (nb - 1) // 2
    triples = nb * (nb - 1) * (nb - 2) // 6
    return 8.0 * (terms * pairs + groups * triples) * wl.pos.shape[1]


def coupling_roofline(key: str, path: str, coupling_ms: float, useful=None):
    """MFMA flops per coupling launch from a committed rocprofv3 counter run
    (taken on the current coupling source), over the live coupling-stage time
    of this run (which also holds the 0.5 ms FP64 reduction of partials)."""
    fpath = os.path.join(ROOT, "profiles", "coupling_mfma.json")
    if not os.path.exists(fpath):
        return None
    try:
        d = json.load(open(fpath))
    except Exception:
        return None
    if d.get("coupling_source_sha256_16") != coupling_source_hash() or d.get("workload") != key:
        return None
    e = d.get("paths", {}).get(path)
    if not e:
        return None
    achieved = e["mfma_flops"] / (coupling_ms * 1e-3)
    out = {"kernel": "k_couple4f", "bound": "mfma", "dtype": e["mfma_dtype"], "achieved": achieved / 1e12,
           "peak": e["peak"] / 1e12, "unit": "TFLOP/s", "frac": achieved / e["peak"], "mfma_flops": e["mfma_flops"],
           "stage_ms": coupling_ms, "source": d.get("source")}
    if useful:
        # the algorithmic minimum over the same time: against the path's MFMA
        # peak and against the FP32 vector peak (S formation runs there)
        u = useful / (coupling_ms * 1e-3)
        out.update(useful_flops=useful, useful_achieved=u / 1e12, useful_frac=u / e["peak"],
                   useful_frac_fp32_vector=u / FP32_VECTOR_PEAK)
    return out


def sphere_flops(D: int, L: int, pairs: float) -> float:
    """FP32-equivalent operations of the curved-space harmonic stage (the
    unit D-sphere and hyperbolic space alike; FP64 counted twice, the FP64
    vector peak being half the FP32 one) over its in-range pairs: an FP64 dot
    product of the D + 1 coordinates (2D + 1 operations) for the bin, D FP64
    tangent projections (2D + 1 each), the squared norm (2D - 1) and its
    reciprocal square root, then the harmonics and their accumulation as
    flops_per_pair counts them past the geometry (D = 2: 6 per azimuthal
    step, 2 per real output).  Pairs beyond the bins count nothing, as on the
    flat path: tiles out of reach are skipped whole and the rest fail an FP32
    pre-test."""
    geo_flat = D + D + (2 * D - 1) + 1 + D
    harm = flops_per_pair(D, L) - geo_flat
    return (2.0 * (2 * D + 1) + 2 * (D * (2 * D + 1) + (2 * D - 1)) + 1 + harm) * pairs


def grid_stage_bytes(wl) -> float:
    """Algorithmic HBM bytes of one pass of the gridded harmonic stage: the
    weights (read X, write w64, w32 and the complex FFT input), the forward
    FFT of w (D passes, read + write), the batched inverse FFTs over every
    (bin, state) with the spectral product taken on the first pass's load
    (D passes, read + write, plus the spectrum of w once), and the row
    transposes (complex FP64 in, complex FP32 out, weights)."""
    D = wl.D
    ng = float(np.prod(wl.field.shape))
    nst = {2: wl.lmax + 1, 3: (wl.lmax + 1) * (wl.lmax + 2) // 2}[D]
    nbs = (len(wl.edges) - 1) * nst
    return (36 + 32 * D + 16 + 8) * ng + (32 * D + 16 + 8) * nbs * ng


def mixed_vs_plain(results, head):
    """The metric's comparison: the headline split-precision path against
    plain FP32, per step and in the coupling stage (the only stage the split
    changes), with which of the two is faster."""
    if head == "plain" or "plain" not in results or head not in results:
        return None
    m, p = results[head], results["plain"]
    return {"mixed_path": head, "mixed_ms_per_step": m["ms_per_step"], "plain_ms_per_step": p["ms_per_step"],
            "speedup": p["ms_per_step"] / m["ms_per_step"],
            "mixed_coupling_ms": m["stage_ms_per_step"]["coupling"],
            "plain_coupling_ms": p["stage_ms_per_step"]["coupling"],
            "faster": "mixed" if m["ms_per_step"] < p["ms_per_step"] else "plain",
            "note": "the split changes only the coupling's MFMA slices; S is formed on the vector ALU in "
                    "FP32 either way, and the split operands' extra registers cost occupancy"}


def cpu_baseline(wl, plan_factory, pos, w, sample_per_role: int, field=None, target_s: float = 12.0):
    """Time the FP64 oracle on a bounded sample of primaries (both roles):
    first `sample_per_role` primaries per role, then, if that took well under
    `target_s`, a sample scaled to about `target_s` of CPU work (at most each
    role's size).  The GPU paths' errors are taken on the timed sample."""
    import oracle
    nd = wl.n_data
    n = wl.pos.shape[1]
    Lmax = wl.Lmax

    def sample(per):
        r = [(0, min(per, nd))]
        if n > nd:
            r.append((nd, nd + min(per, n - nd)))
        return r

    def timed(r):
        prims = np.concatenate([np.arange(a, b) for a, b in r])
        t0 = time.perf_counter()
        z, pairs = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w, prims=prims, Lmax=Lmax,
                               sphere=wl.sphere, hyperbolic=wl.hyperbolic)
        return prims, z, pairs, time.perf_counter() - t0

    ranges = sample(sample_per_role)
    prims, z, pairs, dt = timed(ranges)
    if dt < 0.5 * target_s:
        per = int(sample_per_role * target_s / max(dt, 1e-3))
        bigger = sample(per)
        if sum(b - a for a, b in bigger) > len(prims):
            ranges = bigger
            prims, z, pairs, dt = timed(ranges)
    ref = oracle.reported_part(z, oracle.lambda_labels(wl.D, wl.N, wl.lmax, Lmax), wl.D, wl.N, los=Lmax is not None)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    errs = {}
    for prec in ("plain",) + MIXED:
        plan = plan_factory(prec)
        for a, b in ranges:
            if field is not None:
                plan.accumulate_grid(field, a, b)
            else:
                plan.accumulate(pos, w, a, b)
        got = plan.finalize()
        gp = plan.pair_count()[0]
        labels = oracle.lambda_labels(wl.D, wl.N, wl.lmax, Lmax)
        if wl.D == 2:
            # complex output: one row per (Lambda, Re/Im)
            got = np.concatenate([got.real, got.imag])
            ref_rows = np.concatenate([ref.real, ref.imag])
            labels = np.concatenate([labels, labels])
        else:
            ref_rows = ref
        errs[prec] = multipole_errors(got, ref_rows, labels) | {"pairs_match": bool(gp == pairs)}
        plan.close()
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    base = {"value": pairs / dt, "unit": "pairs/s", "cores": cores, "cpu_model": cpu_model, "kind": "oracle",
            "sample": f"{len(prims)} primaries ({'+'.join(f'[{a},{b})' for a, b in ranges)}) against all "
                      f"{wl.pos.shape[1]} secondaries, {pairs} in-range pairs, {dt:.1f} s",
            "seconds": dt}
    if wl.name.startswith("D3-N4-clustered"):
        base["c1_one_core"] = c1_one_core()
    return base, errs


def run_batch(precisions, steps: int, warmup: int, tune: bool = True):
    """The batched workload: 64 D = 3, N = 4 catalogues (data sizes
    log-uniform in [20k, 300k], clustered as c2, plus 3x randoms at w = -1/3)
    in one npcf_accumulate_batch per step (captured HIP graph, replayed).
    Reports aggregate pairs/s over the wall time of accumulate_batch +
    finalize of every catalogue, and percentiles of the per-catalogue
    completion times taken from device-clock timestamps."""
    import torch
    from paper_2106_10278_amd import NPCF, inputs
    sizes = inputs.c4_batch_sizes()
    pos, w = [], []
    ref = None
    for c, nd in enumerate(sizes):
        wl = inputs.c4_catalogue(c, nd)
        ref = ref or wl
        pos.append(torch.from_numpy(np.ascontiguousarray(wl.pos)).to("cuda:0"))
        w.append(torch.from_numpy(np.ascontiguousarray(wl.w)).to("cuda:0"))
    npts = int(sum(int(x.shape[1]) for x in pos))
    out = {"workload": f"D3-N4-lmax5 batch of {len(sizes)} catalogues (data log-uniform in [20k, 300k], "
                       f"clustered as c2, + 3x randoms w=-1/3), {npts} points",
           "catalogues": len(sizes), "points": npts, "paths": {}}
    for prec in precisions:
        big = int(np.argmax([int(x.shape[1]) for x in pos]))
        plan = NPCF(3, 4, 5, ref.edges, ref.box, precision=prec, max_points=int(pos[big].shape[1]))
        tuning = plan.autotune(pos[big], w[big]) if tune else None   # tile shapes from the largest catalogue
        walls, lat, pairs = [], [], 0
        for it in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.accumulate_batch(pos, w)
            res = [plan.finalize_batch(c) for c in range(len(sizes))]
            torch.cuda.synchronize()
            if it >= warmup:
                walls.append(time.perf_counter() - t0)
                lat.extend(r[1] for r in res)
                pairs += sum(r[2] for r in res)
        plan.close()
        wall = float(np.sum(walls))
        out["paths"][prec] = {
            "pairs_per_s": pairs / wall, "wall_ms_per_batch": 1e3 * wall / steps, "pairs_per_batch": pairs // steps,
            "latency_ms": {q: float(np.percentile(lat, v)) for q, v in (("p50", 50), ("p90", 90), ("p99", 99))}
            | {"max": float(np.max(lat))}, "tuning": tuning}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--cpu-sample", type=int, default=128, help="oracle primaries per role for cpu_baseline "
                    "(first sample; scaled up to about --cpu-seconds of CPU work)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU work the oracle sample is scaled to")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="mixed_fp16,mixed_bf16x6,plain,mixed_bf16")
    ap.add_argument("--batch-steps", type=int, default=1, help="timed passes of the batched workload (0: skip)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes (no autotuner)")
    ap.add_argument("--tuning", default="",
                    help="fixed 'cell_subdiv,couple_block[,curved_bins_per_pass]' instead of the autotuner")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
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
    # gridded workloads: the field on the grid; the nodes are the catalogue
    field = torch.from_numpy(np.ascontiguousarray(wl.field)).to("cuda:0") if wl.field is not None else None

    def factory(prec):
        return NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, precision=prec, max_points=n,
                    Lmax=wl.Lmax, sphere=wl.sphere, hyperbolic=wl.hyperbolic)

    results = {}
    plan_labels = None
    for prec in args.precisions.split(","):
        plan = factory(prec)
        plan_labels = plan.lambda_labels
        if args.tuning:
            knobs = [int(x) for x in args.tuning.split(",")]
            plan.set_tuning(cell_subdiv=knobs[0], couple_block=knobs[1])
            if len(knobs) > 2:
                plan.apply_tuning(curved_bins_per_pass=knobs[2])
            tuning = plan.tuning() | {"fixed": True}
        elif field is None:
            tuning = plan.autotune(pos, w) if not args.no_tune else None
        else:
            tuning = None   # no cell grid on the gridded path
        for _ in range(args.warmup):
            plan.reset()
            if field is not None:
                plan.accumulate_grid(field)
            else:
                plan.accumulate(pos, w)
            plan.finalize()
        out, pairs, ms, stage, launches, wall = run_steps(plan, pos, w, args.steps, field)
        results[prec] = {"pairs_per_s": pairs / wall, "ms_per_step": 1e3 * wall / args.steps,
                         "ms_median": float(np.median(ms)), "pairs_per_step": pairs // args.steps,
                         "stage_ms_per_step": {k: v / args.steps for k, v in stage.items()},
                         "harmonic_ms_per_launch": stage["harmonic"] / launches, "tuning": tuning}
        plan.close()

    cpu = None
    errs = None
    if not args.no_cpu:
        cpu, errs = cpu_baseline(wl, factory, pos, w, args.cpu_sample, field, args.cpu_seconds)

    # headline: the fastest split-precision path within 1e-5 of the oracle,
    # with a 10% margin for the sample of primaries (BF16 hi+lo sits at the
    # bar on c2: 9.4e-6 to 1.04e-5 over samples); without the oracle check,
    # the FP16 hi+lo path, which carries 22 bits
    cands = [p for p in MIXED if p in results and (errs is None or errs[p]["max_rel_err"] <= 0.9e-5)]
    if errs is None:
        cands = [p for p in ("mixed_fp16",) if p in results] or cands
    head = (max(cands, key=lambda p: results[p]["pairs_per_s"]) if cands
            else ("plain" if "plain" in results else list(results)[0]))
    r = results[head]
    key = f"D{wl.D}-N{wl.N}-lmax{wl.lmax}-{wl.name}"
    fpp = scope_flops_per_pair(wl.D, wl.lmax)
    achieved = fpp * r["pairs_per_step"] / (r["harmonic_ms_per_launch"] * 1e-3)
    roof = {"kernel": harmonic_kernel_name(wl.D, wl.lmax), "bound": "alu", "achieved": achieved / 1e12,
            "peak": FP32_VECTOR_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
            "traffic": load_traffic(key), "flops_per_pair": fpp,
            "flops_per_pair_instruction_level": flops_per_pair(wl.D, wl.lmax),
            "launch_ms": r["harmonic_ms_per_launch"]}
    if wl.sphere or wl.hyperbolic:
        fl = sphere_flops(wl.D, wl.lmax, r["pairs_per_step"])
        ach = fl / (r["harmonic_ms_per_launch"] * 1e-3)
        roof = {"kernel": "k_sphere", "bound": "alu", "achieved": ach / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": ach / FP32_VECTOR_PEAK, "traffic": None,
                "flops_per_pass": fl, "launch_ms": r["harmonic_ms_per_launch"]}
    if field is not None:
        # the gridded harmonic stage is FFT passes over HBM, not pair arithmetic
        gb = grid_stage_bytes(wl)
        ach = gb / (r["stage_ms_per_step"]["harmonic"] * 1e-3)
        roof = {"kernel": "gridded harmonic stage (k_grid_weights, k_fft_axis passes, k_grid_rows)", "bound": "hbm",
                "achieved": ach / 1e9, "peak": 8000.0, "unit": "GB/s", "frac": ach / 8.0e12, "traffic": None,
                "bytes_per_pass": gb, "launch_ms": r["stage_ms_per_step"]["harmonic"]}

    batch = None
    if args.batch_steps > 0 and args.workload == "c2":
        batch = run_batch([head, "plain"] if head != "plain" else ["plain"], args.batch_steps, 1, not args.no_tune)

    line = {
        "metric": "pairs/s + 4PCF wall time, mixed vs plain on one GPU at rel err <=1e-5",
        "value": r["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE.get(head, head), "headline_path": head,
        "data": "synthetic",
        "config": {"workload": key, "n_points": n, "n_data": wl.n_data, "D": wl.D, "N": wl.N, "lmax": wl.lmax,
                   "nbins": len(wl.edges) - 1, "r_range": [float(wl.edges[0]), float(wl.edges[-1])],
                   "box": float(wl.box[0]), "geometry": (f"unit {wl.D}-sphere" if wl.sphere else
                                (f"hyperbolic {wl.D}-space" if wl.hyperbolic else "flat")),
                   "parallelism": "single GPU"},
        "paths": results,
        "roofline": roof,
        "mixed_vs_plain": mixed_vs_plain(results, head),
        "coupling_roofline": coupling_roofline(key, head, r["stage_ms_per_step"]["coupling"],
                                               coupling_useful_flops(wl, plan_labels)),
        "cpu_baseline": cpu,
        "parity_vs_oracle": errs,
        "batch": batch,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
