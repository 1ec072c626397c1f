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


def condition_scale(wl, btuple_mode=0, prims=None, periodic=True, Lmax=None):
    """Sum of the magnitudes of every term of the estimator,
    (1/V) sum_i |w_i| sum_terms |C| prod_k |a_i^{b_k}[s_k]|, per (Lambda, b-tuple),
    from the oracle's a_lm and coupling coefficients (eq. NPCF-estimator-discrete
    with every term replaced by its absolute value).  A sum evaluated with unit
    roundoff u has forward error bounded by about u times this scale, so errors
    are judged against it where the multipole itself cancels."""
    sphere = getattr(wl, "sphere", False)
    hyp = getattr(wl, "hyperbolic", False)
    a, _ = oracle.alm(wl.D, wl.lmax, wl.edges, wl.box, wl.pos, wl.w, prims=prims, periodic=periodic, sphere=sphere,
                      hyperbolic=hyp)
    if hyp:
        V = float(wl.box[0])   # the region's volume
    elif sphere:
        V = 4 * np.pi if wl.D == 2 else 2 * np.pi ** 2   # the unit 2- or 3-sphere's volume
    else:
        V = float(np.prod(np.asarray(wl.box, dtype=np.float64)[: wl.D]))
    lam, s, c = oracle.coupling_terms(wl.D, wl.N, wl.lmax, Lmax)
    nb = len(wl.edges) - 1
    bts = oracle.btuple_labels(nb, wl.N, btuple_mode)
    nlam = len(oracle.lambda_labels(wl.D, wl.N, wl.lmax, Lmax))
    w = np.abs(wl.w if prims is None else wl.w[prims])
    A = np.abs(a)
    out = np.zeros((nlam, len(bts)))
    if wl.N == 5:
        # four legs: gather the b-tuples' legs per chunk of terms
        for t0 in range(0, len(lam), 4096):
            sl = slice(t0, t0 + 4096)
            X = w[:, None, None] * A[:, bts[:, 0]][:, :, s[sl, 0]]
            for k in range(1, 4):
                X = X * A[:, bts[:, k]][:, :, s[sl, k]]
            np.add.at(out, lam[sl], np.abs(c[sl])[:, None] * X.sum(axis=0).T)
        return out / V
    for t in range(len(lam)):
        if wl.N == 3:
            m = np.einsum("i,ij,ik->jk", w, A[:, :, s[t, 0]], A[:, :, s[t, 1]])
            out[lam[t]] += abs(c[t]) * m[bts[:, 0], bts[:, 1]]
        else:
            m = np.einsum("i,ij,ik,il->jkl", w, A[:, :, s[t, 0]], A[:, :, s[t, 1]], A[:, :, s[t, 2]])
            out[lam[t]] += abs(c[t]) * m[bts[:, 0], bts[:, 1], bts[:, 2]]
    return out / V


def conditioned_error(got, ref, scale):
    """max over multipoles of max_b |got - ref| / max_b scale."""
    got, ref = np.asarray(got), np.asarray(ref)
    errs = np.array([np.max(np.abs(got[i] - ref[i])) / max(np.max(scale[i]), 1e-300) for i in range(ref.shape[0])])
    return float(errs.max()) if errs.size else 0.0, errs


def oracle_reported(wl, prims=None, btuple_mode=0, Lmax=None):
    z, pairs = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w, prims=prims,
                           btuple_mode=btuple_mode, Lmax=Lmax, sphere=getattr(wl, "sphere", False),
                           hyperbolic=getattr(wl, "hyperbolic", False))
    labels = oracle.lambda_labels(wl.D, wl.N, wl.lmax, Lmax)
    return oracle.reported_part(z, labels, wl.D, wl.N, los=Lmax is not None), pairs, z


def gpu_run(wl, ranges=None, precision="plain", btuple_mode=0, device="cuda:0", plan=None, Lmax=None):
    import torch
    from paper_2106_10278_amd import NPCF
    pos = torch.from_numpy(np.ascontiguousarray(wl.pos)).to(device)
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).to(device)
    n = wl.pos.shape[1]
    if plan is None:
        plan = NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, btuple_mode=btuple_mode, precision=precision,
                    max_points=n, Lmax=Lmax, sphere=getattr(wl, "sphere", False),
                    hyperbolic=getattr(wl, "hyperbolic", False))
    if ranges is None:
        ranges = [(0, n)]
    for a, b in ranges:
        plan.accumulate(pos, w, a, b)
    out = plan.finalize()
    pairs = plan.pair_count()[0]
    return out, pairs, plan


def alm_error(got, ref, wl, prims, D, lmax, sphere=False, hyperbolic=False):
    """Largest |got - ref| of a^b_[l] values, each over a bound on the sum of
    the magnitudes of its terms: |w_k conj(Y_s)| <= |w_k| sqrt(dim_l / |S^{D-1}|)
    (the addition theorem bounds every harmonic of order l), so with
    A_0 = a^b_0 evaluated with |w|, which is sum_k |w_k| / (v_b sqrt|S^{D-1}|),
    the bound of state s is A_0 sqrt(dim_l) (dim_l = 1, 2l + 1, (l + 1)^2 for
    D = 2, 3, 4).  Judged value by value, small multipoles are held to their
    own scale rather than to the largest |a|.  `got` and `ref` are in the
    library's stored-state order, [prim][bin][state]."""
    from paper_2106_10278_amd import stored_state_labels
    a_abs, _ = oracle.alm(D, lmax, wl.edges, wl.box, wl.pos, np.abs(wl.w), prims=prims, sphere=sphere,
                          hyperbolic=hyperbolic)
    olab = [tuple(int(x) for x in r) for r in oracle.state_labels(D, lmax)]
    zero = (0,) if D == 2 else ((0, 0) if D == 3 else (0, 0, 0))
    A0 = np.abs(a_abs[:, :, olab.index(zero)])
    st = stored_state_labels(D, lmax)
    top = st[:, 0] if D == 2 else (st[:, 1] if D == 3 else st[:, 2])
    dim = np.ones(len(st)) if D == 2 else ((2 * top + 1.0) if D == 3 else (top + 1.0) ** 2)
    bound = A0[:, :, None] * np.sqrt(dim)[None, None, :]
    bound = np.maximum(bound, 1e-300)
    return float(np.max(np.abs(np.asarray(got) - np.asarray(ref)) / bound))


def strict_where_well_conditioned(got, ref, scale, kappa_max=3.0):
    """Strict per-multipole errors on the rows whose condition number
    kappa = max_b S / max_b |ref| (S: sum of the magnitudes of the estimator's
    terms) is at most kappa_max.  A sum evaluated with unit roundoff u has
    error below about u S, so on such a row the strict error is within
    kappa_max of the conditioned one; rows above it are multipoles that cancel
    to a small fraction of their terms.  Returns (largest strict error over
    the well-conditioned rows, their count, kappa of every row)."""
    got, ref, scale = np.asarray(got), np.asarray(ref), np.asarray(scale)
    kappa = np.array([np.max(scale[i]) / max(np.max(np.abs(ref[i])), 1e-300) for i in range(ref.shape[0])])
    _, errs = per_multipole_error(got, ref)
    sel = kappa <= kappa_max
    return (float(np.max(errs[sel])) if np.any(sel) else 0.0), int(np.sum(sel)), kappa


def curved_widths(plan):
    """The bins per pass a curved-space plan accepts (its kernel's two widths,
    or one when they coincide), found by trying every value: the rule stays
    in the library.  The plan keeps its default afterwards."""
    from paper_2106_10278_amd.binding import NPCFError
    default = plan.tuning()["curved_bins_per_pass"]
    ok = []
    for g in range(1, 17):
        try:
            plan.apply_tuning(curved_bins_per_pass=g)
            ok.append(g)
        except NPCFError:
            pass
    plan.apply_tuning(curved_bins_per_pass=default)
    return ok


def curved_plan(wl, width):
    """A plan for a curved-space workload at its kernel's wide or narrow
    (default) width."""
    from paper_2106_10278_amd import NPCF
    plan = NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, max_points=wl.pos.shape[1],
                sphere=getattr(wl, "sphere", False), hyperbolic=getattr(wl, "hyperbolic", False))
    widths = curved_widths(plan)
    plan.apply_tuning(curved_bins_per_pass=min(widths) if width == "narrow" else max(widths))
    return plan



def _fma(a, b, c):
    """a * b + c rounded once (exact rational arithmetic, then one rounding)."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def fused_distance_catalogue(seed=5, n_fill=200):
    """A D = 3 periodic catalogue (box 1024, a power of two, so lattice offsets
    times the lattice scale are exact in FP64) with one planted pair whose
    squared distance, summed axis by axis with every product and sum rounded,
    lies one ulp below the outermost squared edge, while the same sum with
    the products fused into FMAs (the compiler's contraction of
    x*x + y*y + z*z) lands on the edge: the definition counts the pair, the
    fused form does not.  Returns (workload, r2 by the definition, r2 fused,
    squared outer edge)."""
    import math
    from paper_2106_10278_amd import inputs
    L = 1024.0
    sc = L / 2.0 ** 32
    rng = np.random.default_rng(seed)
    for _ in range(100000):
        d = rng.integers(2 ** 26, 2 ** 27, size=3) * rng.choice([-1, 1], size=3)
        v = [float(x) * sc for x in d]
        r2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]
        r2f = _fma(v[2], v[2], _fma(v[1], v[1], v[0] * v[0]))
        if not r2 < r2f:
            continue
        e = math.sqrt(r2f)
        for step in (0, 1, -1, 2, -2):
            ee = e
            for _ in range(abs(step)):
                ee = math.nextafter(ee, math.inf if step > 0 else -math.inf)
            if ee * ee == r2f:
                p = np.array([300.0, 400.0, 500.0])
                q = p + np.array(v)
                fill = inputs.uniform(rng, n_fill, [L] * 3)
                pos = np.concatenate([p[:, None], q[:, None], fill], axis=1)
                n = pos.shape[1]
                w = rng.uniform(0.5, 1.5, size=n)
                edges = np.array([ee / 3, 2 * ee / 3, ee])
                wl = inputs.Workload("fused-distance", 3, 3, 2, edges, [L] * 3, pos, w, n)
                return wl, r2, r2f, ee * ee
    raise RuntimeError("no planted pair found")


def pair_count_by_definition(wl):
    """In-range ordered pairs (self pairs excluded) with the squared distance
    summed axis by axis, every product and sum rounded (numpy applies no
    contraction), minimum image in a periodic box."""
    pos = np.asarray(wl.pos, dtype=np.float64)
    box = np.asarray(wl.box, dtype=np.float64)
    e2lo, e2hi = wl.edges[0] * wl.edges[0], wl.edges[-1] * wl.edges[-1]
    n = pos.shape[1]
    count = 0
    for j in range(n):
        r2 = np.zeros(n)
        for k in range(wl.D):
            v = pos[k] - pos[k, j]
            v = v - box[k] * np.rint(v / box[k])
            r2 = r2 + v * v
        ok = (r2 >= e2lo) & (r2 < e2hi)
        ok[j] = False
        count += int(ok.sum())
    return count


def fused_dot_sphere_catalogue(seed=9, n_fill=150):
    """Points on the unit 2-sphere with one planted pair whose cosine, the
    dot product summed left to right with every product and sum rounded,
    lies one or more ulps above cos of the outermost edge, while the same sum
    with the products fused into FMAs lands on it: the definition counts the
    pair (cos e_last < c), the fused form does not.  Returns (workload,
    cosine by the definition, fused cosine, cos of the outer edge)."""
    import math
    from paper_2106_10278_amd import inputs
    rng = np.random.default_rng(seed)
    for _ in range(100000):
        p = inputs.sphere_points(rng, 1)[:, 0]
        q = inputs.sphere_points(rng, 1)[:, 0]
        c = (p[0] * q[0] + p[1] * q[1]) + p[2] * q[2]
        cf = _fma(p[2], q[2], _fma(p[1], q[1], p[0] * q[0]))
        if not (c > cf and -0.9 < cf < 0.5):
            continue
        e = math.acos(cf)
        for step in (0, 1, -1, 2, -2, 3, -3):
            ee = e
            for _ in range(abs(step)):
                ee = math.nextafter(ee, math.inf if step > 0 else -math.inf)
            if math.cos(ee) == cf:
                fill = inputs.sphere_points(rng, n_fill)
                pos = np.concatenate([p[:, None], q[:, None], fill], axis=1)
                n = pos.shape[1]
                w = rng.uniform(0.5, 1.5, size=n)
                edges = np.array([ee / 4, ee / 2, ee])
                wl = inputs.Workload("fused-dot-sphere", 2, 3, 3, edges, [1.0, 1.0], pos, w, n, sphere=True)
                return wl, c, cf, math.cos(ee)
    raise RuntimeError("no planted pair found")


def sphere_pair_count_by_definition(wl):
    """In-range ordered pairs on the sphere (self pairs excluded): cosine
    summed left to right with every product and sum rounded (numpy applies no
    contraction), cos e_last < c <= cos e_0."""
    import math
    pos = np.asarray(wl.pos, dtype=np.float64)
    chi, clo = math.cos(wl.edges[0]), math.cos(wl.edges[-1])
    n = pos.shape[1]
    count = 0
    for j in range(n):
        c = (pos[0, j] * pos[0] + pos[1, j] * pos[1]) + pos[2, j] * pos[2]
        ok = (c <= chi) & (c > clo)
        ok[j] = False
        count += int(ok.sum())
    return count
