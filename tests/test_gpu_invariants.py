"""Invariants of the estimator checked on the GPU path itself (GPU against
GPU, within the precision tolerance), as the oracle pins check them in FP64:
weight scaling zeta(c w) = c^N zeta(w); lattice translations of the periodic
box; proper symmetries of the cube (every component unchanged) and improper
ones (odd-parity components change sign, eq. basis-parity-conj); a random
rotation of a catalogue in an open box; the l = 0 row as weighted counts."""
import math

import numpy as np
import pytest

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import condition_scale, conditioned_error, gpu_run

pytestmark = pytest.mark.gpu


def _run(wl, pos=None, w=None, periodic=True, precision="plain", mode=1):
    import torch
    from paper_2106_10278_amd import NPCF
    pos = wl.pos if pos is None else pos
    w = wl.w if w is None else w
    plan = NPCF(wl.D, wl.N, wl.lmax, wl.edges, wl.box, periodic=periodic, btuple_mode=mode, precision=precision,
                max_points=pos.shape[1])
    plan.accumulate(torch.from_numpy(np.ascontiguousarray(pos)).cuda(), torch.from_numpy(np.ascontiguousarray(w)).cuda())
    out = plan.finalize()
    pairs = plan.pair_count()[0]
    plan.close()
    return out, pairs


def _parity(wl):
    lab = oracle.lambda_labels(wl.D, wl.N, wl.lmax)
    if wl.N == 5:
        return lab[:, 0] + lab[:, 1] + lab[:, 3] + lab[:, 4]
    return 2 * lab[:, 0] if wl.N == 3 else lab.sum(axis=1)


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (3, 5, 2), (2, 4, 4), (4, 3, 3)])
@pytest.mark.parametrize("precision", ["plain", "mixed_bf16x6"])
def test_weight_scaling_and_translation(D, N, lmax, precision):
    wl = inputs.tiny(D, N, lmax, 300, seed=800 + 10 * D + N, box_side=10.0, rmax=4.0, nbins=3)
    print(f"[case] invariants D={D} N={N} {precision}", flush=True)
    z, p = _run(wl, precision=precision)
    scale = condition_scale(wl, 1)
    z2, p2 = _run(wl, w=2.5 * wl.w, precision=precision)
    assert p2 == p
    cerr, _ = conditioned_error(z2 / 2.5 ** N, z, scale)
    assert cerr <= 2e-6
    shift = inputs.to_lattice(wl.pos + np.array([1.75, -2.5, 3.125, 0.5])[:D, None], wl.box)
    z3, p3 = _run(wl, pos=shift, precision=precision)
    assert p3 == p
    cerr, _ = conditioned_error(z3, z, scale)
    assert cerr <= 2e-6


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (3, 5, 2), (4, 3, 2)])
def test_cube_symmetries(D, N, lmax):
    wl = inputs.tiny(D, N, lmax, 300, seed=820 + 10 * D + N, box_side=10.0, rmax=4.0, nbins=3)
    print(f"[case] cube symmetries D={D} N={N}", flush=True)
    z, p = _run(wl)
    scale = condition_scale(wl, 1)
    par = _parity(wl)
    rng = np.random.default_rng(31)
    for _ in range(3):
        perm = rng.permutation(D)
        flips = rng.integers(0, 2, size=D)
        pos = wl.pos[list(perm)].copy()
        for ax, f in enumerate(flips):
            if f:
                pos[ax] = np.mod(wl.box[ax] - pos[ax], wl.box[ax])
        det = np.linalg.det(np.eye(D)[perm]) * np.prod([-1 if f else 1 for f in flips])
        z2, p2 = _run(wl, pos=inputs.to_lattice(pos, wl.box))
        assert p2 == p
        sign = np.where((par % 2 == 1) & (det < 0), -1.0, 1.0)
        cerr, _ = conditioned_error(z2, sign[:, None] * z, scale)
        assert cerr <= 2e-6


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (3, 3, 5)])
def test_open_box_rotation(D, N, lmax):
    """Points in a ball far from the walls of an open box: a random rotation
    about the ball's centre leaves every isotropic component unchanged."""
    rng = np.random.default_rng(51)
    n, L, R = 400, 40.0, 8.0
    x = rng.normal(size=(D, n))
    x = x / np.linalg.norm(x, axis=0) * (R * rng.uniform(0, 1, size=n) ** (1.0 / D))
    q, r = np.linalg.qr(rng.normal(size=(D, D)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    c = L / 2
    wl = inputs.Workload("ball", D, N, lmax, np.linspace(1.0, 5.0, 4), [L] * D, inputs.to_lattice(x + c, [L] * D),
                         rng.uniform(-0.5, 1.5, size=n), n)
    print(f"[case] open-box rotation D={D} N={N}", flush=True)
    z, p = _run(wl, periodic=False)
    z2, _ = _run(wl, pos=inputs.to_lattice(q @ x + c, [L] * D), periodic=False)
    scale = condition_scale(wl, 1, periodic=False)
    cerr, _ = conditioned_error(z2, z, scale)
    # the rotated points are snapped back to the 2^-32 lattice (moves of ~1e-8):
    # with ~4e4 pairs no distance of this seed lies that close to an edge
    assert cerr <= 2e-6


def test_l0_row_is_weighted_count():
    wl = inputs.tiny(3, 4, 3, 300, seed=77, box_side=10.0, rmax=4.0, nbins=3)
    print("[case] l = 0 row", flush=True)
    z, _ = _run(wl)
    lab = oracle.lambda_labels(3, 4, 3)
    i0 = int(np.nonzero(np.all(lab == 0, axis=1))[0][0])
    nb = 3
    vb = np.array([oracle.bin_volume(3, wl.edges[b], wl.edges[b + 1]) for b in range(nb)])
    bt = oracle.btuple_labels(nb, 4, 1)
    ref = np.zeros(len(bt))
    box = np.asarray(wl.box)[:, None]
    e2 = wl.edges ** 2
    for j in range(wl.pos.shape[1]):
        d = wl.pos - wl.pos[:, j:j + 1]
        d -= box * np.round(d / box)
        r2 = (d * d).sum(0)
        ok = (r2 >= e2[0]) & (r2 < e2[-1])
        b = np.searchsorted(e2, r2[ok], side="right") - 1
        W = np.bincount(b, weights=wl.w[ok], minlength=nb) / vb
        ref += wl.w[j] * np.prod(W[bt], axis=1)
    ref /= np.prod(wl.box) * (4 * math.pi) ** 1.5
    assert np.max(np.abs(z[i0] - ref)) <= 2e-6 * np.max(np.abs(ref))
