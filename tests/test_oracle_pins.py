"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (mpmath Ferrers functions, SciPy spherical harmonics and Gegenbauer
polynomials, SymPy Wigner/Clebsch-Gordan symbols), a closed form, an
invariance, an exact count printed in the paper, or a brute-force O(n^N)
evaluation of the naive estimator at tiny n (the paper's own check that the
naive and separable estimators agree, section Applications, Fig. 3 caption).
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.special import eval_gegenbauer, roots_legendre, sph_harm_y
from sympy.physics.wigner import clebsch_gordan, wigner_3j

import labels_indep
import oracle
from paper_2106_10278_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sphere_area(D):
    return 2.0 * math.pi ** (D / 2) / math.gamma(D / 2)


def rand_unit(rng, D):
    x = rng.normal(size=D)
    return x / np.linalg.norm(x)


def rand_rotation(rng, D):
    q, r = np.linalg.qr(rng.normal(size=(D, D)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# --------------------------------------------------------------------------
# Single-particle basis
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mu", [0, 0.5, 1, 1.5, 2, 2.5, 3, 3.5, 5.5])
def test_ferrers_matches_mpmath(mu):
    """Ferrers functions of the first kind (DLMF 14.3) used by eq. hypersph-def."""
    for n in range(0, 7):
        for x in [-0.93, -0.4, 0.013, 0.31, 0.88]:
            # DLMF 14.3.1: P^{-mu}_nu(x) = ((1-x)/(1+x))^{mu/2} F(nu+1, -nu; mu+1; (1-x)/2) / Gamma(mu+1)
            nu = mu + n
            ref = float(((1 - mpmath.mpf(x)) / (1 + mpmath.mpf(x))) ** (mpmath.mpf(mu) / 2)
                        * mpmath.hyp2f1(nu + 1, -nu, mu + 1, (1 - mpmath.mpf(x)) / 2) / mpmath.gamma(mu + 1))
            got = oracle.ferrers_neg(mu, n, x)
            assert got == pytest.approx(ref, rel=1e-11, abs=1e-14), (mu, n, x)


def test_d3_harmonics_match_scipy():
    """D = 3 closed form of section Hyperspherical Harmonics: the P^{-l1}_{l2}
    form equals (-1)^m times SciPy's Condon-Shortley Y_l^m (DLMF 14.9.3)."""
    rng = np.random.default_rng(0)
    lab = oracle.state_labels(3, 7)
    for _ in range(20):
        x = rng.normal(size=3)
        r = np.linalg.norm(x)
        th, ph = np.arccos(x[2] / r), np.arctan2(x[1], x[0])
        got = oracle.harmonics(3, 7, x)
        ref = np.array([(-1.0) ** int(m) * sph_harm_y(int(l), int(m), th, ph) for m, l in lab])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_d2_harmonics_closed_form():
    """D = 2: Y_l = e^{i l theta_1} / sqrt(2 pi)."""
    for th in [0.1, 1.3, 2.9, -2.0]:
        got = oracle.harmonics(2, 6, np.array([3.0 * math.cos(th), 3.0 * math.sin(th)]))
        lab = oracle.state_labels(2, 6)[:, 0]
        np.testing.assert_allclose(got, np.exp(1j * lab * th) / math.sqrt(2 * math.pi), atol=1e-14)


@pytest.mark.parametrize("D,lmax", [(2, 5), (3, 4), (4, 3)])
def test_state_count_formula(D, lmax):
    """Number of states of total angular momentum l: binom(l+D-3, D-3)(2l+D-2)/(D-2)
    for D >= 3, one for D = 2 (section Connection to Angular Momentum Eigenstates)."""
    lab = oracle.state_labels(D, lmax)
    for l in range(lmax + 1):
        cnt = int(np.sum(lab[:, -1] == l))
        if D == 2:
            assert int(np.sum(lab[:, 0] == l)) == 1
            continue
        ref = math.comb(l + D - 3, D - 3) * (2 * l + D - 2) // (D - 2)
        assert cnt == ref
        if D == 4:
            assert cnt == (l + 1) ** 2


def _sphere_quadrature(D, nq):
    """Product rule on S^{D-1}: uniform in theta_1, Gauss-Legendre in theta_K
    with the measure sin^{K-1}(theta_K) d theta_K."""
    t1 = np.arange(2 * nq) * (2 * math.pi / (2 * nq))
    w1 = np.full(2 * nq, 2 * math.pi / (2 * nq))
    grids = [(t1, w1)]
    g, gw = roots_legendre(nq)
    th = 0.5 * math.pi * (g + 1.0)
    for K in range(2, D):
        grids.append((th, 0.5 * math.pi * gw * np.sin(th) ** (K - 1)))
    pts = []
    wts = []
    for idx in np.ndindex(*[len(gr[0]) for gr in grids]):
        ang = [grids[k][0][idx[k]] for k in range(D - 1)]
        wt = np.prod([grids[k][1][idx[k]] for k in range(D - 1)])
        # x_1 = prod_{K>=2} sin th_K cos th_1, x_2 = prod sin th_K sin th_1,
        # x_{K+1} = prod_{J>K} sin th_J cos th_K, x_D = cos th_{D-1}
        x = np.zeros(D)
        s = 1.0
        for K in range(D - 1, 1, -1):
            x[K] = s * math.cos(ang[K - 1])
            s *= math.sin(ang[K - 1])
        x[0] = s * math.cos(ang[0])
        x[1] = s * math.sin(ang[0])
        pts.append(x)
        wts.append(wt)
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("D,lmax,nq", [(2, 6, 16), (3, 5, 32), (4, 3, 24)])
def test_orthonormality(D, lmax, nq):
    """Orthonormality of the hyperspherical harmonics on S^{D-1}."""
    pts, wts = _sphere_quadrature(D, nq)
    Y = np.array([oracle.harmonics(D, lmax, p) for p in pts])
    assert wts.sum() == pytest.approx(sphere_area(D), rel=1e-12)
    G = (Y * wts[:, None]).T @ Y.conj()
    np.testing.assert_allclose(G, np.eye(Y.shape[1]), atol=1e-11)


@pytest.mark.parametrize("D,lmax", [(2, 6), (3, 6), (4, 5)])
def test_addition_theorem(D, lmax):
    """sum over states of total l of Y(x) Y*(y) = dim/|S^{D-1}| * C^{(D/2-1)}_l(x.y)/C^{(D/2-1)}_l(1)
    (Chebyshev T_l for D = 2)."""
    rng = np.random.default_rng(D)
    lab = oracle.state_labels(D, lmax)
    tot = np.abs(lab[:, 0]) if D == 2 else lab[:, -1]
    for _ in range(6):
        x, y = rand_unit(rng, D), rand_unit(rng, D)
        t = float(x @ y)
        Yx, Yy = oracle.harmonics(D, lmax, x), oracle.harmonics(D, lmax, y)
        for l in range(lmax + 1):
            sel = tot == l
            s = np.sum(Yx[sel] * Yy[sel].conj())
            dim = int(sel.sum())
            if D == 2:
                g = math.cos(l * math.acos(max(-1.0, min(1.0, t))))
            else:
                a = D / 2 - 1
                g = eval_gegenbauer(l, a, t) / eval_gegenbauer(l, a, 1.0)
            assert s.real == pytest.approx(dim / sphere_area(D) * g, abs=1e-12)
            assert abs(s.imag) < 1e-12


@pytest.mark.parametrize("D,lmax", [(2, 5), (3, 5), (4, 4)])
def test_conjugation_and_parity(D, lmax):
    """eq. complex-conj-hypersph: Y* = (-1)^{l1} Y_{(-l1)...} for D >= 3
    (Y*_l = Y_{-l} in D = 2) and P[Y] = (-1)^{l_{D-1}} Y."""
    rng = np.random.default_rng(7)
    lab = [tuple(r) for r in oracle.state_labels(D, lmax)]
    index = {s: i for i, s in enumerate(lab)}
    for _ in range(5):
        x = rng.normal(size=D)
        Y, Ym = oracle.harmonics(D, lmax, x), oracle.harmonics(D, lmax, -x)
        for i, s in enumerate(lab):
            flip = (-s[0],) + s[1:]
            sign = 1.0 if D == 2 else (-1.0) ** s[0]
            assert Y[i].conjugate() == pytest.approx(sign * Y[index[flip]], abs=1e-13)
            assert Ym[i] == pytest.approx((-1.0) ** s[-1] * Y[i], abs=1e-13)


# --------------------------------------------------------------------------
# Coupling
# --------------------------------------------------------------------------

def test_wigner3j_matches_sympy():
    for j1 in range(0, 5):
        for j2 in range(0, 5):
            for j3 in range(abs(j1 - j2), j1 + j2 + 1):
                for m1 in range(-j1, j1 + 1):
                    for m2 in range(-j2, j2 + 1):
                        m3 = -m1 - m2
                        if abs(m3) > j3:
                            continue
                        ref = float(wigner_3j(j1, j2, j3, m1, m2, m3))
                        assert oracle.wigner3j(j1, j2, j3, m1, m2, m3) == pytest.approx(ref, abs=1e-13)


def test_cg3_matches_sympy_and_orthogonality():
    """eq. CG-examples (D = 3) is the standard Clebsch-Gordan coefficient;
    eq. CG-orthonorm holds."""
    for j1 in range(0, 4):
        for j2 in range(0, 4):
            for J in range(abs(j1 - j2), j1 + j2 + 1):
                for m1 in range(-j1, j1 + 1):
                    for m2 in range(-j2, j2 + 1):
                        M = m1 + m2
                        if abs(M) > J:
                            continue
                        ref = float(clebsch_gordan(j1, j2, J, m1, m2, M))
                        assert oracle.cg3(j1, m1, j2, m2, J, M) == pytest.approx(ref, abs=1e-13)
            for J in range(abs(j1 - j2), j1 + j2 + 1):
                for Jp in range(abs(j1 - j2), j1 + j2 + 1):
                    for M in range(-min(J, Jp), min(J, Jp) + 1):
                        s = sum(oracle.cg3(j1, m1, j2, M - m1, J, M) * oracle.cg3(j1, m1, j2, M - m1, Jp, M)
                                for m1 in range(-j1, j1 + 1) if abs(M - m1) <= j2)
                        assert s == pytest.approx(1.0 if J == Jp else 0.0, abs=1e-12)


def _basis_function(D, N, lmax):
    """P^0_Lambda(rhat_1..rhat_{N-1}) = sum C prod Y (eq. N-1-particle-basis-wavefunction),
    assembled from the oracle's harmonics and coupling terms."""
    lam, s, c = oracle.coupling_terms(D, N, lmax)
    nlam = len(oracle.lambda_labels(D, N, lmax))

    def P(*dirs):
        Ys = [oracle.harmonics(D, lmax, d) for d in dirs]
        out = np.zeros(nlam, dtype=complex)
        prod = c * Ys[0][s[:, 0]] * Ys[1][s[:, 1]]
        if N == 4:
            prod = prod * Ys[2][s[:, 2]]
        np.add.at(out, lam, prod)
        return out

    return P


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 4), (3, 3, 5), (4, 3, 4), (2, 4, 4), (2, 3, 4)])
def test_isotropic_basis_rotation_invariance_and_parity(D, N, lmax):
    """vec L = 0 states are invariant under SO(D); eq. basis-parity-conj:
    P* = (-1)^{sum l} P and P(-r) = (-1)^{sum l} P."""
    rng = np.random.default_rng(11)
    P = _basis_function(D, N, lmax)
    labels = oracle.lambda_labels(D, N, lmax)
    if D == 2:
        tot = np.zeros(len(labels), dtype=int)  # sum of l1 is zero
        par = labels[:, 0] + labels[:, 1] + (labels[:, 2] if N == 4 else 0)
    else:
        tot = 2 * labels[:, 0] if N == 3 else labels.sum(axis=1)
        par = tot
    for _ in range(4):
        dirs = [rand_unit(rng, D) for _ in range(N - 1)]
        R = rand_rotation(rng, D)
        p0 = P(*dirs)
        p1 = P(*[R @ d for d in dirs])
        np.testing.assert_allclose(p1, p0, atol=1e-12)
        pm = P(*[-d for d in dirs])
        np.testing.assert_allclose(pm, ((-1.0) ** par) * p0, atol=1e-12)
        if D >= 3:
            np.testing.assert_allclose(p0.conj(), ((-1.0) ** tot) * p0, atol=1e-12)
    assert np.max(np.abs(P(*[rand_unit(rng, D) for _ in range(N - 1)]))) > 1e-3


def test_d3_n3_coupling_closed_form():
    """<l m, l -m | 0 0> = (-1)^{l-m}/sqrt(2l+1) (DLMF 34.3.1 with the CG relation)."""
    lam, s, c = oracle.coupling_terms(3, 3, 5)
    lab = oracle.state_labels(3, 5)
    for L, (a, b), cc in zip(lam, s[:, :2], c):
        m, l = lab[a]
        assert lab[b][0] == -m and lab[b][1] == l == L
        assert cc == pytest.approx((-1.0) ** (l - m) / math.sqrt(2 * l + 1), abs=1e-14)


def test_paper_component_counts():
    """Counts printed in section Applications (golden fixture)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    assert len(oracle.lambda_labels(2, 4, 4)) == g["d2_n4_lmax4_angular"]
    assert len(oracle.btuple_labels(10, 4)) == g["n4_nbins10_radial"]
    assert math.comb(10, 4) == g["n5_nbins10_radial"]
    assert len(oracle.btuple_labels(10, 5)) == g["n5_nbins10_radial"]
    lab5 = oracle.lambda_labels(3, 5, 4)
    even = (lab5[:, 0] + lab5[:, 1] + lab5[:, 3] + lab5[:, 4]) % 2 == 0
    assert int(even.sum()) == g["n5_lmax4_angular_even"]


def test_bin_volumes_sum_to_shell():
    for D in (2, 3, 4):
        e = np.array([0.7, 1.1, 2.0, 3.5])
        tot = sum(oracle.bin_volume(D, e[b], e[b + 1]) for b in range(3))
        ball = lambda r: math.pi ** (D / 2) / math.gamma(D / 2 + 1) * r ** D
        assert tot == pytest.approx(ball(e[-1]) - ball(e[0]), rel=1e-13)


# --------------------------------------------------------------------------
# Separable estimator == naive estimator (brute force, tiny n)
# --------------------------------------------------------------------------

def _neighbours(wl, j, periodic=True):
    d = wl.pos - wl.pos[:, j:j + 1]
    box = np.asarray(wl.box)[:, None]
    if periodic:
        d = d - box * np.round(d / box)
    r2 = np.sum(d * d, axis=0)
    e2 = wl.edges ** 2
    ok = (r2 >= e2[0]) & (r2 < e2[-1])
    idx = np.nonzero(ok)[0]
    b = np.searchsorted(e2, r2[idx], side="right") - 1
    return idx, b, d[:, idx].T


def _indep_basis(D, N, lmax):
    """P^0_Lambda from SciPy/SymPy/closed forms, independent of the oracle
    (labels too: enumerated from SymPy coefficients, not from the oracle)."""
    labels = labels_indep.labels(D, N, lmax)
    if D == 2:
        def P(*dirs):
            ph = [np.arctan2(d[:, 1], d[:, 0]) for d in dirs]
            ls = [labels[:, 0], labels[:, 1]] + ([labels[:, 2]] if N == 4 else [])
            tot = 0.0
            for k in range(N - 1):
                shape = [1] * (N - 1)
                shape[k] = -1
                tot = tot + ls[k].reshape((-1,) + (1,) * (N - 1)) * ph[k].reshape(shape)[None]
            return np.exp(1j * tot) / (2 * math.pi) ** ((N - 1) / 2)
        return P
    if N == 3:
        def P(d1, d2):
            t = np.clip(d1 @ d2.T, -1.0, 1.0)
            out = []
            for l in labels[:, 0]:
                dim = math.comb(l + D - 3, D - 3) * (2 * l + D - 2) / (D - 2)
                a = D / 2 - 1
                g = eval_gegenbauer(int(l), a, t) / eval_gegenbauer(int(l), a, 1.0)
                out.append((-1.0) ** l * math.sqrt(dim) / sphere_area(D) * g)
            return np.array(out)
        return P
    assert D == 3 and N == 4

    def Yall(d):
        th = np.arccos(np.clip(d[:, 2], -1, 1))
        ph = np.arctan2(d[:, 1], d[:, 0])
        return {(l, m): (-1.0) ** m * sph_harm_y(l, m, th, ph) for l in range(lmax + 1) for m in range(-l, l + 1)}

    coup = []
    for l1, l2, l3 in labels:
        terms = []
        for m1 in range(-l1, l1 + 1):
            for m2 in range(-l2, l2 + 1):
                m3 = -m1 - m2
                if abs(m3) > l3:
                    continue
                c = sum(float(clebsch_gordan(l1, l2, l3, m1, m2, M)) * float(clebsch_gordan(l3, l3, 0, M, m3, 0))
                        for M in [m1 + m2] if abs(M) <= l3)
                if c != 0.0:
                    terms.append((m1, m2, m3, c))
        coup.append((l1, l2, l3, terms))

    def P(d1, d2, d3):
        Y1, Y2, Y3 = Yall(d1), Yall(d2), Yall(d3)
        out = np.zeros((len(labels), len(d1), len(d2), len(d3)), dtype=complex)
        for i, (l1, l2, l3, terms) in enumerate(coup):
            for m1, m2, m3, c in terms:
                out[i] += c * np.einsum("a,b,c->abc", Y1[(l1, m1)], Y2[(l2, m2)], Y3[(l3, m3)])
        return out

    return P


def _brute_force(wl, btuple_mode, periodic=True):
    """eq. NPCF-estimator-intro-discrete with B = P^0_Lambda prod Theta^{b_i}/v_{b_i},
    coefficients extracted with conj(P) (eq. zeta-basis-coeff), sums over all
    secondaries unrestricted."""
    D, N = wl.D, wl.N
    nb = len(wl.edges) - 1
    vb = np.array([sphere_area(D) * (wl.edges[b + 1] ** D - wl.edges[b] ** D) / D for b in range(nb)])
    labels = labels_indep.labels(D, N, wl.lmax)
    P = _indep_basis(D, N, wl.lmax)
    full = np.zeros((len(labels),) + (nb,) * (N - 1), dtype=complex)
    for j in range(wl.pos.shape[1]):
        idx, b, d = _neighbours(wl, j, periodic)
        if len(idx) == 0:
            continue
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        ww = wl.w[idx] / vb[b]
        pv = np.conj(P(*([u] * (N - 1))))
        if N == 3:
            contrib = pv * ww[None, :, None] * ww[None, None, :]
            for i1 in range(len(idx)):
                np.add.at(full, (slice(None), b[i1], b), wl.w[j] * contrib[:, i1, :])
        else:
            contrib = pv * ww[None, :, None, None] * ww[None, None, :, None] * ww[None, None, None, :]
            for i1 in range(len(idx)):
                for i2 in range(len(idx)):
                    np.add.at(full, (slice(None), b[i1], b[i2], b), wl.w[j] * contrib[:, i1, i2, :])
    full /= np.prod(wl.box)
    bt = oracle.btuple_labels(nb, N, btuple_mode)
    return np.stack([full[(slice(None),) + tuple(bt[q])] for q in range(len(bt))], axis=1)


@pytest.mark.parametrize("D,N,lmax,n,mode", [
    (3, 4, 2, 30, 0), (3, 4, 2, 24, 1), (3, 3, 4, 40, 1), (4, 3, 3, 40, 1),
    (2, 4, 3, 30, 1), (2, 3, 4, 40, 1), (2, 4, 3, 30, 0)])
def test_separable_equals_naive(D, N, lmax, n, mode):
    """The paper's naive-vs-separable agreement, to rounding."""
    box = {2: 6.0, 3: 8.0, 4: 6.0}[D]
    wl = inputs.tiny(D, N, lmax, n, seed=100 + D * 10 + N, box_side=box, rmax=2.8, nbins=3)
    ref = _brute_force(wl, mode)
    got, _ = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=mode)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("D,N,lmax,n", [(3, 4, 2, 30), (3, 3, 3, 40), (4, 3, 2, 40), (2, 4, 3, 30)])
def test_separable_equals_naive_open_box(D, N, lmax, n):
    """Open box (no wrap-around): the separable estimator equals the naive one
    computed with plain Euclidean separations; the box is small enough that
    many pairs would wrap if it were periodic, so the two boxes differ."""
    box = {2: 4.0, 3: 5.0, 4: 4.5}[D]
    wl = inputs.tiny(D, N, lmax, n, seed=300 + D * 10 + N, box_side=box, rmax=2.2, nbins=3)
    ref = _brute_force(wl, 1, periodic=False)
    got, pairs = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1, periodic=False)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)
    # pair count: ordered pairs with e_0 <= r < e_nb, no wrap
    cnt = sum(len(_neighbours(wl, j, periodic=False)[0]) for j in range(n))
    assert pairs == cnt
    cnt_per = sum(len(_neighbours(wl, j)[0]) for j in range(n))
    assert cnt_per != cnt


def test_open_box_equals_periodic_away_from_walls():
    """Points at least r_max from every wall have no wrapped pairs: the open
    and the periodic estimators agree exactly."""
    rng = np.random.default_rng(17)
    D, N, lmax, n, L, rmax = 3, 4, 3, 60, 20.0, 3.0
    pos = rng.uniform(rmax, L - rmax, size=(D, n))
    wl = inputs.Workload("inner", D, N, lmax, np.linspace(0.75, rmax, 4), [L] * D,
                         inputs.to_lattice(pos, [L] * D), rng.uniform(-0.5, 1.5, size=n), n)
    a, pa = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, periodic=True)
    b, pb = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, periodic=False)
    assert pa == pb and pa > 0
    np.testing.assert_array_equal(a, b)


# --------------------------------------------------------------------------
# Invariants of the estimator
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (3, 3, 4), (4, 3, 3), (2, 4, 4)])
def test_l0_is_weighted_count(D, N, lmax):
    """zeta_{0...0}^b = sum_j w_j prod_i W_{b_i}(j) / (V_D prod v_{b_i} |S^{D-1}|^{(N-1)/2})."""
    wl = inputs.tiny(D, N, lmax, 60, seed=5, box_side=8.0, rmax=3.0, nbins=3)
    nb = 3
    got, _ = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1)
    labels = oracle.lambda_labels(D, N, lmax)
    i0 = int(np.nonzero(np.all(labels == 0, axis=1))[0][0])
    vb = np.array([oracle.bin_volume(D, wl.edges[b], wl.edges[b + 1]) for b in range(nb)])
    bt = oracle.btuple_labels(nb, N, 1)
    ref = np.zeros(len(bt))
    for j in range(wl.pos.shape[1]):
        idx, b, _ = _neighbours(wl, j)
        W = np.bincount(b, weights=wl.w[idx], minlength=nb) / vb
        ref += wl.w[j] * np.prod(W[bt], axis=1)
    ref /= np.prod(wl.box) * sphere_area(D) ** ((N - 1) / 2)
    np.testing.assert_allclose(got[i0].real, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    assert np.max(np.abs(got[i0].imag)) < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (3, 3, 4), (4, 3, 3)])
def test_parity_real_imaginary(D, N, lmax):
    """Real field, vec L = 0: even sum l gives a real coefficient, odd an imaginary one."""
    wl = inputs.tiny(D, N, lmax, 50, seed=9, box_side=8.0, rmax=3.0, nbins=3)
    z, _ = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w)
    labels = oracle.lambda_labels(D, N, lmax)
    tot = 2 * labels[:, 0] if N == 3 else labels.sum(axis=1)
    scale = np.abs(z).max()
    for i in range(len(labels)):
        other = z[i].imag if tot[i] % 2 == 0 else z[i].real
        assert np.max(np.abs(other)) < 1e-13 * scale
    if N == 4:
        assert np.max(np.abs(z[tot % 2 == 1].imag)) > 1e-6 * scale


def _apply_cube_symmetry(wl, perm, flips):
    pos = wl.pos[list(perm)].copy()
    for ax, f in enumerate(flips):
        if f:
            pos[ax] = np.mod(wl.box[ax] - pos[ax], wl.box[ax])
    return pos


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (2, 4, 3), (4, 3, 2)])
def test_lattice_symmetries(D, N, lmax):
    """Exact symmetries of the periodic box: proper ones leave every component
    unchanged; improper ones flip the odd-parity components (eq. basis-parity-conj)."""
    wl = inputs.tiny(D, N, lmax, 40, seed=21, box_side=7.0, rmax=3.0, nbins=3)
    z, _ = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w)
    labels = oracle.lambda_labels(D, N, lmax)
    if D == 2:
        par = labels[:, 0] + labels[:, 1] + labels[:, 2]
    else:
        par = 2 * labels[:, 0] if N == 3 else labels.sum(axis=1)
    rng = np.random.default_rng(3)
    scale = np.abs(z).max()
    for _ in range(3):
        perm = rng.permutation(D)
        flips = rng.integers(0, 2, size=D)
        det = np.linalg.det(np.eye(D)[perm]) * np.prod([-1 if f else 1 for f in flips])
        z2, _ = oracle.npcf(D, N, lmax, wl.edges, wl.box, _apply_cube_symmetry(wl, perm, flips), wl.w)
        if D == 2:
            # SO(2) acts on l by a phase e^{i sum(l) alpha} = 1; reflections conjugate (l -> -l)
            if det > 0:
                np.testing.assert_allclose(z2, z, atol=1e-12 * scale)
            continue
        sign = np.where((par % 2 == 1) & (det < 0), -1.0, 1.0)
        np.testing.assert_allclose(z2, sign[:, None] * z, atol=1e-12 * scale)


def test_translation_and_weight_scaling():
    wl = inputs.tiny(3, 4, 3, 40, seed=4, box_side=7.0, rmax=3.0, nbins=3)
    z, p = oracle.npcf(3, 4, 3, wl.edges, wl.box, wl.pos, wl.w)
    shift = inputs.to_lattice(wl.pos + np.array([[1.75], [-2.5], [3.125]]), wl.box)
    z2, p2 = oracle.npcf(3, 4, 3, wl.edges, wl.box, shift, wl.w)
    assert p2 == p
    np.testing.assert_allclose(z2, z, rtol=0, atol=1e-13 * np.abs(z).max())
    z3, _ = oracle.npcf(3, 4, 3, wl.edges, wl.box, wl.pos, 2.5 * wl.w)
    np.testing.assert_allclose(z3, 2.5 ** 4 * z, rtol=1e-12, atol=1e-14 * np.abs(z3).max())


def _twins(wl):
    """The catalogue with every point taken twice."""
    return inputs.Workload(wl.name + "-twins", wl.D, wl.N, wl.lmax, wl.edges, wl.box,
                           np.concatenate([wl.pos, wl.pos], axis=1), np.concatenate([wl.w, wl.w]),
                           2 * wl.pos.shape[1])


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (2, 3, 4), (4, 3, 2)])
def test_coincident_twins_scale(D, N, lmax):
    """Every point taken twice: a primary's twin lies at zero separation, outside
    every bin (the first edge is positive), and every other neighbour counts
    twice, so each of the twice as many primaries has twice the a^b_l:
    zeta scales by 2^N and the pair count by 4."""
    wl = inputs.tiny(D, N, lmax, 70, seed=41, box_side=8.0, rmax=3.0, nbins=3)
    tw = _twins(wl)
    z1, p1 = oracle.npcf(D, N, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1)
    z2, p2 = oracle.npcf(D, N, lmax, tw.edges, tw.box, tw.pos, tw.w, btuple_mode=1)
    assert p2 == 4 * p1
    scale = np.abs(z1).max()
    assert np.max(np.abs(z2 - 2.0 ** N * z1)) <= 1e-12 * 2.0 ** N * scale


def test_primary_additivity():
    """Eq. NPCF-estimator-discrete sums over primaries: disjoint ranges add up."""
    wl = inputs.tiny(3, 4, 2, 50, seed=8, box_side=7.0, rmax=3.0, nbins=3)
    z, p = oracle.npcf(3, 4, 2, wl.edges, wl.box, wl.pos, wl.w)
    za, pa = oracle.npcf(3, 4, 2, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(0, 17))
    zb, pb = oracle.npcf(3, 4, 2, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(17, 50))
    assert pa + pb == p
    np.testing.assert_allclose(za + zb, z, rtol=1e-13, atol=1e-15 * np.abs(z).max())


# --------------------------------------------------------------------------
# Line-of-sight basis P^{0L}_{l1 l2} (section "Large-Scale Structure")
# --------------------------------------------------------------------------

def _los_basis(lmax, Lmax):
    """P^{0L}_{l1 l2}(d1, d2) = (-1)^{l2-l1} sqrt(2L+1) sum_m (l1 l2 L; m -m 0)
    Y_{l1 m}(d1) Y_{l2,-m}(d2), from SciPy harmonics and SymPy 3j symbols."""
    labels = labels_indep.line_of_sight(lmax, Lmax)

    def Yall(d):
        th = np.arccos(np.clip(d[:, 2], -1, 1))
        ph = np.arctan2(d[:, 1], d[:, 0])
        return {(l, m): (-1.0) ** m * sph_harm_y(l, m, th, ph) for l in range(lmax + 1) for m in range(-l, l + 1)}

    def P(d1, d2):
        Y1, Y2 = Yall(d1), Yall(d2)
        out = np.zeros((len(labels), len(d1), len(d2)), dtype=complex)
        for i, (l1, l2, L) in enumerate(labels):
            pre = (-1.0) ** (l2 - l1) * math.sqrt(2 * L + 1)
            for m in range(-min(l1, l2), min(l1, l2) + 1):
                c = float(wigner_3j(int(l1), int(l2), int(L), m, -m, 0))
                if c != 0.0:
                    out[i] += pre * c * np.outer(Y1[(int(l1), m)], Y2[(int(l2), -m)])
        return out

    return labels, P


def test_los_basis_l0_is_isotropic():
    """L = 0 forces l1 = l2 = l: the line-of-sight components equal the
    isotropic 3PCF ones (eq. for P^{0L} with the 3j value at L = 0)."""
    wl = inputs.tiny(3, 3, 4, 80, seed=41, box_side=8.0, rmax=3.0, nbins=3)
    iso, _ = oracle.npcf(3, 3, 4, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1)
    los, _ = oracle.npcf(3, 3, 4, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1, Lmax=0)
    lab = oracle.lambda_labels(3, 3, 4, 0)
    assert np.all(lab[:, 0] == lab[:, 1]) and np.all(lab[:, 2] == 0)
    np.testing.assert_allclose(los, iso[lab[:, 0]], rtol=0, atol=1e-13 * np.max(np.abs(iso)))


@pytest.mark.parametrize("lmax,Lmax,mode", [(2, 4, 1), (3, 2, 0), (2, 1, 1)])
def test_los_separable_equals_naive(lmax, Lmax, mode):
    """Separable line-of-sight estimator equals the naive pair sum with an
    independently built basis (coefficients extracted with conj(P))."""
    wl = inputs.tiny(3, 3, lmax, 40, seed=55 + lmax, box_side=8.0, rmax=2.8, nbins=3)
    labels, P = _los_basis(lmax, Lmax)
    nb = 3
    vb = np.array([oracle.bin_volume(3, wl.edges[b], wl.edges[b + 1]) for b in range(nb)])
    full = np.zeros((len(labels), nb, nb), dtype=complex)
    for j in range(wl.pos.shape[1]):
        idx, b, d = _neighbours(wl, j)
        if len(idx) == 0:
            continue
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        ww = wl.w[idx] / vb[b]
        pv = np.conj(P(u, u)) * ww[None, :, None] * ww[None, None, :]
        for i1 in range(len(idx)):
            np.add.at(full, (slice(None), b[i1], b), wl.w[j] * pv[:, i1, :])
    full /= np.prod(wl.box)
    bt = oracle.btuple_labels(nb, 3, mode)
    ref = full[:, bt[:, 0], bt[:, 1]]
    got, _ = oracle.npcf(3, 3, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=mode, Lmax=Lmax)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


def test_los_rotation_and_parity():
    """A quarter turn about the line of sight (axis 3) maps the periodic cube
    onto itself and leaves every P^{0L} component unchanged; a quarter turn
    about axis 1 leaves the L = 0 (isotropic) components unchanged but not the
    L > 0 ones.  The part the parity rule drops (Im for even l1+l2+L, Re for
    odd) vanishes for real weights."""
    L_box = 8.0
    wl = inputs.tiny(3, 3, 3, 120, seed=77, box_side=L_box, rmax=3.0, nbins=3)
    # anisotropic input: stretch the catalogue along the line of sight
    pos = wl.pos.copy()
    pos[2] = np.mod(pos[2] * 1.0, L_box)
    rng = np.random.default_rng(3)
    pos[2] = np.mod(pos[2] + 0.25 * rng.standard_normal(pos.shape[1]) * (pos[0] > L_box / 2), L_box)
    pos = inputs.to_lattice(pos, wl.box)
    args = (3, 3, 3, wl.edges, wl.box)
    z0, _ = oracle.npcf(*args, pos, wl.w, btuple_mode=1, Lmax=4)
    rz = np.stack([np.mod(-pos[1], L_box), pos[0], pos[2]])
    rx = np.stack([pos[0], np.mod(-pos[2], L_box), pos[1]])
    zz, _ = oracle.npcf(*args, rz, wl.w, btuple_mode=1, Lmax=4)
    zx, _ = oracle.npcf(*args, rx, wl.w, btuple_mode=1, Lmax=4)
    lab = oracle.lambda_labels(3, 3, 3, 4)
    sc = np.max(np.abs(z0))
    np.testing.assert_allclose(zz, z0, rtol=0, atol=1e-12 * sc)
    iso = lab[:, 2] == 0
    np.testing.assert_allclose(zx[iso], z0[iso], rtol=0, atol=1e-12 * sc)
    assert np.max(np.abs(zx[~iso] - z0[~iso])) > 1e-6 * sc
    odd = (lab.sum(axis=1) % 2) == 1
    dropped = np.where(odd[:, None], z0.real, z0.imag)
    assert np.max(np.abs(dropped)) <= 1e-12 * sc


# --------------------------------------------------------------------------
# Isotropic 5PCF (D = 3, N = 5; section "Hydrodynamic Turbulence")
# --------------------------------------------------------------------------

def _parity_sum5(labels):
    return labels[:, 0] + labels[:, 1] + labels[:, 3] + labels[:, 4]


_W3J = {}


def _w3j(*a):
    if a not in _W3J:
        _W3J[a] = float(wigner_3j(*a))
    return _W3J[a]


def _explicit_c5(l1, l2, l12, l3, l4, m1, m2, m3, m4):
    """The section's explicit 5PCF coefficient with the prefactor sqrt(2 l12 + 1):
    (-1)^{l1+l2+l3+l4} (-1)^{l12-m12} sqrt(2 l12+1) (l1 l2 l12; m1 m2 -m12)(l12 l3 l4; m12 m3 m4)."""
    m12 = m1 + m2
    if m12 + m3 + m4 != 0 or abs(m12) > l12:
        return 0.0
    return ((-1.0) ** (l1 + l2 + l3 + l4 + l12 - m12) * math.sqrt(2 * l12 + 1)
            * _w3j(l1, l2, l12, m1, m2, -m12) * _w3j(l12, l3, l4, m12, m3, m4))


@pytest.mark.parametrize("lmax", [2, 3])
def test_5pcf_coupling_is_the_explicit_3j_form(lmax):
    """The oracle builds C from the CG chain of eq. Coupling-C; it must equal
    the explicit two-3j form (SymPy) term by term, and list every non-zero
    term of it."""
    labels = oracle.lambda_labels(3, 5, lmax)
    st = oracle.state_labels(3, lmax)
    lam, s, c = oracle.coupling_terms(3, 5, lmax)
    got = {}
    for L, ss, cc in zip(lam, s, c):
        ms = tuple(int(st[k][0]) for k in ss)
        assert tuple(int(st[k][1]) for k in ss) == tuple(int(v) for v in labels[L][[0, 1, 3, 4]])
        got[(int(L),) + ms] = cc
    nz = 0
    for L, (l1, l2, l12, l3, l4) in enumerate(labels):
        l1, l2, l12, l3, l4 = map(int, (l1, l2, l12, l3, l4))
        for m1 in range(-l1, l1 + 1):
            for m2 in range(-l2, l2 + 1):
                for m3 in range(-l3, l3 + 1):
                    m4 = -m1 - m2 - m3
                    if abs(m4) > l4:
                        continue
                    ref = _explicit_c5(l1, l2, l12, l3, l4, m1, m2, m3, m4)
                    key = (L, m1, m2, m3, m4)
                    if abs(ref) < 1e-15:
                        assert abs(got.get(key, 0.0)) < 1e-13
                        continue
                    nz += 1
                    assert got[key] == pytest.approx(ref, rel=1e-12, abs=1e-14)
    # terms whose exact value is zero by cancellation appear in the oracle as
    # rounding noise (checked above to stay below 1e-13); the rest match one to one
    assert nz == sum(1 for v in got.values() if abs(v) >= 1e-13)


def test_5pcf_basis_rotation_invariance_and_parity():
    """P^0_Lambda of the 5PCF is SO(3)-invariant; P(-r) = P* = (-1)^{l1+l2+l3+l4} P."""
    lmax = 2
    lam, s, c = oracle.coupling_terms(3, 5, lmax)
    labels = oracle.lambda_labels(3, 5, lmax)
    par = _parity_sum5(labels)

    def P(*dirs):
        Ys = [oracle.harmonics(3, lmax, d) for d in dirs]
        out = np.zeros(len(labels), dtype=complex)
        np.add.at(out, lam, c * Ys[0][s[:, 0]] * Ys[1][s[:, 1]] * Ys[2][s[:, 2]] * Ys[3][s[:, 3]])
        return out

    rng = np.random.default_rng(12)
    for _ in range(3):
        dirs = [rand_unit(rng, 3) for _ in range(4)]
        R = rand_rotation(rng, 3)
        p0 = P(*dirs)
        np.testing.assert_allclose(P(*[R @ d for d in dirs]), p0, atol=1e-12)
        np.testing.assert_allclose(P(*[-d for d in dirs]), ((-1.0) ** par) * p0, atol=1e-12)
        np.testing.assert_allclose(p0.conj(), ((-1.0) ** par) * p0, atol=1e-12)
    assert np.max(np.abs(p0[par % 2 == 1])) > 1e-3


def _brute_force5(wl, btuple_mode):
    """Naive 5PCF: unrestricted sum over 4-tuples of secondaries of
    prod_i w Theta^{b_i}/v_{b_i} conj(P_Lambda), P from SciPy harmonics and the
    explicit 3j form (independent of the oracle)."""
    lmax = wl.lmax
    nb = len(wl.edges) - 1
    vb = np.array([sphere_area(3) * (wl.edges[b + 1] ** 3 - wl.edges[b] ** 3) / 3 for b in range(nb)])
    labels = labels_indep.d3_n5(lmax)
    coup = []
    for l1, l2, l12, l3, l4 in labels:
        l1, l2, l12, l3, l4 = map(int, (l1, l2, l12, l3, l4))
        terms = []
        for m1 in range(-l1, l1 + 1):
            for m2 in range(-l2, l2 + 1):
                for m3 in range(-l3, l3 + 1):
                    m4 = -m1 - m2 - m3
                    if abs(m4) <= l4:
                        v = _explicit_c5(l1, l2, l12, l3, l4, m1, m2, m3, m4)
                        if v != 0.0:
                            terms.append(((l1, m1), (l2, m2), (l3, m3), (l4, m4), v))
        coup.append(terms)
    full = np.zeros((len(labels),) + (nb,) * 4, dtype=complex)
    for j in range(wl.pos.shape[1]):
        idx, b, d = _neighbours(wl, j)
        if len(idx) == 0:
            continue
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        th = np.arccos(np.clip(u[:, 2], -1, 1))
        ph = np.arctan2(u[:, 1], u[:, 0])
        Y = {(l, m): (-1.0) ** m * sph_harm_y(l, m, th, ph) for l in range(lmax + 1) for m in range(-l, l + 1)}
        Bm = np.zeros((len(idx), nb))
        Bm[np.arange(len(idx)), b] = wl.w[idx] / vb[b]
        for i, terms in enumerate(coup):
            pv = np.zeros((len(idx),) * 4, dtype=complex)
            for k1, k2, k3, k4, v in terms:
                pv += v * np.multiply.outer(np.multiply.outer(Y[k1], Y[k2]), np.multiply.outer(Y[k3], Y[k4]))
            full[i] += wl.w[j] * np.einsum("pqrs,pa,qb,rc,sd->abcd", np.conj(pv), Bm, Bm, Bm, Bm, optimize=True)
    full /= np.prod(wl.box)
    bt = oracle.btuple_labels(nb, 5, btuple_mode)
    return full[:, bt[:, 0], bt[:, 1], bt[:, 2], bt[:, 3]]


@pytest.mark.parametrize("lmax,n,nbins,mode", [(2, 40, 3, 1), (1, 50, 5, 0)])
def test_5pcf_separable_equals_naive(lmax, n, nbins, mode):
    """The paper's naive-vs-separable check for its isotropic 5PCF, to rounding."""
    wl = inputs.tiny(3, 5, lmax, n, seed=500 + lmax, box_side=8.0, rmax=2.8, nbins=nbins)
    ref = _brute_force5(wl, mode)
    got, _ = oracle.npcf(3, 5, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=mode)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


def test_5pcf_l0_is_weighted_count_and_parity():
    """zeta_{00000}^b = sum_j w_j prod_i W_{b_i}(j) / (V prod v_{b_i} (4 pi)^2);
    even l1+l2+l3+l4 gives real coefficients, odd imaginary ones."""
    lmax, nb = 2, 3
    wl = inputs.tiny(3, 5, lmax, 60, seed=6, box_side=8.0, rmax=3.0, nbins=nb)
    z, _ = oracle.npcf(3, 5, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1)
    labels = oracle.lambda_labels(3, 5, lmax)
    i0 = int(np.nonzero(np.all(labels == 0, axis=1))[0][0])
    vb = np.array([oracle.bin_volume(3, wl.edges[b], wl.edges[b + 1]) for b in range(nb)])
    bt = oracle.btuple_labels(nb, 5, 1)
    ref = np.zeros(len(bt))
    for j in range(wl.pos.shape[1]):
        idx, b, _ = _neighbours(wl, j)
        W = np.bincount(b, weights=wl.w[idx], minlength=nb) / vb
        ref += wl.w[j] * np.prod(W[bt], axis=1)
    ref /= np.prod(wl.box) * (4 * math.pi) ** 2
    np.testing.assert_allclose(z[i0].real, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    par = _parity_sum5(labels)
    scale = np.abs(z).max()
    dropped = np.where((par % 2 == 1)[:, None], z.real, z.imag)
    assert np.max(np.abs(dropped)) < 1e-13 * scale
    assert np.max(np.abs(z[par % 2 == 1].imag)) > 1e-6 * scale


def test_5pcf_lattice_symmetries():
    """Proper symmetries of the periodic cube leave every 5PCF component
    unchanged; improper ones flip the odd-parity ones."""
    lmax = 2
    wl = inputs.tiny(3, 5, lmax, 40, seed=22, box_side=7.0, rmax=3.0, nbins=3)
    z, _ = oracle.npcf(3, 5, lmax, wl.edges, wl.box, wl.pos, wl.w, btuple_mode=1)
    par = _parity_sum5(oracle.lambda_labels(3, 5, lmax))
    scale = np.abs(z).max()
    for perm, flips in [((1, 2, 0), (0, 0, 0)), ((0, 1, 2), (1, 0, 0)), ((2, 0, 1), (1, 1, 0))]:
        det = np.linalg.det(np.eye(3)[list(perm)]) * np.prod([-1 if f else 1 for f in flips])
        z2, _ = oracle.npcf(3, 5, lmax, wl.edges, wl.box, _apply_cube_symmetry(wl, perm, flips), wl.w, btuple_mode=1)
        sign = np.where((par % 2 == 1) & (det < 0), -1.0, 1.0)
        np.testing.assert_allclose(z2, sign[:, None] * z, atol=1e-12 * scale)


# --------------------------------------------------------------------------
# Points on the unit 2-sphere (D = 2 harmonics; section "Cosmic Microwave Background")
# --------------------------------------------------------------------------

def _sphere_points(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(3, n))
    return x / np.linalg.norm(x, axis=0), rng.uniform(-0.5, 1.5, size=n)


def _sphere_area_quad(e0, e1):
    from scipy.integrate import quad
    return 2 * math.pi * quad(math.sin, e0, e1, epsabs=1e-13, epsrel=1e-12)[0]


def _sphere_brute(pos, w, edges, N, lmax, btuple_mode):
    """Naive estimator on S^2: for each primary p, unrestricted (N-1)-tuples of
    secondaries in the angular bins, basis (2 pi)^{-(N-1)/2} e^{i sum l_k phi_k}
    with phi measured from the spherical-coordinate direction e_theta of p (a
    frame other than the oracle's), coefficients through conj(P), over 4 pi."""
    labels = labels_indep.d2(N, lmax)
    nb = len(edges) - 1
    vb = np.array([_sphere_area_quad(edges[b], edges[b + 1]) for b in range(nb)])
    n = pos.shape[1]
    full = np.zeros((len(labels),) + (nb,) * (N - 1), dtype=complex)
    for j in range(n):
        p = pos[:, j]
        th = math.acos(np.clip(p[2], -1, 1))
        ph = math.atan2(p[1], p[0])
        et = np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)])
        ep = np.array([-math.sin(ph), math.cos(ph), 0.0])
        ang = np.arccos(np.clip(pos.T @ p, -1, 1))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        idx = np.nonzero(ok)[0]
        if len(idx) == 0:
            continue
        b = np.searchsorted(edges, ang[idx], side="right") - 1
        phi = np.arctan2(pos[:, idx].T @ ep, pos[:, idx].T @ et)
        Bm = np.zeros((len(idx), nb))
        Bm[np.arange(len(idx)), b] = w[idx] / vb[b]
        ls = [labels[:, k] for k in range(N - 1)]
        if N == 3:
            P = np.exp(1j * (ls[0][:, None, None] * phi[None, :, None] + ls[1][:, None, None] * phi[None, None, :]))
            full += w[j] * np.einsum("lpq,pa,qb->lab", np.conj(P), Bm, Bm) / (2 * math.pi)
        else:
            P = np.exp(1j * (ls[0][:, None, None, None] * phi[None, :, None, None]
                             + ls[1][:, None, None, None] * phi[None, None, :, None]
                             + ls[2][:, None, None, None] * phi[None, None, None, :]))
            full += w[j] * np.einsum("lpqr,pa,qb,rc->labc", np.conj(P), Bm, Bm, Bm, optimize=True) / (2 * math.pi) ** 1.5
    full /= 4 * math.pi
    bt = oracle.btuple_labels(nb, N, btuple_mode)
    return full[(slice(None),) + tuple(bt[:, k] for k in range(N - 1))]


@pytest.mark.parametrize("N,lmax,mode", [(4, 3, 1), (3, 5, 1), (4, 2, 0)])
def test_sphere_separable_equals_naive(N, lmax, mode):
    edges = np.array([0.35, 0.6, 0.9, 1.3, 1.9]) if mode == 0 else np.array([0.3, 0.7, 1.2, 1.7])
    pos, w = _sphere_points(60, 40 + N + lmax)
    ref = _sphere_brute(pos, w, edges, N, lmax, mode)
    got, _ = oracle.npcf(2, N, lmax, edges, [1.0, 1.0], pos, w, btuple_mode=mode, sphere=True)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


def test_sphere_rotation_invariance_and_l0():
    """Any rotation of the sphere leaves every isotropic component unchanged;
    zeta_{000}^b = sum_p w_p prod_i W_{b_i}(p) / (4 pi prod v_{b_i} (2 pi)^{(N-1)/2})
    with the bin areas from quadrature."""
    N, lmax = 4, 3
    edges = np.array([0.3, 0.7, 1.2, 1.7])
    pos, w = _sphere_points(200, 9)
    z, pairs = oracle.npcf(2, N, lmax, edges, [1.0, 1.0], pos, w, btuple_mode=1, sphere=True)
    R = rand_rotation(np.random.default_rng(5), 3)
    z2, pairs2 = oracle.npcf(2, N, lmax, edges, [1.0, 1.0], R @ pos, w, btuple_mode=1, sphere=True)
    assert pairs2 == pairs
    np.testing.assert_allclose(z2, z, rtol=0, atol=1e-12 * np.abs(z).max())
    nb = len(edges) - 1
    vb = np.array([_sphere_area_quad(edges[b], edges[b + 1]) for b in range(nb)])
    labels = oracle.lambda_labels(2, N, lmax)
    i0 = int(np.nonzero(np.all(labels == 0, axis=1))[0][0])
    bt = oracle.btuple_labels(nb, N, 1)
    ref = np.zeros(len(bt))
    for j in range(pos.shape[1]):
        ang = np.arccos(np.clip(pos.T @ pos[:, j], -1, 1))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        b = np.searchsorted(edges, ang[ok], side="right") - 1
        W = np.bincount(b, weights=w[ok], minlength=nb) / vb
        ref += w[j] * np.prod(W[bt], axis=1)
    ref /= 4 * math.pi * (2 * math.pi) ** ((N - 1) / 2)
    np.testing.assert_allclose(z[i0].real, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_sphere_alm_frame_phase():
    """a_l of the oracle in its tangent frame equals, up to the phase e^{-i l alpha}
    of the frame's rotation alpha, the sum in the spherical-coordinate frame."""
    pos, w = _sphere_points(80, 3)
    edges = np.array([0.4, 1.0, 1.6])
    lmax = 4
    a, _ = oracle.alm(2, lmax, edges, [1.0, 1.0], pos, w, sphere=True)
    lab = oracle.state_labels(2, lmax)[:, 0]
    vb = np.array([_sphere_area_quad(edges[b], edges[b + 1]) for b in range(2)])
    for j in (0, 17, 55):
        p = pos[:, j]
        th, ph = math.acos(p[2]), math.atan2(p[1], p[0])
        et = np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)])
        ep = np.array([-math.sin(ph), math.cos(ph), 0.0])
        ang = np.arccos(np.clip(pos.T @ p, -1, 1))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        idx = np.nonzero(ok)[0]
        b = np.searchsorted(edges, ang[idx], side="right") - 1
        phi = np.arctan2(pos[:, idx].T @ ep, pos[:, idx].T @ et)
        ref = np.zeros((2, len(lab)), dtype=complex)
        for k in range(len(idx)):
            ref[b[k]] += w[idx[k]] * np.exp(-1j * lab * phi[k]) / math.sqrt(2 * math.pi) / vb[b[k]]
        # the two frames differ by one rotation angle per primary: a = ref * e^{i l alpha}
        l1 = int(np.nonzero(lab == 1)[0][0])
        alpha = np.angle(a[j, :, l1].sum() / ref[:, l1].sum())
        np.testing.assert_allclose(a[j], ref * np.exp(1j * lab * alpha)[None, :], rtol=0, atol=1e-12 * np.abs(ref).max())


# --------------------------------------------------------------------------
# Unit 3-sphere (section "Constant-Curvature Metric", k = 1: chi(r) = sin r)
# --------------------------------------------------------------------------

def _s3_points(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(4, n))
    return x / np.linalg.norm(x, axis=0), rng.uniform(-0.5, 1.5, size=n)


def _s3_volume_quad(e0, e1):
    """|S^2| int sin^2 r dr over the bin, by quadrature (eq. metric's volume element)."""
    from scipy.integrate import quad
    return 4 * math.pi * quad(lambda r: math.sin(r) ** 2, e0, e1, epsabs=1e-13, epsrel=1e-12)[0]


def _second_frame(p):
    """An orthonormal, positively oriented frame of the tangent space at p
    (Gram-Schmidt of the coordinate axes), unlike the oracle's quaternion one."""
    q, _ = np.linalg.qr(np.column_stack([p, np.eye(4)]))
    f = q[:, 1:4] * np.sign(q[:, 0] @ p)
    if np.linalg.det(np.column_stack([p, f])) < 0:
        f[:, 2] = -f[:, 2]
    return f


def _s3_brute(pos, w, edges, N, lmax, btuple_mode):
    """Naive estimator on S^3: unrestricted (N-1)-tuples of secondaries in the
    geodesic bins, directions in the second frame, basis from SciPy harmonics
    and SymPy Clebsch-Gordan coefficients, coefficients through conj(P), bin
    volumes by quadrature, divided by the 3-sphere's volume 2 pi^2."""
    nb = len(edges) - 1
    vb = np.array([_s3_volume_quad(edges[b], edges[b + 1]) for b in range(nb)])
    labels = labels_indep.labels(3, N, lmax)
    P = _indep_basis(3, N, lmax)
    full = np.zeros((len(labels),) + (nb,) * (N - 1), dtype=complex)
    for j in range(pos.shape[1]):
        p = pos[:, j]
        ang = np.arccos(np.clip(pos.T @ p, -1.0, 1.0))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        idx = np.nonzero(ok)[0]
        if len(idx) == 0:
            continue
        b = np.searchsorted(edges, ang[idx], side="right") - 1
        t = pos[:, idx].T @ _second_frame(p)
        u = t / np.linalg.norm(t, axis=1, keepdims=True)
        ww = w[idx] / vb[b]
        pv = np.conj(P(*([u] * (N - 1))))
        if N == 3:
            contrib = pv * ww[None, :, None] * ww[None, None, :]
            for i1 in range(len(idx)):
                np.add.at(full, (slice(None), b[i1], b), w[j] * contrib[:, i1, :])
        else:
            contrib = pv * ww[None, :, None, None] * ww[None, None, :, None] * ww[None, None, None, :]
            for i1 in range(len(idx)):
                for i2 in range(len(idx)):
                    np.add.at(full, (slice(None), b[i1], b[i2], b), w[j] * contrib[:, i1, i2, :])
    full /= 2 * math.pi ** 2
    bt = oracle.btuple_labels(nb, N, btuple_mode)
    return full[(slice(None),) + tuple(bt[:, k] for k in range(N - 1))]


@pytest.mark.parametrize("N,lmax,mode,n", [(3, 4, 1, 50), (4, 3, 1, 28), (4, 2, 0, 34)])
def test_s3_separable_equals_naive(N, lmax, mode, n):
    """The separable estimator on S^3 equals the naive tuple sum built in
    another tangent frame with an independent basis (isotropic components do
    not depend on the frame)."""
    edges = np.array([0.3, 0.7, 1.2, 1.7]) if mode == 1 else np.array([0.35, 0.6, 0.9, 1.3, 1.9])
    pos, w = _s3_points(n, 60 + N + lmax)
    ref = _s3_brute(pos, w, edges, N, lmax, mode)
    got, _ = oracle.npcf(3, N, lmax, edges, [1.0] * 3, pos, w, btuple_mode=mode, sphere=True)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


def test_s3_rotation_invariance_parity_and_l0():
    """A random SO(4) rotation leaves every isotropic component unchanged; a
    reflection keeps the even-parity ones and flips the odd ones (the frame's
    orientation is reversed); the l = 0 row equals the weighted triplet count
    sum_j w_j W_b1(j) W_b2(j) W_b3(j) / (2 pi^2 prod v_b (4 pi)^{3/2}) with
    bin volumes by quadrature."""
    rng = np.random.default_rng(7)
    pos, w = _s3_points(80, 8)
    edges = np.array([0.4, 0.8, 1.3, 1.9])
    args = (3, 4, 3, edges, [1.0] * 3)
    z0, p0 = oracle.npcf(*args, pos, w, btuple_mode=1, sphere=True)
    R, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    zr, pr = oracle.npcf(*args, R @ pos, w, btuple_mode=1, sphere=True)
    sc = np.max(np.abs(z0))
    assert pr == p0
    np.testing.assert_allclose(zr, z0, rtol=0, atol=1e-11 * sc)
    F = np.diag([1.0, 1.0, 1.0, -1.0])
    zf, _ = oracle.npcf(*args, F @ pos, w, btuple_mode=1, sphere=True)
    lab = oracle.lambda_labels(3, 4, 3)
    odd = lab.sum(axis=1) % 2 == 1
    np.testing.assert_allclose(zf[~odd], z0[~odd], rtol=0, atol=1e-11 * sc)
    np.testing.assert_allclose(zf[odd], -z0[odd], rtol=0, atol=1e-11 * sc)
    assert np.max(np.abs(z0[odd])) > 1e-6 * sc
    # l = 0: weighted counts
    nb = 3
    vb = np.array([_s3_volume_quad(edges[b], edges[b + 1]) for b in range(nb)])
    Wb = np.zeros((pos.shape[1], nb))
    for j in range(pos.shape[1]):
        ang = np.arccos(np.clip(pos.T @ pos[:, j], -1, 1))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        b = np.searchsorted(edges, ang[ok], side="right") - 1
        np.add.at(Wb[j], b, w[ok])
    bt = oracle.btuple_labels(nb, 4, 1)
    ref = np.array([np.sum(w * Wb[:, t[0]] * Wb[:, t[1]] * Wb[:, t[2]]) / (vb[t[0]] * vb[t[1]] * vb[t[2]])
                    for t in bt]) / (2 * math.pi ** 2 * (4 * math.pi) ** 1.5)
    i0 = int(np.nonzero((lab == 0).all(axis=1))[0][0])
    np.testing.assert_allclose(z0[i0].real, ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(ref)))


def test_s3_bin_volumes_fill_the_sphere():
    """Bins covering [1e-5, pi) hold the 3-sphere's volume 2 pi^2 up to the
    first bin's 1e-15 (each bin's volume against quadrature of the metric's
    volume element), and every pair is in range: the pair count is n (n - 1).
    An innermost edge whose cosine rounds to 1 is rejected (the self pair
    could not be told apart from a pair at that distance)."""
    edges = np.array([1e-5, 0.5, 1.0, 2.0, math.pi])
    pos, w = _s3_points(30, 3)
    tot = sum(_s3_volume_quad(edges[b], edges[b + 1]) for b in range(4))
    assert tot == pytest.approx(2 * math.pi ** 2, rel=1e-9)
    _, pairs = oracle.npcf(3, 3, 1, edges, [1.0] * 3, pos, w, sphere=True)
    assert pairs == 30 * 29
    with pytest.raises(ValueError):
        oracle.npcf(3, 3, 1, np.array([1e-9, 1.0]), [1.0] * 3, pos, w, sphere=True)


# ---------------------------------------------------------------------------
# Hyperbolic space H^D (section "Constant-Curvature Metric", k = -1,
# chi(r) = sinh r), hyperboloid model in R^{D,1}.
# ---------------------------------------------------------------------------

def _mink(a, b):
    """<a, b> = a0 b0 - a1 b1 - .. (columns of a against the vector b)."""
    return a[0] * b[0] - np.tensordot(b[1:], a[1:], axes=(0, 0))


def _h_points(D, n, seed, R=1.2):
    """n points of H^D: tangent vectors at the origin with N(0, (R/2)^2)
    coordinates, mapped by the exponential map to (cosh r, sinh r y/r)."""
    rng = np.random.default_rng(seed)
    y = rng.normal(0.0, R / 2, size=(D, n))
    r = np.linalg.norm(y, axis=0)
    return np.vstack([np.cosh(r), np.sinh(r) * y / r]), rng.uniform(-0.5, 1.5, size=n)


def _h_volume_quad(D, e0, e1):
    """|S^{D-1}| int sinh^{D-1} r dr over the bin, by quadrature (eq. metric's volume element)."""
    from scipy.integrate import quad
    area = 2 * math.pi if D == 2 else 4 * math.pi
    return area * quad(lambda r: math.sinh(r) ** (D - 1), e0, e1, epsabs=1e-13, epsrel=1e-12)[0]


def _h_second_frame(p, D):
    """An orthonormal, positively oriented frame of the tangent space at p
    (Gram-Schmidt in the Minkowski metric of the projected spatial axes),
    unlike the oracle's boost frame."""
    frame = []
    for i in range(1, D + 1):
        a = np.zeros(D + 1)
        a[i] = 1.0
        v = a - _mink(a[:, None], p)[0] * p
        for e in frame:
            v = v + _mink(v[:, None], e)[0] * e
        frame.append(v / math.sqrt(-_mink(v[:, None], v)[0]))
    if np.linalg.det(np.column_stack([p] + frame)) < 0:
        frame[-1] = -frame[-1]
    return frame


def _h_brute(pos, w, edges, D, N, lmax, btuple_mode, V):
    """Naive estimator in H^D: unrestricted (N-1)-tuples of secondaries in the
    geodesic bins (theta = arccosh <p, q>), directions in the second frame,
    basis from SciPy harmonics and SymPy coefficients, coefficients through
    conj(P), bin volumes by quadrature, divided by V."""
    nb = len(edges) - 1
    vb = np.array([_h_volume_quad(D, edges[b], edges[b + 1]) for b in range(nb)])
    labels = labels_indep.labels(D, N, lmax)
    P = _indep_basis(D, N, lmax)
    full = np.zeros((len(labels),) + (nb,) * (N - 1), dtype=complex)
    for j in range(pos.shape[1]):
        p = pos[:, j]
        c = _mink(pos, p)
        ang = np.arccosh(np.maximum(c, 1.0))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        idx = np.nonzero(ok)[0]
        if len(idx) == 0:
            continue
        b = np.searchsorted(edges, ang[idx], side="right") - 1
        t = np.column_stack([-_mink(pos[:, idx], e) for e in _h_second_frame(p, D)])
        u = t / np.linalg.norm(t, axis=1, keepdims=True)
        ww = w[idx] / vb[b]
        pv = np.conj(P(*([u] * (N - 1))))
        if N == 3:
            contrib = pv * ww[None, :, None] * ww[None, None, :]
            for i1 in range(len(idx)):
                np.add.at(full, (slice(None), b[i1], b), w[j] * contrib[:, i1, :])
        else:
            contrib = pv * ww[None, :, None, None] * ww[None, None, :, None] * ww[None, None, None, :]
            for i1 in range(len(idx)):
                for i2 in range(len(idx)):
                    np.add.at(full, (slice(None), b[i1], b[i2], b), w[j] * contrib[:, i1, i2, :])
    full /= V
    bt = oracle.btuple_labels(nb, N, btuple_mode)
    return full[(slice(None),) + tuple(bt[:, k] for k in range(N - 1))]


@pytest.mark.parametrize("D,N,lmax,mode,n", [(3, 3, 4, 1, 50), (3, 4, 3, 1, 28), (3, 4, 2, 0, 34),
                                             (2, 3, 4, 1, 60), (2, 4, 3, 0, 40)])
def test_hyp_separable_equals_naive(D, N, lmax, mode, n):
    """The separable estimator in H^D equals the naive tuple sum built in
    another tangent frame with an independent basis (isotropic components do
    not depend on the frame)."""
    edges = np.array([0.2, 0.5, 0.9, 1.4]) if mode == 1 else np.array([0.25, 0.5, 0.8, 1.1, 1.6])
    pos, w = _h_points(D, n, 70 + 3 * D + N + lmax)
    V = 7.5
    ref = _h_brute(pos, w, edges, D, N, lmax, mode, V)
    got, _ = oracle.npcf(D, N, lmax, edges, [V, 1.0, 1.0], pos, w, btuple_mode=mode, hyperbolic=True)
    scale = np.max(np.abs(ref))
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * scale)


def _lorentz(D, rng):
    """A random proper orthochronous Lorentz transformation of R^{D,1}: a
    spatial rotation, then a boost of rapidity 0.7 along a random direction."""
    Q, _ = np.linalg.qr(rng.normal(size=(D, D)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    Rt = np.eye(D + 1)
    Rt[1:, 1:] = Q
    nvec = rng.normal(size=D)
    nvec /= np.linalg.norm(nvec)
    phi = 0.7
    B = np.eye(D + 1)
    B[0, 0] = math.cosh(phi)
    B[0, 1:] = B[1:, 0] = math.sinh(phi) * nvec
    B[1:, 1:] += (math.cosh(phi) - 1.0) * np.outer(nvec, nvec)
    return B @ Rt


def test_hyp_isometry_invariance_parity_and_l0():
    """A random isometry of H^3 (rotation and boost) leaves every isotropic
    component unchanged; a reflection of one spatial axis keeps the
    even-parity ones and flips the odd ones; the l = 0 row equals the weighted
    triplet count sum_j w_j W_b1(j) W_b2(j) W_b3(j) / (V prod v_b (4 pi)^{3/2})
    with bin volumes by quadrature."""
    rng = np.random.default_rng(11)
    pos, w = _h_points(3, 70, 12)
    edges = np.array([0.3, 0.7, 1.1, 1.6])
    V = 4.0
    args = (3, 4, 3, edges, [V, 1.0, 1.0])
    z0, p0 = oracle.npcf(*args, pos, w, btuple_mode=1, hyperbolic=True)
    L = _lorentz(3, rng)
    zr, pr = oracle.npcf(*args, L @ pos, w, btuple_mode=1, hyperbolic=True)
    sc = np.max(np.abs(z0))
    assert pr == p0
    np.testing.assert_allclose(zr, z0, rtol=0, atol=1e-9 * sc)
    F = np.diag([1.0, 1.0, 1.0, -1.0])
    zf, _ = oracle.npcf(*args, F @ pos, w, btuple_mode=1, hyperbolic=True)
    lab = oracle.lambda_labels(3, 4, 3)
    odd = lab.sum(axis=1) % 2 == 1
    np.testing.assert_allclose(zf[~odd], z0[~odd], rtol=0, atol=1e-11 * sc)
    np.testing.assert_allclose(zf[odd], -z0[odd], rtol=0, atol=1e-11 * sc)
    assert np.max(np.abs(z0[odd])) > 1e-6 * sc
    nb = 3
    vb = np.array([_h_volume_quad(3, edges[b], edges[b + 1]) for b in range(nb)])
    Wb = np.zeros((pos.shape[1], nb))
    for j in range(pos.shape[1]):
        ang = np.arccosh(np.maximum(_mink(pos, pos[:, j]), 1.0))
        ok = (ang >= edges[0]) & (ang < edges[-1])
        ok[j] = False
        b = np.searchsorted(edges, ang[ok], side="right") - 1
        np.add.at(Wb[j], b, w[ok])
    bt = oracle.btuple_labels(nb, 4, 1)
    ref = np.array([np.sum(w * Wb[:, t[0]] * Wb[:, t[1]] * Wb[:, t[2]]) / (vb[t[0]] * vb[t[1]] * vb[t[2]])
                    for t in bt]) / (V * (4 * math.pi) ** 1.5)
    i0 = int(np.nonzero((lab == 0).all(axis=1))[0][0])
    np.testing.assert_allclose(z0[i0].real, ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(ref)))


@pytest.mark.parametrize("D,N,lmax", [(3, 4, 3), (3, 3, 4), (2, 4, 4)])
def test_hyp_flat_limit(D, N, lmax):
    """Far below the curvature scale H^D is flat: a catalogue within 1e-3 of
    the origin, lifted by the exponential map, gives the flat open-box
    estimator of the tangent coordinates (the oracle's flat path, with the
    same bins and V) up to relative corrections of order r^2 ~ 1e-6."""
    eps = 1e-3
    rng = np.random.default_rng(40 + D + N)
    n = 60
    y = rng.uniform(-eps, eps, size=(D, n))
    w = rng.uniform(0.5, 1.5, size=n)
    r = np.linalg.norm(y, axis=0)
    pos = np.vstack([np.cosh(r), np.sinh(r) * y / r])
    edges = eps * np.array([0.2, 0.5, 0.9, 1.4, 2.0])
    box = 1.0
    zh, ph = oracle.npcf(D, N, lmax, edges, [box ** D, 1.0, 1.0], pos, w, hyperbolic=True)
    zf, pf = oracle.npcf(D, N, lmax, edges, [box] * D, y + box / 2, w, periodic=False)
    assert ph == pf
    np.testing.assert_allclose(zh, zf, rtol=0, atol=3e-5 * np.max(np.abs(zf)))


def test_hyp_rejects_and_self_pair():
    """Every distinct pair within range is counted once and the self pair
    never (excluded by index); an innermost edge with cosh(e0) < 1 + 1e-9 and
    a non-positive volume are rejected."""
    pos, w = _h_points(3, 25, 5, R=0.5)
    edges = np.array([1e-4, 0.5, 3.0, 6.0])
    _, pairs = oracle.npcf(3, 3, 1, edges, [1.0, 1.0, 1.0], pos, w, hyperbolic=True)
    assert pairs == 25 * 24
    with pytest.raises(ValueError):
        oracle.npcf(3, 3, 1, np.array([1e-6, 1.0]), [1.0] * 3, pos, w, hyperbolic=True)
    with pytest.raises(ValueError):
        oracle.npcf(3, 3, 1, np.array([0.1, 1.0]), [0.0, 1.0, 1.0], pos, w, hyperbolic=True)


def test_oracle_distance_is_not_fused():
    """The oracle's squared distance rounds every product and sum (the
    definition's arithmetic): on a planted pair whose fused sum lands on the
    outer edge and whose rounded sum lies one ulp inside it, the oracle counts
    the pair, as the plain numpy count does."""
    from npcf_testutil import fused_distance_catalogue, pair_count_by_definition
    wl, r2, r2f, e2 = fused_distance_catalogue()
    assert r2 < e2 <= r2f   # the pair separates the two arithmetics
    _, pairs = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w)
    assert pairs == pair_count_by_definition(wl)


def test_oracle_sphere_cosine_is_not_fused():
    """The oracle's cosine on the sphere rounds every product and sum: a
    planted pair whose rounded cosine lies above cos of the outer edge and
    whose fused cosine lands on it is counted, as the plain numpy count does."""
    from npcf_testutil import fused_dot_sphere_catalogue, sphere_pair_count_by_definition
    wl, c, cf, clo = fused_dot_sphere_catalogue()
    assert c > clo >= cf   # the pair separates the two arithmetics
    _, pairs = oracle.npcf(wl.D, wl.N, wl.lmax, wl.edges, wl.box, wl.pos, wl.w, sphere=True)
    assert pairs == sphere_pair_count_by_definition(wl)
