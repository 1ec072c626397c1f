"""Label sets of the isotropic (and line-of-sight) bases, enumerated without
the oracle: a label is kept when the basis function it names is not
identically zero, decided from SymPy's Clebsch-Gordan / 3j values or, in
D = 2, from the rotation average of exp(i sum l theta).

The candidates are every tuple of non-negative (D = 2: signed) orders up to
the bounds; the triangle conditions of eq. addition-triangle-conditions are
not written out here, they follow from which coefficients SymPy finds
non-zero.  Output order is lexicographic, the order the library documents.
"""
from __future__ import annotations

import functools

import numpy as np
from sympy.physics.wigner import clebsch_gordan, wigner_3j


@functools.lru_cache(maxsize=None)
def _w3j(j1, j2, j3, m1, m2, m3):
    return float(wigner_3j(j1, j2, j3, m1, m2, m3))


@functools.lru_cache(maxsize=None)
def _cg(j1, m1, j2, m2, J, M):
    return float(clebsch_gordan(j1, j2, J, m1, m2, M))


def _d3_pair_couples(l1, l2, l3):
    """Some <l1 m1 l2 m2 | l3 m1+m2> is non-zero (the N = 4 basis of eq.
    Coupling-C then has a non-zero term, since <l3 M l3 -M | 0 0> never vanishes)."""
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            if abs(m1 + m2) <= l3 and _cg(l1, m1, l2, m2, l3, m1 + m2) != 0.0:
                return True
    return False


def d3_n4(lmax):
    out = [(l1, l2, l3) for l1 in range(lmax + 1) for l2 in range(lmax + 1) for l3 in range(lmax + 1)
           if _d3_pair_couples(l1, l2, l3)]
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def isotropic_n3(D, lmax):
    """N = 3, D >= 3: labels (l, 0, 0).  In D = 3 the pairs of orders that
    couple to zero are found from SymPy (<l m, l' -m | 0 0> non-zero), which
    leaves only l = l'; in D = 4 the N = 3 basis is the Gegenbauer function
    C^{(1)}_l of the angle between the two directions, non-zero for every l."""
    out = set()
    for l in range(lmax + 1):
        for lp in range(lmax + 1):
            if D == 3:
                ok = any(_cg(l, m, lp, -m, 0, 0) != 0.0 for m in range(-min(l, lp), min(l, lp) + 1))
            else:
                ok = l == lp
            if ok:
                assert l == lp
                out.add((l, 0, 0))
    return np.array(sorted(out), dtype=np.int32).reshape(-1, 3)


def _d2_average(ls):
    """Rotation average of exp(i sum l theta) over a uniform grid finer than the orders."""
    t = np.arange(128) * (2 * np.pi / 128)
    return abs(np.mean(np.exp(1j * sum(ls) * t)))


def d2(N, lmax):
    """D = 2, N = 3 or 4: signed orders with a non-vanishing rotation average,
    first order >= 0 (the other half is the complex conjugate); labels padded
    to three entries as the library reports them."""
    out = []
    rng = range(-lmax, lmax + 1)
    if N == 3:
        for l1 in range(lmax + 1):
            for l2 in rng:
                if _d2_average((l1, l2)) > 0.5:
                    out.append((l1, l2, 0))
    else:
        for l1 in range(lmax + 1):
            for l2 in rng:
                for l3 in rng:
                    if _d2_average((l1, l2, l3)) > 0.5:
                        out.append((l1, l2, l3))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def _n5_nonzero(l1, l2, l12, l3, l4):
    """Some product (l1 l2 l12; m1 m2 -m12)(l12 l3 l4; m12 m3 m4) is non-zero."""
    for m12 in range(-l12, l12 + 1):
        for m1 in range(-l1, l1 + 1):
            m2 = m12 - m1
            if abs(m2) > l2 or _w3j(l1, l2, l12, m1, m2, -m12) == 0.0:
                continue
            for m3 in range(-l3, l3 + 1):
                m4 = -m12 - m3
                if abs(m4) <= l4 and _w3j(l12, l3, l4, m12, m3, m4) != 0.0:
                    return True
    return False


def d3_n5(lmax):
    """(l1, l2, l12, l3, l4), l_i <= lmax, intermediate l12 up to 2 lmax."""
    out = []
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for l12 in range(2 * lmax + 1):
                for l3 in range(lmax + 1):
                    for l4 in range(lmax + 1):
                        if _n5_nonzero(l1, l2, l12, l3, l4):
                            out.append((l1, l2, l12, l3, l4))
    return np.array(out, dtype=np.int32).reshape(-1, 5)


def line_of_sight(lmax, Lmax):
    """(l1, l2, L): sum_m (l1 l2 L; m -m 0) Y_{l1 m} Y_{l2 -m} is not identically zero."""
    out = []
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for L in range(Lmax + 1):
                if any(_w3j(l1, l2, L, m, -m, 0) != 0.0 for m in range(-min(l1, l2), min(l1, l2) + 1)):
                    out.append((l1, l2, L))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def labels(D, N, lmax, Lmax=None):
    """The label set of the library's output for (D, N, lmax[, Lmax])."""
    if Lmax is not None:
        return line_of_sight(lmax, Lmax)
    if D == 2:
        return d2(N, lmax)
    if N == 3:
        return isotropic_n3(D, lmax)
    if N == 4:
        return d3_n4(lmax)
    return d3_n5(lmax)


def odd_parity(D, N, lab, los=False):
    """Labels whose basis is imaginary (odd sum of the top orders, eq. basis-parity-conj;
    l1 + l2 + L for the line-of-sight basis)."""
    if los:
        return lab.sum(axis=1) % 2 == 1
    if N == 5:
        return (lab[:, 0] + lab[:, 1] + lab[:, 3] + lab[:, 4]) % 2 == 1
    if N == 3 and D >= 3:
        return np.zeros(len(lab), dtype=bool)  # (l, 0, 0): the parity sum is 2 l
    return lab.sum(axis=1) % 2 == 1
