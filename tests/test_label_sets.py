"""Label sets pinned independently of the oracle (eq. addition-triangle-conditions,
eq. selection-rules, and the component counts of the sections "Cosmic
Microwave Background" and "Hydrodynamic Turbulence").

The expected sets come from ``labels_indep`` (SymPy coefficients and D = 2
rotation averages, no oracle code).  A label that the oracle's enumeration
dropped or invented changes the set or its size and fails here; the GPU
planner's labels are held to the same sets in ``test_gpu_parity.py``.
"""
import json
import os

import numpy as np
import pytest

import oracle
import labels_indep as li

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("D,N,lmax,Lmax,total,odd", [
    # D = 3, N = 4, lmax 5: the benchmark configuration's 111 triples
    (3, 4, 5, None, 111, 42),
    (3, 4, 2, None, 15, 4),
    (3, 4, 8, None, 369, 154),
    # D = 2, N = 4: 35 at lmax 4 is the paper's CMB count; 117 at |l| <= 8 the turbulence configuration's
    (2, 4, 4, None, 35, 0),
    (2, 4, 8, None, 117, 0),
    (2, 3, 4, None, 5, 0),
    (3, 3, 5, None, 6, 0),
    (4, 3, 6, None, 7, 0),
    # N = 5, lmax 4: 1085 labels, of which the paper's 585 even and 500 odd
    (3, 5, 4, None, 1085, 500),
    # line-of-sight 3PCF, lmax 5, L <= 6
    (3, 3, 5, 6, 126, 48),
])
def test_label_counts(D, N, lmax, Lmax, total, odd):
    lab = li.labels(D, N, lmax, Lmax)
    assert len(lab) == total
    assert int(li.odd_parity(D, N, lab, los=Lmax is not None).sum()) == odd


@pytest.mark.parametrize("D,N,lmax,Lmax", [
    (3, 4, 5, None), (3, 4, 3, None), (3, 4, 8, None), (2, 4, 4, None), (2, 4, 8, None),
    (2, 3, 6, None), (3, 3, 5, None), (4, 3, 6, None), (3, 5, 4, None), (3, 5, 2, None),
    (3, 3, 5, 6), (3, 3, 4, 8), (3, 3, 3, 0)])
def test_oracle_labels_equal_independent_sets(D, N, lmax, Lmax):
    """The oracle lists exactly the independently enumerated labels, in lexicographic order."""
    got = oracle.lambda_labels(D, N, lmax, Lmax)
    ref = li.labels(D, N, lmax, Lmax)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)


def test_paper_counts_from_independent_sets():
    """The paper's printed counts, from the independent enumeration."""
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    assert len(li.labels(2, 4, 4)) == g["d2_n4_lmax4_angular"]
    lab5 = li.labels(3, 5, 4)
    assert int((~li.odd_parity(3, 5, lab5)).sum()) == g["n5_lmax4_angular_even"]


@pytest.mark.gpu
@pytest.mark.parametrize("D,N,lmax,Lmax", [
    (3, 4, 5, None), (3, 4, 8, None), (2, 4, 8, None), (2, 3, 6, None), (3, 3, 5, None), (4, 3, 6, None),
    (3, 5, 4, None), (3, 3, 5, 6)])
def test_plan_labels_equal_independent_sets(D, N, lmax, Lmax):
    """The GPU planner's labels (npcf_describe) are the independently enumerated set."""
    from paper_2106_10278_amd import NPCF
    edges = np.linspace(1.0, 3.0, 6)
    plan = NPCF(D, N, lmax, edges, [10.0] * D, max_points=64, Lmax=Lmax)
    ref = li.labels(D, N, lmax, Lmax)
    got = plan.lambda_labels[:, : ref.shape[1]]
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)
    plan.close()
