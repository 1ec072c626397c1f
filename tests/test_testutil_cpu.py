"""CPU checks of the test helpers' conditioning scale (the sum of the
magnitudes of the estimator's terms), which the GPU parity tests use."""
import numpy as np

import oracle
from paper_2106_10278_amd import inputs
from npcf_testutil import condition_scale, conditioned_error, oracle_reported


def test_scale_bounds_zeta():
    for D, N, L in [(3, 3, 3), (3, 4, 2), (2, 4, 3), (4, 3, 2)]:
        wl = inputs.tiny(D, N, L, 150, 7, box_side=10.0, rmax=3.0, nbins=3)
        ref, _, _ = oracle_reported(wl)
        sc = condition_scale(wl)
        assert sc.shape == ref.shape
        assert np.all(sc >= np.abs(ref) * (1 - 1e-12))


def test_scale_equals_monopole_for_positive_weights():
    """With w > 0 every term of the Lambda = 0 3PCF is w_i |a_00|^2 C >= 0 with C > 0,
    so the magnitude sum is zeta itself (eq. NPCF-estimator-discrete)."""
    wl = inputs.tiny(3, 3, 2, 200, 9, box_side=10.0, rmax=3.0, nbins=3, weights="ones")
    ref, _, _ = oracle_reported(wl, btuple_mode=1)
    sc = condition_scale(wl, btuple_mode=1)
    lab = oracle.lambda_labels(3, 3, 2)
    i0 = int(np.nonzero(lab[:, 0] == 0)[0][0])
    assert np.allclose(sc[i0], ref[i0], rtol=1e-12)


def test_conditioned_error_is_scale_relative():
    ref = np.array([[1.0, -1.0], [1e-3, 2e-3]])
    sc = np.array([[2.0, 2.0], [1.0, 1.0]])
    got = ref + np.array([[1e-6, 0.0], [0.0, 1e-6]])
    err, errs = conditioned_error(got, ref, sc)
    assert np.allclose(errs, [5e-7, 1e-6]) and err == errs.max()
