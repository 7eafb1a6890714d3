"""The problems of the GPU threshold tests (Sec. 3.2, Eqs. 9-11) really
exercise the threshold: on the oracle's assembled blocks every case drops
eigenvalues, and none of its eigenvalues lies within a factor 3 of
1e-13 * lambda_max, so the dropped set is decided by the FP64 data and not
by the rounding of one eigensolver or another (a backward-stable solver
moves an eigenvalue by at most about m * eps * lambda_max, under half of
the threshold for m <= 192)."""
import numpy as np
import pytest

from tests.gpu_common import THRESHOLD_CASES, dropped_count, threshold_case


@pytest.mark.parametrize("name", sorted(THRESHOLD_CASES))
def test_threshold_case_drops_clear_of_the_band(name):
    d, s, spectra = threshold_case(name)
    m = s["elem_dofs"].shape[1]
    assert m == int(name.split("_m")[1])
    total = 0
    for lam in spectra:
        thr = 1e-13 * lam.max()
        assert lam.max() > 0
        assert not np.any((lam > thr / 3) & (lam < 3 * thr))
        total += dropped_count(lam)
    assert total > 0
    # m * eps * lambda_max stays well inside the factor-3 band
    assert m * np.finfo(float).eps < 0.5e-13
