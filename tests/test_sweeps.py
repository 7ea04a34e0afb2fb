"""Host logic of the experiment sweeps (sweeps.py): the spectrum
normalisation and error of Sec. V-A, peak agreement, and the AoA squared
error of eq. (21) with estimates assigned to the true angles (no GPU)."""
import numpy as np
import pytest

import sweeps


def test_normalised_and_error():
    P = np.array([2.0, 4.0, 10.0, 3.0])
    n = sweeps.normalised(P)
    assert n.min() == 0.0 and n.max() == 1.0
    np.testing.assert_allclose(n, [0.0, 0.25, 1.0, 0.125])
    assert sweeps.approx_error(P, P * 7.0 + 1.0) == pytest.approx(0.0, abs=1e-24)
    assert sweeps.approx_error(P, np.array([2.0, 10.0, 4.0, 3.0])) == pytest.approx(
        (0.25 - 1.0) ** 2 + (1.0 - 0.25) ** 2)
    assert np.all(sweeps.normalised(np.ones(5)) == 0.0)


def test_peaks_agree():
    assert sweeps.peaks_agree([10, 51, 99], [50, 100])
    assert not sweeps.peaks_agree([10, 53, 99], [50, 100])
    assert not sweeps.peaks_agree([50], [50, 100])


def test_aoa_sq_error_assignment():
    true = np.array([10.0, 20.0, 30.0])
    # a permutation of exact estimates costs nothing
    assert sweeps.aoa_sq_error([30.0, 10.0, 20.0], true) == 0.0
    # one estimate off by 0.5 deg
    assert sweeps.aoa_sq_error([10.0, 20.5, 30.0], true) == pytest.approx(0.25 / 3)
    # a missing estimate takes the nearest one: 30 -> 20 costs 100
    assert sweeps.aoa_sq_error([10.0, 20.0], true) == pytest.approx(100.0 / 3)
    # the assignment minimises the total, not each angle greedily
    assert sweeps.aoa_sq_error([11.0, 19.0], [10.0, 12.0]) == pytest.approx((1.0 + 49.0) / 2)
    assert np.isnan(sweeps.aoa_sq_error([], true))
