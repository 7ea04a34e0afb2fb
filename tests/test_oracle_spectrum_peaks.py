"""Pins for the oracle's pseudo-spectrum (eqs. (5), (10)) and peak rule (eq. (6)).

The spectrum is pinned by the closed form of a single steering vector
(a Dirichlet kernel, derived from eq. (5) and the ULA steering of Sec. II-B),
by the bound ||U^H a||^2 <= ||a||^2 = M, by the residual form of the
projection, and by the degenerate cases K = 0 and K = M.  The peak rule is
pinned by hand-built arrays whose answers follow from the stated rule.
"""
import numpy as np
import pytest

import fmsynth
import oracle


def _dirichlet_den(M, s, s0):
    """M - |a(theta0)^H a(theta)|^2 / M for the ULA: x = sin(theta) - sin(theta0),
    |sum_m exp(-j pi m x)|^2 = sin^2(M pi x / 2) / sin^2(pi x / 2)."""
    x = s - s0
    num = np.sin(M * np.pi * x / 2) ** 2
    den = np.sin(np.pi * x / 2) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        return M - num / (M * den), den


@pytest.mark.parametrize("M,theta0", [(8, 10.0), (64, -33.3), (257, 71.0)])
def test_single_source_dirichlet_closed_form(M, theta0):
    th0, dth, L = fmsynth.grid(1801)
    a0 = fmsynth.steering_matrix(M, [theta0])[:, 0]
    U = (a0 / np.sqrt(M))[None, :]
    P, den = oracle.pseudospectrum(U, th0, dth, L)
    theta = th0 + np.arange(L) * dth
    ref, sden = _dirichlet_den(M, np.sin(np.deg2rad(theta)), np.sin(np.deg2rad(theta0)))
    ok = sden > 1e-6  # away from the pole (and its aliases at x = +-2)
    assert np.max(np.abs(den[ok] - ref[ok])) <= 1e-11 * M
    # the argmax is the grid point closest to theta0
    assert abs(theta[np.argmax(P)] - theta0) <= dth / 2 + 1e-9


def test_on_grid_source_peaks_exactly_and_is_clamped():
    M = 64
    th0, dth, L = fmsynth.grid(1801)
    l0 = 1234
    theta0 = th0 + l0 * dth
    a0 = fmsynth.steering_matrix(M, [theta0])[:, 0]
    P, den = oracle.pseudospectrum((a0 / np.sqrt(M))[None, :], th0, dth, L)
    assert np.argmax(P) == l0
    assert abs(den[l0]) <= 1e-12 * M
    assert P[l0] <= 1.0 / (M * 2.0 ** -53) * (1 + 1e-15)  # finite after the clamp


def test_spectrum_lower_bound_and_residual_form():
    rng = np.random.default_rng(9)
    M, K = 48, 5
    Q, _ = np.linalg.qr(rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K)))
    Us = np.ascontiguousarray(Q.T)
    th0, dth, L = fmsynth.grid(721)
    P, den = oracle.pseudospectrum(Us, th0, dth, L)
    assert np.all(den <= M * (1 + 1e-13))
    assert np.all(P >= 1.0 / M * (1 - 1e-13))           # P >= 1/M
    theta = th0 + np.arange(L) * dth
    A = fmsynth.steering_matrix(M, theta)               # (M, L)
    resid = A - Q @ (Q.conj().T @ A)
    assert np.max(np.abs(den - np.sum(np.abs(resid) ** 2, axis=0))) <= 1e-11 * M


def test_spectrum_degenerate_K0_and_full_basis():
    M = 16
    th0, dth, L = fmsynth.grid(181)
    P0, den0 = oracle.pseudospectrum(np.zeros((0, M), complex), th0, dth, L)
    assert np.array_equal(den0, np.full(L, float(M)))
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))
    _, denf = oracle.pseudospectrum(np.ascontiguousarray(Q.T), th0, dth, L)
    assert np.max(np.abs(denf)) <= 1e-12 * M


def test_spectrum_phase_reduction_large_M():
    # large element index: the phase m*sin(theta) must be reduced exactly
    M = 4096
    theta0 = 37.123456
    a0 = fmsynth.steering_matrix(M, [theta0])[:, 0]
    th0, dth, L = theta0 - 0.01, 0.0005, 41
    P, den = oracle.pseudospectrum((a0 / np.sqrt(M))[None, :], th0, dth, L)
    theta = th0 + np.arange(L) * dth
    ref, sden = _dirichlet_den(M, np.sin(np.deg2rad(theta)), np.sin(np.deg2rad(theta0)))
    ok = sden > 1e-9
    assert np.max(np.abs(den[ok] - ref[ok]) / np.maximum(ref[ok], 1.0)) <= 1e-8


# ----------------------------------------------------------------------------
# peak rule, eq. (6)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("P,K,idx", [
    ([1, 3, 2, 5, 5, 4, 0, 7], 3, [7, 3, 1]),      # plateau -> leftmost; right endpoint
    ([9, 1, 2], 2, [0, 2]),                          # both endpoints
    ([1, 4, 1, 4, 1], 1, [1]),                       # equal peaks -> lower index
    ([1, 4, 1, 4, 1], 2, [1, 3]),
    ([1, 2, 3, 4], 3, [3]),                          # fewer peaks than K
    ([2, 2, 2], 2, [0]),                             # flat: leftmost only
    ([5.0], 1, [0]),                                 # single point
    ([3, 1, 3, 1, 3, 1], 5, [0, 2, 4]),
    ([0, 1, 0, 2, 0, 3, 0, 2.5], 2, [5, 7]),
])
def test_peak_rule_hand_built(P, K, idx):
    got, val = oracle.peaks(np.array(P, float), K)
    assert got.tolist() == idx
    assert np.array_equal(val, np.array(P, float)[idx])


def test_peaks_K_zero_and_noise_free_sources_on_grid():
    got, _ = oracle.peaks(np.array([1.0, 2.0, 1.0]), 0)
    assert got.size == 0
    M, L = 64, 1801
    th0, dth, _ = fmsynth.grid(L)
    true_l = np.array([400, 900, 1333])
    A = fmsynth.steering_matrix(M, th0 + true_l * dth)
    Q, _ = np.linalg.qr(A)                       # exact signal subspace of a noiseless frame
    P, _ = oracle.pseudospectrum(np.ascontiguousarray(Q.T), th0, dth, L)
    got, _ = oracle.peaks(P, 3)
    assert sorted(got.tolist()) == true_l.tolist()
