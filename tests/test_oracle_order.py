"""Pins for the oracle's model-order estimate: the pre-estimation of K with
Akaike's information criterion (AIC) or the minimum description length (MDL)
that Sec. V-D proposes, evaluated on the eigenvalues of the Method 2 sketch
with the unseen eigenvalues of R completed from its trace.

Pins used:
  * closed forms of the criteria for a single spike over a flat noise floor
    (one eigenvalue lam, M - 1 equal to one): the likelihood term vanishes
    for every k >= 1 and is N (M log((lam + M - 1)/M) - log lam) at k = 0,
    so each criterion at k >= 1 is its penalty alone;
  * a flat spectrum (pure noise) gives K_hat = 0;
  * the completion: n known eigenvalues plus a trace equal the explicit list
    with the M - n missing eigenvalues set to their mean;
  * a sketch that spans the whole space (l = M) sees the eigenvalues of R, so
    the estimate equals the criterion on numpy's eigenvalues of R;
  * invariance to the scale of R; eigenvalues below the rcond threshold are
    treated as unseen (moved into the completion);
  * exact (population) covariances A P A^H + s I and A P A^H give K_hat = K,
    and synthetic frames at the paper's Sec. V-D setting give the true K.
"""
import math

import numpy as np
import pytest

import fmsynth
import oracle

AIC, MDL = oracle.ORDER_AIC, oracle.ORDER_MDL


@pytest.mark.parametrize("M,N,lam", [(4, 10, 4.0), (8, 100, 30.0), (64, 128, 2.5), (200, 400, 1e3)])
def test_single_spike_closed_form(M, N, lam):
    sig = np.array([lam] + [1.0] * (M - 1))
    tr = lam + (M - 1)
    L0 = N * (M * math.log((lam + M - 1) / M) - math.log(lam))
    for kind in (AIC, MDL):
        k, crit = oracle.order_criteria(sig, M, N, tr, kind, rcond=0.0)
        assert crit.shape == (M + 1,)
        assert np.isinf(crit[M])  # r == M: k runs to M - 1
        pen0 = 0.0
        want0 = 2 * L0 + 2 * pen0 if kind == AIC else L0
        assert crit[0] == pytest.approx(want0, rel=1e-12)
        for kk in range(1, M):
            pen = kk * (2 * M - kk)
            want = 2.0 * pen if kind == AIC else 0.5 * pen * math.log(N)
            assert crit[kk] == pytest.approx(want, rel=1e-12, abs=1e-9)
        assert k == int(np.argmin(crit[:M]))


def test_hand_worked_example():
    # eigenvalues (4, 1, 1, 1), N = 10: L(0) = 10 (4 ln(7/4) - ln 4) = 8.52168...,
    # MDL(1) = 3.5 ln 10 = 8.05904..., AIC(0) = 17.0433..., AIC(1) = 14
    k, crit = oracle.order_criteria([4, 1, 1, 1], 4, 10, 7.0, MDL, rcond=0.0)
    assert crit[0] == pytest.approx(8.521687, abs=1e-6)
    assert crit[1] == pytest.approx(8.059048, abs=1e-6)
    assert k == 1
    k, crit = oracle.order_criteria([4, 1, 1, 1], 4, 10, 7.0, AIC, rcond=0.0)
    assert crit[0] == pytest.approx(17.043376, abs=1e-6)
    assert crit[1] == 14.0 and crit[2] == 24.0 and crit[3] == 30.0
    assert k == 1


@pytest.mark.parametrize("kind", [AIC, MDL])
def test_flat_spectrum_gives_zero(kind):
    M = 32
    k, crit = oracle.order_criteria(np.full(8, 2.0), M, 64, 2.0 * M, kind)
    assert k == 0
    assert crit[0] == 0.0


@pytest.mark.parametrize("kind", [AIC, MDL])
def test_completion_equals_explicit_list(kind):
    rng = np.random.default_rng(3)
    M, N = 12, 50
    known = np.sort(rng.uniform(1.5, 20.0, 5))[::-1]
    c = 0.7
    tr = known.sum() + (M - 5) * c
    full = np.concatenate([known, np.full(M - 5, c)])
    k1, crit1 = oracle.order_criteria(known, M, N, tr, kind)
    k2, crit2 = oracle.order_criteria(full, M, N, tr, kind)
    assert k1 == k2
    np.testing.assert_allclose(crit1[:6], crit2[:6], rtol=1e-12)
    assert np.all(np.isinf(crit1[6:]))


@pytest.mark.parametrize("kind", [AIC, MDL])
def test_below_rcond_is_unseen(kind):
    M, N = 40, 80
    sig = np.array([50.0, 20.0, 9.0, 1.2, 1.1, 1.0])
    tr = sig.sum() + (M - 6) * 0.9
    k1, crit1 = oracle.order_criteria(sig, M, N, tr, kind, rcond=1e-6)
    k2, crit2 = oracle.order_criteria(np.concatenate([sig, [1e-9, 0.0]]), M, N, tr, kind,
                                      rcond=1e-6)
    assert k1 == k2
    np.testing.assert_allclose(crit1[:7], crit2[:7], rtol=1e-12)


def _frame_R(M, T, K, snr, seed):
    fr = fmsynth.make_frame(M, T, K, snr, seed=seed, angle_range=(-60.0, 60.0), min_sep=3.0)
    return oracle.covariance(fr.X, threads=oracle.default_threads())


@pytest.mark.parametrize("kind", [AIC, MDL])
def test_full_width_sketch_matches_eigenvalues_of_R(kind):
    M, T, K = 24, 96, 3
    R = _frame_R(M, T, K, 0.0, seed=11)
    Om = fmsynth.make_omega(M, M, 5)
    k, crit, sig = oracle.order_estimate(R, Om, 1, T, kind)
    w = np.sort(np.linalg.eigvalsh(R))[::-1]
    np.testing.assert_allclose(sig, w, rtol=1e-9, atol=1e-12 * w[0])
    k_ref, crit_ref = oracle.order_criteria(w, M, T, float(np.trace(R).real), kind)
    assert k == k_ref == K
    np.testing.assert_allclose(crit[:M], crit_ref[:M], rtol=1e-7)


@pytest.mark.parametrize("kind", [AIC, MDL])
def test_scale_invariance(kind):
    M, T = 64, 128
    R = _frame_R(M, T, 4, -3.0, seed=12)
    Om = fmsynth.make_omega(M, 16, 6)
    k1, crit1, _ = oracle.order_estimate(R, Om, 2, T, kind)
    k2, crit2, _ = oracle.order_estimate(R * 37.5, Om, 2, T, kind)
    assert k1 == k2
    np.testing.assert_allclose(crit1[np.isfinite(crit1)], crit2[np.isfinite(crit2)], rtol=1e-8)


@pytest.mark.parametrize("noise", [0.5, 0.0])
@pytest.mark.parametrize("kind", [AIC, MDL])
def test_population_covariance(kind, noise):
    M, K = 64, 3
    A = fmsynth.steering_matrix(M, np.array([-30.0, 5.0, 41.0]))
    R = (A * np.array([4.0, 2.0, 1.0])) @ A.conj().T + noise * np.eye(M)
    Om = fmsynth.make_omega(M, 12, 7)
    k, _crit, sig = oracle.order_estimate(R, Om, 2, 200, kind)
    assert k == K
    assert sig[0] > sig[K - 1] > (sig[K] if sig[K] > 0 else -1.0)


@pytest.mark.parametrize("kind", [AIC, MDL])
def test_paper_setting_recovers_k(kind):
    # Sec. V-D's setting: M = 200, N = 2M, K = 10 at 0 dB
    M, T, K = 200, 400, 10
    R = _frame_R(M, T, K, 0.0, seed=5)
    Om = fmsynth.make_omega(M, 24, 7)
    k, _crit, _sig = oracle.order_estimate(R, Om, 2, T, kind)
    assert k == K
