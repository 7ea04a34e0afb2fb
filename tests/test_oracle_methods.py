"""Pins for the oracle's subspace estimators: standard MUSIC (eq. (4)),
Method 1 (Alg. 1) and Method 2 (Alg. 2).

Pins used:
  * exactness statements of the paper: a rank-K covariance is recovered
    exactly by the Nystrom sketch (Fig. 2; Lemmas 5 and 6, Appendix), and the
    sketch is exact when it spans the whole space (p = M, l = M);
  * the definition of the approximation, eq. (9), evaluated with library
    routines (numpy pinv/eigh) against the oracle's rank-restriction route;
  * the probabilistic bounds of Theorems 1-3 (Sec. IV) over many seeds;
  * the peak-preservation argument of Sec. IV-E;
  * invariance to the order of the sampled index set.
"""
import json
import os

import numpy as np
import pytest

import fmsynth
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def proj(U_cols):
    """Orthogonal projector onto the span of the given columns (numpy QR)."""
    Q, _ = np.linalg.qr(U_cols)
    return Q @ Q.conj().T


def us_proj(Us):
    """Projector U_s U_s^H from the [K][M] storage."""
    return Us.T @ Us.conj()


def exact_rank_k_cov(M, thetas, powers):
    A = fmsynth.steering_matrix(M, thetas)
    return (A * np.asarray(powers, float)) @ A.conj().T, A


def top_k_projector_lapack(R, K):
    w, V = np.linalg.eigh(R)
    return proj(V[:, ::-1][:, :K])


# ----------------------------------------------------------------------------
# Fig. 2: rank-4 matrix, I = {1, 4, 2, 9}, error < 1e-12
# ----------------------------------------------------------------------------

def test_fig2_rank4_nystrom_exact():
    g = json.load(open(os.path.join(GOLDEN, "fig2_nystrom_rank4.json")))
    n, r = g["n"], g["rank"]
    rng = np.random.default_rng(2019)
    B = rng.standard_normal((n, r))
    S = B @ B.T                                         # real, rank 4, as in the figure
    Us, sig, rank = oracle.subspace_sample(S.astype(complex), np.array(g["index_set"]), r)
    assert rank == r
    St = (Us.T * sig) @ Us.conj()                       # C W C^H = U~ Sigma_B U~^H
    err = np.linalg.norm(St - S) / np.linalg.norm(S)
    assert err < g["max_relative_error"]


# ----------------------------------------------------------------------------
# exactness: rank-K covariance and full sketches (Lemmas 5, 6)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("M,K,p", [(32, 3, 3), (64, 4, 12), (100, 7, 30)])
def test_method1_exact_on_rank_k(M, K, p):
    rng = np.random.default_rng(M + K)
    th = fmsynth.draw_angles(rng, K, -70, 70, 3.0)
    R, A = exact_rank_k_cov(M, th, rng.uniform(0.5, 2.0, K))
    idx = fmsynth.make_idx(M, p, seed=M * K)
    Us, sig, rank = oracle.subspace_sample(R, idx, K)
    assert rank == K
    assert np.max(np.abs(us_proj(Us) - proj(A))) <= 1e-10
    assert np.max(np.abs(Us.conj() @ Us.T - np.eye(K))) <= 1e-12


@pytest.mark.parametrize("M,K,l,q", [(32, 3, 3, 0), (64, 4, 12, 1), (100, 7, 15, 2)])
def test_method2_exact_on_rank_k(M, K, l, q):
    rng = np.random.default_rng(M + K + 1)
    th = fmsynth.draw_angles(rng, K, -70, 70, 3.0)
    R, A = exact_rank_k_cov(M, th, rng.uniform(0.5, 2.0, K))
    Om = fmsynth.make_omega(M, l, seed=M * l)
    Us, sig, rank = oracle.subspace_project(R, Om, q, K)
    assert rank == K
    assert np.max(np.abs(us_proj(Us) - proj(A))) <= 1e-10


def test_full_sketches_equal_standard_music():
    fr = fmsynth.make_frame(40, 80, 3, 0.0, seed=21)
    R = oracle.covariance(fr.X)
    Pref = top_k_projector_lapack(R, 3)
    U1, _, r1 = oracle.subspace_sample(R, np.arange(40, dtype=np.int32)[::-1].copy(), 3)
    U2, _, r2 = oracle.subspace_project(R, fmsynth.make_omega(40, 40, 5), 1, 3)
    Um, w = oracle.music_subspace(R, 3)
    assert r1 == 40 and r2 == 40
    for U in (U1, U2, Um):
        assert np.max(np.abs(us_proj(U) - Pref)) <= 1e-9
    assert np.max(np.abs(w - np.linalg.eigvalsh(R)[::-1])) <= 1e-12 * w[0]


# ----------------------------------------------------------------------------
# eq. (9) by library routines vs the oracle's rank restriction (Alg. 1/2 step 2)
# ----------------------------------------------------------------------------

def _top_k_of(St, K):
    w, V = np.linalg.eigh((St + St.conj().T) / 2)
    return proj(V[:, ::-1][:, :K]), w[::-1][:K]


def test_method1_equals_definition_of_eq9():
    fr = fmsynth.make_frame(64, 128, 3, 10.0, seed=5, angle_range=(-60, 60), min_sep=5)
    R = oracle.covariance(fr.X)
    idx = fmsynth.make_idx(64, 44, seed=5)
    Us, sig, _ = oracle.subspace_sample(R, idx, 3)
    Cm = R[:, idx]
    W = np.linalg.pinv(R[np.ix_(idx, idx)], rcond=1e-6, hermitian=True)
    Pdef, wdef = _top_k_of(Cm @ W @ Cm.conj().T, 3)
    assert np.max(np.abs(us_proj(Us) - Pdef)) <= 1e-9
    assert np.max(np.abs(sig - wdef)) <= 1e-10 * wdef[0]


def test_method2_equals_definition_of_eq9():
    fr = fmsynth.make_frame(64, 128, 3, 0.0, seed=6, angle_range=(-60, 60), min_sep=5)
    R = oracle.covariance(fr.X)
    Om = fmsynth.make_omega(64, 11, seed=6).astype(complex)
    q = 2
    Y = Om
    for _ in range(q):
        Y = R @ Y
    V, _ = np.linalg.qr(Y)                       # orth(S^q Omega)
    Cm = R @ V
    W = np.linalg.pinv(V.conj().T @ Cm, rcond=1e-6, hermitian=True)
    Pdef, wdef = _top_k_of(Cm @ W @ Cm.conj().T, 3)
    Us, sig, _ = oracle.subspace_project(R, Om.real.astype(np.float32), q, 3)
    assert np.max(np.abs(us_proj(Us) - Pdef)) <= 1e-9
    assert np.max(np.abs(sig - wdef)) <= 1e-10 * wdef[0]


def test_method1_invariant_to_index_order():
    fr = fmsynth.make_frame(50, 100, 4, 5.0, seed=8)
    R = oracle.covariance(fr.X)
    idx = fmsynth.make_idx(50, 20, seed=8)
    U1, s1, _ = oracle.subspace_sample(R, idx, 4)
    U2, s2, _ = oracle.subspace_sample(R, np.ascontiguousarray(idx[::-1]), 4)
    assert np.max(np.abs(us_proj(U1) - us_proj(U2))) <= 1e-10
    assert np.max(np.abs(s1 - s2)) <= 1e-10 * s1[0]


def test_method2_power_iterations_reduce_error():
    # Theorem 2: the error decays like (sigma_{K+1}/sigma_K)^(t+1)
    errs = {0: [], 1: [], 2: []}
    for seed in range(6):
        fr = fmsynth.make_frame(64, 128, 4, -5.0, seed=100 + seed)
        R = oracle.covariance(fr.X)
        Pref = top_k_projector_lapack(R, 4)
        Om = fmsynth.make_omega(64, 4, seed=100 + seed)
        for q in errs:
            Us, _, _ = oracle.subspace_project(R, Om, q, 4)
            errs[q].append(np.linalg.norm(us_proj(Us) - Pref, 2))
    med = {q: np.median(v) for q, v in errs.items()}
    assert med[2] < med[1] < med[0]


# ----------------------------------------------------------------------------
# Theorems 1-3: relative bounds on sqrt(P / P~), checked over many seeds
# ----------------------------------------------------------------------------

def _music_and_eigs(R, K, th0, dth, L):
    Um, w = oracle.music_subspace(R, K)
    P, _ = oracle.pseudospectrum(Um, th0, dth, L)
    return P, w, Um


def _coherence(Um):
    M, K = Um.shape[1], Um.shape[0]
    return M / K * np.max(np.sum(np.abs(Um) ** 2, axis=0))


def _violation_budget(delta, n):
    return delta + 3 * np.sqrt(delta * (1 - delta) / n)


def test_theorem1_lower_bound_method1():
    M, T, K, delta, n = 96, 192, 3, 0.1, 24
    th0, dth, L = fmsynth.grid(361)
    viol = 0
    for seed in range(n):
        fr = fmsynth.make_frame(M, T, K, 5.0, seed=300 + seed, angle_range=(0, 80), min_sep=5)
        R = oracle.covariance(fr.X)
        P, w, Um = _music_and_eigs(R, K, th0, dth, L)
        mu = _coherence(Um)
        p = int(min(M, np.ceil(4.5 * mu * K * np.log(K / delta))))
        rho = w[K] / w[K - 1]
        kappa = 1 + 2 * np.sqrt(M ** 2 / p) * rho
        idx = fmsynth.make_idx(M, p, seed=300 + seed)
        _, _, rank = oracle.subspace_sample(R, idx, K)
        Ut, _, _ = oracle.subspace_sample(R, idx, rank)   # orthonormal basis of S~
        Pt, _ = oracle.pseudospectrum(Ut, th0, dth, L)
        viol += np.any(np.sqrt(P / Pt) > kappa * (1 + 1e-12))
    assert viol <= _violation_budget(delta, n) * n


@pytest.mark.parametrize("t", [1, 2])
def test_theorems2_3_bounds_method2(t):
    # Sec. V-C setting scaled down: K = 9 in [0, 80] deg, SNR 1 dB, l = K
    M, T, K, delta, n = 128, 256, 9, 0.1, 20
    th0, dth, L = fmsynth.grid(361)
    viol_lo = viol_hi = 0
    for seed in range(n):
        fr = fmsynth.make_frame(M, T, K, 1.0, seed=500 + seed, angle_range=(0, 80), min_sep=4)
        R = oracle.covariance(fr.X)
        P, w, _ = _music_and_eigs(R, K, th0, dth, L)
        rho = w[K] / w[K - 1]
        alpha = np.sqrt(M ** 2 * K) / delta * rho ** (t + 1)
        Ut, _, _ = oracle.subspace_project(R, fmsynth.make_omega(M, K, 500 + seed), t, K)
        Pt, _ = oracle.pseudospectrum(Ut, th0, dth, L)
        ratio = np.sqrt(P / Pt)
        viol_lo += np.any(ratio > (1 + alpha) * (1 + 1e-12))
        viol_hi += np.any(ratio < (1 - alpha) * (1 - 1e-12))
    assert viol_lo <= _violation_budget(delta, n) * n
    assert viol_hi <= _violation_budget(delta, n) * n


# ----------------------------------------------------------------------------
# Sec. IV-E: the fast spectra keep the peaks of standard MUSIC
# ----------------------------------------------------------------------------

def test_fast_methods_keep_music_peaks_config1_shape():
    cfg = fmsynth.CONFIGS["c1"]
    th0, dth, L = fmsynth.grid(cfg["L"])
    for seed in range(5):
        fr, _ = fmsynth.config_frame("c1", seed=700 + seed)
        K = fr.K
        ref = oracle.run_frame(fr.X, K, "music", th0, dth, L)
        f1 = oracle.run_frame(fr.X, K, "sample", th0, dth, L,
                              idx=fmsynth.make_idx(fr.M, cfg["p"], 700 + seed))
        f2 = oracle.run_frame(fr.X, K, "project", th0, dth, L,
                              Omega=fmsynth.make_omega(fr.M, cfg["l"], 700 + seed), q=cfg["q"])
        for f in (f1, f2):
            assert len(f["peak_idx"]) == len(ref["peak_idx"]) == K
            for pk in ref["peak_idx"]:
                assert np.min(np.abs(f["peak_idx"] - pk)) <= 1
        # and the peaks sit at the true angles to within the resolution of the frame
        est = np.sort(th0 + ref["peak_idx"] * dth)
        assert np.max(np.abs(est - np.sort(fr.thetas_deg))) < 1.0


def test_noiseless_on_grid_sources_music_peaks_exact():
    M, T = 64, 128
    th0, dth, L = fmsynth.grid(1801)
    true_l = np.array([350, 1000, 1500])
    fr = fmsynth.make_frame(M, T, 3, 0.0, seed=1, thetas_deg=th0 + true_l * dth, noiseless=True)
    out = oracle.run_frame(fr.X, 3, "music", th0, dth, L)
    assert sorted(out["peak_idx"].tolist()) == true_l.tolist()
    _, A = exact_rank_k_cov(M, th0 + true_l * dth, [1, 1, 1])
    # complex64 rounding of X is the only error source
    assert np.max(np.abs(us_proj(out["Us"]) - proj(A))) <= 1e-6
