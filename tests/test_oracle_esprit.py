"""Pins for the oracle's ESPRIT on a signal subspace (least-squares ESPRIT on
the two shifted subarrays, the extension to other subspace estimators that
the conclusion proposes) and its general complex eigenvalue solver.

Pins used:
  * the eigenvalue solver against LAPACK (numpy.linalg.eigvals) on random,
    Hermitian, triangular, diagonal and defective-free matrices with repeated
    eigenvalues, and the 2x2 closed form;
  * ESPRIT against its definition evaluated with library routines
    (numpy.linalg.lstsq for Psi, numpy.linalg.eigvals for its eigenvalues);
  * exact recovery of the angles from a noiseless steering subspace, the
    one-source closed form phi = <u_0..M-2, u_1..M-1> / ||u_0..M-2||^2,
    invariance to a unitary mixing of the subspace's columns, and angles
    within a small fraction of a degree at high SNR.
"""
import numpy as np
import pytest

import fmsynth
import oracle


def _match(w, ref):
    """max over w of the distance to the nearest reference eigenvalue"""
    return max(np.min(np.abs(ref - x)) for x in w)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 31, 64])
def test_eigvals_random_against_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    w, st = oracle.eigvals(A)
    assert st >= 0
    ref = np.linalg.eigvals(A)
    scale = max(1.0, np.max(np.abs(ref)))
    assert _match(w, ref) <= 1e-12 * scale
    assert _match(ref, w) <= 1e-12 * scale


def test_eigvals_special_matrices():
    rng = np.random.default_rng(7)
    n = 12
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = B + B.conj().T                          # Hermitian: real eigenvalues
    w, _ = oracle.eigvals(H)
    np.testing.assert_allclose(np.sort(w.real), np.linalg.eigvalsh(H), atol=1e-12)
    assert np.max(np.abs(w.imag)) <= 1e-12
    Tu = np.triu(B)                             # triangular: the diagonal
    w, _ = oracle.eigvals(Tu)
    assert _match(w, np.diag(Tu)) <= 1e-12 and _match(np.diag(Tu), w) <= 1e-12
    D = np.diag(np.array([2, 2, 2, -1j, -1j, 3 + 4j]))
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)))
    w, _ = oracle.eigvals(Q @ D @ Q.conj().T)   # normal, repeated eigenvalues
    assert _match(w, np.diag(D)) <= 1e-12 and _match(np.diag(D), w) <= 1e-12
    a, b, c, d = 1 + 2j, -0.5j, 3.0, 2 - 1j     # 2x2 closed form
    tr, det = a + d, a * d - b * c
    roots = np.array([tr / 2 + np.sqrt(tr * tr / 4 - det), tr / 2 - np.sqrt(tr * tr / 4 - det)])
    w, _ = oracle.eigvals(np.array([[a, b], [c, d]]))
    assert _match(w, roots) <= 1e-14 * 4 and _match(roots, w) <= 1e-14 * 4


def _library_esprit(Us):
    U = Us.T                                    # M x K
    psi = np.linalg.lstsq(U[:-1], U[1:], rcond=None)[0]
    phi = np.linalg.eigvals(psi)
    return np.sort(np.degrees(np.arcsin(np.clip(-np.angle(phi) / np.pi, -1, 1))))


def _steering_subspace(M, thetas):
    A = fmsynth.steering_matrix(M, np.asarray(thetas))
    Q, _ = np.linalg.qr(A)
    return Q.T.copy()                            # [K][M]


@pytest.mark.parametrize("M,thetas", [(16, [10.0]), (64, [-40.0, 3.0, 25.5]),
                                      (200, list(np.linspace(-60, 60, 9))),
                                      (33, [-5.0, 5.0])])
def test_esprit_noiseless_exact(M, thetas):
    Us = _steering_subspace(M, thetas)
    doa, st = oracle.esprit(Us)
    assert st >= 0
    np.testing.assert_allclose(doa, np.sort(thetas), atol=1e-9)


def test_esprit_single_source_closed_form():
    rng = np.random.default_rng(3)
    M = 40
    u = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    u /= np.linalg.norm(u)
    phi = np.vdot(u[:-1], u[1:]) / np.vdot(u[:-1], u[:-1])
    want = np.degrees(np.arcsin(np.clip(-np.angle(phi) / np.pi, -1, 1)))
    doa, _ = oracle.esprit(u[None, :])
    assert doa[0] == pytest.approx(want, abs=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_esprit_matches_library_definition_and_unitary_mixing(seed):
    M, T, K = 96, 192, 5
    fr = fmsynth.make_frame(M, T, K, 5.0, seed=seed, angle_range=(-60, 60), min_sep=4)
    Us, _w = oracle.music_subspace(oracle.covariance(fr.X), K)
    doa, st = oracle.esprit(Us)
    assert st >= 0
    np.testing.assert_allclose(doa, _library_esprit(Us), atol=1e-10)
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K)))
    doa2, _ = oracle.esprit((Us.T @ Q).T.copy())
    np.testing.assert_allclose(doa2, doa, atol=1e-9)


def test_esprit_high_snr_angles():
    M, T, K = 128, 512, 4
    fr = fmsynth.make_frame(M, T, K, 20.0, seed=9, angle_range=(-50, 50), min_sep=5)
    Us, _w = oracle.music_subspace(oracle.covariance(fr.X), K)
    doa, _ = oracle.esprit(Us)
    assert np.max(np.abs(doa - np.sort(fr.thetas_deg))) < 0.02
