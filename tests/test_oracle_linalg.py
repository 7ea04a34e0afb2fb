"""Pins for the oracle's covariance and dense linear-algebra building blocks.

Each test compares the oracle with something other than itself: an
independent library routine (numpy/LAPACK), an exact integer result, a
closed form, or an invariant the mathematics fixes.
"""
import numpy as np
import pytest

import fmsynth
import oracle


def _rand_herm(rng, n):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A + A.conj().T


# ----------------------------------------------------------------------------
# covariance, eqs. (2)-(3)
# ----------------------------------------------------------------------------

def test_covariance_matches_library_matmul():
    rng = np.random.default_rng(1)
    X = (rng.standard_normal((17, 33)) + 1j * rng.standard_normal((17, 33))).astype(np.complex64)
    R = oracle.covariance(X)
    Xd = X.astype(np.complex128)
    ref = Xd @ Xd.conj().T / X.shape[1]
    assert np.max(np.abs(R - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_covariance_integer_frame_exact():
    # integer entries: every partial sum is an exact integer in double
    X = fmsynth.make_integer_frame(8, 64, seed=3)
    R = oracle.covariance(X)
    re = X.real.astype(np.int64)
    im = X.imag.astype(np.int64)
    # X X^H with exact integer arithmetic: (a+ib)(c-id) = (ac+bd) + i(bc-ad)
    RR = re @ re.T + im @ im.T
    RI = im @ re.T - re @ im.T
    assert np.array_equal(R.real * 64, RR.astype(np.float64))
    assert np.array_equal(R.imag * 64, RI.astype(np.float64))


def test_covariance_invariants():
    fr = fmsynth.make_frame(24, 40, 3, 5.0, seed=11)
    R = oracle.covariance(fr.X)
    assert np.array_equal(R, R.conj().T)            # Hermitian, bit for bit
    assert np.all(np.diag(R).imag == 0)             # real diagonal
    tr = np.trace(R).real
    fro = np.sum(np.abs(fr.X.astype(np.complex128)) ** 2) / fr.T
    assert abs(tr - fro) <= 1e-12 * fro             # trace(R) = ||X||_F^2 / T
    w = np.linalg.eigvalsh(R)
    assert w.min() >= -1e-12 * w.max()              # positive semidefinite


def test_covariance_rank_deficient_when_T_lt_M():
    rng = np.random.default_rng(5)
    X = (rng.standard_normal((12, 4)) + 1j * rng.standard_normal((12, 4))).astype(np.complex64)
    w = np.linalg.eigvalsh(oracle.covariance(X))
    assert np.sum(w > 1e-10 * w.max()) == 4


# ----------------------------------------------------------------------------
# Jacobi eigen-decomposition (eq. (4) for Hermitian S)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 40, 64])
def test_eigh_matches_lapack(n):
    rng = np.random.default_rng(n)
    A = _rand_herm(rng, n)
    w, V, sw = oracle.eigh(A)
    assert sw >= 0
    wl, Vl = np.linalg.eigh(A)
    wl, Vl = wl[::-1], Vl[:, ::-1]
    scale = np.max(np.abs(wl))
    assert np.max(np.abs(w - wl)) <= 1e-12 * scale
    # eigenvector projectors wherever the eigenvalue is separated
    gaps = np.abs(np.subtract.outer(wl, wl)) + np.eye(n) * 1e300
    for k in range(n):
        if gaps[k].min() > 1e-6 * scale:
            Pk = np.outer(V[:, k], V[:, k].conj())
            Pl = np.outer(Vl[:, k], Vl[:, k].conj())
            assert np.max(np.abs(Pk - Pl)) <= 1e-9
    assert np.max(np.abs(A @ V - V * w)) <= 1e-12 * n * scale
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) <= 1e-13 * n


def test_eigh_2x2_closed_form():
    a, d, b = 1.5, -0.25, 0.7 - 1.2j
    w, V, _ = oracle.eigh(np.array([[a, b], [np.conj(b), d]]))
    mid, rad = (a + d) / 2, np.sqrt(((a - d) / 2) ** 2 + abs(b) ** 2)
    assert np.allclose(w, [mid + rad, mid - rad], rtol=0, atol=1e-15)


def test_eigh_known_spectrum_with_degeneracy():
    rng = np.random.default_rng(7)
    n = 12
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.array([9, 7, 7, 7, 4, 2, 1, 0.5, 0.5, 0.1, 0.0, -3.0])
    A = (Q * lam) @ Q.conj().T
    w, V, _ = oracle.eigh(A)
    assert np.max(np.abs(w - lam)) <= 1e-13 * 9
    # projector on the 3-fold cluster is unique even though the basis is not
    Pc = V[:, 1:4] @ V[:, 1:4].conj().T
    Pq = Q[:, 1:4] @ Q[:, 1:4].conj().T
    assert np.max(np.abs(Pc - Pq)) <= 1e-12


def test_eigh_diagonal_input_sorted_no_sweeps():
    w, V, sw = oracle.eigh(np.diag([1.0, 5.0, 3.0]).astype(complex))
    assert sw == 0
    assert np.array_equal(w, [5.0, 3.0, 1.0])
    assert np.array_equal(np.abs(V), np.eye(3)[:, [1, 2, 0]])


# ----------------------------------------------------------------------------
# one-sided Jacobi SVD, MGS2 orth, eigen pseudo-inverse
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(5, 1), (10, 4), (64, 16), (200, 40)])
def test_svd_matches_lapack(m, n):
    rng = np.random.default_rng(m * n)
    Cm = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    U, s, V, sw = oracle.svd(Cm)
    assert sw >= 0
    sl = np.linalg.svd(Cm, compute_uv=False)
    assert np.max(np.abs(s - sl)) <= 1e-13 * sl[0] * n
    assert np.max(np.abs((U * s) @ V.conj().T - Cm)) <= 1e-13 * sl[0] * n
    assert np.max(np.abs(U.conj().T @ U - np.eye(n))) <= 1e-12
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) <= 1e-12


def test_svd_rank_deficient_has_zero_columns():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((30, 2)) + 1j * rng.standard_normal((30, 2))
    Cm = np.concatenate([B, B @ np.array([[1, 2j], [0.5, -1]])], axis=1)  # rank 2
    U, s, V, _ = oracle.svd(Cm)
    assert np.all(s[2:] <= 1e-13 * s[0])
    assert np.max(np.abs((U * s) @ V.conj().T - Cm)) <= 1e-12 * s[0]


def test_orth_spans_column_space():
    rng = np.random.default_rng(3)
    Cm = rng.standard_normal((50, 7)) + 1j * rng.standard_normal((50, 7))
    Q, r = oracle.orth(Cm)
    assert r == 7
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(7))) <= 1e-14 * 10
    Ql, _ = np.linalg.qr(Cm)
    assert np.max(np.abs(Q @ Q.conj().T - Ql @ Ql.conj().T)) <= 1e-13


def test_orth_drops_dependent_columns():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))
    Cm = np.concatenate([B, B[:, :1] * (2 - 1j), B[:, 1:] @ np.ones((2, 1))], axis=1)
    Q, r = oracle.orth(Cm)
    assert r == 3
    Ql, _ = np.linalg.qr(B)
    assert np.max(np.abs(Q @ Q.conj().T - Ql @ Ql.conj().T)) <= 1e-12


def test_pinv_matches_library_and_penrose():
    rng = np.random.default_rng(6)
    n = 9
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.array([10, 5, 2, 1, 1e-3, 1e-4, 1e-7, 0, 0])
    A = (Q * lam) @ Q.conj().T
    A = (A + A.conj().T) / 2
    Ap, r = oracle.pinv_herm(A, 1e-6)
    assert r == 6  # threshold 10 * 1e-6 = 1e-5 keeps 10, 5, 2, 1, 1e-3, 1e-4
    ref = np.linalg.pinv(A, rcond=1e-6, hermitian=True)
    assert np.max(np.abs(Ap - ref)) <= 1e-8 * np.max(np.abs(ref))
    # Moore-Penrose conditions restricted to the kept eigenspace
    At = (Q[:, :6] * lam[:6]) @ Q[:, :6].conj().T
    assert np.max(np.abs(At @ Ap @ At - At)) <= 1e-10
    assert np.max(np.abs(Ap @ At @ Ap - Ap)) <= 1e-6 * np.max(np.abs(Ap))
    assert np.max(np.abs(Ap - Ap.conj().T)) <= 1e-10


def test_orth_stays_orthonormal_when_ill_conditioned():
    # nearly dependent columns (condition ~1e9): a single Gram-Schmidt pass
    # loses orthogonality, the re-orthogonalised one does not
    rng = np.random.default_rng(12)
    B = rng.standard_normal((60, 6)) + 1j * rng.standard_normal((60, 6))
    Cm = B @ np.diag(10.0 ** (-1.6 * np.arange(6))) @ (
        np.eye(6) + 1e-3 * rng.standard_normal((6, 6)))
    Cm[:, 1:] += Cm[:, :1]
    Q, r = oracle.orth(Cm)
    assert r == 6
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(6))) <= 1e-13
