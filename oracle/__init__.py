"""FP64 CPU oracle for the fast-MUSIC hot path (test infrastructure only).

This package is the checker, not the product.  Only the test-suite, the
``__graft_entry__.smoke`` check and the benchmark's ``cpu_baseline`` leg may
import it; the HIP library never does, and it never imports the library.

The arithmetic lives in ``fm_oracle.c`` (plain C, double precision, loops
written from the paper's definitions); this module only marshals numpy
arrays through ctypes.  ``build()`` compiles the shared object with gcc.

Paper: Li, Wang, Zhang, Cao, Zhao, "Ultra-Fast Accurate AoA Estimation via
Automotive Massive-MIMO Radar", arXiv:1911.07434.
  - covariance          eqs. (2)-(3)
  - eigen-decomposition eq. (4)           (cyclic Jacobi)
  - MUSIC spectrum      eqs. (5), (10)
  - peaks               eq. (6)
  - Method 1            Alg. 1, eqs. (8)-(9), rank restriction of Sec. III-A
  - Method 2            Alg. 2, eq. (11)
  - ESPRIT on U_s      the conclusion's extension to other subspace
                        estimators (least-squares ESPRIT: a reading)
  - order of the model  Sec. V-D (AIC / MDL pre-estimation of K from the
                        sketch eigenvalues; completion of the unseen
                        eigenvalues from the trace is a reading)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

RCOND_DEFAULT = 1e-6


def build(force: bool = True) -> str:
    """Compile ``fm_oracle.c`` into ``liboracle.so`` (gcc -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-fcx-fortran-rules", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    lib.om_covariance.argtypes = [P, C.c_int, C.c_int, C.c_long, P, C.c_int]
    lib.om_covariance.restype = None
    lib.om_eigh.argtypes = [P, C.c_int, P, P]
    lib.om_eigh.restype = C.c_int
    lib.om_svd.argtypes = [P, C.c_int, C.c_int, P, P, P]
    lib.om_svd.restype = C.c_int
    lib.om_orth.argtypes = [P, C.c_int, C.c_int, P]
    lib.om_orth.restype = C.c_int
    lib.om_pinv_herm.argtypes = [P, C.c_int, C.c_double, P]
    lib.om_pinv_herm.restype = C.c_int
    lib.om_music_subspace.argtypes = [P, C.c_int, C.c_int, P, P]
    lib.om_music_subspace.restype = C.c_int
    lib.om_fast_music_sample.argtypes = [P, C.c_int, P, C.c_int, C.c_int, C.c_double, P, P]
    lib.om_fast_music_sample.restype = C.c_int
    lib.om_fast_music_project.argtypes = [P, C.c_int, P, C.c_int, C.c_int, C.c_int,
                                          C.c_double, P, P]
    lib.om_fast_music_project.restype = C.c_int
    lib.om_pseudospectrum.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double,
                                      C.c_int, P, P, C.c_int]
    lib.om_pseudospectrum.restype = None
    lib.om_peaks.argtypes = [P, C.c_int, C.c_int, P, P]
    lib.om_peaks.restype = C.c_int
    lib.om_order.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, P]
    lib.om_order.restype = C.c_int
    lib.om_eigvals.argtypes = [P, C.c_int, P]
    lib.om_eigvals.restype = C.c_int
    lib.om_esprit.argtypes = [P, C.c_int, C.c_int, P]
    lib.om_esprit.restype = C.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# --------------------------------------------------------------------------
# stage functions
# --------------------------------------------------------------------------

def covariance(X: np.ndarray, threads: int = 1) -> np.ndarray:
    """R = X X^H / T (eqs. (2)-(3)).  X: complex64 (M, T) -> complex128 (M, M)."""
    X = np.ascontiguousarray(X, dtype=np.complex64)
    M, T = X.shape
    R = np.zeros((M, M), np.complex128)
    _load().om_covariance(_p(X), M, T, T, _p(R), threads)
    return R


def eigh(A: np.ndarray):
    """Jacobi eigen-decomposition of a Hermitian matrix (eq. (4)).

    Returns (w descending, V with eigenvectors in columns, sweeps)."""
    A = _c128(A)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), np.complex128)
    sw = _load().om_eigh(_p(A), n, _p(w), _p(V))
    return w, V, sw


def svd(Cm: np.ndarray):
    """Thin SVD by one-sided Jacobi: C = U diag(s) V^H (m >= n)."""
    Cm = _c128(Cm)
    m, n = Cm.shape
    U = np.zeros((m, n), np.complex128)
    s = np.zeros(n)
    V = np.zeros((n, n), np.complex128)
    sw = _load().om_svd(_p(Cm), m, n, _p(U), _p(s), _p(V))
    return U, s, V, sw


def orth(Cm: np.ndarray):
    """Orthonormal basis (MGS, two passes) of the columns of C -> (Q[:, :r], r)."""
    Cm = _c128(Cm)
    m, n = Cm.shape
    Q = np.zeros((m, n), np.complex128)
    r = _load().om_orth(_p(Cm), m, n, _p(Q))
    return Q[:, :r], r


def pinv_herm(A: np.ndarray, rcond: float = RCOND_DEFAULT):
    """Eigen-based pseudo-inverse of a Hermitian PSD matrix -> (A^+, rank)."""
    A = _c128(A)
    n = A.shape[0]
    Ap = np.zeros((n, n), np.complex128)
    r = _load().om_pinv_herm(_p(A), n, rcond, _p(Ap))
    return Ap, r


def music_subspace(R: np.ndarray, K: int):
    """Standard MUSIC: K leading eigenvectors of R -> (Us [K][M], all eigenvalues)."""
    R = _c128(R)
    M = R.shape[0]
    Us = np.zeros((K, M), np.complex128)
    w = np.zeros(M)
    sw = _load().om_music_subspace(_p(R), M, K, _p(Us), _p(w))
    if sw < 0:
        raise RuntimeError("Jacobi eigensolver did not converge")
    return Us, w


def subspace_sample(R: np.ndarray, idx: np.ndarray, K: int, rcond: float = RCOND_DEFAULT):
    """Fast MUSIC Method 1 (Alg. 1) -> (Us [K][M], sigma[K], rank of W)."""
    R = _c128(R)
    M = R.shape[0]
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    p = idx.shape[0]
    Us = np.zeros((K, M), np.complex128)
    sig = np.zeros(K)
    r = _load().om_fast_music_sample(_p(R), M, _p(idx), p, K, rcond, _p(Us), _p(sig))
    return Us, sig, r


def subspace_project(R: np.ndarray, Omega: np.ndarray, q: int, K: int,
                     rcond: float = RCOND_DEFAULT):
    """Fast MUSIC Method 2 (Alg. 2) -> (Us [K][M], sigma[K], rank of W)."""
    R = _c128(R)
    M = R.shape[0]
    Omega = np.ascontiguousarray(Omega, dtype=np.float32)
    l = Omega.shape[1]
    Us = np.zeros((K, M), np.complex128)
    sig = np.zeros(K)
    r = _load().om_fast_music_project(_p(R), M, _p(Omega), l, q, K, rcond, _p(Us), _p(sig))
    return Us, sig, r


def pseudospectrum(Us: np.ndarray, theta0_deg: float, dtheta_deg: float, L: int,
                   threads: int = 1):
    """MUSIC pseudo-spectrum over theta0 + l*dtheta (eqs. (5), (10)) -> (P, den)."""
    Us = _c128(Us)
    K, M = Us.shape
    den = np.zeros(L)
    P = np.zeros(L)
    _load().om_pseudospectrum(_p(Us), M, K, theta0_deg, dtheta_deg, L, _p(den), _p(P),
                              threads)
    return P, den


def peaks(P: np.ndarray, K: int):
    """Peak picking (eq. (6)) -> (idx int32[n], val float64[n])."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    L = P.shape[0]
    idx = np.zeros(max(K, 1), np.int32)
    val = np.zeros(max(K, 1))
    n = _load().om_peaks(_p(P), L, K, _p(idx), _p(val))
    return idx[:n].copy(), val[:n].copy()


ORDER_AIC, ORDER_MDL = 0, 1


def order_criteria(sig, M: int, N: int, trR: float, kind: int, rcond: float = RCOND_DEFAULT):
    """AIC (kind 0) / MDL (kind 1) over the sketch eigenvalues (Sec. V-D)
    -> (K_hat, crit[n + 1]); crit is +inf where not evaluated."""
    sig = np.ascontiguousarray(sig, dtype=np.float64)
    n = sig.shape[0]
    crit = np.zeros(n + 1)
    k = _load().om_order(_p(sig), n, M, N, float(trR), rcond, kind, _p(crit))
    return k, crit


def order_estimate(R: np.ndarray, Omega: np.ndarray, q: int, N: int, kind: int,
                   rcond: float = RCOND_DEFAULT):
    """Pre-estimation of K (Sec. V-D): all l eigenvalues of the Method 2 sketch
    of R, the trace of R, then the criterion -> (K_hat, crit, sig)."""
    R = _c128(R)
    l = np.asarray(Omega).shape[1]
    _Us, sig, _ = subspace_project(R, Omega, q, l, rcond)
    trR = float(np.sum(np.real(np.diag(R))))
    k, crit = order_criteria(sig, R.shape[0], N, trR, kind, rcond)
    return k, crit, sig


def eigvals(A: np.ndarray):
    """Eigenvalues of a general complex matrix (Hessenberg + shifted QR) -> (w, steps)."""
    A = _c128(A)
    n = A.shape[0]
    w = np.zeros(n, np.complex128)
    st = _load().om_eigvals(_p(A), n, _p(w))
    return w, st


def esprit(Us: np.ndarray):
    """Least-squares ESPRIT on U_s [K][M] -> (angles in degrees ascending, steps)."""
    Us = _c128(Us)
    K, M = Us.shape
    doa = np.zeros(K)
    st = _load().om_esprit(_p(Us), M, K, _p(doa))
    return doa, st


# --------------------------------------------------------------------------
# whole pipelines
# --------------------------------------------------------------------------

def run_frame(X, K, variant, theta0_deg, dtheta_deg, L, *, Omega=None, q=2, idx=None,
              rcond=RCOND_DEFAULT, threads=1):
    """Covariance -> subspace (variant 'project' | 'sample' | 'music') -> spectrum -> peaks."""
    R = covariance(X, threads)
    if variant == "project":
        Us, sig, _ = subspace_project(R, Omega, q, K, rcond)
    elif variant == "sample":
        Us, sig, _ = subspace_sample(R, idx, K, rcond)
    elif variant == "music":
        Us, w = music_subspace(R, K)
        sig = w[:K]
    else:
        raise ValueError(variant)
    P, den = pseudospectrum(Us, theta0_deg, dtheta_deg, L, threads)
    pidx, pval = peaks(P, K)
    return dict(R=R, Us=Us, sigma=sig, P=P, den=den, peak_idx=pidx, peak_val=pval)
