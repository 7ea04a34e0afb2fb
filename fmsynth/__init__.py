"""Seeded synthetic radar frames (inputs only -- no estimation arithmetic).

This module generates the inputs that both the HIP library and the FP64 oracle
consume: snapshot matrices X of a half-wavelength uniform linear array, the
Gaussian test matrices Omega of the projection variant and the column index
sets of the sampling variant.  It holds none of the estimator's arithmetic
(no covariance, subspace, spectrum or peak code), so the two sides under
test share nothing but these arrays.

Signal model (the paper's Sec. II-A, with its experiments starting directly
from the snapshot matrix, Sec. V-A):
  x_m(t) = sum_k a_m(theta_k) s_k(t) + n_m(t),   m = 0..M-1, t = 0..T-1
  a_m(theta) = exp(-j pi m sin(theta))            (d = lambda/2)
  s_k(t) ~ CN(0, 1) i.i.d. (unit-power sources)
  n_m(t) ~ CN(0, sigma^2), sigma^2 = 10^(-SNR/10)  (SNR per source per element)
X is rounded to complex64 once; everything downstream sees those bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Frame:
    X: np.ndarray            # complex64 (M, T)
    thetas_deg: np.ndarray   # float64 (K,) true angles
    snr_db: float
    seed: int
    M: int = field(init=False)
    T: int = field(init=False)
    K: int = field(init=False)

    def __post_init__(self):
        self.M, self.T = self.X.shape
        self.K = int(self.thetas_deg.shape[0])


def _rng(seed: int, stream: int) -> np.random.Generator:
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, int(stream)])
    return np.random.Generator(np.random.PCG64(ss))


def draw_angles(rng: np.random.Generator, K: int, lo: float, hi: float,
                min_sep: float, max_tries: int = 100000) -> np.ndarray:
    """K angles uniform in [lo, hi] (degrees) with pairwise separation >= min_sep."""
    for _ in range(max_tries):
        th = np.sort(rng.uniform(lo, hi, size=K))
        if K < 2 or np.min(np.diff(th)) >= min_sep:
            return th
    raise RuntimeError("could not place the requested angles")


def draw_pairs(rng: np.random.Generator, n_pairs: int, spacing: float, lo: float,
               hi: float, min_center_sep: float) -> np.ndarray:
    """n_pairs pairs (c, c + spacing) with centres uniform in [lo, hi - spacing]."""
    c = draw_angles(rng, n_pairs, lo, hi - spacing, min_center_sep)
    return np.sort(np.concatenate([c, c + spacing]))


def steering_matrix(M: int, thetas_deg: np.ndarray) -> np.ndarray:
    """A[m, k] = exp(-j pi m sin(theta_k)), float64 phases -> complex128 (M, K)."""
    s = np.sin(np.deg2rad(np.asarray(thetas_deg, np.float64)))
    ph = np.outer(np.arange(M, dtype=np.float64), s)
    ph = np.mod(ph, 2.0)
    return np.exp(-1j * np.pi * ph)


def make_frame(M: int, T: int, K: int, snr_db: float, seed: int, *,
               angle_range=(-75.0, 75.0), min_sep: float = 1.0,
               thetas_deg=None, noiseless: bool = False, pairs: float | None = None,
               pair_center_sep: float = 2.0) -> Frame:
    """One synthetic frame.  thetas_deg overrides the random angles."""
    rng = _rng(seed, 0)
    if thetas_deg is not None:
        th = np.asarray(thetas_deg, np.float64)
    elif pairs is not None:
        th = draw_pairs(rng, K // 2, pairs, angle_range[0], angle_range[1], pair_center_sep)
    else:
        th = draw_angles(rng, K, angle_range[0], angle_range[1], min_sep)
    K = th.shape[0]
    A = steering_matrix(M, th)
    S = (rng.standard_normal((K, T)) + 1j * rng.standard_normal((K, T))) / np.sqrt(2.0)
    X = A @ S
    if not noiseless:
        sig = np.sqrt(10.0 ** (-snr_db / 10.0))
        nz = rng.standard_normal((M, 2 * T), dtype=np.float32).view(np.complex64)
        X = X + (sig / np.sqrt(2.0)) * nz
    return Frame(X=np.ascontiguousarray(X.astype(np.complex64)), thetas_deg=th,
                 snr_db=float(snr_db), seed=int(seed))


def make_integer_frame(M: int, T: int, seed: int, bound: int = 8) -> np.ndarray:
    """complex64 (M, T) with integer re/im in [-bound, bound] (exact in FP16/BF16/FP32)."""
    rng = _rng(seed, 3)
    re = rng.integers(-bound, bound + 1, size=(M, T))
    im = rng.integers(-bound, bound + 1, size=(M, T))
    return np.ascontiguousarray((re + 1j * im).astype(np.complex64))


def make_omega(M: int, l: int, seed: int) -> np.ndarray:
    """Real Gaussian test matrix Omega ~ N(0, 1), float32 (M, l)  (Alg. 2 step 1)."""
    return np.ascontiguousarray(_rng(seed, 1).standard_normal((M, l), dtype=np.float32))


def make_idx(M: int, p: int, seed: int) -> np.ndarray:
    """p distinct column indices drawn uniformly from {0..M-1}, int32 (Alg. 1 step 1)."""
    return np.ascontiguousarray(_rng(seed, 2).choice(M, size=p, replace=False).astype(np.int32))


def grid(L: int, theta0_deg: float = -90.0, span_deg: float = 180.0):
    """Uniform grid theta_l = theta0 + l * dtheta over [theta0, theta0 + span]."""
    return theta0_deg, span_deg / (L - 1), L


# --------------------------------------------------------------------------
# workload configurations (shapes of the paper's simulations, scaled up)
# --------------------------------------------------------------------------

def sketch_sizes(M: int, K: int, l_cap: int = 40):
    """l = K + 8 (<= l_cap, <= M) and p = min(4 l, M)."""
    l = min(K + 8, l_cap, M)
    p = min(4 * l, M)
    return l, p


CONFIGS = {
    # plain MUSIC single frame, M=64, T=128, K=3, SNR 10 dB, 0.1 deg grid
    "c1": dict(M=64, T=128, K=3, snr_db=10.0, angle_range=(-60.0, 60.0), min_sep=5.0,
               L=1801, l=11, p=44, q=2),
    # massive-MIMO single frame, M=1024, T=2048, K=8, SNR 0 dB, 0.01 deg grid
    "c2": dict(M=1024, T=2048, K=8, snr_db=0.0, angle_range=(-75.0, 75.0), min_sep=1.0,
               L=18001, l=16, p=64, q=2),
    # mixed precision, M=4096, T=8192, K=16 as pairs 0.5 deg apart, 0.005 deg grid
    "c4": dict(M=4096, T=8192, K=16, snr_db=0.0, angle_range=(-75.0, 75.0), min_sep=2.0,
               L=36001, l=24, p=96, q=2, pairs=0.5),
}


def config_frame(name: str, seed: int, **over) -> tuple[Frame, dict]:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    fr = make_frame(cfg["M"], cfg["T"], cfg["K"], cfg["snr_db"], seed,
                    angle_range=cfg["angle_range"], min_sep=cfg["min_sep"],
                    pairs=cfg.get("pairs"))
    return fr, cfg


def uneven_batch(n: int, seed: int, Ms=(256, 512, 1024, 2048), K_range=(1, 16),
                 snr_range=(-5.0, 20.0), T_rel=(0.5, 2.0)):
    """Frame shapes of the uneven-batch workload: M from Ms, T ~ U[M/2, 2M],
    K ~ U[K_range], SNR ~ U[snr_range].  Returns a list of dicts (no data)."""
    rng = _rng(seed, 4)
    out = []
    for i in range(n):
        M = int(rng.choice(Ms))
        T = int(rng.integers(int(M * T_rel[0]), int(M * T_rel[1]) + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        snr = float(rng.uniform(*snr_range))
        l, p = sketch_sizes(M, K)
        out.append(dict(M=M, T=T, K=K, snr_db=snr, l=l, p=p, q=2, seed=seed * 100003 + i))
    return out


def make_batch_device(M: int, T: int, K: int, snr_db: float, n: int, seed: int, *,
                      angle_range=(-75.0, 75.0), min_sep: float = 1.0, device="cuda",
                      pairs: float | None = None, pair_center_sep: float = 2.0):
    """n frames of the same shape generated on the GPU (for throughput runs).

    Same signal model as make_frame (angles drawn on the host with the same
    rule -- pairs `pairs` degrees apart when given -- sources and noise drawn
    with a seeded torch generator on the device).  Returns (X complex64
    (n, M, T) on the device, angles (n, K)).
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    rng = _rng(seed, 5)
    if pairs is not None:
        th = np.stack([draw_pairs(rng, K // 2, pairs, angle_range[0], angle_range[1],
                                  pair_center_sep) for _ in range(n)])
    else:
        th = np.stack([draw_angles(rng, K, angle_range[0], angle_range[1], min_sep)
                       for _ in range(n)])
    A = torch.from_numpy(np.stack([steering_matrix(M, t) for t in th]).astype(np.complex64))
    A = A.to(device)                                           # (n, M, K)
    S = torch.complex(torch.randn((n, K, T), generator=g, device=device),
                      torch.randn((n, K, T), generator=g, device=device)) / np.sqrt(2.0)
    X = torch.bmm(A.contiguous(), S.contiguous())
    sig = float(np.sqrt(10.0 ** (-snr_db / 10.0) / 2.0))
    X += sig * torch.complex(torch.randn((n, M, T), generator=g, device=device),
                             torch.randn((n, M, T), generator=g, device=device))
    return X.contiguous(), th


def make_omega_device(M: int, l: int, n: int, seed: int, device="cuda"):
    """n real Gaussian test matrices (n, M, l) float32 on the device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + 7777)
    return torch.randn((n, M, l), generator=g, device=device, dtype=torch.float32)
