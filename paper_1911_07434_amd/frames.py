"""Device buffers of one frame and its fm_frame descriptor.

A DeviceFrame owns (as torch tensors on the GPU) the inputs, outputs and
randomness of one frame and builds the fm_frame record a Plan consumes.  It
does no arithmetic of its own.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import (FM_FP32, FM_METHOD_PROJECT, FM_METHOD_PROJECT_X, FM_METHOD_SAMPLE,
               FM_METHOD_SAMPLE_X, FM_RCOND_DEFAULT, fm_frame)

SAMPLE_METHODS = (FM_METHOD_SAMPLE, FM_METHOD_SAMPLE_X)


@dataclass
class FrameSpec:
    M: int
    T: int
    K: int
    method: int = FM_METHOD_PROJECT
    n: int = 16            # l (Method 2) or p (Method 1)
    q: int = 2
    L: int = 18001
    theta0_deg: float = -90.0
    dtheta_deg: float = 0.01
    rcond: float = FM_RCOND_DEFAULT
    order_rule: int | None = None  # FM_ORDER_AIC / FM_ORDER_MDL: also estimate K (Sec. V-D)
    esprit: bool = False           # also the ESPRIT angles of U_s (K <= 32)
    spec_prec: int = 0             # FM_FP32: polynomial pass; FM_FP16: split hi+lo projection


class DeviceFrame:
    def __init__(self, spec: FrameSpec, X=None, rnd=None, device="cuda"):
        import torch
        s = spec
        self.spec = s
        dev = torch.device(device)
        self.X = (torch.as_tensor(X).to(dev) if X is not None
                  else torch.empty((s.M, s.T), dtype=torch.complex64, device=dev))
        self.R = torch.empty((s.M, s.M), dtype=torch.complex64, device=dev)
        if s.method not in SAMPLE_METHODS:
            self.Omega = (torch.as_tensor(rnd).to(dev) if rnd is not None
                          else torch.empty((s.M, s.n), dtype=torch.float32, device=dev))
            self.idx = None
        else:
            self.idx = (torch.as_tensor(np.asarray(rnd, np.int32)).to(dev) if rnd is not None
                        else torch.empty((s.n,), dtype=torch.int32, device=dev))
            self.Omega = None
        self.Us = torch.zeros((s.K, s.M), dtype=torch.complex128, device=dev)
        self.sigma = torch.zeros((s.K,), dtype=torch.float64, device=dev)
        self.status = torch.zeros((1,), dtype=torch.int32, device=dev)
        self.P = torch.zeros((s.L,), dtype=torch.float32, device=dev)
        self.peak_idx = torch.zeros((s.K,), dtype=torch.int32, device=dev)
        self.peak_val = torch.zeros((s.K,), dtype=torch.float32, device=dev)
        self.n_found = torch.zeros((1,), dtype=torch.int32, device=dev)
        if s.order_rule is not None:
            self.K_hat = torch.full((1,), -1, dtype=torch.int32, device=dev)
            self.order_crit = torch.zeros((s.n + 1,), dtype=torch.float64, device=dev)
        else:
            self.K_hat = self.order_crit = None
        self.doa = (torch.zeros((s.K,), dtype=torch.float64, device=dev) if s.esprit
                    else None)

    def descriptor(self) -> fm_frame:
        s = self.spec
        f = fm_frame()
        f.X = self.X.data_ptr()
        f.ldx = self.X.stride(0)
        f.M, f.T = s.M, s.T
        f.R = self.R.data_ptr()
        f.ldr = self.R.stride(0)
        f.K, f.method, f.n, f.q = s.K, s.method, s.n, s.q
        f.rcond = s.rcond
        f.Omega = self.Omega.data_ptr() if self.Omega is not None else None
        f.idx = self.idx.data_ptr() if self.idx is not None else None
        f.Us = self.Us.data_ptr()
        f.sigma = self.sigma.data_ptr()
        f.status = self.status.data_ptr()
        f.L = s.L
        f.theta0_deg, f.dtheta_deg = s.theta0_deg, s.dtheta_deg
        f.P = self.P.data_ptr()
        f.peak_idx = self.peak_idx.data_ptr()
        f.peak_val = self.peak_val.data_ptr()
        f.n_found = self.n_found.data_ptr()
        if s.order_rule is not None:
            f.K_hat = self.K_hat.data_ptr()
            f.order_crit = self.order_crit.data_ptr()
            f.order_rule = s.order_rule
        if self.doa is not None:
            f.esprit_deg = self.doa.data_ptr()
        f.spec_prec = s.spec_prec
        return f

    def results(self) -> dict:
        """Copy the outputs back to host numpy arrays."""
        nf = int(self.n_found.cpu()[0])
        out = dict(R=self.R.cpu().numpy(), Us=self.Us.cpu().numpy(),
                   sigma=self.sigma.cpu().numpy(), status=int(self.status.cpu()[0]),
                   P=self.P.cpu().numpy(), peak_idx=self.peak_idx.cpu().numpy()[:nf],
                   peak_val=self.peak_val.cpu().numpy()[:nf], n_found=nf)
        if self.K_hat is not None:
            out["K_hat"] = int(self.K_hat.cpu()[0])
            out["order_crit"] = self.order_crit.cpu().numpy()
        if self.doa is not None:
            out["doa"] = self.doa.cpu().numpy()
        return out


def run_single(ctx, fr: DeviceFrame, prec=0, stream=None):
    """All four stages of one frame through the single-frame entry points, as
    a plan at precision `prec` runs them: the covariance and the Method 2
    sketch at `prec`, Method 1 and Method 2 from X (no covariance) in FP32,
    the spectrum at the frame's spec_prec (FP32: the polynomial pass)."""
    s = fr.spec
    if s.method == FM_METHOD_PROJECT_X:
        # Method 2 from the snapshots: no covariance (FP32 products)
        ctx.fm_subspace_project_x(fr.X, fr.Omega, s.q, s.K, fr.Us, fr.sigma, fr.status, s.rcond,
                                  FM_FP32, stream)
    elif s.method == FM_METHOD_SAMPLE_X:
        ctx.fm_subspace_sample_x(fr.X, fr.idx, s.K, fr.Us, fr.sigma, fr.status, s.rcond, stream)
    else:
        ctx.fm_covariance(fr.X, fr.R, prec, stream)
    if s.method == FM_METHOD_PROJECT:
        ctx.fm_subspace_project(fr.R, fr.Omega, s.q, s.K, fr.Us, fr.sigma, fr.status, s.rcond,
                                prec, stream)
    elif s.method == FM_METHOD_SAMPLE:
        ctx.fm_subspace_sample(fr.R, fr.idx, s.K, fr.Us, fr.sigma, fr.status, s.rcond, stream)
    ctx.fm_pseudospectrum(fr.Us, s.theta0_deg, s.dtheta_deg, s.L, fr.P, s.spec_prec, stream)
    ctx.fm_peaks(fr.P, s.K, fr.peak_idx, fr.peak_val, fr.n_found, stream)


def sampling_length(K_hat: int, M: int, factor: float = 1.2) -> int:
    """Method 1's sampling length from an estimated number of sources: the
    over-estimate p = ceil(1.2 K_hat) of Sec. V-D (Fig. 6), at least 1, at
    most M."""
    import math
    return max(1, min(M, math.ceil(factor * K_hat - 1e-9)))


def estimate_order_single(ctx, fr: DeviceFrame, rule: int, prec=FM_FP32, stream=None):
    """Model order of one frame through the single-frame entry points (the
    pre-estimation of Sec. V-D): covariance, the frame's sketch with every
    direction kept (its K must equal n, so sigma holds all n eigenvalues),
    then fm_order.  Writes fr.K_hat (and fr.order_crit)."""
    import torch
    s = fr.spec
    if s.K != s.n:
        raise ValueError("order estimate needs the sketch with every direction kept (K == n)")
    if fr.K_hat is None:
        fr.K_hat = torch.full((1,), -1, dtype=torch.int32, device=fr.X.device)
        fr.order_crit = torch.zeros((s.n + 1,), dtype=torch.float64, device=fr.X.device)
    ctx.fm_covariance(fr.X, fr.R, prec, stream)
    if s.method == FM_METHOD_PROJECT:
        ctx.fm_subspace_project(fr.R, fr.Omega, s.q, s.K, fr.Us, fr.sigma, fr.status, s.rcond,
                                prec, stream)
    elif s.method == FM_METHOD_SAMPLE:
        ctx.fm_subspace_sample(fr.R, fr.idx, s.K, fr.Us, fr.sigma, fr.status, s.rcond, stream)
    else:
        raise ValueError("order estimate needs R (Method 1 or 2 on R)")
    ord_status = torch.zeros((1,), dtype=torch.int32, device=fr.X.device)
    ctx.fm_order(fr.R, s.T, fr.sigma, fr.K_hat, ord_status,
                 rule if rule is not None else s.order_rule, fr.order_crit, s.rcond, stream)
    return ord_status
