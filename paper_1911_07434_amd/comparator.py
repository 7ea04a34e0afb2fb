"""Standard MUSIC on the same GPU: the comparator of the fast methods.

Eq. (4)'s full eigendecomposition of R replaces the randomized subspace:
R = X X^H / T from the library's covariance kernel, every eigenpair of R
from torch.linalg.eigh (rocSOLVER, complex64), the K leading eigenvectors as
U_s, then the library's pseudo-spectrum and peak kernels (eqs. (5)-(6)).
This is the O(M^3) route the paper's methods avoid; it is timed beside them
and checked against the FP64 oracle's standard MUSIC.
"""
from __future__ import annotations


def plain_music_batch(ctx, frames, K, theta0_deg, dtheta_deg, L, stream=None):
    """Run standard MUSIC on `frames` (DeviceFrame objects of equal M, with
    their X filled); writes each frame's P, peak_idx, peak_val and n_found.
    The eigen-solve of all frames is one batched call."""
    import torch
    M = frames[0].spec.M
    Rs = torch.empty((len(frames), M, M), dtype=torch.complex64, device=frames[0].X.device)
    for i, d in enumerate(frames):
        ctx.fm_covariance(d.X, Rs[i], stream=stream)
    _w, V = torch.linalg.eigh(Rs)                    # ascending eigenvalues
    Us = V[:, :, M - K:].flip(-1).transpose(1, 2).to(torch.complex128).contiguous()
    for i, d in enumerate(frames):
        ctx.fm_pseudospectrum(Us[i], theta0_deg, dtheta_deg, L, d.P, stream=stream)
        ctx.fm_peaks(d.P, K, d.peak_idx, d.peak_val, d.n_found, stream=stream)
