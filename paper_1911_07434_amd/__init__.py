"""MI355X (gfx950) fast-MUSIC angle-of-arrival path -- Python binding.

Thin ctypes marshalling over the C ABI declared in ``include/fastmusic.h``
(libfastmusic.so, built in-tree by ``paper_1911_07434_amd.build``).  Every
stage runs in the library's HIP kernels; PyTorch is used only to own device
memory and to supply the current HIP stream.  There is no CPU fallback: if
the shared library is missing, every entry point raises.

Paper: Li, Wang, Zhang, Cao, Zhao, "Ultra-Fast Accurate AoA Estimation via
Automotive Massive-MIMO Radar", arXiv:1911.07434.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfastmusic.so")

FM_OK, FM_E_ARG, FM_E_HIP, FM_E_WORKSPACE, FM_E_UNSUPPORTED = 0, 1, 2, 3, 4
FM_FP32, FM_BF16, FM_FP16, FM_FP16X3, FM_BF16X3 = 0, 1, 2, 3, 4
FM_METHOD_PROJECT, FM_METHOD_SAMPLE, FM_METHOD_PROJECT_X, FM_METHOD_SAMPLE_X = 0, 1, 2, 3
FM_ST_NONFINITE, FM_ST_EIG_MAXIT, FM_ST_RANK_DEFICIENT, FM_ST_FEW_PEAKS, FM_ST_BAD_INDEX = (
    1, 4, 8, 16, 32)
FM_ST_ORTH_FALLBACK, FM_ST_ORDER_AT_LIMIT, FM_ST_CORE_TRUNCATED = 2, 64, 128
FM_ST_NOTES = FM_ST_ORTH_FALLBACK | FM_ST_CORE_TRUNCATED


def status_errors(status) -> int:
    """The status bits of a frame that are not FM_ST_NOTES (0: a clean result)."""
    return int(status) & ~FM_ST_NOTES
FM_ORDER_AIC, FM_ORDER_MDL = 0, 1
FM_RCOND_DEFAULT = 1e-6
FM_KNOB_COV_SCHEDULE, FM_KNOB_SPEC_ANGLES, FM_KNOB_SPEC16_ANGLES = 0, 1, 2
FM_NOALLOC_SCRATCH_BYTES = 16 << 20

# every symbol of include/fastmusic.h
EXPORTS = (
    "fm_create", "fm_destroy", "fm_status_string", "fm_last_error", "fm_workspace_bytes",
    "fm_covariance", "fm_subspace_sample", "fm_subspace_project", "fm_pseudospectrum",
    "fm_peaks", "fm_plan_create", "fm_plan_destroy", "fm_plan_workspace_bytes",
    "fm_plan_covariance", "fm_plan_subspace", "fm_plan_pseudospectrum", "fm_plan_peaks",
    "fm_plan_run", "fm_plan_bytes", "fm_plan_create_in", "fm_set_knob", "fm_get_knob",
    "fm_subspace_project_x", "fm_subspace_sample_x", "fm_order", "fm_esprit",
    "fm_subspace_project_noalloc",
)


class FmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fastmusic status {status}: {msg}")
        self.status = status


class fm_frame(C.Structure):
    """Mirror of the C struct fm_frame (one frame of a plan)."""
    _fields_ = [
        ("X", C.c_void_p), ("ldx", C.c_int64), ("M", C.c_int), ("T", C.c_int),
        ("R", C.c_void_p), ("ldr", C.c_int64),
        ("K", C.c_int), ("method", C.c_int), ("n", C.c_int), ("q", C.c_int),
        ("rcond", C.c_double),
        ("Omega", C.c_void_p), ("idx", C.c_void_p),
        ("Us", C.c_void_p), ("sigma", C.c_void_p), ("status", C.c_void_p),
        ("L", C.c_int), ("theta0_deg", C.c_double), ("dtheta_deg", C.c_double),
        ("P", C.c_void_p), ("peak_idx", C.c_void_p), ("peak_val", C.c_void_p),
        ("n_found", C.c_void_p),
        ("K_hat", C.c_void_p), ("order_crit", C.c_void_p), ("order_rule", C.c_int),
        ("esprit_deg", C.c_void_p),
        ("spec_prec", C.c_int),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfastmusic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_1911_07434_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(path)
    P, I, D, Z, I64 = C.c_void_p, C.c_int, C.c_double, C.c_size_t, C.c_int64
    sig = {
        "fm_create": ([I, Z, C.POINTER(P)], I),
        "fm_destroy": ([P], I),
        "fm_status_string": ([I], C.c_char_p),
        "fm_last_error": ([P], C.c_char_p),
        "fm_workspace_bytes": ([I, I, I, I], Z),
        "fm_covariance": ([P, P, P, I, I, I64, P, I64, I], I),
        "fm_subspace_sample": ([P, P, P, I, I64, P, I, I, D, P, P, P], I),
        "fm_subspace_project": ([P, P, P, I, I64, P, I, I, I, D, I, P, P, P], I),
        "fm_pseudospectrum": ([P, P, P, I, I, D, D, I, I, P], I),
        "fm_peaks": ([P, P, P, I, I, P, P, P], I),
        "fm_plan_create": ([P, C.POINTER(fm_frame), I, I, C.POINTER(P)], I),
        "fm_plan_destroy": ([P], I),
        "fm_plan_workspace_bytes": ([P], Z),
        "fm_plan_covariance": ([P, P], I),
        "fm_plan_subspace": ([P, P], I),
        "fm_plan_pseudospectrum": ([P, P], I),
        "fm_plan_peaks": ([P, P], I),
        "fm_plan_run": ([P, P, I], I),
        "fm_plan_bytes": ([P, C.POINTER(fm_frame), I, I], Z),
        "fm_plan_create_in": ([P, C.POINTER(fm_frame), I, I, P, Z, P, C.POINTER(P)], I),
        "fm_set_knob": ([P, I, I, I], I),
        "fm_subspace_project_x": ([P, P, P, I, I, I64, P, I, I, I, D, I, P, P, P], I),
        "fm_subspace_sample_x": ([P, P, P, I, I, I64, P, I, I, D, P, P, P], I),
        "fm_get_knob": ([P, I, I], I),
        "fm_order": ([P, P, P, I, I64, I, P, I, D, I, P, P, P], I),
        "fm_esprit": ([P, P, P, I, I, P, P], I),
        "fm_subspace_project_noalloc": ([P, P, P, I, I64, P, I, I, I, D, I, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int | None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """Owns an fm_ctx (device + arena).  Use one per host thread."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        self.lib = load_library()
        self.h = C.c_void_p()
        st = self.lib.fm_create(device, workspace_bytes, C.byref(self.h))
        if st != FM_OK:
            raise FmError(st, f"fm_create(device={device}) failed")
        self.device = device

    def close(self):
        if self.h:
            self.lib.fm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != FM_OK:
            raise FmError(st, self.lib.fm_last_error(self.h).decode())

    # -- tuning knobs ---------------------------------------------------------

    def set_knob(self, knob: int, bucket: int, value: int):
        self.check(self.lib.fm_set_knob(self.h, knob, bucket, value))

    def get_knob(self, knob: int, bucket: int) -> int:
        return self.lib.fm_get_knob(self.h, knob, bucket)

    # -- single-frame stages (device tensors in, device tensors out) --------

    def fm_covariance(self, X, R, prec=FM_FP32, stream=None):
        M, T = X.shape
        self.check(self.lib.fm_covariance(self.h, _stream(stream), _ptr(X), M, T, X.stride(0),
                                          _ptr(R), R.stride(0), prec))
        return R

    def fm_subspace_sample(self, R, idx, K, Us, sigma, status, rcond=FM_RCOND_DEFAULT,
                           stream=None):
        M = R.shape[0]
        self.check(self.lib.fm_subspace_sample(self.h, _stream(stream), _ptr(R), M, R.stride(0),
                                               _ptr(idx), idx.shape[0], K, rcond, _ptr(Us),
                                               _ptr(sigma), _ptr(status)))

    def fm_subspace_project(self, R, Omega, q, K, Us, sigma, status, rcond=FM_RCOND_DEFAULT,
                            prec=FM_FP32, stream=None):
        M = R.shape[0]
        self.check(self.lib.fm_subspace_project(self.h, _stream(stream), _ptr(R), M,
                                                R.stride(0), _ptr(Omega), Omega.shape[1], q, K,
                                                rcond, prec, _ptr(Us), _ptr(sigma),
                                                _ptr(status)))

    def fm_subspace_project_noalloc(self, R, Omega, q, K, Us, sigma, status,
                                    rcond=FM_RCOND_DEFAULT, prec=FM_FP32, stream=None):
        """fm_subspace_project with the library's fixed device scratch array as
        its workspace: allocates nothing (FM_NOALLOC_SCRATCH_BYTES at most)."""
        M = R.shape[0]
        self.check(self.lib.fm_subspace_project_noalloc(
            self.h, _stream(stream), _ptr(R), M, R.stride(0), _ptr(Omega), Omega.shape[1], q, K,
            rcond, prec, _ptr(Us), _ptr(sigma), _ptr(status)))

    def fm_subspace_project_x(self, X, Omega, q, K, Us, sigma, status, rcond=FM_RCOND_DEFAULT,
                              prec=FM_FP32, stream=None):
        M, T = X.shape
        self.check(self.lib.fm_subspace_project_x(self.h, _stream(stream), _ptr(X), M, T,
                                                  X.stride(0), _ptr(Omega), Omega.shape[1], q,
                                                  K, rcond, prec, _ptr(Us), _ptr(sigma),
                                                  _ptr(status)))

    def fm_subspace_sample_x(self, X, idx, K, Us, sigma, status, rcond=FM_RCOND_DEFAULT,
                             stream=None):
        M, T = X.shape
        self.check(self.lib.fm_subspace_sample_x(self.h, _stream(stream), _ptr(X), M, T,
                                                 X.stride(0), _ptr(idx), idx.shape[0], K, rcond,
                                                 _ptr(Us), _ptr(sigma), _ptr(status)))

    def fm_order(self, R, T, eig, K_hat, status, rule=FM_ORDER_MDL, crit=None,
                 rcond=FM_RCOND_DEFAULT, stream=None):
        M = R.shape[0]
        self.check(self.lib.fm_order(self.h, _stream(stream), _ptr(R), M, R.stride(0), T,
                                     _ptr(eig), eig.shape[0], rcond, rule, _ptr(K_hat),
                                     _ptr(crit), _ptr(status)))

    def fm_esprit(self, Us, doa, status, stream=None):
        K, M = Us.shape
        self.check(self.lib.fm_esprit(self.h, _stream(stream), _ptr(Us), M, K, _ptr(doa),
                                      _ptr(status)))

    def fm_pseudospectrum(self, Us, theta0_deg, dtheta_deg, L, P, prec=FM_FP32, stream=None):
        K, M = Us.shape
        self.check(self.lib.fm_pseudospectrum(self.h, _stream(stream), _ptr(Us), M, K,
                                              float(theta0_deg), float(dtheta_deg), L, prec,
                                              _ptr(P)))

    def fm_peaks(self, P, K, idx, val, n_found, stream=None):
        self.check(self.lib.fm_peaks(self.h, _stream(stream), _ptr(P), P.shape[0], K,
                                     _ptr(idx), _ptr(val), _ptr(n_found)))


def plan_bytes(ctx: Context, frames: list[fm_frame], prec=FM_FP32) -> int:
    arr = (fm_frame * len(frames))(*frames)
    return int(ctx.lib.fm_plan_bytes(ctx.h, arr, len(frames), prec))


class Plan:
    """A batch of frames (fm_frame list) run through one launch per stage.

    With dev_mem (a device pointer) and dev_bytes the plan lives in that
    caller-owned block and is uploaded asynchronously on `stream`
    (fm_plan_create_in); otherwise it allocates (fm_plan_create)."""

    def __init__(self, ctx: Context, frames: list[fm_frame], prec=FM_FP32, dev_mem=None,
                 dev_bytes=0, stream=None):
        self.ctx = ctx
        self.frames = (fm_frame * len(frames))(*frames)
        self.h = C.c_void_p()
        if dev_mem is None:
            ctx.check(ctx.lib.fm_plan_create(ctx.h, self.frames, len(frames), prec,
                                             C.byref(self.h)))
        else:
            ctx.check(ctx.lib.fm_plan_create_in(ctx.h, self.frames, len(frames), prec, dev_mem,
                                                dev_bytes, _stream(stream), C.byref(self.h)))

    def close(self):
        if self.h:
            self.ctx.lib.fm_plan_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        return self.ctx.lib.fm_plan_workspace_bytes(self.h)

    def covariance(self, stream=None):
        self.ctx.check(self.ctx.lib.fm_plan_covariance(self.h, _stream(stream)))

    def subspace(self, stream=None):
        self.ctx.check(self.ctx.lib.fm_plan_subspace(self.h, _stream(stream)))

    def pseudospectrum(self, stream=None):
        self.ctx.check(self.ctx.lib.fm_plan_pseudospectrum(self.h, _stream(stream)))

    def peaks(self, stream=None):
        self.ctx.check(self.ctx.lib.fm_plan_peaks(self.h, _stream(stream)))

    def run(self, use_graph: bool = False, stream=None):
        self.ctx.check(self.ctx.lib.fm_plan_run(self.h, _stream(stream), int(use_graph)))
