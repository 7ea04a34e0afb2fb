"""Large-array mixed precision against the FP64 oracle, per SNR.

M = 4096 channels, T = 8192 snapshots, K = 16 sources as eight pairs 0.5 deg
apart, SNR in {-10, 0, 10, 30} dB, Method 2 with l = 24, q = 2, and a
36001-angle grid at 0.005 deg.  The covariance runs with FP32, FP16 and
BF16 operands (FP32 accumulation), and with split FP16 / BF16 hi + lo
operands; the oracle runs the whole pipeline in
FP64 on the same complex64 snapshots and Gaussian test matrix.  The error
of every path is printed per SNR.
"""
import numpy as np
import pytest

import fmsynth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_07434_amd as fm  # noqa: E402
from paper_1911_07434_amd.frames import DeviceFrame, FrameSpec  # noqa: E402

M, T, K, L_SK, Q, L = 4096, 8192, 16, 24, 2, 36001
# FP32 path 1e-3 dB, mixed paths 1e-2 dB.  BF16 operands (8-bit mantissa)
# meet the mixed budget up to 10 dB; at 30 dB the peak-region denominators
# are so small that BF16 rounding of the snapshots moves them by ~0.015 dB
# (measured on an MI355X): that one cell is a strict expected failure below
# (its status and AoA checks still run in the per-SNR test).  The split
# precisions (hi + lo halves, three 16-bit products) carry FP32-level error
# and are held to the FP32 bar at every SNR.
# "+spec16": the same covariance precision with the split hi + lo FP16
# steering projection as the spectrum pass (fm_frame.spec_prec = FM_FP16)
BARS_DB = {"fp32": 1e-3, "fp16": 1e-2, "bf16": 1e-2, "fp16x3": 1e-3, "bf16x3": 1e-3,
           "fp32+spec16": 1e-3, "fp16+spec16": 1e-2}
PRECS = (("fp32", fm.FM_FP32), ("fp16", fm.FM_FP16), ("bf16", fm.FM_BF16),
         ("fp16x3", fm.FM_FP16X3), ("bf16x3", fm.FM_BF16X3),
         ("fp32+spec16", fm.FM_FP32), ("fp16+spec16", fm.FM_FP16))
# the dB bar of this cell is asserted in its own strict-xfail test
KNOWN_OVER_BAR = {("bf16", 30.0)}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0, 256 << 20)
    yield c
    c.close()


_cache = {}


def _run_snr(ctx, snr):
    """GPU results at every precision and the oracle's, for one SNR (cached)."""
    if snr in _cache:
        return _cache[snr]
    seed = 4000 + int(snr)
    fr = fmsynth.make_frame(M, T, K, snr, seed, angle_range=(-75.0, 75.0), pairs=0.5,
                            pair_center_sep=2.0)
    Om = fmsynth.make_omega(M, L_SK, seed)
    th0, dth, _ = fmsynth.grid(L)
    X = torch.from_numpy(fr.X).cuda()
    Omd = torch.from_numpy(Om).cuda()
    got = {}
    for name, prec in PRECS:
        spec = FrameSpec(M=M, T=T, K=K, method=fm.FM_METHOD_PROJECT, n=L_SK, q=Q, L=L,
                         theta0_deg=th0, dtheta_deg=dth,
                         spec_prec=fm.FM_FP16 if name.endswith("+spec16") else fm.FM_FP32)
        d = DeviceFrame(spec, X=X, rnd=Omd)
        plan = fm.Plan(ctx, [d.descriptor()], prec=prec)
        plan.run()
        torch.cuda.synchronize()
        plan.close()
        r = d.results()
        got[name] = {k: r[k] for k in ("P", "status", "peak_idx")}
        del d, r
    thr = oracle.default_threads()
    R = oracle.covariance(fr.X, threads=thr)
    Us, sig, _ = oracle.subspace_project(R, Om, Q, K)
    del R
    Po, _ = oracle.pseudospectrum(Us, th0, dth, L, threads=thr)
    pi_o, _ = oracle.peaks(Po, K)
    errs = {}
    for name, g in got.items():
        errs[name] = float(np.max(np.abs(10 * np.log10(g["P"].astype(np.float64) / Po))))
        near = all(np.min(np.abs(g["peak_idx"] - p)) <= 1 for p in pi_o)
        print(f"config4 SNR {snr:+.0f} dB {name}: max |dP| = {errs[name]:.3g} dB, "
              f"peaks within one step: {near}, status {g['status']}", flush=True)
    _cache[snr] = (got, errs, pi_o)
    return _cache[snr]


@pytest.mark.parametrize("snr", [-10.0, 0.0, 10.0, 30.0])
def test_config4_mixed_precision_per_snr(ctx, snr):
    got, errs, pi_o = _run_snr(ctx, snr)
    for name, bar in BARS_DB.items():
        assert fm.status_errors(got[name]["status"]) == 0, name
        if (name, snr) not in KNOWN_OVER_BAR:
            assert errs[name] <= bar, (name, errs[name])
        for p in pi_o:
            assert np.min(np.abs(got[name]["peak_idx"] - p)) <= 1, name


@pytest.mark.xfail(strict=True, reason="BF16 rounding of the snapshots: about 1.5e-2 dB at "
                                       "30 dB SNR, over the 1e-2 dB mixed-path bar")
def test_config4_bf16_30db_mixed_bar(ctx):
    _got, errs, _pi = _run_snr(ctx, 30.0)
    assert errs["bf16"] <= BARS_DB["bf16"]
