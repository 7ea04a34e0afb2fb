"""ESPRIT on the fast subspace (least-squares ESPRIT on U_s) on the GPU,
through the C ABI, against the oracle:

* on identical U_s bits (the oracle's FP64 subspaces, K = 1..32, ragged M):
  angles within 1e-9 degrees of the oracle's ESPRIT;
* end to end from the snapshots (GPU Method 2 subspace, then ESPRIT) against
  the oracle's Method 2 + ESPRIT on the same X: within 1e-4 degrees, and at
  high SNR within 0.05 degrees of the true angles;
* the angles formed inside a plan (per frame at the end of the subspace
  stage) are bit-identical to fm_esprit on the plan's own U_s;
* invalid arguments are rejected (K > 32 unsupported).
"""
import numpy as np
import pytest

import fmsynth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_07434_amd as fm  # noqa: E402
from paper_1911_07434_amd.frames import DeviceFrame, FrameSpec  # noqa: E402


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0, 64 << 20)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def _gpu_esprit(ctx, Us):
    Ud = torch.from_numpy(np.ascontiguousarray(Us)).cuda()
    K = Us.shape[0]
    doa = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.fm_esprit(Ud, doa, st)
    torch.cuda.synchronize()
    return doa.cpu().numpy(), int(st.cpu()[0])


@pytest.mark.parametrize("M,T,K,snr", [(64, 128, 1, 10.0), (97, 200, 3, 5.0), (200, 400, 10, 0.0),
                                       (256, 512, 16, 5.0), (130, 300, 32, 15.0),
                                       (1024, 2048, 8, 0.0)])
def test_esprit_identical_subspace(ctx, M, T, K, snr):
    # many sources: an evenly spread set (random placement with a minimum
    # separation would rarely succeed)
    th = np.linspace(-62.0, 62.0, K) + 0.37 if K >= 16 else None
    fr = fmsynth.make_frame(M, T, K, snr, seed=M + K, angle_range=(-60, 60), min_sep=2.0,
                            thetas_deg=th)
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    # an FP64 subspace from the oracle (Method 2, l = K + 8) is the common input
    Us, _s, _ = oracle.subspace_project(R, fmsynth.make_omega(M, min(M, K + 8), M), 2, K)
    ref, st_o = oracle.esprit(Us)
    got, st = _gpu_esprit(ctx, Us)
    d = float(np.max(np.abs(got - ref)))
    say(f"ESPRIT M={M} K={K}: max |d| {d:.3g} deg (oracle QR steps {st_o})")
    assert st == 0 and st_o >= 0
    assert d <= 1e-9


@pytest.mark.parametrize("M,T,K,snr,l", [(200, 400, 6, 20.0, 12), (1024, 2048, 8, 10.0, 16)])
def test_esprit_end_to_end(ctx, M, T, K, snr, l):
    fr = fmsynth.make_frame(M, T, K, snr, seed=7 * M + K, angle_range=(-60, 60), min_sep=3.0)
    Om = fmsynth.make_omega(M, l, M + l)
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(torch.from_numpy(fr.X).cuda(), R)
    ctx.fm_subspace_project(R, torch.from_numpy(Om).cuda(), 2, K, Us, sig, st)
    doa = torch.zeros(K, dtype=torch.float64, device="cuda")
    est = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.fm_esprit(Us, doa, est)
    torch.cuda.synchronize()
    got = doa.cpu().numpy()
    Ro = oracle.covariance(fr.X, threads=oracle.default_threads())
    Uo, _so, _ = oracle.subspace_project(Ro, Om, 2, K)
    ref, _ = oracle.esprit(Uo)
    d = float(np.max(np.abs(got - ref)))
    e = float(np.max(np.abs(got - np.sort(fr.thetas_deg))))
    say(f"ESPRIT end to end M={M} K={K}: vs oracle {d:.3g} deg, vs truth {e:.3g} deg")
    assert int(est.cpu()[0]) == 0
    assert d <= 1e-4
    assert e <= 0.05


def test_esprit_in_plan_matches_single_calls(ctx):
    th0, dth, L = fmsynth.grid(721)
    devs = []
    for i, (M, T, K) in enumerate([(128, 256, 4), (200, 300, 10), (96, 200, 2), (128, 512, 7)]):
        fr = fmsynth.make_frame(M, T, K, 10.0, seed=40 + i, angle_range=(-60, 60), min_sep=3)
        spec = FrameSpec(M=M, T=T, K=K, n=K + 8, q=2, L=L, theta0_deg=th0, dtheta_deg=dth,
                         esprit=True)
        devs.append(DeviceFrame(spec, X=torch.from_numpy(fr.X),
                                rnd=torch.from_numpy(fmsynth.make_omega(M, K + 8, 50 + i))))
    plan = fm.Plan(ctx, [d.descriptor() for d in devs])
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    plan.close()
    for d in devs:
        g = d.results()
        single, st = _gpu_esprit(ctx, g["Us"])
        say(f"plan M={d.spec.M} K={d.spec.K}: {np.round(g['doa'], 3).tolist()}")
        assert np.array_equal(g["doa"], single)
        assert g["status"] & fm.FM_ST_EIG_MAXIT == 0 and st == 0


def test_esprit_validation(ctx):
    M, K = 64, 33
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    doa = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_esprit(Us, doa, st)
    assert e.value.status == fm.FM_E_UNSUPPORTED
    with pytest.raises(fm.FmError) as e:
        ctx.fm_esprit(torch.zeros((4, 4), dtype=torch.complex128, device="cuda"), doa, st)
    assert e.value.status == fm.FM_E_ARG
