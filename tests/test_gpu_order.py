"""Model-order estimate (the pre-estimation of K of Sec. V-D) on the GPU,
through the C ABI, against the oracle.

* fm_order after the Method 2 sketch with every direction kept (K = n): K_hat
  identical to the oracle's (criterion in FP64 on both sides), the n sketch
  eigenvalues within 1e-5 of the largest, the criterion curves within 1e-3
  (relative) and their difference below the oracle's own decision margin;
* the same estimate inside a batched plan (formed from the workspace
  eigenvalues at the end of the subspace stage) is bit-identical to the
  single-frame calls, for frames whose K is only a guess;
* a sketch too narrow for the sources reports K_hat = n and
  FM_ST_ORDER_AT_LIMIT; invalid arguments are rejected;
* the paper's recipe for an unknown K (estimate, then Method 1 with
  p = ceil(1.2 K_hat), Fig. 6) matches the oracle's run of the same recipe
  end to end (<= 1e-3 dB, every oracle AoA within one grid step).
"""
import numpy as np
import pytest

import fmsynth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_07434_amd as fm  # noqa: E402
from paper_1911_07434_amd.frames import (DeviceFrame, FrameSpec, estimate_order_single,  # noqa: E402
                                         run_single, sampling_length)

RULES = {"aic": fm.FM_ORDER_AIC, "mdl": fm.FM_ORDER_MDL}


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0, 256 << 20)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def _frame(M, T, K, snr, seed):
    return fmsynth.make_frame(M, T, K, snr, seed=seed, angle_range=(-60.0, 60.0), min_sep=3.0)


def _gpu_order(ctx, X, l, q, rule, seed):
    M, T = X.shape
    Om = fmsynth.make_omega(M, l, seed)
    spec = FrameSpec(M=M, T=T, K=l, n=l, q=q, L=1, order_rule=rule)
    d = DeviceFrame(spec, X=torch.from_numpy(X), rnd=torch.from_numpy(Om))
    ost = estimate_order_single(ctx, d, rule)
    torch.cuda.synchronize()
    return (int(d.K_hat.cpu()[0]), d.order_crit.cpu().numpy(), d.sigma.cpu().numpy(),
            int(ost.cpu()[0]), int(d.status.cpu()[0]), Om)


@pytest.mark.parametrize("rule", ["mdl", "aic"])
@pytest.mark.parametrize("M,T,K,snr,l,q", [
    (200, 400, 10, 0.0, 24, 2),      # Sec. V-D's setting
    (1024, 2048, 8, 0.0, 16, 2),     # the bench frame
    (256, 512, 8, -5.0, 32, 2),
    (130, 333, 3, 10.0, 9, 1),       # ragged shapes
    (64, 100, 5, 5.0, 12, 0),
])
def test_order_matches_oracle(ctx, rule, M, T, K, snr, l, q):
    say(f"order {rule} M={M} T={T} K={K} snr={snr} l={l} q={q}")
    fr = _frame(M, T, K, snr, seed=M + 7 * T + K)
    kg, cg, sg, ost, sst, Om = _gpu_order(ctx, fr.X, l, q, RULES[rule], seed=M + l)
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    ko, co, so = oracle.order_estimate(R, Om, q, T, RULES[rule])
    fin = np.isfinite(co)
    assert np.array_equal(fin, np.isfinite(cg))
    srt = np.sort(co[fin])
    margin = srt[1] - srt[0] if srt.size > 1 else np.inf
    dc = np.max(np.abs(cg[fin] - co[fin]))
    say(f"  K_hat gpu {kg} oracle {ko}; eig max |d|/eig0 {np.max(np.abs(sg - so)) / so[0]:.3g};"
        f" crit max |d| {dc:.3g} (oracle margin {margin:.3g})")
    assert ko == K                        # the estimate itself is right here
    assert kg == ko
    assert np.max(np.abs(sg - so)) <= 1e-5 * so[0]
    np.testing.assert_allclose(cg[fin], co[fin], rtol=1e-3, atol=1e-6)
    assert dc < margin
    assert ost == 0 and sst == 0


def test_order_at_limit_and_noiseless(ctx):
    M, T = 64, 256
    # more sources than the sketch is wide: every sketch direction is signal
    fr = _frame(M, T, 10, 20.0, seed=3)
    kg, _cg, _sg, ost, _sst, Om = _gpu_order(ctx, fr.X, 8, 2, fm.FM_ORDER_MDL, seed=4)
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    ko, _co, _so = oracle.order_estimate(R, Om, 2, T, fm.FM_ORDER_MDL)
    say(f"at limit: gpu {kg} oracle {ko} status {ost}")
    assert kg == ko == 8
    assert ost == fm.FM_ST_ORDER_AT_LIMIT
    # noiseless rank-3 snapshots: the kept eigenvalues hold the whole trace
    A = fmsynth.steering_matrix(M, np.array([-20.0, 10.0, 35.0]))
    rng = np.random.default_rng(9)
    S = (rng.standard_normal((3, T)) + 1j * rng.standard_normal((3, T))) / np.sqrt(2)
    X = (A @ S).astype(np.complex64)
    kg, _cg, _sg, ost, _sst, Om = _gpu_order(ctx, X, 8, 2, fm.FM_ORDER_MDL, seed=5)
    ko, _co, _so = oracle.order_estimate(oracle.covariance(X), Om, 2, T, fm.FM_ORDER_MDL)
    say(f"noiseless: gpu {kg} oracle {ko}")
    assert kg == ko == 3
    assert ost == 0


def test_order_validation(ctx):
    M, T, n = 32, 64, 8
    R = torch.zeros((M, M), dtype=torch.complex64, device="cuda")
    eig = torch.ones(n, dtype=torch.float64, device="cuda")
    kh = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for kw in [dict(rule=7), dict(rcond=-1.0)]:
        with pytest.raises(fm.FmError) as e:
            ctx.fm_order(R, T, eig, kh, st, **kw)
        assert e.value.status == fm.FM_E_ARG
    with pytest.raises(fm.FmError) as e:
        ctx.fm_order(R, 0, eig, kh, st)
    assert e.value.status == fm.FM_E_ARG
    big = torch.ones(M + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_order(R, T, big, kh, st)
    assert e.value.status == fm.FM_E_ARG
    # a plan frame formed from X has no R to take the trace of
    spec = FrameSpec(M=M, T=T, K=2, n=n, q=1, L=64, method=fm.FM_METHOD_PROJECT_X,
                     order_rule=fm.FM_ORDER_MDL)
    d = DeviceFrame(spec)
    with pytest.raises(fm.FmError) as e:
        fm.Plan(ctx, [d.descriptor()])
    assert e.value.status == fm.FM_E_ARG


def test_order_in_plan_matches_single_calls(ctx):
    shapes = [(200, 400, 10, 0.0, 24), (96, 200, 4, 5.0, 12), (256, 300, 6, -3.0, 20),
              (64, 64, 2, 10.0, 6)]
    devs, singles = [], []
    for i, (M, T, K, snr, l) in enumerate(shapes):
        fr = _frame(M, T, K, snr, seed=100 + i)
        Om = fmsynth.make_omega(M, l, 200 + i)
        rule = fm.FM_ORDER_MDL if i % 2 == 0 else fm.FM_ORDER_AIC
        # the plan frame's K is a guess (2); the estimate uses all l eigenvalues
        spec = FrameSpec(M=M, T=T, K=2, n=l, q=2, L=361, theta0_deg=-90.0, dtheta_deg=0.5,
                         order_rule=rule)
        devs.append(DeviceFrame(spec, X=torch.from_numpy(fr.X), rnd=torch.from_numpy(Om)))
        s1 = FrameSpec(M=M, T=T, K=l, n=l, q=2, L=1, order_rule=rule)
        d1 = DeviceFrame(s1, X=torch.from_numpy(fr.X), rnd=torch.from_numpy(Om))
        estimate_order_single(ctx, d1, rule)
        singles.append(d1)
    plan = fm.Plan(ctx, [d.descriptor() for d in devs])
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    plan.close()
    for (M, T, K, _snr, l), d, d1 in zip(shapes, devs, singles):
        g = d.results()
        k1 = int(d1.K_hat.cpu()[0])
        say(f"plan M={M} K={K} l={l}: K_hat {g['K_hat']} single {k1}")
        assert g["K_hat"] == k1 == K
        assert np.array_equal(g["order_crit"], d1.order_crit.cpu().numpy())
        assert g["status"] & fm.FM_ST_ORDER_AT_LIMIT == 0


def test_unknown_k_recipe_end_to_end(ctx):
    # Sec. V-D: K unknown -> estimate it (MDL over a Method 2 sketch), then run
    # Method 1 with p = ceil(1.2 K_hat) and K = K_hat (Fig. 6's sizing)
    M, T, K = 200, 400, 10
    fr = fmsynth.make_frame(M, T, K, 0.0, seed=77, angle_range=(-60.0, 60.0), min_sep=4.0)
    kg, _cg, _sg, _ost, _sst, Om = _gpu_order(ctx, fr.X, 24, 2, fm.FM_ORDER_MDL, seed=78)
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    ko, _co, _so = oracle.order_estimate(R, Om, 2, T, fm.FM_ORDER_MDL)
    assert kg == ko == K
    p = sampling_length(kg, M)
    assert p == 12
    idx = fmsynth.make_idx(M, p, 79)
    th0, dth, L = fmsynth.grid(3601)
    spec = FrameSpec(M=M, T=T, K=kg, n=p, method=fm.FM_METHOD_SAMPLE, L=L, theta0_deg=th0,
                     dtheta_deg=dth)
    d = DeviceFrame(spec, X=torch.from_numpy(fr.X), rnd=torch.from_numpy(idx))
    run_single(ctx, d)
    torch.cuda.synchronize()
    g = d.results()
    ref = oracle.run_frame(fr.X, ko, "sample", th0, dth, L, idx=idx,
                           threads=oracle.default_threads())
    err = float(np.max(np.abs(10 * np.log10(g["P"].astype(np.float64) / ref["P"]))))
    say(f"unknown-K recipe: K_hat {kg}, p {p}, max |dP| {err:.3g} dB")
    assert err <= 1e-3
    assert g["n_found"] == len(ref["peak_idx"])
    for pk in ref["peak_idx"]:
        assert np.min(np.abs(g["peak_idx"] - pk)) <= 1
