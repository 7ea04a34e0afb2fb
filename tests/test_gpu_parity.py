"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (written in each test):
  * covariance: bit-exact on small-integer frames with power-of-two T;
    relative Frobenius error <= 1e-6 otherwise (FP32 accumulation);
  * pseudo-spectrum: max |10 log10(P_gpu / P_oracle)| <= 1e-3 dB on the FP32
    path, both for the spectrum stage alone (same U_s bits) and end to end;
    the compensated FP16 spectrum pass meets the same bar on the same U_s
    bits; 16-bit plans end to end <= 1e-2 dB;
  * peaks: bit-exact on identical float32 spectra; end to end, every oracle
    peak within one grid step of a GPU peak and the same count;
  * subspace: projector distance small and the spectra of both subspaces
    within 1e-3 dB;
  * a frame gives bit-identical results alone and inside an uneven batch.
"""
import numpy as np
import pytest

import fmsynth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_07434_amd as fm  # noqa: E402
from paper_1911_07434_amd.frames import DeviceFrame, FrameSpec, run_single  # noqa: E402

DB_FP32 = 1e-3


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0, 256 << 20)
    yield c
    c.close()


def db_err(Pg, Po):
    return float(np.max(np.abs(10.0 * np.log10(np.asarray(Pg, np.float64) / Po))))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def proj(Us):
    return Us.T @ Us.conj()


def say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------------------------
# stage 1: covariance
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("M,T", [(8, 64), (200, 512), (129, 1024), (256, 2048)])
def test_covariance_integer_bitwise(ctx, M, T):
    say(f"cov int M={M} T={T}")
    X = fmsynth.make_integer_frame(M, T, seed=M + T)
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(dev(X), R)
    torch.cuda.synchronize()
    Rg = R.cpu().numpy()
    Ro = oracle.covariance(X)
    assert np.array_equal(Rg.astype(np.complex128), Ro)


@pytest.mark.parametrize("M,T", [(64, 128), (300, 777), (1, 5), (130, 3), (1024, 2048)])
def test_covariance_gaussian(ctx, M, T):
    say(f"cov gauss M={M} T={T}")
    fr = fmsynth.make_frame(M, T, min(3, M), 0.0, seed=M * 7 + T)
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(dev(fr.X), R)
    torch.cuda.synchronize()
    Rg = R.cpu().numpy()
    Ro = oracle.covariance(fr.X, threads=oracle.default_threads())
    err = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
    say(f"  relative Frobenius error {err:.3g}")
    assert err <= 1e-6
    assert np.array_equal(Rg, Rg.conj().T)
    assert np.all(np.diag(Rg).imag == 0)


@pytest.mark.parametrize("M,T", [(1024, 2048), (200, 1029), (97, 1536), (64, 519)])
def test_covariance_segments_parallel_equals_sequential_bitwise(ctx, M, T):
    # fm_covariance runs the FP32 T segments one wave each with an in-order
    # reduction; a plan whose blocks fill the GPU runs them in turn on one
    # wave: the same sums in the same order, so the same bits
    say(f"cov segments M={M} T={T}")
    fr = fmsynth.make_frame(M, T, 3, 5.0, seed=M + 3 * T)
    X = dev(fr.X)
    R1 = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(X, R1)
    nfr = 2048 // ((M + 63) // 64 * ((M + 63) // 64 + 1)) + 1
    specs = [DeviceFrame(FrameSpec(M=M, T=T, K=3, n=8, L=181, theta0_deg=-90.0,
                                   dtheta_deg=1.0), X=X,
                         rnd=torch.from_numpy(fmsynth.make_omega(M, 8, 1))) for _ in range(nfr)]
    plan = fm.Plan(ctx, [d.descriptor() for d in specs])
    plan.covariance()
    torch.cuda.synchronize()
    a = R1.cpu().numpy()
    for d in specs[:3]:
        assert np.array_equal(a, d.R.cpu().numpy())
    Ro = oracle.covariance(fr.X, threads=oracle.default_threads())
    assert np.linalg.norm(a - Ro) / np.linalg.norm(Ro) <= 1e-6
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("M,n", [(1024, 16), (300, 24)])
def test_sketch_segments_parallel_equals_sequential_bitwise(ctx, prec, M, n):
    # single-frame Method 2 runs each product's channel segments on separate
    # workgroups with an in-order reduction; a plan with enough row blocks
    # runs them in turn in one workgroup: the same bits
    say(f"sketch segments M={M} n={n} {prec}")
    p = {"fp32": fm.FM_FP32, "fp16": fm.FM_FP16}[prec]
    T, K, q = 2 * M, 4, 2
    fr = fmsynth.make_frame(M, T, K, 5.0, seed=M + n)
    X = dev(fr.X)
    Om = torch.from_numpy(fmsynth.make_omega(M, n, 5))
    alone = DeviceFrame(FrameSpec(M=M, T=T, K=K, n=n, q=q, L=181, theta0_deg=-90.0,
                                  dtheta_deg=1.0), X=X, rnd=Om)
    run_single(ctx, alone, prec=p)
    nfr = 512 // ((M + 127) // 128) + 1
    devs = [DeviceFrame(FrameSpec(M=M, T=T, K=K, n=n, q=q, L=181, theta0_deg=-90.0,
                                  dtheta_deg=1.0), X=X, rnd=Om) for _ in range(nfr)]
    plan = fm.Plan(ctx, [d.descriptor() for d in devs], prec=p)
    plan.run()
    torch.cuda.synchronize()
    a = alone.results()
    for d in devs[:2]:
        b = d.results()
        assert np.array_equal(a["Us"], b["Us"])
        assert np.array_equal(a["sigma"], b["sigma"])
        assert np.array_equal(a["P"], b["P"])
    plan.close()


def test_covariance_leading_dimensions(ctx):
    M, T = 70, 90
    fr = fmsynth.make_frame(M, T, 2, 5.0, seed=3)
    Xbig = np.zeros((M, T + 13), np.complex64)
    Xbig[:, :T] = fr.X
    Xd = dev(Xbig)
    Rbig = torch.zeros((M, M + 5), dtype=torch.complex64, device="cuda")
    lib = ctx.lib
    st = lib.fm_covariance(ctx.h, fm._stream(), Xd.data_ptr(), M, T, T + 13, Rbig.data_ptr(),
                           M + 5, fm.FM_FP32)
    assert st == fm.FM_OK
    torch.cuda.synchronize()
    Rg = Rbig.cpu().numpy()
    Ro = oracle.covariance(fr.X)
    assert np.linalg.norm(Rg[:, :M] - Ro) / np.linalg.norm(Ro) <= 1e-6
    assert np.all(Rg[:, M:] == 0)


# ----------------------------------------------------------------------------
# stage 3: pseudo-spectrum on the same U_s bits
# ----------------------------------------------------------------------------

SPEC_PRECS = {"fp32": fm.FM_FP32, "fp16": fm.FM_FP16}


def _spectrum_case(ctx, Us, th0, dth, L, prec="fp32"):
    K, M = Us.shape
    P = torch.empty(L, dtype=torch.float32, device="cuda")
    ctx.fm_pseudospectrum(dev(Us), th0, dth, L, P, prec=SPEC_PRECS[prec])
    torch.cuda.synchronize()
    Po, deno = oracle.pseudospectrum(Us, th0, dth, L, threads=oracle.default_threads())
    return P.cpu().numpy(), Po, deno


# The compensated FP16 pass (hi + lo operands, ~22-bit products, FP32
# accumulation) is held to the FP32 bar as well.
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_spectrum_on_oracle_subspace(ctx, name, prec):
    cfg = fmsynth.CONFIGS[name]
    say(f"spectrum {name} {prec}")
    fr, _ = fmsynth.config_frame(name, seed=11)
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    Us, _, _ = oracle.subspace_project(R, fmsynth.make_omega(fr.M, cfg["l"], 11), cfg["q"], fr.K)
    th0, dth, L = fmsynth.grid(cfg["L"])
    Pg, Po, _ = _spectrum_case(ctx, Us, th0, dth, L, prec)
    say(f"  max |dP| = {db_err(Pg, Po):.3g} dB")
    assert db_err(Pg, Po) <= DB_FP32


# K spans every row-block class of both passes; M and L leave ragged chunks
# and angle tiles
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("M,K,L", [(2, 1, 7), (17, 5, 333), (100, 33, 1000), (256, 64, 4097),
                                   (1000, 8, 2049), (77, 9, 515), (300, 16, 700),
                                   (129, 17, 257), (64, 24, 1025), (96, 40, 999),
                                   (200, 48, 321), (150, 57, 130)])
def test_spectrum_random_orthonormal(ctx, M, K, L, prec):
    rng = np.random.default_rng(M + K)
    Q, _ = np.linalg.qr(rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K)))
    th0, dth = -80.0, 160.0 / max(L - 1, 1)
    Pg, Po, _ = _spectrum_case(ctx, np.ascontiguousarray(Q.T), th0, dth, L, prec)
    assert db_err(Pg, Po) <= DB_FP32


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_spectrum_single_source_pole_and_dirichlet(ctx, prec):
    M, L = 512, 18001
    th0, dth, _ = fmsynth.grid(L)
    l0 = 12345
    a0 = fmsynth.steering_matrix(M, [th0 + l0 * dth])[:, 0]
    Pg, Po, _ = _spectrum_case(ctx, (a0 / np.sqrt(M))[None, :], th0, dth, L, prec)
    assert int(np.argmax(Pg)) == l0
    ok = np.abs(np.arange(L) - l0) > 0
    assert db_err(Pg[ok], Po[ok]) <= DB_FP32
    # the pole is clamped to a finite value
    assert np.isfinite(Pg[l0]) and Pg[l0] > 1e6


# the FP64 recompute of main-lobe angles with ragged channel counts (a
# partial 64-channel block, a partial group of four blocks) and a partial
# group of four sources: a steering vector in the subspace puts a pole on the
# grid, so its lobe is listed for the recompute
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("M,K", [(300, 6), (1000, 9), (70, 5)])
def test_spectrum_refine_ragged(ctx, M, K, prec):
    L = 4097
    th0, dth = -80.0, 160.0 / (L - 1)
    l0 = 2345
    a0 = fmsynth.steering_matrix(M, [th0 + l0 * dth])[:, 0] / np.sqrt(M)
    rng = np.random.default_rng(M * K)
    G = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    G[:, 0] = a0
    Q, _ = np.linalg.qr(G)
    Pg, Po, _ = _spectrum_case(ctx, np.ascontiguousarray(Q.T), th0, dth, L, prec)
    assert int(np.argmax(Pg)) == l0
    ok = np.abs(np.arange(L) - l0) > 0
    assert db_err(Pg[ok], Po[ok]) <= DB_FP32
    assert np.isfinite(Pg[l0]) and Pg[l0] > 1e6


# ----------------------------------------------------------------------------
# stage 4: peaks on identical float32 spectra (bit-exact)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("case", range(10))
def test_peaks_bitexact(ctx, case):
    # lengths on both sides of the scan's forms: positions held in registers
    # (L <= 24576), flags in a bit mask (L <= 32768), full rescan beyond
    rng = np.random.default_rng(case)
    L = [1, 2, 5, 1000, 18001, 40000, 1025, 24576, 24577, 30000][case]
    K = [1, 2, 3, 8, 40, 64, 5, 16, 16, 33][case]
    P = rng.integers(0, 6, size=L).astype(np.float32)      # many ties and plateaus
    if case >= 3:
        P = np.round(rng.random(L) * 50).astype(np.float32)
    Pd = dev(P)
    idx = torch.zeros(K, dtype=torch.int32, device="cuda")
    val = torch.zeros(K, dtype=torch.float32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.fm_peaks(Pd, K, idx, val, nf)
    torch.cuda.synchronize()
    n = int(nf.cpu()[0])
    oi, ov = oracle.peaks(P.astype(np.float64), K)
    assert n == len(oi)
    assert np.array_equal(idx.cpu().numpy()[:n], oi)
    assert np.array_equal(val.cpu().numpy()[:n].astype(np.float64), ov)


def test_peaks_many_local_maxima_fallback(ctx):
    # alternating spectrum: L/2 local maxima, more than the LDS candidate list
    L, K = 40001, 10
    P = np.where(np.arange(L) % 2 == 0, 1.0, 0.0).astype(np.float32)
    P += (np.arange(L) % 997).astype(np.float32) * 1e-3
    Pd = dev(P)
    idx = torch.zeros(K, dtype=torch.int32, device="cuda")
    val = torch.zeros(K, dtype=torch.float32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.fm_peaks(Pd, K, idx, val, nf)
    torch.cuda.synchronize()
    oi, _ = oracle.peaks(P.astype(np.float64), K)
    assert np.array_equal(idx.cpu().numpy()[: int(nf.cpu()[0])], oi)


# ----------------------------------------------------------------------------
# stage 2: subspace on the same covariance bits
# ----------------------------------------------------------------------------

def _subspace_case(ctx, R64, method, rnd, n, q, K, prec=fm.FM_FP32):
    M = R64.shape[0]
    Rd = dev(R64.astype(np.complex64))
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    if method == "project":
        ctx.fm_subspace_project(Rd, dev(rnd), q, K, Us, sig, st, prec=prec)
    else:
        ctx.fm_subspace_sample(Rd, dev(rnd), K, Us, sig, st)
    torch.cuda.synchronize()
    # the oracle consumes the same complex64 covariance bits
    Rq = Rd.cpu().numpy().astype(np.complex128)
    if method == "project":
        Uo, so, _ = oracle.subspace_project(Rq, rnd, q, K)
    else:
        Uo, so, _ = oracle.subspace_sample(Rq, rnd, K)
    return Us.cpu().numpy(), sig.cpu().numpy(), int(st.cpu()[0]), Uo, so


# The compensated FP16 sketch (hi + lo operands, ~22-bit products) is held
# to the same bars as the FP32 one.
@pytest.mark.parametrize("name,method,prec", [("c1", "project", "fp32"), ("c1", "sample", "fp32"),
                                              ("c2", "project", "fp32"), ("c2", "sample", "fp32"),
                                              ("c1", "project", "fp16"), ("c2", "project", "fp16")])
def test_subspace_matches_oracle(ctx, name, method, prec):
    cfg = fmsynth.CONFIGS[name]
    say(f"subspace {name} {method} {prec}")
    fr, _ = fmsynth.config_frame(name, seed=23)
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    if method == "project":
        rnd, n = fmsynth.make_omega(fr.M, cfg["l"], 23), cfg["l"]
    else:
        rnd, n = fmsynth.make_idx(fr.M, cfg["p"], 23), cfg["p"]
    Ug, sg, st, Uo, so = _subspace_case(ctx, R, method, rnd, n, cfg["q"], fr.K,
                                        SPEC_PRECS[prec])
    assert st == 0
    assert np.max(np.abs(Ug.conj() @ Ug.T - np.eye(fr.K))) <= 1e-9
    say(f"  projector distance {np.linalg.norm(proj(Ug) - proj(Uo), 2):.3g}")
    assert np.linalg.norm(proj(Ug) - proj(Uo), 2) <= 1e-6
    assert np.max(np.abs(sg - so) / so) <= 1e-6
    th0, dth, L = fmsynth.grid(cfg["L"])
    Pg, _ = oracle.pseudospectrum(Ug, th0, dth, L, threads=oracle.default_threads())
    Po, _ = oracle.pseudospectrum(Uo, th0, dth, L, threads=oracle.default_threads())
    assert db_err(Pg, Po) <= DB_FP32


@pytest.mark.parametrize("M,K,n,q,method", [
    (40, 3, 3, 0, "project"), (40, 3, 40, 1, "project"), (97, 1, 9, 3, "project"),
    (65, 6, 64, 2, "project"), (40, 4, 40, 0, "sample"), (150, 5, 96, 0, "sample"),
    (300, 7, 160, 0, "sample"), (33, 2, 2, 0, "sample"),
    (40, 3, 3, 0, "project16"), (40, 3, 40, 1, "project16"), (97, 1, 9, 3, "project16"),
    (130, 6, 32, 2, "project16"), (65, 6, 64, 2, "project16"), (33, 5, 17, 1, "project16")])
def test_subspace_edge_shapes(ctx, M, K, n, q, method):
    say(f"subspace edge M={M} K={K} n={n} q={q} {method}")
    fr = fmsynth.make_frame(M, 2 * M, K, 10.0, seed=M + n, angle_range=(-60, 60), min_sep=3)
    R = oracle.covariance(fr.X)
    prec = fm.FM_FP16 if method == "project16" else fm.FM_FP32
    method = "project" if method == "project16" else method
    rnd = fmsynth.make_omega(M, n, M) if method == "project" else fmsynth.make_idx(M, n, M)
    Ug, sg, st, Uo, so = _subspace_case(ctx, R, method, rnd, n, q, K, prec)
    assert st == 0
    assert np.linalg.norm(proj(Ug) - proj(Uo), 2) <= 1e-5
    assert np.max(np.abs(sg - so) / so) <= 1e-5


# Method 2 without forming R: every product R V is X (X^H V) / T.  The oracle
# is Method 2 on the FP64 covariance of the same complex64 X (the identity is
# exact), so the bars are those of the FP32 Method 2 path.
@pytest.mark.parametrize("M,T,K,n,q", [
    (64, 128, 3, 11, 2), (1024, 2048, 8, 16, 2), (40, 80, 3, 3, 0), (97, 50, 1, 9, 3),
    (130, 333, 6, 32, 2), (65, 100, 6, 64, 1), (200, 31, 4, 12, 2), (256, 4096, 5, 40, 0)])
def test_subspace_from_x_matches_oracle(ctx, M, T, K, n, q):
    say(f"subspace from X M={M} T={T} K={K} l={n} q={q}")
    fr = fmsynth.make_frame(M, T, K, 10.0, seed=M + T, angle_range=(-60, 60), min_sep=2)
    Om = fmsynth.make_omega(M, n, M + T)
    Xd = dev(fr.X)
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.fm_subspace_project_x(Xd, dev(Om), q, K, Us, sig, st)
    torch.cuda.synchronize()
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    Uo, so, _ = oracle.subspace_project(R, Om, q, K)
    Ug, sg = Us.cpu().numpy(), sig.cpu().numpy()
    d = np.linalg.norm(proj(Ug) - proj(Uo), 2)
    say(f"  projector distance {d:.3g}, sigma rel {np.max(np.abs(sg - so) / so):.3g}")
    assert int(st.cpu()[0]) == 0
    assert d <= 1e-5
    assert np.max(np.abs(sg - so) / so) <= 1e-5
    if M == 1024:
        th0, dth, L = fmsynth.grid(18001)
        Pg, _ = oracle.pseudospectrum(Ug, th0, dth, L, threads=oracle.default_threads())
        Po, _ = oracle.pseudospectrum(Uo, th0, dth, L, threads=oracle.default_threads())
        assert db_err(Pg, Po) <= DB_FP32


@pytest.mark.parametrize("M,T,K,p", [(64, 128, 3, 44), (1024, 2048, 8, 64), (97, 50, 2, 9),
                                     (130, 333, 6, 33), (200, 31, 4, 64), (65, 100, 1, 1)])
def test_subspace_sample_from_x_matches_oracle(ctx, M, T, K, p):
    say(f"Method 1 from X M={M} T={T} K={K} p={p}")
    fr = fmsynth.make_frame(M, T, K, 10.0, seed=3 * M + T, angle_range=(-60, 60), min_sep=2)
    idx = fmsynth.make_idx(M, p, M + p)
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.fm_subspace_sample_x(dev(fr.X), dev(idx), K, Us, sig, st)
    torch.cuda.synchronize()
    R = oracle.covariance(fr.X, threads=oracle.default_threads())
    Uo, so, _ = oracle.subspace_sample(R, idx, K)
    Ug, sg = Us.cpu().numpy(), sig.cpu().numpy()
    d = np.linalg.norm(proj(Ug) - proj(Uo), 2)
    say(f"  projector distance {d:.3g}, sigma rel {np.max(np.abs(sg - so) / so):.3g}")
    # with T < p the core R(I, I) has rank <= T: its pseudo-inverse drops p - T
    # directions and says so
    assert int(st.cpu()[0]) == (fm.FM_ST_CORE_TRUNCATED if T < p else 0)
    assert d <= 1e-5
    assert np.max(np.abs(sg - so) / so) <= 1e-5


def test_subspace_sample_from_x_reports_bad_index(ctx):
    M, T, K = 64, 96, 2
    fr = fmsynth.make_frame(M, T, K, 10.0, seed=5)
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for bad in ([1, 5, 5, 9], [0, 3, 70, 2]):   # repeated, out of range
        ctx.fm_subspace_sample_x(dev(fr.X), dev(np.array(bad, np.int32)), K, Us, sig, st)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) & fm.FM_ST_BAD_INDEX


def test_subspace_from_x_validation(ctx):
    X = torch.zeros((16, 8), dtype=torch.complex64, device="cuda")
    Om = torch.zeros((16, 4), dtype=torch.float32, device="cuda")
    Us = torch.zeros((2, 16), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_project_x(X, Om, 1, 2, Us, sig, st, prec=fm.FM_FP16)
    assert e.value.status == fm.FM_E_UNSUPPORTED
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_project_x(X, Om, 1, 5, Us, sig, st)          # K > l
    assert e.value.status == fm.FM_E_ARG
    big = torch.arange(65, dtype=torch.int32, device="cuda") % 16
    Xb = torch.zeros((128, 8), dtype=torch.complex64, device="cuda")
    Ub = torch.zeros((2, 128), dtype=torch.complex128, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_sample_x(Xb, big, 2, Ub, sig, st)            # p > 64
    assert e.value.status == fm.FM_E_UNSUPPORTED
    small = fm.Context(0, 4096)
    with pytest.raises(fm.FmError) as e:
        small.fm_subspace_project_x(X, Om, 1, 2, Us, sig, st)       # arena too small
    assert e.value.status == fm.FM_E_WORKSPACE
    small.close()


def test_subspace_noiseless_rank_k(ctx):
    # exactly rank-K covariance: both methods recover span(A) (Lemmas 5, 6)
    M, K = 128, 4
    th = np.array([-40.0, -12.5, 20.0, 55.0])
    A = fmsynth.steering_matrix(M, th)
    R = A @ A.conj().T
    for method, rnd, n in (("project", fmsynth.make_omega(M, 12, 1), 12),
                           ("sample", fmsynth.make_idx(M, 16, 1), 16)):
        Ug, sg, st, Uo, so = _subspace_case(ctx, R, method, rnd, n, 2, K)
        Qa, _ = np.linalg.qr(A)
        # the core has rank K < n: its pseudo-inverse drops n - K directions;
        # the rank-K sketch's Cholesky QR meets a zero pivot (eigen route)
        want = fm.FM_ST_CORE_TRUNCATED | (fm.FM_ST_ORTH_FALLBACK if method == "project" else 0)
        assert st == want, (method, st)
        assert np.linalg.norm(proj(Ug) - Qa @ Qa.conj().T, 2) <= 1e-5


def test_subspace_reports_bad_index_and_rank_deficiency(ctx):
    M, K = 32, 3
    fr = fmsynth.make_frame(M, 64, K, 10.0, seed=4)
    R = oracle.covariance(fr.X)
    idx = np.array([1, 5, 5, 9, 30], np.int32)
    Ug, sg, st, _, _ = _subspace_case(ctx, R, "sample", idx, 5, 0, K)
    assert st & fm.FM_ST_BAD_INDEX
    # rank-1 covariance, K = 3: only one direction survives
    a = fmsynth.steering_matrix(M, [10.0])
    R1 = a @ a.conj().T
    Ug, sg, st, _, _ = _subspace_case(ctx, R1, "project", fmsynth.make_omega(M, 6, 2), 6, 1, K)
    assert st & fm.FM_ST_RANK_DEFICIENT
    assert sg[1] == 0 and sg[2] == 0


# ----------------------------------------------------------------------------
# end to end: X -> peaks, single frame, against the oracle pipeline
# ----------------------------------------------------------------------------

def _end_to_end(ctx, name, method, seed):
    cfg = fmsynth.CONFIGS[name]
    fr, _ = fmsynth.config_frame(name, seed=seed)
    th0, dth, L = fmsynth.grid(cfg["L"])
    if method == "project":
        rnd, n, m = fmsynth.make_omega(fr.M, cfg["l"], seed), cfg["l"], fm.FM_METHOD_PROJECT
    else:
        rnd, n, m = fmsynth.make_idx(fr.M, cfg["p"], seed), cfg["p"], fm.FM_METHOD_SAMPLE
    spec = FrameSpec(M=fr.M, T=fr.T, K=fr.K, method=m, n=n, q=cfg["q"], L=L, theta0_deg=th0,
                     dtheta_deg=dth)
    d = DeviceFrame(spec, X=torch.from_numpy(fr.X), rnd=torch.from_numpy(rnd))
    run_single(ctx, d)
    torch.cuda.synchronize()
    got = d.results()
    kw = dict(Omega=rnd, q=cfg["q"]) if method == "project" else dict(idx=rnd)
    ref = oracle.run_frame(fr.X, fr.K, method, th0, dth, L, threads=oracle.default_threads(), **kw)
    return got, ref


@pytest.mark.parametrize("name,method,seed", [("c1", "project", 1), ("c1", "sample", 2),
                                              ("c1", "project", 3), ("c2", "project", 4),
                                              ("c2", "sample", 5)])
def test_end_to_end_matches_oracle(ctx, name, method, seed):
    say(f"end-to-end {name} {method} seed={seed}")
    got, ref = _end_to_end(ctx, name, method, seed)
    assert got["status"] == 0
    assert db_err(got["P"], ref["P"]) <= DB_FP32
    assert got["n_found"] == len(ref["peak_idx"])
    for pk in ref["peak_idx"]:
        assert np.min(np.abs(got["peak_idx"] - pk)) <= 1
    for pk in got["peak_idx"]:
        assert np.min(np.abs(ref["peak_idx"] - pk)) <= 1


# ----------------------------------------------------------------------------
# batches: each frame bit-identical alone and in an uneven mix
# ----------------------------------------------------------------------------

def _mixed_frames(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M = int(rng.choice([64, 100, 256, 512]))
        T = int(rng.integers(M // 2, 2 * M + 1))
        K = int(rng.integers(1, 9))
        l, p = fmsynth.sketch_sizes(M, K)
        method = (fm.FM_METHOD_SAMPLE_X if i % 5 == 4 else
                  fm.FM_METHOD_SAMPLE if i % 3 == 2 else
                  fm.FM_METHOD_PROJECT_X if i % 4 == 3 else fm.FM_METHOD_PROJECT)
        sample = method in (fm.FM_METHOD_SAMPLE, fm.FM_METHOD_SAMPLE_X)
        if method == fm.FM_METHOD_SAMPLE_X:
            p = min(p, 64)
        n_ = p if sample else l
        q = int(rng.integers(0, 3))
        L = int(rng.choice([181, 1801, 3001]))
        fr = fmsynth.make_frame(M, T, K, float(rng.uniform(-5, 20)), seed=seed * 1000 + i)
        rnd = fmsynth.make_idx(M, n_, i) if sample else fmsynth.make_omega(M, n_, i)
        th0, dth, _ = fmsynth.grid(L)
        spec = FrameSpec(M=M, T=T, K=K, method=method, n=n_, q=q, L=L, theta0_deg=th0,
                         dtheta_deg=dth)
        out.append((spec, fr.X, rnd))
    return out


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_alone_bitwise(ctx, use_graph):
    frames = _mixed_frames(9, seed=5)
    alone = []
    for spec, X, rnd in frames:
        d = DeviceFrame(spec, X=torch.from_numpy(X), rnd=torch.from_numpy(rnd))
        run_single(ctx, d)
        torch.cuda.synchronize()
        alone.append(d.results())
    devs = [DeviceFrame(s, X=torch.from_numpy(X), rnd=torch.from_numpy(r)) for s, X, r in frames]
    plan = fm.Plan(ctx, [d.descriptor() for d in devs])
    for rep in range(3 if use_graph else 1):
        for d in devs:
            d.P.zero_()
            d.Us.zero_()
        plan.run(use_graph=use_graph)
        torch.cuda.synchronize()
        for a, d in zip(alone, devs):
            b = d.results()
            if d.spec.method not in (fm.FM_METHOD_PROJECT_X, fm.FM_METHOD_SAMPLE_X):  # no R
                assert np.array_equal(a["R"], b["R"])
            assert np.array_equal(a["Us"], b["Us"])
            assert np.array_equal(a["sigma"], b["sigma"])
            assert np.array_equal(a["P"], b["P"])
            assert np.array_equal(a["peak_idx"], b["peak_idx"])
            assert a["status"] == b["status"]
    plan.close()


# ----------------------------------------------------------------------------
# argument validation: rejected synchronously, nothing launched
# ----------------------------------------------------------------------------

def test_argument_validation(ctx):
    R = torch.zeros((16, 16), dtype=torch.complex64, device="cuda")
    Om = torch.zeros((16, 4), dtype=torch.float32, device="cuda")
    Us = torch.zeros((5, 16), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(5, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_project(R, Om, 2, 5, Us, sig, st)      # K > l
    assert e.value.status == fm.FM_E_ARG
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_project(R, Om, 17, 2, Us, sig, st)     # q out of range
    assert e.value.status == fm.FM_E_ARG
    P = torch.zeros(10, dtype=torch.float32, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_pseudospectrum(Us, 0.0, -1.0, 10, P)             # dtheta <= 0
    assert e.value.status == fm.FM_E_ARG
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_project(R, Om, 2, 3, Us, sig, st, prec=7)        # no such precision
    assert e.value.status == fm.FM_E_ARG
    with pytest.raises(fm.FmError) as e:
        ctx.fm_pseudospectrum(Us, 0.0, 1.0, 10, P, prec=fm.FM_BF16)  # FP32 or FP16 only
    assert e.value.status == fm.FM_E_UNSUPPORTED
    small = fm.Context(0, 1024)
    with pytest.raises(fm.FmError) as e:
        small.fm_subspace_project(R, Om, 2, 3, Us, sig, st)     # arena too small
    assert e.value.status == fm.FM_E_WORKSPACE
    small.close()


# ----------------------------------------------------------------------------
# 16-bit covariance operands (FP32 accumulation)
# ----------------------------------------------------------------------------

DB_MIXED = 1e-2
PRECS = {"fp16": fm.FM_FP16, "bf16": fm.FM_BF16, "fp16x3": fm.FM_FP16X3,
         "bf16x3": fm.FM_BF16X3}


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp16x3", "bf16x3"])
@pytest.mark.parametrize("M,T", [(8, 64), (200, 512), (257, 2048), (130, 8)])
def test_covariance16_integer_bitwise(ctx, prec, M, T):
    # |re|, |im| <= 8 are exact in FP16 and BF16 (the split precisions' lo
    # halves are zero); every partial sum is an exact integer in FP32, so the
    # result is the oracle's bit for bit
    say(f"cov16 int {prec} M={M} T={T}")
    X = fmsynth.make_integer_frame(M, T, seed=3 * M + T)
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(dev(X), R, prec=PRECS[prec])
    torch.cuda.synchronize()
    assert np.array_equal(R.cpu().numpy().astype(np.complex128), oracle.covariance(X))


# bound: rounding each snapshot to 16 bits perturbs every product x_i conj(x_j)
# by at most 2u relative (u = 2^-11 for FP16, 2^-8 for BF16); with many
# snapshots the errors average down, with T = 3 they do not
@pytest.mark.parametrize("prec,tol", [("fp16", 2 * 2.0 ** -11), ("bf16", 2 * 2.0 ** -8)])
@pytest.mark.parametrize("M,T", [(64, 128), (300, 777), (130, 3), (1024, 2048)])
def test_covariance16_gaussian(ctx, prec, tol, M, T):
    say(f"cov16 gauss {prec} M={M} T={T}")
    fr = fmsynth.make_frame(M, T, 3, 0.0, seed=M + 5 * T)
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(dev(fr.X), R, prec=PRECS[prec])
    torch.cuda.synchronize()
    Rg = R.cpu().numpy()
    Ro = oracle.covariance(fr.X, threads=oracle.default_threads())
    assert np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro) <= tol
    assert np.array_equal(Rg, Rg.conj().T)
    assert np.all(np.diag(Rg).imag == 0)


# split operands x = hi + lo: the representation error of each snapshot is at
# most u_s |x| with u_s = 2^-22 (FP16 halves) or 2^-17 (BF16 halves), and the
# dropped lo*lo term at most u_s^2-ish, so each product moves by about 2 u_s
# relative on top of the FP32 accumulation error that the FP32 path's 1e-6
# bar already covers
@pytest.mark.parametrize("prec,tol", [("fp16x3", 1e-6 + 2 * 2.0 ** -22),
                                      ("bf16x3", 1e-6 + 2 * 2.0 ** -17)])
@pytest.mark.parametrize("M,T", [(64, 128), (300, 777), (130, 3), (1, 5), (1024, 2048)])
def test_covariance_split_gaussian(ctx, prec, tol, M, T):
    say(f"cov split gauss {prec} M={M} T={T}")
    fr = fmsynth.make_frame(M, T, min(3, M), 0.0, seed=M + 11 * T)
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(dev(fr.X), R, prec=PRECS[prec])
    torch.cuda.synchronize()
    Rg = R.cpu().numpy()
    Ro = oracle.covariance(fr.X, threads=oracle.default_threads())
    err = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
    say(f"  relative Frobenius error {err:.3g}")
    assert err <= tol
    assert np.array_equal(Rg, Rg.conj().T)
    assert np.all(np.diag(Rg).imag == 0)


def _plan_one(ctx, name, method, seed, prec):
    cfg = fmsynth.CONFIGS[name]
    fr, _ = fmsynth.config_frame(name, seed=seed)
    th0, dth, L = fmsynth.grid(cfg["L"])
    if method == "project":
        rnd, n, m = fmsynth.make_omega(fr.M, cfg["l"], seed), cfg["l"], fm.FM_METHOD_PROJECT
    else:
        rnd, n, m = fmsynth.make_idx(fr.M, cfg["p"], seed), cfg["p"], fm.FM_METHOD_SAMPLE
    spec = FrameSpec(M=fr.M, T=fr.T, K=fr.K, method=m, n=n, q=cfg["q"], L=L, theta0_deg=th0,
                     dtheta_deg=dth)
    d = DeviceFrame(spec, X=torch.from_numpy(fr.X), rnd=torch.from_numpy(rnd))
    plan = fm.Plan(ctx, [d.descriptor()], prec=prec)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    kw = dict(Omega=rnd, q=cfg["q"]) if method == "project" else dict(idx=rnd)
    ref = oracle.run_frame(fr.X, fr.K, method, th0, dth, L, threads=oracle.default_threads(), **kw)
    return d.results(), ref


@pytest.mark.parametrize("name,method,seed", [("c1", "project", 31), ("c2", "project", 32),
                                              ("c2", "sample", 33)])
def test_mixed_fp16_end_to_end(ctx, name, method, seed):
    say(f"mixed fp16 {name} {method}")
    got, ref = _plan_one(ctx, name, method, seed, fm.FM_FP16)
    err = db_err(got["P"], ref["P"])
    say(f"  max |dP| = {err:.3g} dB")
    assert got["status"] == 0
    assert err <= DB_MIXED
    assert got["n_found"] == len(ref["peak_idx"])
    for pk in ref["peak_idx"]:
        assert np.min(np.abs(got["peak_idx"] - pk)) <= 1


# split precisions carry FP32-level error: the FP32 path's spectrum bar
@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("name,method,seed", [("c1", "project", 41), ("c2", "project", 42),
                                              ("c2", "sample", 43)])
def test_split_end_to_end(ctx, prec, name, method, seed):
    say(f"split {prec} {name} {method}")
    got, ref = _plan_one(ctx, name, method, seed, PRECS[prec])
    err = db_err(got["P"], ref["P"])
    say(f"  max |dP| = {err:.3g} dB")
    assert got["status"] == 0
    assert err <= DB_FP32
    assert got["n_found"] == len(ref["peak_idx"])
    for pk in ref["peak_idx"]:
        assert np.min(np.abs(got["peak_idx"] - pk)) <= 1


def test_split_precision_calls(ctx):
    # FP16X3 takes the compensated FP16 spectrum pass; BF16X3 has none
    M, K = 64, 2
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    Us[0, 0] = 1.0
    Us[1, 1] = 1.0
    P = torch.empty(91, dtype=torch.float32, device="cuda")
    Pr = torch.empty(91, dtype=torch.float32, device="cuda")
    ctx.fm_pseudospectrum(Us, -90.0, 2.0, 91, P, prec=fm.FM_FP16X3)
    ctx.fm_pseudospectrum(Us, -90.0, 2.0, 91, Pr, prec=fm.FM_FP16)
    torch.cuda.synchronize()
    assert torch.equal(P, Pr)
    with pytest.raises(fm.FmError) as e:
        ctx.fm_pseudospectrum(Us, -90.0, 2.0, 91, P, prec=fm.FM_BF16X3)
    assert e.value.status == fm.FM_E_UNSUPPORTED
    R = torch.zeros((M, M), dtype=torch.complex64, device="cuda")
    X = torch.zeros((M, 4), dtype=torch.complex64, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_covariance(X, R, prec=5)                                 # no such precision
    assert e.value.status == fm.FM_E_ARG


def test_mixed_plan_equals_single_calls_bitwise(ctx):
    frames = _mixed_frames(5, seed=9)
    for prec in (fm.FM_FP16, fm.FM_BF16, fm.FM_FP16X3, fm.FM_BF16X3):
        alone = []
        for spec, X, rnd in frames:
            d = DeviceFrame(spec, X=torch.from_numpy(X), rnd=torch.from_numpy(rnd))
            run_single(ctx, d, prec=prec)
            torch.cuda.synchronize()
            alone.append(d.results())
        devs = [DeviceFrame(s, X=torch.from_numpy(X), rnd=torch.from_numpy(r))
                for s, X, r in frames]
        plan = fm.Plan(ctx, [d.descriptor() for d in devs], prec=prec)
        plan.run()
        torch.cuda.synchronize()
        for a, d in zip(alone, devs):
            b = d.results()
            if d.spec.method not in (fm.FM_METHOD_PROJECT_X, fm.FM_METHOD_SAMPLE_X):  # no R
                assert np.array_equal(a["R"], b["R"])
            assert np.array_equal(a["P"], b["P"])
        plan.close()


# ----------------------------------------------------------------------------
# config 2 end to end over several seeds, FP32 / FP16 / BF16 plans against the
# FP64 oracle of the same randomized algorithm on the same frame
# ----------------------------------------------------------------------------

_c2_oracle = {}


def _c2_frame(method, seed):
    """(frame, random input, oracle result) of a config-2 frame (cached)."""
    key = (method, seed)
    if key not in _c2_oracle:
        cfg = fmsynth.CONFIGS["c2"]
        fr, _ = fmsynth.config_frame("c2", seed=seed)
        th0, dth, L = fmsynth.grid(cfg["L"])
        if method == "project":
            rnd = fmsynth.make_omega(fr.M, cfg["l"], seed)
            kw = dict(Omega=rnd, q=cfg["q"])
        else:
            rnd = fmsynth.make_idx(fr.M, cfg["p"], seed)
            kw = dict(idx=rnd)
        ref = oracle.run_frame(fr.X, fr.K, method, th0, dth, L,
                               threads=oracle.default_threads(), **kw)
        _c2_oracle[key] = (fr, rnd, {k: ref[k] for k in ("P", "peak_idx")})
    return _c2_oracle[key]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("method,seed", [("project", 51), ("project", 52), ("project", 53),
                                         ("sample", 54), ("sample", 55), ("sample", 56)])
def test_c2_end_to_end_seeds(ctx, method, seed, prec):
    fr, rnd, ref = _c2_frame(method, seed)
    cfg = fmsynth.CONFIGS["c2"]
    th0, dth, L = fmsynth.grid(cfg["L"])
    m = fm.FM_METHOD_PROJECT if method == "project" else fm.FM_METHOD_SAMPLE
    n = cfg["l"] if method == "project" else cfg["p"]
    spec = FrameSpec(M=fr.M, T=fr.T, K=fr.K, method=m, n=n, q=cfg["q"], L=L, theta0_deg=th0,
                     dtheta_deg=dth)
    d = DeviceFrame(spec, X=torch.from_numpy(fr.X), rnd=torch.from_numpy(rnd))
    plan = fm.Plan(ctx, [d.descriptor()], prec=fm.FM_FP32 if prec == "fp32" else PRECS[prec])
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    got = d.results()
    err = db_err(got["P"], ref["P"])
    say(f"c2 {method} seed {seed} {prec}: max |dP| = {err:.3g} dB")
    assert got["status"] == 0
    assert err <= (DB_FP32 if prec == "fp32" else DB_MIXED)
    assert got["n_found"] == len(ref["peak_idx"])
    for pk in ref["peak_idx"]:
        assert np.min(np.abs(got["peak_idx"] - pk)) <= 1
    for pk in got["peak_idx"]:
        assert np.min(np.abs(ref["peak_idx"] - pk)) <= 1


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_nonfinite_snapshot_is_reported(ctx, prec):
    # one NaN (or Inf) snapshot value reaches every entry of the final sketch
    # Gram matrix: every method reports FM_ST_NONFINITE
    M, T, K = 64, 128, 3
    th0, dth, L = fmsynth.grid(361)
    for bad in (np.nan, np.inf):
        fr = fmsynth.make_frame(M, T, K, 10.0, seed=8)
        X = fr.X.copy()
        X[5, 17] = complex(bad, 0.0)
        devs = []
        for m, n in ((fm.FM_METHOD_PROJECT, 8), (fm.FM_METHOD_SAMPLE, 12),
                     (fm.FM_METHOD_PROJECT_X, 8), (fm.FM_METHOD_SAMPLE_X, 12)):
            sample = m in (fm.FM_METHOD_SAMPLE, fm.FM_METHOD_SAMPLE_X)
            rnd = fmsynth.make_idx(M, n, 3) if sample else fmsynth.make_omega(M, n, 3)
            spec = FrameSpec(M=M, T=T, K=K, method=m, n=n, q=1, L=L, theta0_deg=th0,
                             dtheta_deg=dth)
            devs.append(DeviceFrame(spec, X=torch.from_numpy(X), rnd=torch.from_numpy(rnd)))
        plan = fm.Plan(ctx, [d.descriptor() for d in devs],
                       prec=fm.FM_FP32 if prec == "fp32" else PRECS[prec])
        plan.run()
        torch.cuda.synchronize()
        plan.close()
        for d in devs:
            st = int(d.status.cpu()[0])
            say(f"{prec} method {d.spec.method} X[5,17] = {bad}: status {st}")
            assert st & fm.FM_ST_NONFINITE
        # a clean frame reports nothing
        good = DeviceFrame(FrameSpec(M=M, T=T, K=K, n=8, q=1, L=L, theta0_deg=th0,
                                     dtheta_deg=dth),
                           X=torch.from_numpy(fr.X), rnd=torch.from_numpy(fmsynth.make_omega(M, 8, 3)))
        plan = fm.Plan(ctx, [good.descriptor()], prec=fm.FM_FP32 if prec == "fp32" else PRECS[prec])
        plan.run()
        torch.cuda.synchronize()
        plan.close()
        assert int(good.status.cpu()[0]) == 0


def test_plan_spec16_pass_equals_single_calls_bitwise(ctx):
    # frames whose spectrum runs the split hi + lo FP16 projection inside a
    # plan (fm_frame.spec_prec = FM_FP16), mixed with polynomial-pass frames,
    # at FP32 and FP16 covariance: bit-identical to the single-frame calls
    import dataclasses
    frames = _mixed_frames(8, seed=19)
    frames = [(dataclasses.replace(sp, spec_prec=fm.FM_FP16 if i % 2 == 0 else fm.FM_FP32), X, r)
              for i, (sp, X, r) in enumerate(frames)]
    for prec in (fm.FM_FP32, fm.FM_FP16):
        alone = []
        for spec, X, rnd in frames:
            d = DeviceFrame(spec, X=torch.from_numpy(X), rnd=torch.from_numpy(rnd))
            run_single(ctx, d, prec=prec)
            torch.cuda.synchronize()
            alone.append(d.results())
        devs = [DeviceFrame(s, X=torch.from_numpy(X), rnd=torch.from_numpy(r))
                for s, X, r in frames]
        plan = fm.Plan(ctx, [d.descriptor() for d in devs], prec=prec)
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for a, d in zip(alone, devs):
            b = d.results()
            assert np.array_equal(a["P"], b["P"]), d.spec
            assert np.array_equal(a["peak_idx"], b["peak_idx"])
        plan.close()


def test_plan_rejects_bf16_spectrum_pass(ctx):
    fr = fmsynth.make_frame(64, 64, 2, 10.0, seed=3)
    spec = FrameSpec(M=64, T=64, K=2, n=8, L=181, theta0_deg=-90.0, dtheta_deg=1.0,
                     spec_prec=fm.FM_BF16)
    d = DeviceFrame(spec, X=torch.from_numpy(fr.X),
                    rnd=torch.from_numpy(fmsynth.make_omega(64, 8, 3)))
    with pytest.raises(fm.FmError) as e:
        fm.Plan(ctx, [d.descriptor()])
    assert e.value.status == fm.FM_E_UNSUPPORTED


# ----------------------------------------------------------------------------
# the batch forms of every stage against the one-frame forms, bitwise: a plan
# of 64 frames (M = 1024) runs the covariance and sketch products without
# channel segments in separate workgroups, the four-lag form of the lag sums
# and 128-angle polynomial tiles; a plan of one of its frames runs segment
# workgroups with in-order reductions, one lag per lane and 64-angle tiles
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [fm.FM_FP32, fm.FM_FP16])
def test_plan_forms_batch_equals_one_frame_bitwise(ctx, prec):
    M, T, K, B, L = 1024, 256, 8, 64, 18001
    X, _ = fmsynth.make_batch_device(M, T, K, 0.0, B, 31)
    Om = fmsynth.make_omega_device(M, 16, B, 31)
    th0, dth, _ = fmsynth.grid(L)
    spec = FrameSpec(M=M, T=T, K=K, method=fm.FM_METHOD_PROJECT, n=16, q=2, L=L,
                     theta0_deg=th0, dtheta_deg=dth)
    assert ctx.get_knob(fm.FM_KNOB_SPEC_ANGLES, 0) == 128  # the built-in tile (wider than 64)
    devs = [DeviceFrame(spec, X=X[i], rnd=Om[i]) for i in range(B)]
    plan = fm.Plan(ctx, [d.descriptor() for d in devs], prec=prec)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    for i in (0, 37, B - 1):
        one = DeviceFrame(spec, X=X[i], rnd=Om[i])
        p1 = fm.Plan(ctx, [one.descriptor()], prec=prec)
        p1.run()
        torch.cuda.synchronize()
        p1.close()
        a, b = devs[i].results(), one.results()
        for key in ("R", "Us", "sigma", "P", "peak_idx"):
            assert np.array_equal(a[key], b[key]), (i, key)
        assert a["status"] == b["status"] == 0
