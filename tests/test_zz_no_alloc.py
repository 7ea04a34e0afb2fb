"""fm_subspace_project_noalloc (workspace in the library's fixed device array,
no allocation) against fm_subspace_project (workspace in the context's
arena): the same kernels on the same inputs, so the results must be
bit-identical -- on two calls in a row, the second with a smaller input
(the array keeps the first call's contents), and at both precisions.  A
request larger than the array is rejected before anything is launched."""
import numpy as np
import pytest

import fmsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_07434_amd as fm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0, 64 << 20)
    yield c
    c.close()


def _case(ctx, M, T, K, l, q, prec, seed):
    fr = fmsynth.make_frame(M, T, K, 5.0, seed=seed)
    X = torch.from_numpy(fr.X).cuda()
    R = torch.empty((M, M), dtype=torch.complex64, device="cuda")
    ctx.fm_covariance(X, R)
    Om = torch.from_numpy(fmsynth.make_omega(M, l, seed)).cuda()
    out = []
    for call in (ctx.fm_subspace_project, ctx.fm_subspace_project_noalloc):
        Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
        sig = torch.zeros(K, dtype=torch.float64, device="cuda")
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        call(R, Om, q, K, Us, sig, st, prec=prec)
        torch.cuda.synchronize()
        out.append((Us.cpu().numpy(), sig.cpu().numpy(), int(st.cpu()[0])))
    return out


@pytest.mark.parametrize("prec", [fm.FM_FP32, fm.FM_FP16])
def test_noalloc_equals_arena_call_bitwise(ctx, prec):
    # first call at M = 1024, then a smaller one (M = 200) into the same array
    for M, T, K, l, q, seed in ((1024, 2048, 8, 16, 2, 91), (200, 300, 5, 12, 1, 92)):
        (Ua, sa, ta), (Ub, sb, tb) = _case(ctx, M, T, K, l, q, prec, seed)
        print(f"prec {prec} M={M}: status {ta} / {tb}", flush=True)
        assert fm.status_errors(ta) == 0
        assert np.array_equal(Ua, Ub)
        assert np.array_equal(sa, sb)
        assert ta == tb


def test_noalloc_rejects_requests_over_the_limit(ctx):
    lib = ctx.lib
    M, l, K = 8192, 64, 64
    assert lib.fm_workspace_bytes(M, l, K, 0) > fm.FM_NOALLOC_SCRATCH_BYTES
    # real buffers of the full size: nothing may be read even if the check failed
    R = torch.zeros((M, M), dtype=torch.complex64, device="cuda")
    Om = torch.zeros((M, l), dtype=torch.float32, device="cuda")
    Us = torch.zeros((K, M), dtype=torch.complex128, device="cuda")
    sig = torch.zeros(K, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(fm.FmError) as e:
        ctx.fm_subspace_project_noalloc(R, Om, 1, K, Us, sig, st)
    assert e.value.status == fm.FM_E_WORKSPACE
    torch.cuda.synchronize()
