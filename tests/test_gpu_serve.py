"""Serving on the GPU: frames that arrive while others run are batched
continuously, each with its own snapshots generated into the pool, and
every frame's results are bit-identical to running it alone (the same
snapshots generated again, then the single-frame entry points)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_07434_amd as fm  # noqa: E402
from paper_1911_07434_amd.serve import GpuExecutor, Server, WallClock, poisson_arrivals  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0, 256 << 20)
    yield c
    c.close()


def _unpack(raw, lay, req):
    b = raw.cpu().numpy()
    M, K, L = req.M, req.K, req.L

    def take(name, dtype, count):
        return np.frombuffer(b[lay[name]:lay[name] + count * np.dtype(dtype).itemsize].tobytes(),
                             dtype=dtype)
    return dict(X=take("X", np.complex64, M * req.T).reshape(M, req.T),
                R=take("R", np.complex64, M * M).reshape(M, M),
                Us=take("Us", np.complex128, K * M).reshape(K, M),
                sigma=take("sigma", np.float64, K), status=int(take("status", np.int32, 1)[0]),
                P=take("P", np.float32, L), n=int(take("nf", np.int32, 1)[0]),
                pidx=take("pidx", np.int32, K))


@pytest.mark.parametrize("max_batch_cost", [None, 2e-4])
def test_served_frames_equal_alone_bitwise(ctx, max_batch_cost):
    # (with the cost cap, batches of these small frames hold up to three)
    Ms = (128, 256, 512)
    reqs = poisson_arrivals(20000.0, 10.0, seed=3, Ms=Ms, T_range=(64, 512), K_range=(1, 12),
                            L=2001, max_frames=48)
    ex = GpuExecutor(ctx, pool_bytes=1 << 30, n_streams=3, keep_results=True)
    clock = WallClock()
    ex.start(clock)
    st = Server(ex, budget_bytes=1 << 30, n_streams=3, max_batch=8, clock=clock,
                max_batch_cost=max_batch_cost).run(reqs)
    torch.cuda.synchronize()
    assert st.completed == len(reqs) and st.failed == 0
    assert st.batches < len(reqs)            # frames were batched together
    for r in reqs:
        raw, lay = ex.results[r.rid]
        got = _unpack(raw, lay, r)
        # the same frame alone
        X = torch.empty((r.M, r.T), dtype=torch.complex64, device="cuda")
        ex.make_X(r, X)
        R = torch.empty((r.M, r.M), dtype=torch.complex64, device="cuda")
        Us = torch.zeros((r.K, r.M), dtype=torch.complex128, device="cuda")
        sig = torch.zeros(r.K, dtype=torch.float64, device="cuda")
        sta = torch.zeros(1, dtype=torch.int32, device="cuda")
        P = torch.zeros(r.L, dtype=torch.float32, device="cuda")
        ctx.fm_covariance(X, R)
        ctx.fm_subspace_project(R, ex._omega(r.M, r.n), r.q, r.K, Us, sig, sta)
        ctx.fm_pseudospectrum(Us, -90.0, 180.0 / (r.L - 1), r.L, P)
        torch.cuda.synchronize()
        assert np.array_equal(got["X"], X.cpu().numpy()), r
        assert np.array_equal(got["R"], R.cpu().numpy()), r
        assert np.array_equal(got["Us"], Us.cpu().numpy()), r
        assert np.array_equal(got["sigma"], sig.cpu().numpy()), r
        assert np.array_equal(got["P"], P.cpu().numpy()), r
        assert got["status"] == int(sta.cpu()[0])
