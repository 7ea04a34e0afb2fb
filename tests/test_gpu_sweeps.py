"""The experiment sweeps (sweeps.py) on the GPU engine, at a few trials:
every sweep runs and reports its fields, and the spectra it is built from
match the oracle (fast methods and standard MUSIC, <= 1e-3 dB on the same
frames, sketches and grid)."""
import numpy as np
import pytest

import fmsynth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import sweeps  # noqa: E402


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sweeps.Engine()
    yield e
    e.close()


def db(a, b):
    return float(np.max(np.abs(10 * np.log10(np.asarray(a, np.float64) / b))))


def test_spectra_match_oracle(eng):
    fm = eng.fm
    M, T, K = 200, 400, 4
    frames = sweeps._frames(eng, 2, M, T, K, 0.0, seed=31)
    for method, n, q, name in [(fm.FM_METHOD_SAMPLE, 8, 0, "sample"),
                               (fm.FM_METHOD_PROJECT, K, 2, "project")]:
        res = eng.run(frames, method, n, K, q=q, seed=5)
        mus = eng.music(res, K)
        for i, (fr, r, m) in enumerate(zip(frames, res, mus)):
            kw = (dict(idx=fmsynth.make_idx(M, n, 5 * 100003 + i)) if name == "sample"
                  else dict(Omega=fmsynth.make_omega(M, n, 5 * 100003 + i), q=q))
            ref = oracle.run_frame(fr.X, K, name, eng.th0, eng.dth, eng.L, **kw)
            ref_m = oracle.run_frame(fr.X, K, "music", eng.th0, eng.dth, eng.L)
            e1, e2 = db(r["P"], ref["P"]), db(m["P"], ref_m["P"])
            print(f"{name} frame {i}: fast {e1:.3g} dB, MUSIC {e2:.3g} dB", flush=True)
            assert e1 <= 1e-3
            assert e2 <= 1e-3


@pytest.mark.parametrize("name", list(sweeps.SWEEPS))
def test_sweep_runs(eng, name):
    out = sweeps.SWEEPS[name](eng, 3)
    assert "setting" in out
    if "rows" in out:
        assert len(out["rows"]) >= 3
        for row in out["rows"].values():
            for v in row.values():
                if isinstance(v, dict):
                    assert all(np.isfinite(x) for x in v.values())
