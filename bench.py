"""Throughput of the fast-MUSIC hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic frames of
the massive-MIMO workload (M = 1024 channels, T = 2048 snapshots, K = 8
sources at SNR 0 dB, 18001-angle grid at 0.01 deg): covariance -> Method 2
subspace (l = K + 8 = 16, q = 2) -> pseudo-spectrum -> peaks, every frame of
the batch in one launch per stage.  `value` is frames per second of that
step (inputs resident in HBM).  In the same run the benchmark also times
Method 1 (p = 4l = 64) and standard MUSIC with a full eigen-decomposition
on the same GPU (rocSOLVER through torch.linalg.eigh for the O(M^3) step,
the library for the other stages), the latency of one frame alone, the
covariance kernel against the FP32 matrix-core roofline (HIP events on the
launch stream), and the FP64 CPU oracle on a bounded sample of frames.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--batch 256]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s fast-MUSIC vs plain MUSIC @M=1024,T=2048; p99 frame latency"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_F16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
M, T, K, L_GRID = 1024, 2048, 8, 18001
L_SKETCH, Q_ITERS, P_SAMPLE = 16, 2, 64
SNR_DB = 0.0


def cov_flops(M, T):
    """Algorithmic FP32 flops of R = X X^H / T with Hermitian symmetry:
    8 real flops per complex multiply-add, M(M+1)/2 entries, T terms."""
    return 8.0 * M * (M + 1) / 2.0 * T


def cov_mfma_flops(M, T, prec):
    """Flops the covariance kernel actually issues on the matrix cores (the
    blocks it computes in full, diagonal ones included): the FP32 kernel
    computes every 32x32 block of the lower triangle with three real products
    per complex product (6 flops per entry and snapshot); the 16-bit kernel
    computes 32x32 blocks of 128x128 tiles (a diagonal tile skips one of its
    four 64x64 quarters) with two real products per complex product (8 flops
    per entry and snapshot), three times that with split operands."""
    if prec == "fp32":
        nb = (M + 31) // 32
        return nb * (nb + 1) // 2 * 1024 * T * 6.0
    nt = (M + 127) // 128
    tiles = nt * (nt + 1) // 2
    subs = (tiles - nt) * 16 + nt * 12
    return subs * 1024 * T * (24.0 if prec.endswith("x3") else 8.0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pmc_traffic(n_frames, prec="fp32"):
    """HBM bytes per covariance launch of `n_frames` frames from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a device copy of known size), if it was taken on the current
    covariance source; else None."""
    name = "covariance_fp32" if prec == "fp32" else f"covariance_{prec}"
    path = os.path.join(ROOT, "profiles", f"{name}_m1024_t2048_pmc.md")
    src = os.path.join(ROOT, "paper_1911_07434_amd", "csrc",
                       "fm_cov.hip" if prec == "fp32" else "fm_cov16.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    m = re.search(r"source_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_frame:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != h:
        return None
    return float(b.group(1)) * n_frames


def serve_legs(ctx, fm, torch, seconds, seed):
    """Serving workload: Poisson arrivals at 2000 frames/s, M uniform over
    {128..4096} (powers of two), T ~ U[64, 4096], K ~ U[1, 32], SNR ~
    U[-10, 30] dB per frame, l = min(K+8, 40), q = 2, 18001-angle grid;
    every frame's own snapshots generated into the pool when its batch is
    launched; continuous batching on several streams (FP32 path three, mixed
    path four: more concurrent, smaller batches cut p50 and p99 at the same
    sustained rate) with HBM-budget admission
    (the budget counts snapshots, covariance, outputs and plans).  The mixed
    path runs again with a budget of four times its mean in-flight bytes,
    which binds: admission waits are reported.  Standard MUSIC (rocSOLVER
    eigen-decomposition per frame) is run on the head of the same arrival
    trace."""
    from paper_1911_07434_amd.serve import GpuExecutor, Server, WallClock, poisson_arrivals
    free, _total = torch.cuda.mem_get_info()
    budget = int(min(200 << 30, free - (24 << 30)))
    streams = {"fp32": 3, "fp16": 4}
    res = {"arrival_rate_hz": 2000.0, "trace_seconds": seconds, "hbm_budget_bytes": budget,
           "streams": streams}
    for pname, prec in (("fp32", fm.FM_FP32), ("fp16", fm.FM_FP16)):
        reqs = poisson_arrivals(2000.0, seconds, seed=seed + 1)
        ns = streams[pname]
        ex = GpuExecutor(ctx, pool_bytes=budget, n_streams=ns, prec=prec)
        # a short trace first: kernel and library start-up stay out of the
        # measured run
        clock = WallClock()
        ex.start(clock)
        Server(ex, budget_bytes=budget, n_streams=ns, max_batch=64, clock=clock).run(
            poisson_arrivals(2000.0, 1.0, seed=seed + 99))
        torch.cuda.synchronize()
        clock = WallClock()
        ex.start(clock)
        st = Server(ex, budget_bytes=budget, n_streams=ns, max_batch=64, clock=clock).run(reqs)
        torch.cuda.synchronize()
        res[pname] = st.summary()
        log(f"serving {pname}: {res[pname]}")
        del ex
        torch.cuda.empty_cache()
    # the mixed path again, with a budget that binds
    bound = int(4 * res["fp16"]["mean_inflight_bytes"]) // 256 * 256
    reqs = poisson_arrivals(2000.0, seconds, seed=seed + 1)
    ex = GpuExecutor(ctx, pool_bytes=bound, n_streams=streams["fp16"], prec=fm.FM_FP16)
    clock = WallClock()
    ex.start(clock)
    st = Server(ex, budget_bytes=bound, n_streams=streams["fp16"], max_batch=64,
                clock=clock).run(reqs)
    torch.cuda.synchronize()
    res["fp16_budget_bound"] = {"hbm_budget_bytes": bound, **st.summary()}
    log(f"serving fp16, budget {bound / 2**30:.2f} GiB: {res['fp16_budget_bound']}")
    del ex
    torch.cuda.empty_cache()
    # standard MUSIC under the same arrivals (head of the trace)
    reqs = poisson_arrivals(2000.0, seconds, seed=seed + 1, max_frames=120)
    ex = PlainMusicExecutor(ctx, pool_bytes=min(budget, 64 << 30), n_streams=2)
    clock = WallClock()
    ex.start(clock)
    st = Server(ex, budget_bytes=min(budget, 64 << 30), n_streams=2, max_batch=64,
                clock=clock).run(reqs)
    torch.cuda.synchronize()
    res["plain_music_head_of_trace"] = st.summary()
    log(f"serving plain MUSIC: {res['plain_music_head_of_trace']}")
    del ex
    torch.cuda.empty_cache()
    return res


def large_leg(fm, torch, ctx, stream, seed, n_frames=8, steps=3):
    """The large-array workload: M = 4096, T = 8192, K = 16 as eight pairs
    0.5 deg apart, SNR 0 dB, Method 2 with l = 24 and q = 2, 36001-angle grid
    (0.005 deg), n_frames frames per plan, at every precision; frames/s,
    stage times, the covariance rate and each precision's largest spectrum
    difference against the FP32 path on the same frames."""
    import fmsynth
    from paper_1911_07434_amd.frames import DeviceFrame, FrameSpec
    M4, T4, K4, l4, q4, L4 = 4096, 8192, 16, 24, 2, 36001
    th0, dth, _ = fmsynth.grid(L4)
    X, _ = fmsynth.make_batch_device(M4, T4, K4, 0.0, n_frames, seed, pairs=0.5)
    Om = fmsynth.make_omega_device(M4, l4, n_frames, seed)
    torch.cuda.synchronize()
    spec = FrameSpec(M=M4, T=T4, K=K4, n=l4, q=q4, L=L4, theta0_deg=th0, dtheta_deg=dth)
    frames = [DeviceFrame(spec, X=X[i], rnd=Om[i]) for i in range(n_frames)]
    names = ("covariance", "subspace", "pseudospectrum", "peaks")
    out = {"workload": f"M={M4} T={T4} K={K4} (pairs 0.5 deg apart) l={l4} q={q4} L={L4} "
                       f"SNR=0dB, {n_frames} frames per plan"}
    P_ref = None
    for pname, prec in (("fp32", fm.FM_FP32), ("fp16", fm.FM_FP16), ("bf16", fm.FM_BF16),
                        ("fp16x3", fm.FM_FP16X3), ("bf16x3", fm.FM_BF16X3)):
        plan = fm.Plan(ctx, [d.descriptor() for d in frames], prec=prec)
        with torch.cuda.stream(stream):
            for st in (plan.covariance, plan.subspace, plan.pseudospectrum, plan.peaks):
                st(stream)
            torch.cuda.synchronize()
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
            for e in ev:
                e[0].record(stream)
                for i, st in enumerate((plan.covariance, plan.subspace, plan.pseudospectrum,
                                        plan.peaks)):
                    st(stream)
                    e[i + 1].record(stream)
            torch.cuda.synchronize()
        sm = {n: float(np.median([e[i].elapsed_time(e[i + 1]) for e in ev]))
              for i, n in enumerate(names)}
        step_ms = float(np.median([e[0].elapsed_time(e[4]) for e in ev]))
        P = [frames[i].P.double().cpu().numpy() for i in range(n_frames)]
        rec = {"frames_per_s": round(n_frames / (step_ms * 1e-3), 1),
               "stage_ms_per_step": {k: round(v, 3) for k, v in sm.items()},
               "covariance_tflops": round(n_frames * cov_flops(M4, T4) / (sm["covariance"] * 1e-3)
                                          / 1e12, 1)}
        if P_ref is None:
            P_ref = P
        else:
            dP = max(float(np.max(np.abs(10 * np.log10(a / b)))) for a, b in zip(P, P_ref))
            rec["max_abs_dP_dB_vs_fp32"] = float(f"{dP:.3g}")
        out[pname] = rec
        log(f"large {pname}: {rec}")
        plan.close()
    return out


def uneven_leg(fm, torch, stream, seed, steps, tune_cache=None):
    """The uneven-batch workload: 512 frames with M from {256, 512, 1024,
    2048}, T ~ U[M/2, 2M], K ~ U[1, 16], SNR ~ U[-5, 20] dB, Method 2 with
    l = K + 8 and q = 2, 18001-angle grid, all in one plan replayed as one
    graph launch.  Timed with the built-in kernel variants, then again after
    the autotuner has chosen variants on these frames (results checked
    bit-identical)."""
    import fmsynth
    from paper_1911_07434_amd import autotune
    from paper_1911_07434_amd.frames import DeviceFrame, FrameSpec
    shapes = fmsynth.uneven_batch(512, seed)
    th0, dth, L = fmsynth.grid(18001)
    t0 = time.time()
    frames = []
    for sh in shapes:
        X, _ = fmsynth.make_batch_device(sh["M"], sh["T"], sh["K"], sh["snr_db"], 1, sh["seed"])
        Om = fmsynth.make_omega_device(sh["M"], sh["l"], 1, sh["seed"])
        spec = FrameSpec(M=sh["M"], T=sh["T"], K=sh["K"], n=sh["l"], q=sh["q"], L=L,
                         theta0_deg=th0, dtheta_deg=dth)
        frames.append(DeviceFrame(spec, X=X[0], rnd=Om[0]))
    torch.cuda.synchronize()
    flops = sum(cov_flops(s["M"], s["T"]) for s in shapes)
    log(f"uneven batch: 512 frames generated in {time.time() - t0:.1f} s, "
        f"covariance {flops / 1e12:.2f} TFLOP per batch")
    descs = [d.descriptor() for d in frames]

    def timed(plan, n):
        with torch.cuda.stream(stream):
            plan.run(use_graph=True, stream=stream)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(n)]
            for a, b in ev:
                a.record(stream)
                plan.run(use_graph=True, stream=stream)
                b.record(stream)
            torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        return {"frames_per_s": round(512.0 / (float(np.median(ms)) * 1e-3), 1),
                "ms_per_launch": {"p10": round(float(np.percentile(ms, 10)), 3),
                                  "p50": round(float(np.median(ms)), 3),
                                  "p90": round(float(np.percentile(ms, 90)), 3)}}

    res = {"frames": 512, "launch": "one hipGraph per batch (all stages, all frames)",
           "covariance_tflop_per_batch": round(flops / 1e12, 3),
           "mean_K": round(float(np.mean([s["K"] for s in shapes])), 2)}
    for pname, prec in (("fp32", fm.FM_FP32), ("fp16", fm.FM_FP16)):
        c = fm.Context(0, 1 << 20)           # built-in variants
        plan = fm.Plan(c, descs, prec=prec)
        base = timed(plan, steps)
        ref = [frames[i].P.cpu().numpy() for i in range(0, 512, 37)]
        plan.close()
        table = autotune.tune(c, frames, prec, reps=3, max_frames=512, stream=stream, log=log)
        if tune_cache:
            key = autotune.cache_key(torch.cuda.get_device_name(0), autotune.library_id(), prec)
            autotune.save(tune_cache, key, table)
        plan = fm.Plan(c, descs, prec=prec)
        tuned = timed(plan, steps)
        same = all(np.array_equal(r, frames[i].P.cpu().numpy())
                   for r, i in zip(ref, range(0, 512, 37)))
        plan.close()
        c.close()
        res[pname] = {"builtin": base, "autotuned": tuned, "tuned_bitwise_equal": bool(same),
                      "knobs": autotune.to_json(table)}
        log(f"uneven {pname}: built-in {base['frames_per_s']} frames/s, autotuned "
            f"{tuned['frames_per_s']} frames/s, bitwise equal {same}")
    del frames
    torch.cuda.empty_cache()
    return res


def _plain_music_executor():
    from paper_1911_07434_amd.serve import GpuExecutor

    class PlainMusic(GpuExecutor):
        """Standard MUSIC per frame: the library's covariance, rocSOLVER's
        eigen-decomposition (torch.linalg.eigh), the library's spectrum and
        peaks -- the comparator, not part of the library."""

        def plan_bytes(self, reqs):
            return 256

        def launch(self, reqs, stream_idx, plan_mem):
            torch = self.torch
            s = self.streams[stream_idx]
            with torch.cuda.stream(s):
                for r in reqs:
                    d = self._descriptor(r)
                    lay, _ = self._layout(r)
                    o = r.mem[0]
                    R = self.pool[o + lay["R"]:o + lay["R"] + r.M * r.M * 8].view(
                        torch.complex64).view(r.M, r.M)
                    X = self.X_view(r)
                    self.make_X(r, X)
                    self.ctx.fm_covariance(X, R, stream=s)
                    _w, V = torch.linalg.eigh(R)
                    Us = V[:, r.M - r.K:].flip(-1).transpose(0, 1).to(torch.complex128).contiguous()
                    P = self.pool[o + lay["P"]:o + lay["P"] + r.L * 4].view(torch.float32)
                    pi = self.pool[o + lay["pidx"]:o + lay["pidx"] + r.K * 4].view(torch.int32)
                    pv = self.pool[o + lay["pval"]:o + lay["pval"] + r.K * 4].view(torch.float32)
                    nf = self.pool[o + lay["nf"]:o + lay["nf"] + 4].view(torch.int32)
                    self.ctx.fm_pseudospectrum(Us, d.theta0_deg, d.dtheta_deg, r.L, P, stream=s)
                    self.ctx.fm_peaks(P, r.K, pi, pv, nf, stream=s)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
            return (None, ev)

        def release(self, handle):
            pass

    return PlainMusic


def PlainMusicExecutor(*a, **k):
    return _plain_music_executor()(*a, **k)


def _time_frames(fn, n_max, budget_s, n_min=1):
    """Run fn(i) for i = 0, 1, ... until budget_s seconds of it (at least
    n_min, at most n_max calls); returns (calls, seconds)."""
    n, t = 0, 0.0
    while n < n_max and (n < n_min or t < budget_s):
        t0 = time.perf_counter()
        fn(n)
        t += time.perf_counter() - t0
        n += 1
    return n, t


CPU_MUSIC_CACHE = os.path.join(ROOT, "profiles", "cpu_oracle_plain_music_m1024_t2048.md")


def _plain_music_frame(i):
    """Seconds of standard MUSIC through the oracle on frame i, one thread."""
    import fmsynth
    import oracle
    th0, dth, _ = fmsynth.grid(L_GRID)
    fr = fmsynth.make_frame(M, T, K, SNR_DB, seed=9100 + i, angle_range=(-75.0, 75.0),
                            min_sep=1.0)
    t0 = time.perf_counter()
    oracle.run_frame(fr.X, K, "music", th0, dth, L_GRID, threads=1)
    return time.perf_counter() - t0


def cpu_plain_music_c2(n_frames):
    """Standard MUSIC (eq. (4): the oracle's full Jacobi eigendecomposition)
    on n_frames frames of the bench workload's shape, each on one host core
    (the frames run side by side in separate processes).  Minutes per frame:
    run on its own (--cpu-plain-music N), its summary kept under profiles/,
    which the default run reports."""
    import concurrent.futures as cf
    os.environ["FM_ORACLE_PROGRESS"] = "1"   # the oracle reports each Jacobi sweep
    with cf.ProcessPoolExecutor(max_workers=n_frames) as ex:
        times = list(ex.map(_plain_music_frame, range(n_frames)))
    for i, t in enumerate(times):
        log(f"plain MUSIC oracle frame {i}: {t:.1f} s on one core")
    return {"frames": n_frames, "cores_per_frame": 1,
            "seconds_per_frame": [round(t, 2) for t in times],
            "frames_per_s": round(n_frames / sum(times), 5)}


def cpu_baseline(X, Om, idx, B, th0, dth):
    """The FP64 oracle timed on this host (a reported baseline, not the
    target): the headline on one core (the paper's timings are single-CPU
    means), the same on all cores of the process, Method 1, the 100 frames
    of the small plain-MUSIC configuration, and the cached standard-MUSIC
    figure at this workload."""
    import fmsynth
    import oracle
    thr = oracle.default_threads()
    Xh = [X[i].cpu().numpy() for i in range(min(B, 16))]
    Omh = [Om[i].cpu().numpy() for i in range(min(B, 16))]

    def m2(threads):
        return lambda i: oracle.run_frame(Xh[i % len(Xh)], K, "project", th0, dth, L_GRID,
                                          Omega=Omh[i % len(Omh)], q=Q_ITERS, threads=threads)
    n1, t1 = _time_frames(m2(1), 16, 8.0, n_min=2)
    log(f"CPU oracle Method 2: {n1 / t1:.4f} frames/s on 1 core ({n1} frames)")
    nn, tn = _time_frames(m2(thr), 16, 4.0, n_min=3)
    log(f"CPU oracle Method 2: {nn / tn:.4f} frames/s on {thr} threads ({nn} frames)")
    nm1, tm1 = _time_frames(
        lambda i: oracle.run_frame(Xh[i % len(Xh)], K, "sample", th0, dth, L_GRID,
                                   idx=idx[i % len(idx)], threads=thr), 16, 3.0, n_min=3)
    log(f"CPU oracle Method 1: {nm1 / tm1:.4f} frames/s on {thr} threads ({nm1} frames)")
    # the small configuration: M = 64, T = 128, K = 3, 1801 angles, 100 frames
    c1 = fmsynth.CONFIGS["c1"]
    th1, dth1, L1 = fmsynth.grid(c1["L"])
    frames1 = [fmsynth.config_frame("c1", seed=5000 + i)[0] for i in range(100)]
    small = {"frames": 100, "cores": 1}
    for name, kw in (("plain_music", {}),
                     ("method1", {"idx": fmsynth.make_idx(c1["M"], c1["p"], 1)}),
                     ("method2", {"Omega": fmsynth.make_omega(c1["M"], c1["l"], 1),
                                  "q": c1["q"]})):
        variant = {"plain_music": "music", "method1": "sample", "method2": "project"}[name]
        t0 = time.perf_counter()
        for fr in frames1:
            oracle.run_frame(fr.X, c1["K"], variant, th1, dth1, L1, threads=1, **kw)
        small[f"{name}_frames_per_s"] = round(100 / (time.perf_counter() - t0), 2)
    log(f"CPU oracle, M=64 frames: {small}")
    cached = None
    if os.path.exists(CPU_MUSIC_CACHE):
        m = re.search(r"frames_per_s:\s*([0-9.eE+-]+)", open(CPU_MUSIC_CACHE).read())
        if m:
            cached = {"frames_per_s": float(m.group(1)), "cores": 1,
                      "source": os.path.relpath(CPU_MUSIC_CACHE, ROOT)}
    return {"value": round(n1 / t1, 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n1} frame(s) of the same workload through the FP64 oracle on one "
                      "host core (covariance, Method 2, spectrum, peaks)",
            "all_cores": {"value": round(nn / tn, 4), "cores": thr, "frames": nn},
            "method1_all_cores": {"value": round(nm1 / tm1, 4), "cores": thr, "frames": nm1},
            "config1_m64": small,
            "plain_music_one_core": cached}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="time only the main step (for profiler runs); same as --legs ''")
    ap.add_argument("--legs", default="compare,alone,large,uneven,serve",
                    help="extra legs after the main step: compare (mixed precision, Method 1, "
                         "standard MUSIC), alone (one frame's latency), large (M=4096 T=8192 frames at "
                         "every precision), uneven (512-frame uneven batch), serve (Poisson "
                         "serving trace)")
    ap.add_argument("--prec", choices=("fp32", "fp16", "bf16", "fp16x3", "bf16x3"),
                    default="fp32",
                    help="covariance operand precision of the main timed step")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the Poisson arrival trace of the serving leg (0 = skip)")
    ap.add_argument("--uneven-steps", type=int, default=5,
                    help="timed graph launches of the 512-frame uneven batch (0 = skip)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file to store the autotuner's choices in")
    ap.add_argument("--cpu-plain-music", type=int, default=0, metavar="N",
                    help="only time N standard-MUSIC oracle frames of the workload on one "
                         "host core (minutes each) and print them as JSON")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 256 MiB device copy first (HBM counter calibration)")
    args = ap.parse_args()
    legs = set() if args.no_extra else {x for x in args.legs.split(",") if x}
    if args.cpu_plain_music > 0:
        print(json.dumps(cpu_plain_music_c2(args.cpu_plain_music)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU form (one process drives one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    import fmsynth
    import paper_1911_07434_amd as fm
    from paper_1911_07434_amd.comparator import plain_music_batch
    from paper_1911_07434_amd.frames import DeviceFrame, FrameSpec

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    ctx = fm.Context(0, 256 << 20)
    B = args.batch
    th0, dth, _ = fmsynth.grid(L_GRID)
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"generating {B} frames M={M} T={T} K={K} on the device")
    t0 = time.time()
    X, _angles = fmsynth.make_batch_device(M, T, K, SNR_DB, B, args.seed)
    Om = fmsynth.make_omega_device(M, L_SKETCH, B, args.seed)
    idx = np.stack([fmsynth.make_idx(M, P_SAMPLE, args.seed * 1000 + i) for i in range(B)])
    torch.cuda.synchronize()
    log(f"  done in {time.time() - t0:.1f} s")

    def make_frames(method):
        out = []
        for i in range(B):
            if method in (fm.FM_METHOD_PROJECT, fm.FM_METHOD_PROJECT_X):
                spec = FrameSpec(M=M, T=T, K=K, method=method, n=L_SKETCH, q=Q_ITERS, L=L_GRID,
                                 theta0_deg=th0, dtheta_deg=dth)
                d = DeviceFrame(spec, X=X[i], rnd=Om[i])
            else:
                spec = FrameSpec(M=M, T=T, K=K, method=method, n=P_SAMPLE, L=L_GRID,
                                 theta0_deg=th0, dtheta_deg=dth)
                d = DeviceFrame(spec, X=X[i], rnd=torch.from_numpy(idx[i]))
            out.append(d)
        return out

    frames2 = make_frames(fm.FM_METHOD_PROJECT)
    precs = {"fp32": fm.FM_FP32, "fp16": fm.FM_FP16, "bf16": fm.FM_BF16,
             "fp16x3": fm.FM_FP16X3, "bf16x3": fm.FM_BF16X3}
    main_prec = precs[args.prec]
    plan2 = fm.Plan(ctx, [d.descriptor() for d in frames2], prec=main_prec)
    log(f"plan workspace {plan2.workspace_bytes() / 2**20:.0f} MiB")

    stage_names = ("covariance", "subspace", "pseudospectrum", "peaks")

    def step(plan, ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.covariance(stream)
        if ev is not None:
            ev[1].record(stream)
        plan.subspace(stream)
        if ev is not None:
            ev[2].record(stream)
        plan.pseudospectrum(stream)
        if ev is not None:
            ev[3].record(stream)
        plan.peaks(stream)
        if ev is not None:
            ev[4].record(stream)

    # ---- main timed step: Method 2 ----------------------------------------
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(plan2)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
        t0 = time.perf_counter()
        for s in range(args.steps):
            step(plan2, evs[s])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    stage_ms = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs]))
                for i, n in enumerate(stage_names)}
    step_ms = np.array([e[0].elapsed_time(e[4]) for e in evs])
    ms_per_step = elapsed * 1e3 / args.steps
    value = B / (elapsed / args.steps)
    st = np.array([int(d.status.cpu()[0]) for d in frames2[:8]])
    log(f"Method 2: {value:.1f} frames/s, {ms_per_step:.2f} ms/step, stages {stage_ms}, "
        f"status {st.tolist()}")

    cov_ms = stage_ms["covariance"]
    achieved = B * cov_flops(M, T) / (cov_ms * 1e-3) / 1e12
    traffic = pmc_traffic(B, args.prec)
    peak = PEAK_FP32_MFMA_TFLOPS if args.prec == "fp32" else PEAK_F16_MFMA_TFLOPS
    kname = "cov_fp32_kernel" if args.prec == "fp32" else "cov16_kernel"
    hw = B * cov_mfma_flops(M, T, args.prec)
    roofline = {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 2),
                "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": traffic,
                # the measured HBM bytes per launch against the HBM peak
                "traffic_frac_of_hbm_peak": (round(traffic / (cov_ms * 1e-3) / (PEAK_HBM_GBS * 1e9), 4)
                                             if traffic else None),
                "launch_ms": round(cov_ms, 4),
                "algorithmic_flops_per_launch": B * cov_flops(M, T),
                # what the matrix cores execute: the FP32 kernel's three-product
                # complex multiply issues fewer flops than the algorithmic count
                "mfma_flops_per_launch": hw,
                "mfma_busy_frac": round(hw / (cov_ms * 1e-3) / 1e12 / peak, 4)}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec if args.prec == "fp32" else args.prec + "+fp32+fp64",
        "data": "synthetic",
        "config": {"workload": f"fast-MUSIC Method 2, M={M} T={T} K={K} l={L_SKETCH} q={Q_ITERS} "
                               f"L={L_GRID} SNR={SNR_DB:g}dB, {B} frames per step",
                   "global_batch": B, "M": M, "T": T, "K": K, "l": L_SKETCH, "q": Q_ITERS,
                   "L": L_GRID, "parallelism": "single GPU, frames batched per launch"},
        "angles_per_s": round(value * K, 1),
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "step_ms_events": {"p10": round(float(np.percentile(step_ms, 10)), 3),
                           "p50": round(float(np.median(step_ms)), 3),
                           "p90": round(float(np.percentile(step_ms, 90)), 3)},
        "roofline": roofline,
    }

    if "compare" in legs:
        # ---- mixed precision: 16-bit covariance operands, same frames ------
        # (the split precisions are checked against the main step's spectra of
        # the first frames)
        n_chk = 8
        P_main = [frames2[i].P.double().cpu().numpy() for i in range(n_chk)]
        mixed = {}
        for pname, prec in (("fp16", fm.FM_FP16), ("bf16", fm.FM_BF16),
                            ("fp16x3", fm.FM_FP16X3), ("bf16x3", fm.FM_BF16X3),
                            ("fp16+spec16", fm.FM_FP16)):
            descs = [d.descriptor() for d in frames2]
            if pname.endswith("+spec16"):
                # the spectrum as the split hi + lo FP16 steering projection
                for f in descs:
                    f.spec_prec = fm.FM_FP16
            planm = fm.Plan(ctx, descs, prec=prec)
            with torch.cuda.stream(stream):
                step(planm)
                torch.cuda.synchronize()
                nm = max(5, args.steps // 2)
                evm = [[torch.cuda.Event(enable_timing=True) for _ in range(5)]
                       for _ in range(nm)]
                t0 = time.perf_counter()
                for sidx in range(nm):
                    step(planm, evm[sidx])
                torch.cuda.synchronize()
                vm = B * nm / (time.perf_counter() - t0)
            sm = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evm]))
                  for i, n in enumerate(stage_names)}
            am = B * cov_flops(M, T) / (sm["covariance"] * 1e-3) / 1e12
            mixed[pname] = {"frames_per_s": round(vm, 2),
                            "stage_ms_per_step": {k: round(v, 4) for k, v in sm.items()},
                            "covariance_tflops": round(am, 1),
                            "covariance_frac_of_16bit_peak": round(am / PEAK_F16_MFMA_TFLOPS, 4)}
            mixed[pname]["covariance_mfma_busy_frac"] = round(
                B * cov_mfma_flops(M, T, pname.split("+")[0]) / (sm["covariance"] * 1e-3) / 1e12
                / PEAK_F16_MFMA_TFLOPS, 4)
            tr = pmc_traffic(B, pname.split("+")[0])
            mixed[pname]["covariance_traffic_frac_of_hbm_peak"] = (
                round(tr / (sm["covariance"] * 1e-3) / (PEAK_HBM_GBS * 1e9), 4) if tr else None)
            dP = max(float(np.max(np.abs(10 * np.log10(
                frames2[i].P.double().cpu().numpy() / P_main[i])))) for i in range(n_chk))
            mixed[pname]["max_abs_dP_dB_vs_main_step"] = float(f"{dP:.3g}")
            log(f"mixed {pname}: {vm:.1f} frames/s, stages {sm}, max |dP| vs main {dP:.3g} dB")
            del planm
        out["mixed_precision"] = mixed
        out["mixed_precision_note"] = ("covariance operands in FP16/BF16 with FP32 "
                                       "accumulation (fp16x3/bf16x3: operands split into "
                                       "16-bit hi+lo halves, three products, FP32-level "
                                       "error); Method 2 sketch on FP16 matrix cores "
                                       "with hi+lo split operands (three products, FP32 "
                                       "accumulation); spectrum FP32 (polynomial pass; "
                                       "+spec16: split hi+lo FP16 steering projection on "
                                       "matrix cores); small dense steps and peak-region "
                                       "denominators FP64")

        # ---- Method 1 on the same frames -----------------------------------
        del plan2
        frames1 = make_frames(fm.FM_METHOD_SAMPLE)
        plan1 = fm.Plan(ctx, [d.descriptor() for d in frames1])
        with torch.cuda.stream(stream):
            step(plan1)
            torch.cuda.synchronize()
            n1 = max(3, args.steps // 4)
            t0 = time.perf_counter()
            for _ in range(n1):
                step(plan1)
            torch.cuda.synchronize()
            v1 = B * n1 / (time.perf_counter() - t0)
        log(f"Method 1: {v1:.1f} frames/s")
        del plan1, frames1
        # Method 1 without forming R (C = X X(I, :)^H / T)
        frames1x = make_frames(fm.FM_METHOD_SAMPLE_X)
        plan1x = fm.Plan(ctx, [d.descriptor() for d in frames1x])
        with torch.cuda.stream(stream):
            step(plan1x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n1):
                step(plan1x)
            torch.cuda.synchronize()
            v1x = B * n1 / (time.perf_counter() - t0)
        log(f"Method 1 without R: {v1x:.1f} frames/s")
        del plan1x, frames1x

        # ---- Method 2 without forming R (products X (X^H V) / T), FP32 -----
        framesx = make_frames(fm.FM_METHOD_PROJECT_X)
        planx = fm.Plan(ctx, [d.descriptor() for d in framesx])
        with torch.cuda.stream(stream):
            step(planx)
            torch.cuda.synchronize()
            nx = max(5, args.steps // 2)
            evx = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(nx)]
            t0 = time.perf_counter()
            for sidx in range(nx):
                step(planx, evx[sidx])
            torch.cuda.synchronize()
            vx = B * nx / (time.perf_counter() - t0)
        smx = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evx]))
               for i, n in enumerate(stage_names)}
        # the same frames' spectra through both routes (identical in exact
        # arithmetic): the covariance route rerun in FP32 on the first four
        from paper_1911_07434_amd.frames import run_single
        with torch.cuda.stream(stream):
            for i in range(4):
                run_single(ctx, frames2[i], fm.FM_FP32, stream)
        torch.cuda.synchronize()
        px = np.stack([framesx[i].P.cpu().numpy() for i in range(4)]).astype(np.float64)
        p2 = np.stack([frames2[i].P.cpu().numpy() for i in range(4)]).astype(np.float64)
        dbx = float(np.max(np.abs(10 * np.log10(px / p2))))
        log(f"Method 2 without R: {vx:.1f} frames/s, stages {smx}, max |dP| vs R route {dbx:.2g} dB")
        out["covariance_free"] = {
            "frames_per_s": round(vx, 2),
            "method1_frames_per_s": round(v1x, 2),
            "stage_ms_per_step": {k: round(v, 4) for k, v in smx.items()},
            "products": "R V as X (X^H V) / T on FP32 MFMA, R never formed",
            "max_abs_dP_db_vs_covariance_route_4_frames": dbx,
        }
        del planx, framesx

        # ---- unknown K: model-order pre-estimation (MDL, Sec. V-D) ---------
        # covariance and the Method 2 sketch of every frame, with the
        # estimate formed from all l eigenvalues at the end of the subspace
        # stage (the remaining stages do not depend on it and are not timed)
        framesk = []
        for i in range(B):
            spec = FrameSpec(M=M, T=T, K=K, n=L_SKETCH, q=Q_ITERS, L=L_GRID, theta0_deg=th0,
                             dtheta_deg=dth, order_rule=fm.FM_ORDER_MDL)
            framesk.append(DeviceFrame(spec, X=X[i], rnd=Om[i]))
        plank = fm.Plan(ctx, [d.descriptor() for d in framesk])
        with torch.cuda.stream(stream):
            plank.covariance(stream)
            plank.subspace(stream)
            torch.cuda.synchronize()
            nk = max(5, args.steps // 2)
            t0 = time.perf_counter()
            for _ in range(nk):
                plank.covariance(stream)
                plank.subspace(stream)
            torch.cuda.synchronize()
            vk = B * nk / (time.perf_counter() - t0)
        khat = np.array([int(d.K_hat.cpu()[0]) for d in framesk])
        log(f"model order (MDL): {vk:.1f} frames/s, K_hat == K for {np.mean(khat == K):.3f} "
            f"of frames, K_hat values {sorted(set(khat.tolist()))}")
        out["order_estimate"] = {
            "rule": "MDL over the l sketch eigenvalues completed from the trace of R",
            "frames_per_s": round(vk, 2),
            "timed": "covariance + Method 2 sketch + estimate",
            "fraction_K_hat_equals_K": round(float(np.mean(khat == K)), 4),
            "K_hat_min_max": [int(khat.min()), int(khat.max())],
        }
        del plank, framesk

        # ---- ESPRIT on the fast subspace, formed in the subspace stage ------
        framese = []
        for i in range(B):
            spec = FrameSpec(M=M, T=T, K=K, n=L_SKETCH, q=Q_ITERS, L=L_GRID, theta0_deg=th0,
                             dtheta_deg=dth, esprit=True)
            framese.append(DeviceFrame(spec, X=X[i], rnd=Om[i]))
        plane = fm.Plan(ctx, [d.descriptor() for d in framese])
        with torch.cuda.stream(stream):
            plane.covariance(stream)
            plane.subspace(stream)
            torch.cuda.synchronize()
            ne = max(5, args.steps // 2)
            t0 = time.perf_counter()
            for _ in range(ne):
                plane.covariance(stream)
                plane.subspace(stream)
            torch.cuda.synchronize()
            ve = B * ne / (time.perf_counter() - t0)
        doa = np.stack([d.doa.cpu().numpy() for d in framese])
        err = np.abs(doa - np.sort(_angles, axis=1))
        log(f"ESPRIT on the fast subspace: {ve:.1f} frames/s (covariance + sketch + ESPRIT), "
            f"median |error| {np.median(err):.3g} deg, p99 {np.percentile(err, 99):.3g} deg")
        out["esprit"] = {
            "frames_per_s": round(ve, 2),
            "timed": "covariance + Method 2 sketch + ESPRIT angles (no spectrum, no peaks)",
            "median_abs_error_deg": round(float(np.median(err)), 5),
            "p99_abs_error_deg": round(float(np.percentile(err, 99)), 4),
        }
        del plane, framese

        # ---- standard MUSIC (full EVD) on the same GPU ---------------------
        nb = min(B, 32)
        with torch.cuda.stream(stream):
            def plain_batch():
                plain_music_batch(ctx, frames2[:nb], K, th0, dth, L_GRID, stream=stream)
            plain_batch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 2
            for _ in range(reps):
                plain_batch()
            torch.cuda.synchronize()
            vplain = nb * reps / (time.perf_counter() - t0)
        log(f"plain MUSIC (rocSOLVER eigh): {vplain:.2f} frames/s")

        out["comparison"] = {
            "method1_frames_per_s": round(v1, 2),
            "plain_music_frames_per_s": round(vplain, 3),
            "plain_music_eig": "torch.linalg.eigh (rocSOLVER), complex64",
            "speedup_method2_vs_plain": round(value / vplain, 1),
            "speedup_method1_vs_plain": round(v1 / vplain, 1),
        }

    if "alone" in legs:
        # ---- one frame alone: latency distribution -------------------------
        # (stage by stage with events between the stages, and the whole frame
        # as one graph replay; FP32 path, then the mixed path)
        def alone(prec):
            lat, lat_g, st = [], [], []
            plan_one = fm.Plan(ctx, [frames2[0].descriptor()], prec=prec)
            with torch.cuda.stream(stream):
                for i in range(3):
                    step(plan_one)
                    plan_one.run(use_graph=True, stream=stream)
                torch.cuda.synchronize()
                for i in range(200):
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
                    step(plan_one, ev)
                    ev[4].synchronize()
                    lat.append(ev[0].elapsed_time(ev[4]))
                    st.append([ev[j].elapsed_time(ev[j + 1]) for j in range(4)])
                for i in range(200):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    plan_one.run(use_graph=True, stream=stream)
                    e1.record(stream)
                    e1.synchronize()
                    lat_g.append(e0.elapsed_time(e1))
            del plan_one
            return {"p50": round(float(np.percentile(lat, 50)), 3),
                    "p99": round(float(np.percentile(lat, 99)), 3),
                    "stage_ms_p50": {n: round(float(np.median([x[j] for x in st])), 4)
                                     for j, n in enumerate(stage_names)},
                    "graph_replay_p50": round(float(np.percentile(lat_g, 50)), 3),
                    "graph_replay_p99": round(float(np.percentile(lat_g, 99)), 3)}
        out["frame_latency_ms_alone"] = alone(fm.FM_FP32)
        out["frame_latency_ms_alone"]["fp16"] = alone(fm.FM_FP16)
        log(f"one frame alone: {out['frame_latency_ms_alone']}")

    # ---- large frames (M = 4096, T = 8192) at every precision -------------
    if "large" in legs:
        out["large_frames"] = large_leg(fm, torch, ctx, stream, args.seed + 11)

    # ---- uneven batch in one graph launch, built-in vs autotuned variants ---
    if "uneven" in legs and args.uneven_steps > 0:
        out["uneven_batch"] = uneven_leg(fm, torch, stream, args.seed + 7, args.uneven_steps,
                                         args.tune_cache)

    # ---- serving: Poisson arrivals of mixed-shape frames ---------------------
    if "serve" in legs and args.serve_seconds > 0:
        del frames2
        torch.cuda.empty_cache()
        out["serving"] = serve_legs(ctx, fm, torch, args.serve_seconds, args.seed)

    # ---- CPU baseline: the FP64 oracle on a bounded sample -----------------
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(X, Om, idx, B, th0, dth)

    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
