"""Continuous-batching serving loop for radar frames on one GPU.

Frames (radar snapshot matrices of different M, T, K) arrive over time.  The
server admits frames against an HBM budget that counts each frame's own
snapshots, covariance, subspace and spectrum (all kept on the device, in one
pool), and whenever one of its streams is idle it launches the frames that
have arrived as one batch (one fm_plan built in pool memory with
fm_plan_create_in: nothing is allocated or synchronised per batch).  Batches
on different streams overlap on the device; a frame that arrives while
others run is picked up by the next idle stream.  Latency = completion of
the frame's batch on the GPU - arrival.

The scheduler (Server) is independent of the GPU: it talks to an executor
(launch / poll / release) and a clock, so the CPU tests drive it with a
simulated executor and a virtual clock.
"""
from __future__ import annotations

import bisect
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

ALIGN = 256


def _al(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


# --------------------------------------------------------------------------
# device memory pool (offsets into one caller-owned block)
# --------------------------------------------------------------------------

class PoolAllocator:
    """First-fit allocator of 256-byte aligned ranges in [0, size)."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free_list = [(0, self.size)]   # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, n: int):
        n = _al(max(n, 1))
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= n:
                if ln == n:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + n, ln - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off
        return None

    def free(self, off: int, n: int):
        n = _al(max(n, 1))
        self.used -= n
        i = bisect.bisect_left(self.free_list, (off, 0))
        self.free_list.insert(i, (off, n))
        # merge with neighbours
        if i + 1 < len(self.free_list) and off + n == self.free_list[i + 1][0]:
            self.free_list[i] = (off, n + self.free_list[i + 1][1])
            self.free_list.pop(i + 1)
        if i > 0 and self.free_list[i - 1][0] + self.free_list[i - 1][1] == off:
            po, pn = self.free_list[i - 1]
            self.free_list[i - 1] = (po, pn + self.free_list[i][1])
            self.free_list.pop(i)

    def largest_free(self) -> int:
        return max((ln for _, ln in self.free_list), default=0)


# --------------------------------------------------------------------------
# requests and the arrival process
# --------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    M: int
    T: int
    K: int
    snr_db: float = 0.0
    n: int = 0              # sketch width (l or p)
    q: int = 2
    L: int = 18001
    method: int = 0         # 0 = Method 2 (projection), 1 = Method 1 (sampling)
    # filled by the server
    admitted: float = float("nan")
    launched: float = float("nan")
    done: float = float("nan")
    status: str = "pending"  # pending | done | failed | rejected
    batch: int = -1
    mem: tuple = ()


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int, *,
                     Ms=(128, 256, 512, 1024, 2048, 4096), T_range=(64, 4096),
                     K_range=(1, 32), snr_range=(-10.0, 30.0), L=18001, l_cap=40,
                     max_frames=None):
    """Poisson arrivals with the mixed-shape frame population of the serving
    workload: M uniform over Ms, T and K uniform integers, SNR uniform."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_frames is not None and len(out) >= max_frames):
            break
        M = int(rng.choice(Ms))
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        K = min(K, M - 1)
        l = min(K + 8, l_cap, M)
        out.append(Request(rid=len(out), arrival=t, M=M, T=T, K=K,
                           snr_db=float(rng.uniform(*snr_range)), n=l, q=2, L=L))
    return out


# --------------------------------------------------------------------------
# clocks
# --------------------------------------------------------------------------

class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, until: float | None):
        # a short nap; arrivals and GPU completions are polled in between
        time.sleep(20e-6)


class VirtualClock:
    """Simulated time for the CPU tests: idle() jumps to the next event."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def idle(self, until: float | None):
        if until is not None and until > self.t:
            self.t = until


# --------------------------------------------------------------------------
# the scheduler
# --------------------------------------------------------------------------

@dataclass
class Batch:
    bid: int
    stream: int
    reqs: list
    handle: object = None
    plan_mem: tuple = ()
    launched: float = 0.0


@dataclass
class ServeStats:
    latencies_ms: np.ndarray
    completed: int
    failed: int
    rejected: int
    duration_s: float
    batches: int
    max_inflight_bytes: int
    max_concurrent_batches: int
    mean_batch: float
    mean_inflight_bytes: float = 0.0
    admission_wait_ms: np.ndarray = field(default_factory=lambda: np.zeros(0))
    quarantined_bytes: int = 0
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = self.latencies_ms
        return {
            "frames_completed": self.completed, "frames_failed": self.failed,
            "frames_rejected": self.rejected,
            "sustained_frames_per_s": round(self.completed / self.duration_s, 1)
            if self.duration_s > 0 else 0.0,
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "max_ms": round(float(np.max(lat)), 3) if lat.size else None,
            "batches": self.batches, "mean_batch": round(self.mean_batch, 2),
            "max_concurrent_batches": self.max_concurrent_batches,
            "max_inflight_bytes": self.max_inflight_bytes,
            "mean_inflight_bytes": int(self.mean_inflight_bytes),
            "admission_wait_p50_ms": (round(float(np.percentile(self.admission_wait_ms, 50)), 3)
                                      if self.admission_wait_ms.size else None),
            "admission_wait_p99_ms": (round(float(np.percentile(self.admission_wait_ms, 99)), 3)
                                      if self.admission_wait_ms.size else None),
            "quarantined_bytes": self.quarantined_bytes, **self.extra,
        }


class Server:
    """Continuous batching: admission by memory budget, FIFO batches, one
    batch in flight per stream, streams overlapping on the device.

    max_batch_cost (optional, in the units of the executor's frame_cost):
    a batch stops growing before its estimated work would pass the cap (its
    first frame is always taken), so that batches stay short when a burst
    of large frames arrives and the streams keep finishing work often."""

    def __init__(self, executor, budget_bytes: int, n_streams: int = 2, max_batch: int = 64,
                 clock=None, stall_timeout_s: float = 30.0, max_batch_cost: float | None = None):
        assert n_streams >= 1
        self.ex = executor
        self.pool = PoolAllocator(budget_bytes)
        self.n_streams = n_streams
        self.max_batch = max_batch
        self.max_batch_cost = max_batch_cost
        self.clock = clock or WallClock()
        self.stall_timeout_s = stall_timeout_s

    def _release(self, req: Request):
        if req.mem:
            self.pool.free(*req.mem)
            req.mem = ()

    def _form_batch(self, queue: deque, now: float, stream: int, bid: int):
        """Take queued requests FIFO while their frame memory fits the budget;
        the head of the queue is never overtaken."""
        taken = []
        cost = 0.0
        while queue and len(taken) < self.max_batch:
            req = queue[0]
            if self.max_batch_cost is not None:
                c = self.ex.frame_cost(req)
                if taken and cost + c > self.max_batch_cost:
                    break
            need = self.ex.frame_bytes(req)
            if need > self.pool.size:
                queue.popleft()
                req.status = "rejected"
                continue
            off = self.pool.alloc(need)
            if off is None:
                break
            queue.popleft()
            req.mem = (off, need)
            req.admitted = now
            taken.append(req)
            if self.max_batch_cost is not None:
                cost += c
        if not taken:
            return None
        pbytes = self.ex.plan_bytes(taken)
        poff = self.pool.alloc(pbytes)
        while poff is None and len(taken) > 1:   # shrink the batch to fit its plan
            last = taken.pop()
            self._release(last)
            queue.appendleft(last)
            pbytes = self.ex.plan_bytes(taken)
            poff = self.pool.alloc(pbytes)
        if poff is None:
            for r in reversed(taken):
                self._release(r)
                queue.appendleft(r)
            return None
        return Batch(bid=bid, stream=stream, reqs=taken, plan_mem=(poff, pbytes))

    def run(self, requests: list) -> ServeStats:
        reqs = sorted(requests, key=lambda r: r.arrival)
        queue: deque = deque()
        inflight: dict[int, Batch] = {}
        nxt = 0
        bid = 0
        sizes = []
        max_conc = 0
        max_bytes = 0
        last_progress = self.clock.now()
        quarantined = 0
        t_prev, used_time = last_progress, 0.0   # time integral of the pool's use
        while nxt < len(reqs) or queue or inflight:
            now = self.clock.now()
            used_time += self.pool.used * (now - t_prev)
            t_prev = now
            progress = False
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
                progress = True
            # completions
            for s in list(inflight):
                b = inflight[s]
                try:
                    t_done = self.ex.poll(b.handle)
                except Exception as e:  # a failed batch: mark, free, carry on
                    t_done, err = now, e
                    for r in b.reqs:
                        r.status = "failed"
                else:
                    err = None
                if t_done is None:
                    continue
                for r in b.reqs:
                    if err is None:
                        r.done = t_done
                        r.status = "done"
                    self._release(r)
                self.pool.free(*b.plan_mem)
                self.ex.release(b.handle)
                del inflight[s]
                progress = True
            # launches on idle streams
            for s in range(self.n_streams):
                if s in inflight or not queue:
                    continue
                b = self._form_batch(queue, now, s, bid)
                if b is None:
                    break
                try:
                    b.handle = self.ex.launch(b.reqs, s, b.plan_mem)
                except Exception:
                    for r in b.reqs:
                        r.status = "failed"
                        self._release(r)
                    self.pool.free(*b.plan_mem)
                    continue
                b.launched = now
                for r in b.reqs:
                    r.launched = now
                    r.batch = bid
                inflight[s] = b
                sizes.append(len(b.reqs))
                bid += 1
                progress = True
            max_conc = max(max_conc, len(inflight))
            max_bytes = max(max_bytes, self.pool.used)
            if progress:
                last_progress = now
            else:
                if inflight and now - last_progress > self.stall_timeout_s:
                    # watchdog: the device made no progress; give up on these
                    # batches.  Their kernels may still write into their frame
                    # and plan memory, so that memory is quarantined (never
                    # handed out again in this run), not freed.
                    for s, b in list(inflight.items()):
                        for r in b.reqs:
                            r.status = "failed"
                            if r.mem:
                                quarantined += r.mem[1]
                                r.mem = ()
                        quarantined += b.plan_mem[1]
                        del inflight[s]
                    last_progress = now
                    continue
                hint = reqs[nxt].arrival if nxt < len(reqs) else None
                h2 = self.ex.next_completion_hint() if inflight else None
                if h2 is not None:
                    hint = h2 if hint is None else min(hint, h2)
                self.clock.idle(hint)
        done = [r for r in reqs if r.status == "done"]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in done])
        wait = np.array([(r.admitted - r.arrival) * 1e3 for r in done])
        end = max((r.done for r in done), default=0.0)
        start = reqs[0].arrival if reqs else 0.0
        span = self.clock.now() - (reqs[0].arrival if reqs else 0.0)
        return ServeStats(
            latencies_ms=lat, completed=len(done),
            failed=sum(r.status == "failed" for r in reqs),
            rejected=sum(r.status == "rejected" for r in reqs),
            duration_s=max(end - start, 1e-9), batches=len(sizes),
            max_inflight_bytes=max_bytes, max_concurrent_batches=max_conc,
            mean_batch=float(np.mean(sizes)) if sizes else 0.0,
            mean_inflight_bytes=used_time / span if span > 0 else 0.0,
            admission_wait_ms=wait, quarantined_bytes=quarantined)


# --------------------------------------------------------------------------
# GPU executor
# --------------------------------------------------------------------------

class GpuExecutor:
    """Runs batches through libfastmusic plans built in a device memory pool.

    Each admitted frame gets its own snapshot matrix X (complex64 [M][T]) in
    its pool memory, generated on the device when its batch is launched (on
    the batch's stream, so it counts in the frame's latency): K sources at
    angles drawn uniformly in [-75, 75] deg, unit-power CN(0, 1) source
    signals and CN(0, sigma^2) noise at the frame's own SNR, X = A S + N
    (the signal model of fmsynth), from a device generator seeded by the
    request id -- so a frame's data do not depend on what it is batched
    with.  Gaussian test matrices are drawn once
    per (M, l) and shared.
    """

    def __init__(self, ctx, pool_bytes: int, n_streams: int = 2, seed: int = 7,
                 prec: int = 0, keep_results: bool = False, **_ignored):
        import torch

        import fmsynth
        from . import FM_RCOND_DEFAULT
        self.torch = torch
        self.fm_pkg = __import__("paper_1911_07434_amd")
        self.ctx = ctx
        self.prec = prec
        self.seed = int(seed)
        self.rcond = FM_RCOND_DEFAULT
        self.keep_results = keep_results
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        self.base = self.pool.data_ptr()
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.gen = torch.Generator(device="cuda")
        self.omega = {}
        self.fmsynth = fmsynth
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_host = None
        self.results = {}

    def start(self, clock):
        """Align the GPU event clock with the server clock."""
        self.torch.cuda.synchronize()
        self.t0_event.record(self.streams[0])
        self.t0_event.synchronize()
        self.t0_host = clock.now()

    def make_X(self, req, out):
        """Write request `req`'s snapshot matrix into `out` (complex64 [M][T],
        contiguous) on the current stream.  Everything is drawn on the device
        (no host-to-device copy, which would wait for the stream): K angles
        uniform in [-75, 75] deg, the steering matrix A with the phase
        m sin(theta) reduced mod 2 in FP64, S and N."""
        torch = self.torch
        M, T, K = req.M, req.T, req.K
        dev = out.device
        self.gen.manual_seed(self.seed * 1000003 + req.rid)
        th = torch.rand(K, generator=self.gen, device=dev, dtype=torch.float64) * 150.0 - 75.0
        x = torch.outer(torch.arange(M, device=dev, dtype=torch.float64),
                        torch.sin(th * (np.pi / 180.0)))
        x = x - 2.0 * torch.floor(x * 0.5)
        A = torch.polar(torch.ones_like(x), -np.pi * x).to(torch.complex64)
        # circularly symmetric complex Gaussians (real and imaginary parts of
        # variance 1/2): unit-power sources S, noise N of power sigma^2; the
        # snapshots X = A S + sigma N: N drawn into X, then one GEMM on it
        S = torch.randn((K, T), generator=self.gen, device=dev, dtype=torch.complex64)
        torch.randn((M, T), generator=self.gen, out=out)
        sig = float(np.float32(np.sqrt(10.0 ** (-req.snr_db / 10.0))))
        out.addmm_(A, S, beta=sig)

    def _omega(self, M, l):
        key = (M, l)
        if key not in self.omega:
            self.omega[key] = self.fmsynth.make_omega_device(M, l, 1, 1000 * M + l)[0].contiguous()
            # drawn on the current stream, read by batches on the executor's
            # streams (which do not wait for it): complete it first
            self.torch.cuda.current_stream().synchronize()
        return self.omega[key]

    @staticmethod
    def _layout(req):
        M, K, L = req.M, req.K, req.L
        parts = [("X", M * req.T * 8), ("R", M * M * 8), ("Us", K * M * 16), ("sigma", K * 8),
                 ("status", 4), ("P", L * 4), ("pidx", K * 4), ("pval", K * 4), ("nf", 4)]
        off, lay = 0, {}
        for name, n in parts:
            lay[name] = off
            off += _al(n)
        return lay, off

    def frame_bytes(self, req) -> int:
        return self._layout(req)[1]

    # sustained rates of the covariance and of the sketch products (flop/s),
    # measured at M = 1024; the cost is a batching estimate, not a bound
    _RATES = {0: (1.4e14, 1.0e14), 1: (6.5e14, 1.0e14)}

    def frame_cost(self, req) -> float:
        """Estimated device seconds of one frame: covariance 4 M^2 T flops,
        sketch products 8 M^2 l (q + 1), a fixed 50 us for the rest."""
        cov_rate, sk_rate = self._RATES[0 if self.prec == 0 else 1]
        M = float(req.M)
        return (4.0 * M * M * req.T / cov_rate + 8.0 * M * M * max(req.n, 1) * (req.q + 1) / sk_rate
                + 5e-5)

    def _descriptor(self, req):
        d = getattr(req, "_desc", None)
        if d is not None and d[0] == req.mem:
            return d[1]
        f = self._make_descriptor(req)
        req._desc = (req.mem, f)
        return f

    def _make_descriptor(self, req):
        fm = self.fm_pkg
        lay, _ = self._layout(req)
        base = self.base + req.mem[0] if req.mem else 0
        f = fm.fm_frame()
        f.X = base + lay["X"]
        f.ldx = req.T
        f.M, f.T = req.M, req.T
        f.R = base + lay["R"]
        f.ldr = req.M
        f.K, f.method, f.n, f.q = req.K, req.method, req.n, req.q
        f.rcond = self.rcond
        f.Omega = self._omega(req.M, req.n).data_ptr()
        f.idx = None
        f.Us = base + lay["Us"]
        f.sigma = base + lay["sigma"]
        f.status = base + lay["status"]
        f.L = req.L
        f.theta0_deg, f.dtheta_deg = -90.0, 180.0 / (req.L - 1)
        f.P = base + lay["P"]
        f.peak_idx = base + lay["pidx"]
        f.peak_val = base + lay["pval"]
        f.n_found = base + lay["nf"]
        return f

    def plan_bytes(self, reqs) -> int:
        fm = self.fm_pkg
        descs = [self._descriptor(r) for r in reqs]   # memory already assigned
        n = fm.plan_bytes(self.ctx, descs, self.prec)
        if n == 0:
            raise RuntimeError(self.ctx.lib.fm_last_error(self.ctx.h).decode())
        return n

    def X_view(self, req):
        """The request's snapshot matrix in its pool memory."""
        lay, _ = self._layout(req)
        o = req.mem[0] + lay["X"]
        return self.pool[o:o + req.M * req.T * 8].view(self.torch.complex64).view(req.M, req.T)

    def launch(self, reqs, stream_idx, plan_mem):
        fm = self.fm_pkg
        s = self.streams[stream_idx]
        with self.torch.cuda.stream(s):
            for r in reqs:
                self.make_X(r, self.X_view(r))
        descs = [self._descriptor(r) for r in reqs]
        plan = fm.Plan(self.ctx, descs, prec=self.prec, dev_mem=self.base + plan_mem[0],
                       dev_bytes=plan_mem[1], stream=s)
        plan.run(stream=s)
        if self.keep_results:
            # copied before the completion event: once the event fires the
            # server may hand this memory to another batch
            for r in reqs:
                self.results[r.rid] = self._snapshot(r, s)
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(s)
        return (plan, ev)

    def _snapshot(self, req, stream):
        """Device copies of a request's outputs (for tests), on its stream."""
        torch = self.torch
        lay, _ = self._layout(req)
        with torch.cuda.stream(stream):
            raw = self.pool[req.mem[0]:req.mem[0] + self.frame_bytes(req)].clone()
        return (raw, lay)

    def poll(self, handle):
        plan, ev = handle
        if not ev.query():
            return None
        return self.t0_host + self.t0_event.elapsed_time(ev) * 1e-3

    def release(self, handle):
        plan, ev = handle
        plan.close()

    def next_completion_hint(self):
        return None
