"""The serving scheduler on the CPU, driven by a simulated executor.

The executor is a duration model (no numerics): a batch occupies its stream
for a time proportional to its frames' covariance work.  It is a test double
for the scheduler only, not a second compute path.
"""
import numpy as np
import pytest

from paper_1911_07434_amd.serve import (PoolAllocator, Request, Server, VirtualClock,
                                        poisson_arrivals)


class FakeExecutor:
    def __init__(self, clock, per_frame_s=1e-3, fail_rids=(), hang_rids=(), plan_bytes=1024):
        self.clock = clock
        self.per_frame_s = per_frame_s
        self.fail_rids = set(fail_rids)
        self.hang_rids = set(hang_rids)
        self._plan_bytes = plan_bytes
        self.busy_until = {}
        self.live = {}
        self.launches = []

    def frame_bytes(self, req):
        return req.M * req.M * 8

    def frame_cost(self, req):
        return self.per_frame_s * (req.M / 1024) ** 2 * req.T / 2048

    def plan_bytes(self, reqs):
        return self._plan_bytes * len(reqs)

    def launch(self, reqs, stream, plan_mem):
        if any(r.rid in self.fail_rids for r in reqs):
            raise RuntimeError("launch failed")
        now = self.clock.now()
        start = max(now, self.busy_until.get(stream, 0.0))
        dur = sum(self.per_frame_s * (r.M / 1024) ** 2 * r.T / 2048 for r in reqs)
        end = float("inf") if any(r.rid in self.hang_rids for r in reqs) else start + dur
        self.busy_until[stream] = end
        h = (stream, end, tuple(r.rid for r in reqs))
        self.live[h] = True
        self.launches.append((now, stream, [r.rid for r in reqs]))
        return h

    def poll(self, h):
        return h[1] if h[1] <= self.clock.now() else None

    def release(self, h):
        del self.live[h]

    def next_completion_hint(self):
        ends = [h[1] for h in self.live if np.isfinite(h[1])]
        return min(ends) if ends else None


def reqs_uniform(n, gap, M=1024, T=2048):
    return [Request(rid=i, arrival=i * gap, M=M, T=T, K=4, n=12) for i in range(n)]


def test_pool_allocator_reuse_and_merge():
    p = PoolAllocator(4096)
    a = p.alloc(1000)
    b = p.alloc(1000)
    c = p.alloc(1000)
    assert (a, b, c) == (0, 1024, 2048)
    assert p.alloc(2000) is None
    p.free(b, 1000)
    p.free(a, 1000)
    assert p.free_list[0] == (0, 2048)
    assert p.alloc(2000) == 0
    p.free(0, 2000)
    p.free(c, 1000)
    assert p.free_list == [(0, 4096)] and p.used == 0


def test_all_frames_complete_and_latency_covers_service():
    clk = VirtualClock()
    ex = FakeExecutor(clk, per_frame_s=1e-3)
    reqs = reqs_uniform(50, 0.01)
    st = Server(ex, budget_bytes=1 << 34, n_streams=2, clock=clk).run(reqs)
    assert st.completed == 50 and st.failed == 0
    assert np.all(st.latencies_ms >= 1.0 - 1e-9)       # at least one frame's service time
    assert st.max_concurrent_batches <= 2


def test_continuous_batching_overlaps_streams_under_load():
    clk = VirtualClock()
    ex = FakeExecutor(clk, per_frame_s=2e-3)
    reqs = reqs_uniform(400, 1e-4)                       # arrivals 20x faster than service
    st = Server(ex, budget_bytes=1 << 36, n_streams=3, max_batch=16, clock=clk).run(reqs)
    assert st.completed == 400
    assert st.max_concurrent_batches == 3
    assert st.mean_batch > 4                             # frames that arrived meanwhile batch up
    streams = {s for _, s, _ in ex.launches}
    assert streams == {0, 1, 2}


def test_admission_respects_memory_budget():
    clk = VirtualClock()
    ex = FakeExecutor(clk, per_frame_s=1e-3, plan_bytes=256)
    frame = 1024 * 1024 * 8
    budget = 2 * frame + 4096                             # two frames (+ plans) at most
    reqs = reqs_uniform(20, 1e-5)
    st = Server(ex, budget_bytes=budget, n_streams=4, max_batch=8, clock=clk).run(reqs)
    assert st.completed == 20
    assert st.max_inflight_bytes <= budget
    assert max(len(r) for _, _, r in ex.launches) <= 2


def test_fifo_no_overtaking_of_a_large_head_frame():
    clk = VirtualClock()
    ex = FakeExecutor(clk, per_frame_s=1e-3, plan_bytes=256)
    small, big = 256, 2048
    budget = big * big * 8 + 8192
    reqs = [Request(rid=0, arrival=0.0, M=big, T=2048, K=4, n=12)]
    reqs += [Request(rid=i, arrival=1e-6 * i, M=small, T=256, K=4, n=12) for i in range(1, 30)]
    reqs.insert(5, Request(rid=99, arrival=2e-6, M=big, T=2048, K=4, n=12))
    Server(ex, budget_bytes=budget, n_streams=2, clock=clk).run(reqs)
    order = [rid for _, _, rids in ex.launches for rid in rids]
    # the second big frame is launched before any small frame that arrived after it
    later_small = [r.rid for r in reqs if r.M == small and r.arrival > 2e-6]
    assert all(order.index(99) < order.index(s) for s in later_small)


def test_oversized_frame_is_rejected_and_the_rest_served():
    clk = VirtualClock()
    ex = FakeExecutor(clk)
    reqs = reqs_uniform(5, 1e-3, M=256)
    reqs.append(Request(rid=5, arrival=1e-3, M=8192, T=64, K=2, n=10))
    st = Server(ex, budget_bytes=256 * 256 * 8 * 8, n_streams=2, clock=clk).run(reqs)
    assert st.rejected == 1 and st.completed == 5
    assert reqs[5].status == "rejected"


def test_failed_launch_is_marked_and_memory_freed():
    clk = VirtualClock()
    ex = FakeExecutor(clk, fail_rids={3})
    reqs = reqs_uniform(10, 5e-3)
    srv = Server(ex, budget_bytes=1 << 34, n_streams=2, max_batch=1, clock=clk)
    st = srv.run(reqs)
    assert st.failed == 1 and st.completed == 9
    assert reqs[3].status == "failed"
    assert srv.pool.used == 0


def test_watchdog_gives_up_on_a_stalled_batch():
    clk = VirtualClock()
    ex = FakeExecutor(clk, hang_rids={2})

    class TickClock(VirtualClock):
        def idle(self, until):
            self.t = until if until is not None and until > self.t else self.t + 1.0

    clk2 = TickClock()
    ex.clock = clk2
    reqs = reqs_uniform(6, 1e-3)
    srv = Server(ex, budget_bytes=1 << 34, n_streams=2, max_batch=1, clock=clk2,
                 stall_timeout_s=5.0)
    st = srv.run(reqs)
    assert reqs[2].status == "failed"
    assert st.completed == 5
    # the stalled batch may still write its memory: quarantined, never reused
    held = ex.frame_bytes(reqs[2]) + ex.plan_bytes([reqs[2]])
    assert st.quarantined_bytes == held
    assert srv.pool.used == held
    assert st.summary()["quarantined_bytes"] == held


def test_poisson_arrivals_population():
    reqs = poisson_arrivals(2000.0, 2.0, seed=1)
    assert 3600 < len(reqs) < 4400                        # ~2000/s
    gaps = np.diff([r.arrival for r in reqs])
    assert abs(np.mean(gaps) - 5e-4) < 5e-5
    assert {r.M for r in reqs} == {128, 256, 512, 1024, 2048, 4096}
    assert min(r.T for r in reqs) >= 64 and max(r.T for r in reqs) <= 4096
    assert all(1 <= r.K <= 32 and r.n == min(r.K + 8, 40) for r in reqs)


def test_budget_binding_run_reports_admission_waits():
    # frames of 8 MiB each, 4 ms of work each, arriving every 1 ms on two
    # streams: a budget of 3 frames (plus plans) makes arrivals wait
    clk = VirtualClock()
    ex = FakeExecutor(clk, per_frame_s=4e-3, plan_bytes=256)
    reqs = reqs_uniform(40, 1e-3)
    clk_free = VirtualClock()
    free = Server(FakeExecutor(clk_free, per_frame_s=4e-3, plan_bytes=256),
                  budget_bytes=1 << 40, n_streams=2, max_batch=4,
                  clock=clk_free).run(reqs_uniform(40, 1e-3))
    budget = 3 * (8 << 20) + 4096
    srv = Server(ex, budget_bytes=budget, n_streams=2, max_batch=4, clock=clk)
    st = srv.run(reqs)
    s = st.summary()
    assert st.completed == 40 and st.rejected == 0
    assert st.max_inflight_bytes <= budget
    assert 0 < st.mean_inflight_bytes <= budget
    assert s["admission_wait_p99_ms"] > 0.0
    # binding the budget delays admission relative to an unbounded run
    assert np.percentile(st.admission_wait_ms, 99) > np.percentile(free.admission_wait_ms, 99)
    assert srv.pool.used == 0


def test_batch_cost_cap_keeps_batches_short_and_fifo():
    # a burst of mixed frames: with the cap, a batch stops growing before its
    # estimated work passes it (a frame over the cap runs alone), the launch
    # order stays the arrival order, and every frame completes
    clk = VirtualClock()
    ex = FakeExecutor(clk, per_frame_s=1e-3)
    rng = np.random.default_rng(3)
    reqs = [Request(rid=i, arrival=1e-5 * i, M=int(rng.choice([256, 1024, 4096])),
                    T=int(rng.integers(64, 4097)), K=4, n=12) for i in range(300)]
    cap = 4e-3
    st = Server(ex, budget_bytes=1 << 40, n_streams=3, max_batch=64, clock=clk,
                max_batch_cost=cap).run(reqs)
    assert st.completed == 300
    by_id = {r.rid: r for r in reqs}
    for _, _, rids in ex.launches:
        if len(rids) > 1:
            assert sum(ex.frame_cost(by_id[i]) for i in rids) <= cap + 1e-12
    order = [rid for _, _, rids in sorted(ex.launches, key=lambda x: x[0]) for rid in rids]
    assert order == sorted(order)
    # without the cap the same burst forms longer batches
    clk2 = VirtualClock()
    ex2 = FakeExecutor(clk2, per_frame_s=1e-3)
    reqs2 = [Request(rid=r.rid, arrival=r.arrival, M=r.M, T=r.T, K=4, n=12) for r in reqs]
    Server(ex2, budget_bytes=1 << 40, n_streams=3, max_batch=64, clock=clk2).run(reqs2)
    assert max(len(r) for _, _, r in ex2.launches) > max(len(r) for _, _, r in ex.launches)
