"""Host-side checks of the serving loop's admission and bookkeeping (no GPU):
a simulated executor stands in for the device."""
import time

import pytest

from paper_2309_00628_amd import inputs
from paper_2309_00628_amd.serving import Request, Server, summarize


class FakeExecutor:
    """Each request 'runs' for a time proportional to its flops."""

    def __init__(self, rate_flops=5e13, ws_bytes=lambda r: 1 << 20, fail_ids=()):
        self.rate = rate_flops
        self.ws = ws_bytes
        self.fail_ids = set(fail_ids)
        self.end = {}
        self.running = set()
        self.max_concurrent = 0

    def need_bytes(self, r):
        return r.m * r.n * 4 + self.ws(r)

    def submit(self, r):
        if r.rid in self.fail_ids:
            raise RuntimeError("injected launch failure")
        self.end[r.rid] = time.perf_counter() + r.flops / self.rate
        self.running.add(r.rid)
        self.max_concurrent = max(self.max_concurrent, len(self.running))

    def done(self, r):
        return time.perf_counter() >= self.end[r.rid]

    def release(self, r):
        self.running.discard(r.rid)


def trace(count, qps, seed=0):
    t = inputs.serving_trace(count, seed, qps, bands=((0.7, 64, 256), (0.3, 256, 512)))
    return [Request(rid=i, m=x["n"], n=x["n"], k=x["n"], dtype=x["dtype"], arrival=x["t"])
            for i, x in enumerate(t)]


def test_all_requests_complete_in_fifo_order_within_budget():
    reqs = trace(60, qps=2000)
    ex = FakeExecutor()
    budget = 6 << 20
    srv = Server(ex, budget, n_slots=4)
    done, wall = srv.run(reqs)
    assert len(done) == 60 and all(not r.error for r in done)
    assert srv.peak_reserved <= budget
    assert srv.max_running <= 4 and ex.max_concurrent <= 4
    arrival_order = [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert srv.admit_order == arrival_order          # first come, first served
    assert all(r.t_admit >= r.arrival - 1e-9 and r.t_done >= r.t_admit for r in done)
    s = summarize(done, wall)
    assert s["completed"] == 60 and s["p50_ms"] <= s["p99_ms"]


def test_requests_overlap_when_they_arrive_together():
    reqs = [Request(rid=i, m=512, n=512, k=512, dtype="f32", arrival=0.0) for i in range(8)]
    ex = FakeExecutor(rate_flops=1e11)
    srv = Server(ex, 1 << 40, n_slots=4)
    done, _ = srv.run(reqs)
    assert srv.max_running == 4            # continuous batching: slots fill up at once
    assert len(done) == 8


def test_budget_limits_concurrency():
    reqs = [Request(rid=i, m=512, n=512, k=512, dtype="f32", arrival=0.0) for i in range(6)]
    ex = FakeExecutor(rate_flops=1e11, ws_bytes=lambda r: 0)
    one = 512 * 512 * 4
    srv = Server(ex, 2 * one, n_slots=8)
    done, _ = srv.run(reqs)
    assert srv.max_running == 2 and srv.peak_reserved == 2 * one
    assert len(done) == 6


def test_oversized_request_is_rejected_not_stalled():
    reqs = [Request(rid=0, m=4096, n=4096, k=64, dtype="f32", arrival=0.0),
            Request(rid=1, m=64, n=64, k=64, dtype="f32", arrival=0.0)]
    srv = Server(FakeExecutor(), 2 << 20, n_slots=2)
    done, _ = srv.run(reqs)
    by = {r.rid: r for r in done}
    assert "budget" in by[0].error and not by[1].error


def test_failed_launch_becomes_an_error_response_and_frees_its_slot():
    reqs = trace(20, qps=5000, seed=3)
    srv = Server(FakeExecutor(fail_ids={2, 7}), 1 << 30, n_slots=1)
    done, _ = srv.run(reqs)
    errs = sorted(r.rid for r in done if r.error)
    assert errs == [2, 7]
    assert len(done) == 20 and srv.reserved == 0


def test_arena_blocks_never_overlap_and_merge_back():
    """The serving arena's first-fit allocator on a random sequence of
    allocations and frees: blocks are aligned, inside the buffer, disjoint,
    and once everything is freed the free list is one block again."""
    import random

    from paper_2309_00628_amd.serving import Arena
    rnd = random.Random(5)
    a = Arena(1 << 20, align=256)
    live = {}
    for step in range(4000):
        if live and (rnd.random() < 0.45 or len(live) > 40):
            off = rnd.choice(sorted(live))
            a.free(off)
            del live[off]
        else:
            nb = rnd.choice([1, 255, 256, 257, 4096, 65536, 300000])
            off = a.alloc(nb)
            if off is None:
                assert sum(sz for _, sz in a.free_list) < 1 << 20
                continue
            size = -(-nb // 256) * 256
            assert off % 256 == 0 and 0 <= off and off + size <= 1 << 20
            for o, s in live.items():
                assert off + size <= o or o + s <= off
            live[off] = size
        assert a.used_bytes == sum(live.values())
    for off in list(live):
        a.free(off)
    assert a.free_list == [(0, 1 << 20)] and a.used_bytes == 0


def test_admission_waits_when_the_arena_is_fragmented():
    """An executor that can refuse to place a request (fragmented arena):
    the server keeps it queued, in order, until a completion makes room."""
    class Fragmented(FakeExecutor):
        def __init__(self):
            super().__init__(rate_flops=1e11, ws_bytes=lambda r: 0)
            self.refusals = 0

        def reserve(self, r):
            # refuse while anything is running
            if self.running:
                self.refusals += 1
                return False
            return True

    reqs = [Request(rid=i, m=256, n=256, k=256, dtype="f32", arrival=0.0) for i in range(5)]
    ex = Fragmented()
    srv = Server(ex, 1 << 30, n_slots=4)
    done, _ = srv.run(reqs)
    assert len(done) == 5 and all(not r.error for r in done)
    assert srv.max_running == 1 and ex.refusals > 0
    assert srv.admit_order == [0, 1, 2, 3, 4]
