"""Serving loop: continuous batching of matrix-product requests on one GPU.

Requests (C = A B with operands already resident on the device) arrive over
time.  The loop admits them first-come first-served whenever a slot is free
and the HBM budget has room for what the request needs while it runs (its
output C and its plan's workspace).  A slot is a HIP stream, so admitted
requests overlap on the device; a request finishing frees its slot and its
budget, and the next queued request is admitted at once, while the others
are still running (continuous batching, not a queue in front of one product
at a time).

The budget is enforced on the device, not only in the books: the GPU
executor allocates one arena of exactly the budget's size when it is built
and places every running request's output and workspace in it (first fit,
256-byte aligned, freed blocks merged with their neighbours).  A request is
admitted only when both blocks can be placed, so the executor's device
memory never exceeds the budget, whatever the mix and however long it runs.

Each request runs the library's product for its size: Strassen-Winograd with
the autotuner's levels and tile for its size class and dtype (float32 or the
split-bfloat16 refined dtype), the plain MFMA GEMM where the tuner says no
level pays.  Kernels use no atomics and plans depend only on (m, n, k,
dtype), so a request's result is bitwise the same alone and in any mix.

The admission and bookkeeping logic is independent of the GPU: ``Server``
drives an executor object (``GpuExecutor`` here, a simulated one in the
tests), so budget accounting, queueing, rejection and completion order are
tested on the host.
"""
import collections
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    m: int
    n: int
    k: int
    dtype: str            # "f32" or "bf16x3"
    arrival: float        # seconds from the start of the run
    A: object = None      # device operands (GpuExecutor) or None
    B: object = None
    C: object = None
    need_bytes: int = 0
    slot: int = -1
    t_admit: float = -1.0
    t_done: float = -1.0
    error: str = ""
    info: dict = field(default_factory=dict)

    @property
    def flops(self):
        return 2.0 * self.m * self.n * self.k

    @property
    def latency(self):
        return self.t_done - self.arrival


class Server:
    """First-come first-served admission under a slot count and an HBM budget."""

    def __init__(self, executor, hbm_budget_bytes, n_slots=4, clock=None, idle_sleep=20e-6):
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.n_slots = int(n_slots)
        self.clock = clock or time.perf_counter
        self.idle_sleep = idle_sleep
        self.reserved = 0
        self.peak_reserved = 0
        self.max_running = 0
        self.admit_order = []

    def run(self, requests):
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue = collections.deque()
        running = {}                       # slot -> request
        free = list(range(self.n_slots))[::-1]
        done = []
        t0 = self.clock()
        while pending or queue or running:
            now = self.clock() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                r.need_bytes = self.ex.need_bytes(r)
                if r.need_bytes > self.budget:
                    r.error = f"needs {r.need_bytes} bytes, budget is {self.budget}"
                    r.t_done = now
                    done.append(r)
                else:
                    queue.append(r)
                progressed = True
            for slot, r in list(running.items()):
                if self.ex.done(r):
                    r.t_done = self.clock() - t0
                    self.ex.release(r)
                    self.reserved -= r.need_bytes
                    del running[slot]
                    free.append(slot)
                    done.append(r)
                    progressed = True
            while (queue and free and self.reserved + queue[0].need_bytes <= self.budget and
                   self._reserve(queue[0])):
                r = queue.popleft()
                r.slot = free.pop()
                self.reserved += r.need_bytes
                self.peak_reserved = max(self.peak_reserved, self.reserved)
                assert self.reserved <= self.budget
                r.t_admit = self.clock() - t0
                try:
                    self.ex.submit(r)
                except Exception as e:          # a failed request frees its slot
                    r.error = str(e)
                    r.t_done = self.clock() - t0
                    self.ex.release(r)
                    self.reserved -= r.need_bytes
                    free.append(r.slot)
                    done.append(r)
                    continue
                running[r.slot] = r
                self.admit_order.append(r.rid)
                self.max_running = max(self.max_running, len(running))
                progressed = True
            if not progressed:
                if not running and not queue and pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                elif self.idle_sleep:
                    time.sleep(self.idle_sleep)
        wall = self.clock() - t0
        return done, wall

    def _reserve(self, r):
        """Ask the executor to place the request's memory (executors without
        an arena always can)."""
        reserve = getattr(self.ex, "reserve", None)
        return True if reserve is None else bool(reserve(r))


class Arena:
    """First-fit allocator of byte ranges in a buffer of ``capacity`` bytes:
    host bookkeeping only (offsets), ``align``-byte aligned blocks, freed
    blocks merged with free neighbours."""

    def __init__(self, capacity, align=256):
        self.capacity = int(capacity)
        self.align = int(align)
        self.free_list = [(0, self.capacity)] if self.capacity > 0 else []   # sorted (offset, size)
        self.used = {}                                                      # offset -> size

    def alloc(self, nbytes):
        size = max(self.align, -(-int(nbytes) // self.align) * self.align)
        for i, (off, sz) in enumerate(self.free_list):
            if sz >= size:
                if sz == size:
                    del self.free_list[i]
                else:
                    self.free_list[i] = (off + size, sz - size)
                self.used[off] = size
                return off
        return None

    def free(self, off):
        size = self.used.pop(off)
        fl = self.free_list
        i = 0
        while i < len(fl) and fl[i][0] < off:
            i += 1
        fl.insert(i, (off, size))
        if i + 1 < len(fl) and fl[i][0] + fl[i][1] == fl[i + 1][0]:       # merge with the next
            fl[i] = (fl[i][0], fl[i][1] + fl[i + 1][1])
            del fl[i + 1]
        if i > 0 and fl[i - 1][0] + fl[i - 1][1] == fl[i][0]:             # and the previous
            fl[i - 1] = (fl[i - 1][0], fl[i - 1][1] + fl[i][1])
            del fl[i]

    @property
    def used_bytes(self):
        return sum(self.used.values())


def summarize(done, wall):
    ok = [r for r in done if not r.error]
    lat = sorted(r.latency * 1e3 for r in ok)

    def pct(q):
        if not lat:
            return float("nan")
        i = min(len(lat) - 1, max(0, int(round(q / 100.0 * (len(lat) - 1)))))
        return lat[i]
    flops = sum(r.flops for r in ok)
    return {"requests": len(done), "completed": len(ok), "rejected": len(done) - len(ok),
            "p50_ms": round(pct(50), 3), "p99_ms": round(pct(99), 3), "max_ms": round(pct(100), 3),
            "req_per_s": round(len(ok) / wall, 2) if wall > 0 else 0.0,
            "tflops": round(flops / wall / 1e12, 3) if wall > 0 else 0.0, "wall_s": round(wall, 4)}


class GpuExecutor:
    """Runs requests on the current GPU through libmm, one HIP stream per slot,
    every running request's output and workspace placed in one device arena
    of ``arena_bytes`` (give it the server's budget).

    Outputs are views into the arena while their request runs.  When a
    request completes, its blocks return to the arena; its output is first
    copied out (and the copy waited for) if ``keep_outputs`` is set or its id
    is in ``keep_rids``, else it is dropped (the caller has consumed it)."""

    def __init__(self, n_slots, arena_bytes, device=None, keep_outputs=True):
        import torch
        from . import api  # noqa: F401  (loads libmm before any stream is made)
        self.torch = torch
        self.keep_outputs = keep_outputs
        self.keep_rids = set()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_slots)]
        self.arena = Arena(arena_bytes)
        self.buf = torch.empty(max(int(arena_bytes), 256), dtype=torch.uint8, device=self.device)
        self.events = {}
        self.blocks = {}

    def choice(self, r):
        from . import tuner
        ch = tuner.choose(r.m, r.n, r.k, r.dtype)
        algo = "winograd" if ch["levels"] > 0 else "naive"
        return (algo, ch["levels"], ch["tile"], bool(ch.get("overlap", False)), bool(ch.get("leaf_u", False)),
                bool(ch.get("trans_b", False)), ch.get("split_k") if ch["levels"] == 0 else None)

    def plan(self, r):
        from . import api
        algo, levels, tile, overlap, leaf_u, trans_b, split_k = self.choice(r)
        return api.get_plan(algo, "grouped" if levels else "auto", r.m, r.n, r.k, 1, levels, r.dtype,
                            max(r.k, 1), max(r.n, 1), max(r.n, 1), False, self.device, tile,
                            overlap=overlap, leaf_u=leaf_u, trans_b=trans_b, split_k=split_k)

    def _sizes(self, r):
        esz = 8 if r.dtype == "f64" else 4
        return r.m * r.n * esz, self.plan(r).ws_bytes

    def need_bytes(self, r):
        c, w = self._sizes(r)
        a = self.arena.align
        return -(-c // a) * a + (-(-w // a) * a if w else 0)

    def reserve(self, r):
        """Place the request's output and workspace in the arena (False, with
        nothing held, when they do not fit now)."""
        c, w = self._sizes(r)
        oc = self.arena.alloc(c)
        if oc is None:
            return False
        ow = None
        if w:
            ow = self.arena.alloc(w)
            if ow is None:
                self.arena.free(oc)
                return False
        self.blocks[r.rid] = (oc, c, ow, w)
        return True

    def submit(self, r):
        torch = self.torch
        s = self.streams[r.slot]
        p = self.plan(r)
        if r.rid not in self.blocks and not self.reserve(r):
            raise RuntimeError("request does not fit in the arena")
        oc, c, ow, w = self.blocks[r.rid]
        tdt = torch.float32 if r.dtype != "f64" else torch.float64
        r.C = self.buf[oc:oc + c].view(tdt).view(r.m, r.n)
        ws = self.buf[ow:ow + w] if w else None
        s.wait_stream(torch.cuda.current_stream(self.device))   # operands were made there
        p(r.A, r.B, r.C, ws=ws, stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        self.events[r.rid] = ev
        r.info = {"algo": p.algo, "levels": p.info["levels"]}

    def done(self, r):
        return self.events[r.rid].query()

    def release(self, r):
        ev = self.events.pop(r.rid, None)
        if r.C is not None and (self.keep_outputs or r.rid in self.keep_rids) and ev is not None:
            # copy the output out of the arena before its block is reused
            cur = self.torch.cuda.current_stream(self.device)
            cur.wait_event(ev)
            r.C = r.C.clone()
            cur.synchronize()
        else:
            r.C = None
        blk = self.blocks.pop(r.rid, None)
        if blk is not None:
            self.arena.free(blk[0])
            if blk[2] is not None:
                self.arena.free(blk[2])


def make_requests(trace, device, keep_outputs=True):
    """Device operands for a serving trace (see inputs.serving_trace); made
    before the run, so their creation is not on any request's latency path."""
    import torch
    reqs = []
    for i, t in enumerate(trace):
        g = torch.Generator(device=device)
        g.manual_seed(int(t["seed"]))
        n = int(t["n"])
        A = torch.rand((n, n), generator=g, device=device, dtype=torch.float32) * 2 - 1
        B = torch.rand((n, n), generator=g, device=device, dtype=torch.float32) * 2 - 1
        reqs.append(Request(rid=i, m=n, n=n, k=n, dtype=t["dtype"], arrival=float(t["t"]), A=A, B=B))
    return reqs
