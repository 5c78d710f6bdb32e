#!/usr/bin/env python3
"""Benchmark: effective TFLOP/s (2mnk/t) of Strassen-Winograd against the
plain MFMA GEMM of the same library, on one MI355X, with the relative error
against the float64 oracle and p50/p99 step latency.

Workload (one "step" = one whole product, every kernel of the path):
square float32 C = A x B, n = 8192, entries i.i.d. U[-1, 1] from a fixed
seed, Strassen-Winograd with two levels (grouped schedule, the autotuner's
options for two levels).  The plain MFMA GEMM (mm_naive) and hipBLASLt
(torch.matmul, context only) run the same product.  Inputs are resident in
HBM before timing starts.

Timing: the GPU first runs the plain product for a fixed wall time (clocks
settle under MFMA load), then W untimed steps of each contender, then the K
timed steps of each contender in R interleaved rounds (the order rotates
from round to round, so no contender always runs first).  ``value`` is
2 n^3 K over the summed wall time of the K Winograd steps; per-round rates
and their medians are reported for all three.

Printed: one JSON line (rank 0).  ``roofline`` is for the dominant kernel,
the grouped MFMA leaf GEMM launch with the most flops: algorithmic flops of
one launch (its leaf products' 2mnk) over that launch's average duration,
measured with HIP events recorded around each launch on the stream the
kernels run on.  ``cpu_baseline`` is the oracle (the double-precision triple
loop) timed on the host on samples of output rows.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_BF16_TFLOPS = 2516.6  # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rounds", type=int, default=5, help="interleaved timing rounds")
    ap.add_argument("--warm-seconds", type=float, default=2.5,
                    help="wall time of plain products run before anything is timed")
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--sched", default="grouped")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline and error check")
    ap.add_argument("--no-extra", action="store_true", help="skip the n=4096 / n=3000 side runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-problem batch")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the depth-first schedules (Two Temp, In-Place, Strassen DFS) at n=4096")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop runs")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the n=8192 split-bfloat16 precision runs")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="host time for the oracle baseline table (all sizes, 1 thread and all cores)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the Winograd steps of the headline (for rocprofv3 runs)")
    ap.add_argument("--profile-set", choices=("gemm", "bf16x3"), default=None,
                    help="for rocprofv3 runs at --n: 'gemm' = the plain float32 product, the fastest "
                         "Winograd plan and torch.matmul (hipBLASLt); 'bf16x3' = the refined "
                         "split-bfloat16 Winograd L=2 and plain products on row-scaled Gaussians")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB float32 buffer 3 times (calibrates HBM byte counters)")
    return ap.parse_args()


def _events(torch, n, stream):
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    for e in evs:              # create the underlying HIP events
        e.record(stream)
    return evs


class Contender:
    """One product to time: ``step()`` enqueues one whole product on the
    current stream."""

    def __init__(self, name, step, plan=None, C=None):
        self.name, self.step, self.plan, self.C = name, step, plan, C
        self.wall_s = 0.0
        self.steps = 0
        self.step_ms = []
        self.round_tflops = []


def plan_contender(torch, L, name, plan, A, B, C, ws):
    lib = L.load()
    wsp, wsb = (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)
    args = (plan._ptr, A.data_ptr(), B.data_ptr(), C.data_ptr(), wsp, wsb)

    def step():
        L.check(lib.mm_plan_execute(*args, torch.cuda.current_stream().cuda_stream))
    c = Contender(name, step, plan, C)
    c.args = args
    c.ws = ws          # the plan reads and writes it: keep it allocated
    return c


def warm_gpu(torch, step, seconds):
    """Run ``step`` until ``seconds`` of wall time have passed (the GPU's
    clocks settle under sustained MFMA load)."""
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        for _ in range(4):
            step()
        torch.cuda.synchronize()


def timed_rounds(torch, contenders, steps, rounds, flops):
    """``steps`` timed steps of every contender, split over ``rounds``
    interleaved rounds; in round r the contenders run in an order rotated by
    r.  Each round's block of steps is bracketed by device synchronisations;
    events around every step give the per-step latencies."""
    s = torch.cuda.current_stream()
    per_round = [steps // rounds + (1 if r < steps % rounds else 0) for r in range(rounds)]
    for r, cnt in enumerate(per_round):
        if cnt == 0:
            continue
        order = contenders[r % len(contenders):] + contenders[:r % len(contenders)]
        for c in order:
            evs = [_events(torch, 2, s) for _ in range(cnt)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for e0, e1 in evs:
                e0.record(s)
                c.step()
                e1.record(s)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c.wall_s += dt
            c.steps += cnt
            c.step_ms += [e0.elapsed_time(e1) for e0, e1 in evs]
            c.round_tflops.append(flops * cnt / dt / 1e12)
    for c in contenders:
        c.tflops = flops * c.steps / c.wall_s / 1e12
        c.wall_ms = c.wall_s * 1e3 / c.steps
        c.median_round_tflops = sorted(c.round_tflops)[len(c.round_tflops) // 2]


def launch_times(torch, L, c, steps):
    """Per-launch durations of a plan contender: ``steps`` more products,
    each with events before and after every launch, recorded on the stream
    that launch runs on (mm_plan_execute_timed).  Returns (per-launch ms
    lists, launch kinds)."""
    import ctypes
    lib = L.load()
    s = torch.cuda.current_stream()
    nops = c.plan.info["launches"]
    nev = 2 * nops
    evsets = [_events(torch, nev, s) for _ in range(steps)]
    ptrs = [(ctypes.c_void_p * nev)(*[e.cuda_event for e in evs]) for evs in evsets]
    torch.cuda.synchronize()
    for i in range(steps):
        L.check(lib.mm_plan_execute_timed(*c.args, s.cuda_stream, ptrs[i], nev))
    torch.cuda.synchronize()
    per_op = [[evs[2 * j].elapsed_time(evs[2 * j + 1]) for evs in evsets] for j in range(nops)]
    kinds = [lib.mm_plan_op_kind(c.plan._ptr, j) for j in range(nops)]
    return per_op, kinds


def time_plan(torch, api, L, plan, A, B, C, ws, steps, warmup):
    """Warm-up steps, then exactly ``steps`` timed steps with one event before
    and one after each step (wall time and per-step latencies), then
    ``steps`` more with events around every launch (per-launch durations).
    An event between two launches of a step delays the second one a little,
    so the step time is taken without them.
    Returns (wall ms per step, per-step ms list, per-launch ms lists, kinds)."""
    c = plan_contender(torch, L, "plan", plan, A, B, C, ws)
    for _ in range(warmup):
        c.step()
    timed_rounds(torch, [c], steps, 1, 2.0)
    per_op, kinds = launch_times(torch, L, c, steps)
    return c.wall_ms, c.step_ms, per_op, kinds


# Element-wise recipes of the plan listing (EwKind in csrc/desc.h).
EW_RECIPES = {0: "copy", 1: "add", 2: "sub", 3: "winograd S", 4: "winograd T", 5: "winograd U", 11: "zero",
              15: "winograd U (accumulate)", 17: "strassen S", 18: "strassen T", 19: "strassen U", 22: "k-split sum"}


def plan_launches(plan, esz):
    """Per launch of a plan (in launch order): its kind ("EW", "GEMM",
    "WINO", "FORK", "JOIN"), stream (0 caller's, 1 auxiliary), algorithmic
    flops (GEMM: 2 m n k per leaf product; WINO: seven such products per
    subproblem) and algorithmic HBM bytes (EW: every valid input element read
    once, every valid output element written once), read off the plan
    listing."""
    out, flops, nbytes, ekinds = [], 0.0, 0.0, set()
    for line in plan.describe().splitlines():
        w = line.split()
        if not w:
            continue
        if line in ("FORK", "JOIN"):
            out.append(dict(kind=line, stream=0, flops=0.0, bytes=0.0))
        elif w[0] == "LAUNCH":
            out.append(dict(kind=w[1], stream=1 if w[-1] == "aux" else 0, flops=flops, bytes=nbytes,
                            grid=int(w[3]) if len(w) > 3 else 0,
                            cfg=int(w[4]) if w[1] in ("GEMM", "WINO") and len(w) > 4 else None,
                            flags=w[5:], recipes=sorted(ekinds)))
            flops, nbytes, ekinds = 0.0, 0.0, set()
        elif w[0] == "GEMM":
            m, n, k = map(int, w[1:4])
            flops += 2.0 * m * n * k
        elif w[0] == "WINO":
            m, n, k = map(int, w[1:4])
            flops += 7 * 2.0 * m * n * k
        elif w[0] == "EW2":
            # two levels in one pass: S/T read the parent block and write three
            # quarters of each upper sum and the 28 lower sums; U reads the 49
            # lower products and writes the four C quadrants
            kind, R, C = map(int, w[1:4])
            ekinds.add(("winograd S" if kind == 0 else "winograd T" if kind == 1 else "winograd U")
                       + " (two levels)")
            blk = R * C * esz
            nbytes += (16 + 12 + 28) * blk if kind in (0, 1) else (49 + 16) * blk
        elif w[0] in ("EW", "TRANS"):
            ekinds.add(EW_RECIPES.get(int(w[1]), w[1]) if w[0] == "EW" else "transpose")
            _, ins, outs = [x.strip() for x in line.split("|")]
            for tok in (ins + " " + outs).split():
                if tok != "-":
                    f = tok.split(":")
                    nbytes += int(f[5]) * int(f[6]) * esz
    return out


def tuned_leaf(tuner, n, levels, dtype="f32"):
    """The autotuner's (tile, overlap, leaf_u, trans_b) choice for an n x n x n
    product at this level count (planner defaults when the tuner has not
    measured that level count for the size class)."""
    o = tuner.options_at(n, n, n, dtype, levels)
    return o if o is not None else (None, False, False, False)


def tuned_plain(tuner, n, dtype="f32"):
    """The autotuner's fastest (tile, k split) for the plain n x n x n product."""
    ch = tuner.choose(n, n, n, dtype)
    if ch["source"] != "tuned":
        return None, None
    if ch.get("best_plain"):
        return ch["best_plain"]["tile"], ch["best_plain"].get("split_k")
    return (ch["tile"], ch.get("split_k")) if ch["levels"] == 0 else (None, None)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def run_product(torch, api, L, algo, sched, n, levels, A, B, steps, warmup, dtype="f32", tile=None,
                overlap=False, leaf_u=False, trans_b=False, split_k=None, pad_to=None):
    plan = api.Plan(algo, sched, n, n, n, cutoff=1, levels=levels, dtype=dtype, tile=tile, overlap=overlap,
                    leaf_u=leaf_u, trans_b=trans_b, split_k=split_k, pad_to=pad_to)
    ws = torch.empty(max(plan.ws_bytes, 256), dtype=torch.uint8, device=A.device)
    C = torch.empty((n, n), dtype=A.dtype, device=A.device)
    wall, step_ms, per_op, kinds = time_plan(torch, api, L, plan, A, B, C, ws, steps, warmup)
    return dict(plan=plan, C=C, wall_ms=wall, p50=pct(step_ms, 50), p99=pct(step_ms, 99),
                per_op=per_op, kinds=kinds, tflops=2.0 * n ** 3 / (wall * 1e-3) / 1e12)


def source_digest():
    """SHA-256 over the library sources (csrc/ and include/) and the build
    script (compiler flags), to tell whether stored counter results were
    taken with the kernels built now."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for d in ("paper_2309_00628_amd/csrc", "include"):
        for name in sorted(os.listdir(os.path.join(root, d))):
            if name.endswith((".hip", ".h", ".cpp")):
                h.update(name.encode())
                with open(os.path.join(root, d, name), "rb") as f:
                    h.update(f.read())
    with open(os.path.join(root, "paper_2309_00628_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


# Template arguments of the float32 leaf kernels per tile configuration
# (MM_PLAN_TILE in include/mm.h): BM, BN, BKC, WGM, WGN.
GEMM_F32_TILES = {0: (128, 128, 8, 4, 2), 1: (256, 128, 8, 4, 2), 2: (128, 256, 8, 2, 4), 3: (256, 256, 8, 4, 2),
                  4: (64, 128, 8, 2, 2), 5: (128, 64, 8, 2, 2), 6: (256, 128, 4, 2, 2), 7: (128, 128, 4, 2, 2),
                  8: (64, 64, 8, 2, 2)}
WINO_TILES = {0: (128, 128, 8, 2, 2), 1: (128, 128, 8, 4, 2), 2: (64, 128, 8, 2, 2)}


def launch_kernel_name(lau):
    """The name rocprofv3 gives the kernel of a float32 leaf launch."""
    if lau["kind"] == "WINO":
        t = WINO_TILES.get(lau["cfg"], WINO_TILES[0])
        return "gemm_wino_kernel<%d, %d, %d, %d, %d, %s>" % (t + ("true" if "fused" in lau["flags"] else "false",))
    t = GEMM_F32_TILES.get(lau["cfg"], GEMM_F32_TILES[0])
    return "gemm_kernel<float, %d, %d, %d, %d, %d, %s>" % (t + ("true" if "bt" in lau["flags"] else "false",))


def measured_traffic(kernel, grid):
    """HBM bytes per launch of (kernel, grid) from the rocprofv3 counter
    summary in profiles/hbm_traffic.json (kernels named with their template
    arguments), or None when there is none or it was taken with other kernel
    sources."""
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic.json")
    try:
        with open(p) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_sha256") != source_digest():
        return None
    for e in data.get("launches", []):
        if e["kernel"] == kernel and e["grid"] == grid:
            return e["bytes_per_launch"]
    return None


def gemm_roofline(res, n, traffic=True):
    """Roofline of the dominant kernel: the leaf-product launch (plain GEMM
    group or fused last Winograd level) with the most flops, on the caller's
    stream (not sharing the GPU with an overlapped S/T pass).  ``traffic``:
    look up its measured HBM bytes (the counter summary covers the headline
    Winograd plan only)."""
    launches = plan_launches(res["plan"], 4)
    best, kind, grid, top = None, 1, None, None
    for lau, d, k in zip(launches, res["per_op"], res["kinds"]):
        if k in (1, 4) and (best is None or lau["flops"] > best[0]):
            kind, grid, top = k, lau["grid"], lau
            best = (lau["flops"], sum(d) / len(d))
    flops, avg_ms = best if best else (0.0, float("nan"))
    achieved = flops / (avg_ms * 1e-3) / 1e12
    kname = launch_kernel_name(top) if top is not None else None
    return dict(bound="mfma", achieved=round(achieved, 2), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / PEAK_FP32_TFLOPS, 4),
                traffic=measured_traffic(kname, grid) if traffic and kname else None,
                kernel=kname + (" (last level: products + U in registers)" if kind == 4
                                else " (grouped leaf products)") if kname else None,
                flops_per_launch=flops, avg_launch_ms=round(avg_ms, 4), grid=grid)


def ew_bandwidth(res, n):
    """Achieved HBM rate of the element-wise launches (algorithmic bytes);
    launches on the auxiliary stream share the GPU with leaf products."""
    launches = plan_launches(res["plan"], 4)
    out = []
    for lau, d, k in zip(launches, res["per_op"], res["kinds"]):
        if k % 8 in (0, 6) or k in (18, 26):  # element-wise, transposing and two-level passes
            ms = sum(d) / len(d)
            gbs = lau["bytes"] / (ms * 1e-3) / 1e9
            out.append(dict(recipes=lau["recipes"], stream="aux" if k in (8, 14, 26) else "main", bytes=lau["bytes"],
                            ms=round(ms, 4),
                            gbs=round(gbs, 1), hbm_frac=round(gbs / PEAK_HBM_GBS, 3)))
    return out


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(inputs, big, seconds):
    """The oracle (double-precision triple loop) timed on the host: at
    n = 512, 3000, 4096 and the headline n, with one thread and with all of
    them, three runs each over a sample of output rows sized so that the
    whole table takes about ``seconds`` of host time.  ``big`` = (A, B) of
    the headline product.  ``value`` is the all-core rate at the headline n."""
    import numpy as np
    from oracle import naive
    nth = naive.max_threads()
    nbig = big[0].shape[0]
    sizes = sorted({512, 3000, 4096, nbig})
    per_run = seconds / (len(sizes) * 2 * 3)
    table = []
    for n in sizes:
        A_np, B_np = big if n == nbig else inputs.pair("uniform", n, n, n, 0, np.float32)
        for th in (1, nth):
            # calibrate the row count so one run takes about per_run seconds
            r0 = th
            t0 = time.perf_counter()
            naive.gemm_rows(A_np, B_np, np.arange(r0), threads=th)
            dt = max(time.perf_counter() - t0, 1e-4)
            rows = int(min(n, max(th, r0 * per_run / dt)))
            rows = max(th, rows // th * th) if rows < n else n
            sample = np.linspace(0, n - 1, rows).astype(np.int64)
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                naive.gemm_rows(A_np, B_np, sample, threads=th)
                ts.append(time.perf_counter() - t0)
            p50, p99 = pct(ts, 50), pct(ts, 99)
            table.append(dict(n=n, threads=th, rows=rows, runs=3, p50_s=round(p50, 4), p99_s=round(p99, 4),
                              gflops=round(2.0 * rows * n * n / p50 / 1e9, 3)))
            print(f"# oracle n={n} threads={th}: {table[-1]}", file=sys.stderr, flush=True)
    head = [t for t in table if t["n"] == nbig and t["threads"] == nth][0]
    return dict(value=round(head["gflops"] / 1e3, 6), unit="TFLOP/s", cores=nth, kind="oracle",
                cpu=cpu_model(),
                sample=f"{head['rows']} of {nbig} output rows of the n={nbig} product per run, 3 runs, "
                       f"{nth} threads (p50 run {head['p50_s']} s); the table gives n = "
                       f"{', '.join(str(s) for s in sizes)} at 1 and {nth} threads",
                table=table)


def sample_rows(n, count=64):
    """Output rows checked against the oracle: ``count`` rows spread over
    the matrix, always including the first and the last."""
    import numpy as np
    return np.unique(np.r_[0, np.linspace(0, n - 1, count).astype(np.int64), n - 1])


def rel_err(C, rows, ref):
    """Relative Frobenius error of C's rows ``rows`` against the oracle's."""
    import numpy as np
    import torch
    got = C[torch.from_numpy(rows).to(C.device)].double().cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def oracle_rows(A_np, B_np, rows):
    from oracle import naive
    return naive.gemm_rows(A_np, B_np, rows)


def profile_set(torch, api, L, inputs, tuner, args):
    """Short runs of a fixed set of products for rocprofv3 (--profile-set)."""
    import numpy as np
    n = args.n
    out = {"profile_set": args.profile_set, "n": n}
    if args.profile_set == "gemm":
        A, B = [torch.from_numpy(x).cuda() for x in inputs.pair("uniform", n, n, n, 0, np.float32)]
        pt, pk = tuned_plain(tuner, n)
        p = run_product(torch, api, L, "naive", "auto", n, 0, A, B, args.steps, args.warmup, tile=pt, split_k=pk)
        out["plain_tflops"] = round(p["tflops"], 2)
        ch = tuner.choose(n, n, n, "f32")
        rec = ch.get("best_recursive") if ch["source"] == "tuned" else None
        lv = ch["levels"] if ch["levels"] > 0 else (rec["levels"] if rec else 1)
        t, o, u, tb = tuned_leaf(tuner, n, lv)
        w = run_product(torch, api, L, "winograd", "grouped", n, lv, A, B, args.steps, args.warmup, tile=t,
                        overlap=o, leaf_u=u, trans_b=tb)
        out["winograd"] = {"levels": lv, "tflops": round(w["tflops"], 2)}
        torch.backends.cuda.matmul.allow_tf32 = False
        C = torch.empty((n, n), device="cuda")
        for _ in range(args.warmup):
            torch.matmul(A, B, out=C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            torch.matmul(A, B, out=C)
        torch.cuda.synchronize()
        out["hipblaslt_tflops"] = round(2.0 * n ** 3 * args.steps / (time.perf_counter() - t0) / 1e12, 2)
    else:
        A = torch.from_numpy(inputs.gauss_rowscaled((n, n), 20)).cuda()
        B = torch.from_numpy(inputs.gauss_rowscaled((n, n), 21)).cuda()
        for name, algo, lv in (("winograd_L2", "winograd", 2), ("plain", "naive", 0)):
            r = run_product(torch, api, L, algo, "grouped" if lv else "auto", n, lv, A, B, args.steps,
                            args.warmup, dtype="bf16x3")
            out[name] = round(r["tflops"], 2)
        out["hipblaslt_bf16"] = bf16_library_rate(torch, A, B, args.steps, args.warmup)["tflops"]
    print(json.dumps(out), flush=True)


def bf16_library_rate(torch, A, B, steps=10, warmup=5):
    """hipBLASLt's bfloat16 GEMM (torch.matmul, one bfloat16 product per
    output, float32 accumulation) on the same operands rounded to bfloat16:
    the MFMA rate the library sustains on this chip with the bfloat16
    matrix cores busy, beside the split-bfloat16 leaves' six products."""
    n = A.shape[0]
    Ab, Bb = A.to(torch.bfloat16).contiguous(), B.to(torch.bfloat16).contiguous()
    Cb = torch.empty((n, n), dtype=torch.bfloat16, device=A.device)
    for _ in range(warmup):
        torch.matmul(Ab, Bb, out=Cb)
    ts = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.matmul(Ab, Bb, out=Cb)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = statistics.median(ts)
    tf = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    return {"tflops": round(tf, 2), "p50_ms": round(ms, 4), "frac_of_bf16_peak": round(tf / PEAK_BF16_TFLOPS, 4)}


def leaf_roofline(res, dt):
    """Roofline of a product's dominant leaf launch; the split-bfloat16 leaves
    run six bfloat16 MFMA products per float product, against the BF16 peak."""
    rl = gemm_roofline(res, 0, traffic=False)
    if dt != "bf16x3":
        return rl
    lau = [x for x, k in zip(plan_launches(res["plan"], 4), res["kinds"]) if k in (1, 9)]
    top = max(lau, key=lambda x: x["flops"]) if lau else None
    bf = 6.0 * rl["flops_per_launch"]
    ach = bf / (rl["avg_launch_ms"] * 1e-3) / 1e12
    return dict(rl, achieved=round(ach, 2), peak=PEAK_BF16_TFLOPS, frac=round(ach / PEAK_BF16_TFLOPS, 4),
                flops_per_launch=bf, kernel=f"gemm_bf16x3_kernel (tile cfg {top['cfg'] if top else None}, "
                                            "6 bf16 products per leaf product)")


def bench_precision(torch, api, L, inputs, tuner, n=8192, steps=10, warmup=10, rows=48):
    """n = 8192, A and B Gaussian with rows scaled by 10^u, u ~ U[-3, 3]:
    split-bfloat16 refined leaves under two Winograd levels (and plain), the
    float32 Winograd and plain products beside them, each with its relative
    Frobenius error against the float64 oracle on a sample of rows."""
    import numpy as np
    from oracle import naive
    A_np = inputs.gauss_rowscaled((n, n), 20)
    B_np = inputs.gauss_rowscaled((n, n), 21)
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    sample = np.linspace(0, n - 1, rows).astype(np.int64)
    ref = naive.gemm_rows(A_np, B_np, sample)
    out = {"workload": f"square n={n}, Gaussian rows scaled by 10^U[-3,3]",
           "oracle_rows": rows}
    for name, algo, lv, dt in (("bf16x3_winograd_L2", "winograd", 2, "bf16x3"),
                               ("bf16x3_plain", "naive", 0, "bf16x3"),
                               ("f32_winograd_L2", "winograd", 2, "f32"),
                               ("f32_plain", "naive", 0, "f32")):
        if lv:
            tile, ov, lu, tb = tuned_leaf(tuner, n, lv, dt)
            sk = None
        else:
            (tile, sk), ov, lu, tb = tuned_plain(tuner, n, dt), False, False, False
        r = run_product(torch, api, L, algo, "grouped" if lv else "auto", n, lv, A, B, steps, warmup,
                        dtype=dt, tile=tile, split_k=sk, overlap=ov, leaf_u=lu, trans_b=tb)
        out[name] = {"tflops": round(r["tflops"], 3), "p50_ms": round(r["p50"], 4),
                     "rel_err": rel_err(r["C"], sample, ref), "tile": tile, "overlap": ov,
                     "roofline": leaf_roofline(r, dt)}
        print(f"# precision {name}: {out[name]}", file=sys.stderr, flush=True)
        del r
    out["speedup_bf16x3_winograd_vs_f32_plain"] = round(out["bf16x3_winograd_L2"]["tflops"] /
                                                        out["f32_plain"]["tflops"], 4)
    out["hipblaslt_bf16"] = bf16_library_rate(torch, A, B)
    print(f"# precision hipblaslt_bf16: {out['hipblaslt_bf16']}", file=sys.stderr, flush=True)
    return out


def bench_schedules(torch, api, L, A, B, n, rows=None, ref=None, steps=20, warmup=10):
    """The paper's schedules beside the grouped one at the headline size:
    Strassen-Winograd Two Temp (Table 2) and In-Place (Table 3), Strassen
    depth first with three temporaries, and both grouped, at one and two
    levels, with the workspace each needs.  The in-place schedule overwrites
    its operands, so it is timed on copies (its run time does not depend on
    the values) and its error is taken from one run on fresh copies."""
    out = {}
    for algo, sched in (("winograd", "two_temp"), ("winograd", "in_place"), ("winograd", "grouped"),
                        ("strassen", "dfs3"), ("strassen", "grouped")):
        for lv in (1, 2):
            clob = sched == "in_place"
            Ax, Bx = (A.clone(), B.clone()) if clob else (A, B)
            r = run_product(torch, api, L, algo, sched, n, lv, Ax, Bx, steps, warmup)
            e = {"tflops": round(r["tflops"], 3), "p50_ms": round(r["p50"], 4),
                 "workspace_mib": round(r["plan"].ws_bytes / 2 ** 20, 1)}
            if rows is not None:
                C = r["C"]
                if clob:
                    Ax.copy_(A)
                    Bx.copy_(B)
                    ws = torch.empty(max(r["plan"].ws_bytes, 256), dtype=torch.uint8, device=A.device)
                    r["plan"](Ax, Bx, C, ws)
                    torch.cuda.synchronize()
                e["rel_err"] = rel_err(C, rows, ref)
            out[f"{algo}_{sched}_L{lv}"] = e
            print(f"# schedule {algo} {sched} L={lv}: {e}", file=sys.stderr, flush=True)
            del r, Ax, Bx
    return out


def bench_fp64_small(torch, api, L, inputs, n=512, cutoff=64, steps=50, warmup=10):
    """float64, n = 512, uniform[-1, 1], recursion cutoff 64 (three levels):
    the plain product and each algorithm / schedule (the depth-first one
    also replayed from a captured hipGraph, which does not shorten it: its
    ~1400 small launches depend on one another, so the time is their GPU-side
    latency, not the host's launch cost), with the relative Frobenius error
    against the oracle's full product."""
    import numpy as np
    from oracle import naive
    A_np, B_np = inputs.pair("uniform", n, n, n, 0, np.float64)
    ref = naive.gemm(A_np, B_np)
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    out = {"workload": f"square fp64 n={n}, uniform[-1,1], cutoff {cutoff}"}
    for name, algo, sched, lv, graph in (("plain", "naive", "auto", 0, False),
                                         ("winograd_grouped", "winograd", "grouped", -1, False),
                                         ("winograd_two_temp", "winograd", "two_temp", -1, False),
                                         ("winograd_two_temp_graph", "winograd", "two_temp", -1, True),
                                         ("strassen_grouped", "strassen", "grouped", -1, False)):
        plan = api.Plan(algo, sched, n, n, n, cutoff=cutoff if lv else 1, levels=lv, dtype="f64", graph=graph)
        ws = torch.empty(max(plan.ws_bytes, 256), dtype=torch.uint8, device=A.device)
        C = torch.empty((n, n), dtype=torch.float64, device=A.device)
        wall, step_ms, _, _ = time_plan(torch, api, L, plan, A, B, C, ws, steps, warmup)
        got = C.cpu().numpy()
        out[name] = {"levels": plan.info.get("levels"), "tflops": round(2.0 * n ** 3 / (wall * 1e-3) / 1e12, 3),
                     "p50_ms": round(pct(step_ms, 50), 4),
                     "rel_err": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
    print(f"# fp64 n={n}: {out}", file=sys.stderr, flush=True)
    return out


def bench_d2(torch, api, L, inputs, tuner, with_ref=True):
    """Square float32 n = 4096 and n = 3000 (not a power of two; with L <= 3
    levels 3000 = 8 * 375 needs no padding beyond the vector width): the
    plain MFMA GEMM, then Strassen-Winograd and Strassen at one and two
    levels, and for n = 3000 Winograd padded to 3072 at one to three levels,
    each with its relative error against the oracle on sampled rows (first
    and last row included)."""
    import numpy as np
    out = {}
    arrays = {}
    for n2 in (4096, 3000):
        A2_np, B2_np = inputs.pair("uniform", n2, n2, n2, 1, np.float32)
        A2, B2 = torch.from_numpy(A2_np).cuda(), torch.from_numpy(B2_np).cuda()
        rows = sample_rows(n2)
        ref = oracle_rows(A2_np, B2_np, rows) if with_ref else None
        pt2, pk2 = tuned_plain(tuner, n2)
        p2 = run_product(torch, api, L, "naive", "auto", n2, 0, A2, B2, 20, 10, tile=pt2, split_k=pk2)
        e = {"plain": {"tflops": round(p2["tflops"], 3), "p99_ms": round(p2["p99"], 4)}}
        if with_ref:
            e["plain"]["rel_err"] = rel_err(p2["C"], rows, ref)
        for lv in (1, 2):
            t2, o2, u2, b2 = tuned_leaf(tuner, n2, lv)
            w2 = run_product(torch, api, L, "winograd", "grouped", n2, lv, A2, B2, 20, 10, tile=t2,
                             overlap=o2, leaf_u=u2, trans_b=b2)
            s2 = run_product(torch, api, L, "strassen", "grouped", n2, lv, A2, B2, 20, 10,
                             tile=None if u2 else t2)
            for name, r in ((f"winograd_L{lv}", w2), (f"strassen_L{lv}", s2)):
                e[name] = {"tflops": round(r["tflops"], 3), "p50_ms": round(r["p50"], 4),
                           "p99_ms": round(r["p99"], 4), "padded_order": r["plan"].info.get("M")}
                if with_ref:
                    e[name]["rel_err"] = rel_err(r["C"], rows, ref)
            e[f"winograd_L{lv}"]["speedup_vs_plain"] = round(w2["tflops"] / p2["tflops"], 4)
            del w2, s2
        if n2 == 3000:
            # the same product zero-padded (virtually) to 3072 = 3 x 2^10, so
            # that the leaves are multiples of the tile edges
            for lv in (1, 2, 3):
                r = run_product(torch, api, L, "winograd", "grouped", n2, lv, A2, B2, 20, 10, pad_to=1024)
                e[f"winograd_L{lv}_pad3072"] = {"tflops": round(r["tflops"], 3), "p50_ms": round(r["p50"], 4),
                                                "padded_order": r["plan"].info.get("M"),
                                                "speedup_vs_plain": round(r["tflops"] / p2["tflops"], 4)}
                if with_ref:
                    e[f"winograd_L{lv}_pad3072"]["rel_err"] = rel_err(r["C"], rows, ref)
                del r
        out[str(n2)] = e
        arrays[n2] = (A2_np, B2_np, A2, B2, rows, ref)
        print(f"# d2 n={n2}: {e}", file=sys.stderr, flush=True)
    return out, arrays


def bench_batched(torch, api, inputs, tuner, count=512, steps=10, warmup=3, seed=7, check=True):
    """512 independent float32 products, m, n, k log-uniform in [64, 2048]
    (multiples of 16), levels per size class from the tuner, run as one
    batched plan replayed from a hipGraph; the relative error of a sample of
    problems (sampled rows, every one against the oracle) is reported."""
    import numpy as np
    shapes = inputs.batched_shapes(count, seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    from paper_2309_00628_amd import _lib as L
    As, Bs, Cs = [], [], []
    for (m, n, k) in shapes:
        As.append(torch.rand((m, k), generator=g, device="cuda") * 2 - 1)
        Bs.append(torch.rand((k, n), generator=g, device="cuda") * 2 - 1)
        Cs.append(torch.empty((m, n), device="cuda"))
    levels = L.batched_levels(shapes)          # the library's tuned level count per size class
    flops = sum(2.0 * m * n * k for (m, n, k) in shapes)
    plan = api.BatchedPlan(As, Bs, Cs, graph=True)  # NULL levels: tuned per size class
    s = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, e0.elapsed_time(e1) / reps

    wall, dev = timed(plan, steps)
    out = {"workload": f"{count} fp32 products, m,n,k log-uniform in [64,2048] (x16), uniform[-1,1]",
           "tflops": round(flops / (wall * 1e-3) / 1e12, 3), "ms_per_batch": round(wall, 4),
           "device_ms_per_batch": round(dev, 4), "launches_per_batch": plan.info["launches"],
           "persistent": False, "levels_source": L.tuning_source() or "rule",
           "levels_histogram": {str(l): levels.count(l) for l in sorted(set(levels))}, "graph": True}
    if check:
        # every problem with a recursion level, the largest problems, and an
        # even spread over the rest
        vol = np.array([m * n * k for (m, n, k) in shapes])
        pick = set(np.argsort(-vol)[:4].tolist()) | {i for i, l in enumerate(levels) if l > 0}
        pick |= set(np.linspace(0, count - 1, 12).astype(int).tolist())
        errs = []
        for i in sorted(pick)[:32]:
            m, n, k = shapes[i]
            rows = sample_rows(m, 8)
            ref = oracle_rows(As[i].cpu().numpy(), Bs[i].cpu().numpy(), rows)
            errs.append(rel_err(Cs[i], rows, ref))
        out["rel_err_max"] = max(errs)
        out["rel_err_checked_problems"] = len(errs)
    naive_plans = [api.get_plan("naive", "auto", m, n, k, 1, 0, "f32", k, n, n, False, As[0].device)
                   for (m, n, k) in shapes]

    def loop_naive():
        for p, a, b, c in zip(naive_plans, As, Bs, Cs):
            p(a, b, c)

    def loop_torch():
        for a, b, c in zip(As, Bs, Cs):
            torch.matmul(a, b, out=c)
    wall_n, _ = timed(loop_naive, 3)
    wall_t, _ = timed(loop_torch, 3)
    out["loop_of_mm_naive_tflops"] = round(flops / (wall_n * 1e-3) / 1e12, 3)
    out["loop_of_torch_matmul_tflops"] = round(flops / (wall_t * 1e-3) / 1e12, 3)
    return out


def bench_serving(torch, inputs, count=160, budget_gib=32, slots=4, seed=11, check=True):
    """Poisson arrivals, square n: 70% in [256,1024], 25% in [1024,4096],
    5% = 8192; dtype 50/50 float32 / split-bfloat16 refined; HBM-budget
    admission into one device arena of the budget's size, one stream per
    slot (one executor for every run).  The outputs of a sample of requests
    of the untimed warm-up run are checked against the oracle on sampled
    rows (a request's result is the same in every run: plans depend only on
    its shape and dtype)."""
    import numpy as np
    from paper_2309_00628_amd import serving
    dev = torch.device("cuda", 0)
    base = inputs.serving_trace(count, seed, qps=1.0)
    reqs = serving.make_requests(base, dev)
    torch.cuda.synchronize()
    ex = serving.GpuExecutor(slots, budget_gib << 30, keep_outputs=False)
    # requests whose outputs are kept for the error check: a spread over
    # the trace covering both dtypes and the three size bands
    keep = set()
    for band in ((256, 1024), (1025, 4096), (8192, 8192)):
        for dt in ("f32", "bf16x3"):
            ids = [i for i, t in enumerate(base) if band[0] <= t["n"] <= band[1] and t["dtype"] == dt]
            keep |= set(ids[:2])

    def run(qps, keep_ids=()):
        for r, t in zip(reqs, base):
            r.arrival = 0.0 if qps is None else t["t"] / qps
            r.t_admit = r.t_done = -1.0
            r.error = ""
            r.C = None
        ex.keep_rids = set(keep_ids)
        srv = serving.Server(ex, budget_gib << 30, n_slots=slots)
        done, wall = srv.run(reqs)
        torch.cuda.synchronize()
        st = serving.summarize(done, wall)
        st["max_concurrent"] = srv.max_running
        st["peak_reserved_gib"] = round(srv.peak_reserved / 2 ** 30, 3)
        return st

    run(None, keep if check else ())            # warm-up (plans; sample outputs kept for the check)
    out = {"workload": f"{count} requests, n: 70% U[256,1024], 25% U[1024,4096], 5% 8192; "
                       "dtype 50/50 f32 / bf16x3; Poisson arrivals",
           "hbm_budget_gib": budget_gib, "slots": slots, "load": {}}
    if check:
        errs = {}
        for i in sorted(keep):
            r = reqs[i]
            if r.C is None:
                continue
            rows = sample_rows(r.m, 8)
            ref = oracle_rows(r.A[torch.from_numpy(rows).to(dev)].cpu().numpy(), r.B.cpu().numpy(),
                              np.arange(len(rows)))
            errs[f"{r.dtype}_n{r.n}_id{i}"] = rel_err(r.C, rows, ref)
            r.C = None
        out["rel_err_sample"] = errs
        out["rel_err_max"] = max(errs.values()) if errs else None
    sat = run(None)
    out["saturation"] = sat
    for f in (0.25, 0.5, 0.75, 0.9):
        qps = f * sat["req_per_s"]
        st = run(qps)
        st["offered_qps"] = round(qps, 2)
        out["load"][str(f)] = st
        print(f"# serving load {f}: {st}", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only (the library runs one process per GPU and has no multi-GPU path); run with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2309_00628_amd import _lib as L
    from paper_2309_00628_amd import api, inputs, tuner

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(args.copy_probe * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4}), flush=True)
        return
    if args.profile_set:
        profile_set(torch, api, L, inputs, tuner, args)
        return
    n, lv = args.n, args.levels
    flops = 2.0 * n ** 3
    A_np, B_np = inputs.pair("uniform", n, n, n, 0, np.float32)
    A = torch.from_numpy(A_np).cuda()
    B = torch.from_numpy(B_np).cuda()
    print(f"# bench n={n} fp32 L={lv}, steps={args.steps} warmup={args.warmup} rounds={args.rounds}",
          file=sys.stderr, flush=True)

    def plan_and_buffers(plan):
        ws = torch.empty(max(plan.ws_bytes, 256), dtype=torch.uint8, device="cuda")
        return ws, torch.empty((n, n), dtype=torch.float32, device="cuda")

    tile, overlap, leaf_u, trans_b = tuned_leaf(tuner, n, lv)
    wplan = api.Plan("winograd", args.sched, n, n, n, cutoff=1, levels=lv, tile=tile, overlap=overlap,
                     leaf_u=leaf_u, trans_b=trans_b)
    win = plan_contender(torch, L, "winograd", wplan, A, B, *reversed(plan_and_buffers(wplan)))
    if args.profile_only:
        warm_gpu(torch, win.step, args.warm_seconds)
        timed_rounds(torch, [win], args.steps, 1, flops)
        per_op, kinds = launch_times(torch, L, win, args.steps)
        print(json.dumps({"profile_only": True, "n": n, "levels": lv, "tflops": round(win.tflops, 3),
                          "roofline": gemm_roofline(dict(plan=wplan, per_op=per_op, kinds=kinds), n)}),
              flush=True)
        return
    plain_tile, plain_split = tuned_plain(tuner, n)
    pplan = api.Plan("naive", "auto", n, n, n, cutoff=1, levels=0, tile=plain_tile, split_k=plain_split)
    plain = plan_contender(torch, L, "plain", pplan, A, B, *reversed(plan_and_buffers(pplan)))
    torch.backends.cuda.matmul.allow_tf32 = False
    Cv = torch.empty((n, n), dtype=torch.float32, device="cuda")
    vendor = Contender("hipblaslt", lambda: torch.matmul(A, B, out=Cv), None, Cv)
    contenders = [win, plain, vendor]

    warm_gpu(torch, plain.step, args.warm_seconds)
    for c in contenders:
        for _ in range(args.warmup):
            c.step()
    timed_rounds(torch, contenders, args.steps, args.rounds, flops)
    for c in contenders:
        print(f"# {c.name}: {c.tflops:.2f} TFLOP/s (rounds {[round(x, 1) for x in c.round_tflops]})",
              file=sys.stderr, flush=True)
    w_ops, w_kinds = launch_times(torch, L, win, args.steps)
    p_ops, p_kinds = launch_times(torch, L, plain, args.steps)
    wres = dict(plan=wplan, per_op=w_ops, kinds=w_kinds)
    pres = dict(plan=pplan, per_op=p_ops, kinds=p_kinds)
    # Strassen (Section 2.2) breadth first at the same levels (context)
    strs = run_product(torch, api, L, "strassen", "grouped", n, lv, A, B, 20, 5, tile=None if leaf_u else tile)
    print(f"# strassen L={lv}: {strs['tflops']:.2f} TFLOP/s", file=sys.stderr, flush=True)

    def summary(c):
        return {"tflops": round(c.tflops, 3), "median_round_tflops": round(c.median_round_tflops, 3),
                "round_tflops": [round(x, 2) for x in c.round_tflops],
                "p50_ms": round(pct(c.step_ms, 50), 4), "p99_ms": round(pct(c.step_ms, 99), 4)}

    out = {
        "metric": "effective TFLOP/s (2mnk/t) Winograd vs plain GEMM at stated rel. err; p99 ms",
        "value": round(win.tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(win.wall_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (uniform[-1,1], seeded)",
        "config": {"workload": f"square fp32 matmul n={n}, Strassen-Winograd {args.sched} L={lv} "
                               f"vs plain MFMA GEMM",
                   "n": n, "levels": lv, "schedule": args.sched, "leaf_tile_cfg": tile,
                   "overlap": overlap, "leaf_u": leaf_u, "trans_b": trans_b},
        "timing": {"warm_seconds": args.warm_seconds, "rounds": args.rounds,
                   "note": "K steps per contender in R interleaved rounds, order rotated per round"},
        "p50_ms": round(pct(win.step_ms, 50), 4),
        "p99_ms": round(pct(win.step_ms, 99), 4),
        "winograd": summary(win),
        "plain_gemm": dict(summary(plain), tile=plain_tile, split_k=plain_split),
        "hipblaslt": summary(vendor),
        "speedup_vs_plain": round(win.tflops / plain.tflops, 4),
        "speedup_vs_plain_median_round": round(win.median_round_tflops / plain.median_round_tflops, 4),
        "speedup_vs_hipblaslt": round(win.tflops / vendor.tflops, 4),
        "strassen_grouped": {"levels": lv, "tflops": round(strs["tflops"], 3),
                             "p50_ms": round(strs["p50"], 4), "p99_ms": round(strs["p99"], 4)},
        "roofline": gemm_roofline(wres, n),
        "plain_gemm_roofline": gemm_roofline(pres, n, traffic=False),
        "addition_kernels": ew_bandwidth(wres, n),
    }
    if not args.no_cpu:
        rows = sample_rows(n)
        ref = oracle_rows(A_np, B_np, rows)
        out["rel_err"] = rel_err(win.C, rows, ref)
        out["plain_gemm"]["rel_err"] = rel_err(plain.C, rows, ref)
        out["hipblaslt"]["rel_err"] = rel_err(vendor.C, rows, ref)
        out["strassen_grouped"]["rel_err"] = rel_err(strs["C"], rows, ref)
        out["rel_err_note"] = (f"relative Frobenius error vs the float64 oracle on {len(rows)} sampled rows "
                               "(first and last included)")
    del strs
    for c in contenders:
        c.C = None
    del win, plain, vendor, contenders, Cv

    if not args.no_extra:
        out["d2"], arrays = bench_d2(torch, api, L, inputs, tuner, with_ref=not args.no_cpu)
        if not args.no_schedules:
            A4_np, B4_np, A4, B4, rows4, ref4 = arrays[4096]
            out["schedules"] = bench_schedules(torch, api, L, A4, B4, 4096,
                                               *((rows4, ref4) if not args.no_cpu else ()))
        del arrays
    if not args.no_precision:
        out["precision"] = bench_precision(torch, api, L, inputs, tuner)
        out["fp64_small"] = bench_fp64_small(torch, api, L, inputs)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, api, inputs, tuner, check=not args.no_cpu)
        print(f"# batched: {out['batched']}", file=sys.stderr, flush=True)
    if not args.no_serving:
        out["serving"] = bench_serving(torch, inputs, check=not args.no_cpu)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inputs, (A_np, B_np), args.cpu_seconds)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
