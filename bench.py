#!/usr/bin/env python3
"""Benchmark: effective TFLOP/s (2mnk/t) of Strassen-Winograd against the
plain MFMA GEMM of the same library, on one MI355X, with the relative error
against the float64 oracle and p50/p99 step latency.

Workload (one "step" = one whole product, every kernel of the path):
square float32 C = A x B, n = 4096, entries i.i.d. U[-1, 1] from a fixed
seed, Strassen-Winograd with the grouped schedule.  The plain MFMA GEMM
(mm_naive) runs the same product for comparison.  Inputs are resident in HBM
before timing starts.

Printed: one JSON line (rank 0).  ``roofline`` is for the dominant kernel,
the grouped MFMA leaf GEMM launch: algorithmic flops of one launch
(7^L leaf products of 2 (n/2^L)^3 flops) over that launch's average duration,
measured with HIP events recorded around each launch on the stream the
kernels run on, during the timed steps.  ``cpu_baseline`` is the oracle (the
double-precision triple loop) timed on the host on a sample of output rows.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # enough untimed steps for the GPU clocks to settle under MFMA load
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--levels", type=int, default=None, help="recursion levels (default: tuned)")
    ap.add_argument("--sched", default="grouped")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline and error check")
    ap.add_argument("--no-extra", action="store_true", help="skip the n=3000 / n=8192 side runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-problem batch")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the depth-first schedules (Two Temp, In-Place, Strassen DFS) at n=4096")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop runs")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the n=8192 split-bfloat16 precision runs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the timed Winograd steps (for rocprofv3 runs)")
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


def time_plan(torch, api, L, plan, A, B, C, ws, steps, warmup):
    """Run warm-up steps, then exactly ``steps`` timed steps with one event
    before and one after each step (the wall time and per-step latencies),
    then ``steps`` more with events before and after every launch, recorded
    on the stream the launch runs on (the per-launch durations).  An event
    between two launches of a step delays the second one a little, so the
    step time is taken without them.
    Returns (wall ms per step, per-step ms list, per-launch ms lists, kinds)."""
    import ctypes
    lib = L.load()
    s = torch.cuda.current_stream()
    nops = plan.info["launches"]
    nev = 2 * nops
    wsp, wsb = (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)
    args = (plan._ptr, A.data_ptr(), B.data_ptr(), C.data_ptr(), wsp, wsb, s.cuda_stream)
    for _ in range(warmup):
        L.check(lib.mm_plan_execute(*args))
    steps_ev = [_events(torch, 2, s) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        steps_ev[i][0].record(s)
        L.check(lib.mm_plan_execute(*args))
        steps_ev[i][1].record(s)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    step_ms = [a.elapsed_time(b) for a, b in steps_ev]
    evsets = [_events(torch, nev, s) for _ in range(steps)]
    ptrs = [(ctypes.c_void_p * nev)(*[e.cuda_event for e in evs]) for evs in evsets]
    torch.cuda.synchronize()
    for i in range(steps):
        L.check(lib.mm_plan_execute_timed(*args, ptrs[i], nev))
    torch.cuda.synchronize()
    per_op = [[evs[2 * j].elapsed_time(evs[2 * j + 1]) for evs in evsets] for j in range(nops)]
    kinds = [lib.mm_plan_op_kind(plan._ptr, j) for j in range(nops)]
    return wall_ms, step_ms, per_op, kinds


def plan_launches(plan, esz):
    """Per launch of a plan (in launch order): its kind ("EW", "GEMM",
    "WINO", "FORK", "JOIN"), stream (0 caller's, 1 auxiliary), algorithmic
    flops (GEMM: 2 m n k per leaf product; WINO: seven such products per
    subproblem) and algorithmic HBM bytes (EW: every valid input element read
    once, every valid output element written once), read off the plan
    listing."""
    out, flops, nbytes = [], 0.0, 0.0
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
                            flags=w[5:]))
            flops, nbytes = 0.0, 0.0
        elif w[0] == "GEMM":
            m, n, k = map(int, w[1:4])
            flops += 2.0 * m * n * k
        elif w[0] == "WINO":
            m, n, k = map(int, w[1:4])
            flops += 7 * 2.0 * m * n * k
        elif w[0] in ("EW", "TRANS"):
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
                overlap=False, leaf_u=False, trans_b=False, split_k=None):
    plan = api.Plan(algo, sched, n, n, n, cutoff=1, levels=levels, dtype=dtype, tile=tile, overlap=overlap,
                    leaf_u=leaf_u, trans_b=trans_b, split_k=split_k)
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
        if k % 8 in (0, 6):  # element-wise and transposing passes
            ms = sum(d) / len(d)
            out.append(dict(stream="aux" if k >= 8 else "main", bytes=lau["bytes"], ms=round(ms, 4),
                            gbs=round(lau["bytes"] / (ms * 1e-3) / 1e9, 1)))
    return out


def cpu_baseline(A_np, B_np, seconds):
    """The oracle (double triple loop, all host cores) on a sample of rows,
    repeated until about ``seconds`` of host time have been spent."""
    import numpy as np
    from oracle import naive
    n = A_np.shape[0]
    rows = 8
    t0 = time.perf_counter()
    naive.gemm_rows(A_np, B_np, np.arange(rows))
    dt = time.perf_counter() - t0
    rows = int(max(8, min(n, rows * seconds / max(dt, 1e-3))))
    sample = np.linspace(0, n - 1, rows).astype(np.int64)
    reps, spent = 0, 0.0
    while True:
        t0 = time.perf_counter()
        ref = naive.gemm_rows(A_np, B_np, sample)
        spent += time.perf_counter() - t0
        reps += 1
        if spent >= 0.8 * seconds or rows < n:
            break
    flops = 2.0 * rows * n * n * reps
    return dict(value=round(flops / spent / 1e12, 6), unit="TFLOP/s", cores=naive.max_threads(),
                kind="oracle",
                sample=f"{reps} pass(es) over {rows} of {n} output rows of the n={n} product "
                       f"({spent:.1f} s, float64 triple loop)"), sample, ref


def rel_err(C, rows, ref):
    import numpy as np
    import torch
    got = C[torch.from_numpy(rows).to(C.device)].double().cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


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
    print(json.dumps(out), flush=True)


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
                     "rel_err": rel_err(r["C"], sample, ref), "tile": tile, "overlap": ov}
        print(f"# precision {name}: {out[name]}", file=sys.stderr, flush=True)
        del r
    out["speedup_bf16x3_winograd_vs_f32_plain"] = round(out["bf16x3_winograd_L2"]["tflops"] /
                                                        out["f32_plain"]["tflops"], 4)
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


def bench_batched(torch, api, inputs, tuner, count=512, steps=10, warmup=3, seed=7):
    """512 independent float32 products, m, n, k log-uniform in [64, 2048]
    (multiples of 16), levels per size class from the tuner, run as one
    level-synchronous batched plan replayed from a hipGraph."""
    shapes = inputs.batched_shapes(count, seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    As, Bs, Cs, levels = [], [], [], []
    for (m, n, k) in shapes:
        As.append(torch.rand((m, k), generator=g, device="cuda") * 2 - 1)
        Bs.append(torch.rand((k, n), generator=g, device="cuda") * 2 - 1)
        Cs.append(torch.empty((m, n), device="cuda"))
        levels.append(tuner.choose(m, n, k, "f32")["levels"])
    flops = sum(2.0 * m * n * k for (m, n, k) in shapes)
    plan = api.BatchedPlan(As, Bs, Cs, cutoff=[1] * count, levels=levels, graph=True)
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
    return {"workload": f"{count} fp32 products, m,n,k log-uniform in [64,2048] (x16), uniform[-1,1]",
            "tflops": round(flops / (wall * 1e-3) / 1e12, 3), "ms_per_batch": round(wall, 4),
            "device_ms_per_batch": round(dev, 4), "launches_per_batch": plan.info["launches"],
            "levels_histogram": {str(l): levels.count(l) for l in sorted(set(levels))},
            "loop_of_mm_naive_tflops": round(flops / (wall_n * 1e-3) / 1e12, 3),
            "loop_of_torch_matmul_tflops": round(flops / (wall_t * 1e-3) / 1e12, 3),
            "graph": True}


def bench_serving(torch, inputs, count=160, budget_gib=32, slots=4, seed=11):
    """Poisson arrivals, square n: 70% in [256,1024], 25% in [1024,4096],
    5% = 8192; dtype 50/50 float32 / split-bfloat16 refined; HBM-budget
    admission, one stream and workspace per slot."""
    from paper_2309_00628_amd import serving
    dev = torch.device("cuda", 0)
    base = inputs.serving_trace(count, seed, qps=1.0)
    reqs = serving.make_requests(base, dev)
    torch.cuda.synchronize()

    def run(qps):
        for r, t in zip(reqs, base):
            r.arrival = 0.0 if qps is None else t["t"] / qps
            r.t_admit = r.t_done = -1.0
            r.error = ""
            r.C = None
        ex = serving.GpuExecutor(slots, keep_outputs=False)
        srv = serving.Server(ex, budget_gib << 30, n_slots=slots)
        done, wall = srv.run(reqs)
        torch.cuda.synchronize()
        st = serving.summarize(done, wall)
        st["max_concurrent"] = srv.max_running
        return st

    run(None)                                   # warm-up: plans, workspaces
    sat = run(None)
    out = {"workload": f"{count} requests, n: 70% U[256,1024], 25% U[1024,4096], 5% 8192; "
                       "dtype 50/50 f32 / bf16x3; Poisson arrivals",
           "hbm_budget_gib": budget_gib, "slots": slots, "saturation": sat, "load": {}}
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
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
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
    n = args.n
    A_np, B_np = inputs.pair("uniform", n, n, n, 0, np.float32)
    A = torch.from_numpy(A_np).cuda()
    B = torch.from_numpy(B_np).cuda()
    print(f"# bench n={n} fp32, steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)

    # level choice: the tuner's cached choice for this size class; without one
    # time L = 1..3 briefly and keep the fastest
    ch = tuner.choose(n, n, n, "f32")
    rec = ch.get("best_recursive") if ch["source"] == "tuned" else None
    if args.levels is None and ch["source"] == "tuned" and ch["levels"] > 0:
        levels = ch["levels"]
    elif args.levels is None and rec:
        levels = rec["levels"]  # the plain product won the size class; time the best recursion
    elif args.levels is None:
        best = None
        for lv in (1, 2, 3):
            r = run_product(torch, api, L, "winograd", args.sched, n, lv, A, B, 5, 2)
            print(f"# tune L={lv}: {r['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
            if best is None or r["tflops"] > best[1]:
                best = (lv, r["tflops"])
        levels = best[0]
    else:
        levels = args.levels

    tile, overlap, leaf_u, trans_b = tuned_leaf(tuner, n, levels)
    win = run_product(torch, api, L, "winograd", args.sched, n, levels, A, B, args.steps, args.warmup,
                      tile=tile, overlap=overlap, leaf_u=leaf_u, trans_b=trans_b)
    print(f"# winograd L={levels}: {win['tflops']:.2f} TFLOP/s", file=sys.stderr, flush=True)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "n": n, "levels": levels,
                          "tflops": round(win["tflops"], 3),
                          "roofline": gemm_roofline(win, n)}), flush=True)
        return
    plain_tile, plain_split = tuned_plain(tuner, n)
    plain = run_product(torch, api, L, "naive", "auto", n, 0, A, B, args.steps, args.warmup,
                        tile=plain_tile, split_k=plain_split)
    print(f"# plain mfma gemm: {plain['tflops']:.2f} TFLOP/s", file=sys.stderr, flush=True)
    # Strassen (Section 2.2) breadth first at the same levels and leaf tile
    # (a tile of the fused leaf-level kernel names another kernel: then the default)
    strs = run_product(torch, api, L, "strassen", "grouped", n, levels, A, B, 20, 10,
                       tile=None if leaf_u else tile)
    print(f"# strassen L={levels}: {strs['tflops']:.2f} TFLOP/s", file=sys.stderr, flush=True)

    # vendor GEMM (hipBLASLt through torch.matmul) as context only
    torch.backends.cuda.matmul.allow_tf32 = False
    for _ in range(3):
        torch.matmul(A, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        torch.matmul(A, B)
    torch.cuda.synchronize()
    vendor_tflops = 2.0 * n ** 3 / ((time.perf_counter() - t0) / args.steps) / 1e12

    out = {
        "metric": "effective TFLOP/s (2mnk/t) Winograd vs plain GEMM at stated rel. err; p99 ms",
        "value": round(win["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(win["wall_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (uniform[-1,1], seeded)",
        "config": {"workload": f"square fp32 matmul n={n}, Strassen-Winograd {args.sched} "
                               f"L={levels} vs plain MFMA GEMM",
                   "n": n, "levels": levels, "schedule": args.sched, "leaf_tile_cfg": tile,
                   "overlap": overlap, "leaf_u": leaf_u, "trans_b": trans_b},
        "p50_ms": round(win["p50"], 4),
        "p99_ms": round(win["p99"], 4),
        "plain_gemm": {"tflops": round(plain["tflops"], 3), "p50_ms": round(plain["p50"], 4),
                       "p99_ms": round(plain["p99"], 4), "tile": plain_tile, "split_k": plain_split},
        "speedup_vs_plain": round(win["tflops"] / plain["tflops"], 4),
        "strassen_grouped": {"levels": levels, "tflops": round(strs["tflops"], 3),
                             "p50_ms": round(strs["p50"], 4), "p99_ms": round(strs["p99"], 4)},
        "vendor_hipblaslt_tflops": round(vendor_tflops, 3),
        "roofline": gemm_roofline(win, n),
        "plain_gemm_roofline": gemm_roofline(plain, n, traffic=False),
        "addition_kernels": ew_bandwidth(win, n),
    }

    if not args.no_cpu:
        cb, rows, ref = cpu_baseline(A_np, B_np, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["rel_err"] = rel_err(win["C"], rows, ref)
        out["plain_rel_err"] = rel_err(plain["C"], rows, ref)
        out["strassen_grouped"]["rel_err"] = rel_err(strs["C"], rows, ref)
        out["rel_err_note"] = "relative Frobenius error vs the float64 oracle on the sampled rows"
    if not args.no_schedules:
        out["schedules"] = bench_schedules(torch, api, L, A, B, n, *((rows, ref) if not args.no_cpu else ()))

    if not args.no_extra:
        extra = {}
        for n2, lvls in ((3000, (1, 2)), (8192, (1, 2))):
            A2_np, B2_np = inputs.pair("uniform", n2, n2, n2, 1, np.float32)
            A2, B2 = torch.from_numpy(A2_np).cuda(), torch.from_numpy(B2_np).cuda()
            pt2, pk2 = tuned_plain(tuner, n2)
            p2 = run_product(torch, api, L, "naive", "auto", n2, 0, A2, B2, 20, 10, tile=pt2, split_k=pk2)
            e = {"plain_tflops": round(p2["tflops"], 3)}
            for lv in lvls:
                t2, o2, u2, b2 = tuned_leaf(tuner, n2, lv)
                w2 = run_product(torch, api, L, "winograd", args.sched, n2, lv, A2, B2, 20, 10, tile=t2,
                                 overlap=o2, leaf_u=u2, trans_b=b2)
                e[f"winograd_L{lv}_tflops"] = round(w2["tflops"], 3)
                e[f"winograd_L{lv}_p99_ms"] = round(w2["p99"], 4)
                s2 = run_product(torch, api, L, "strassen", "grouped", n2, lv, A2, B2, 20, 10,
                                 tile=None if u2 else t2)
                e[f"strassen_L{lv}_tflops"] = round(s2["tflops"], 3)
            extra[str(n2)] = e
            print(f"# extra n={n2}: {e}", file=sys.stderr, flush=True)
            del A2, B2
        out["extra"] = extra

    if not args.no_precision:
        out["precision"] = bench_precision(torch, api, L, inputs, tuner)
        out["fp64_small"] = bench_fp64_small(torch, api, L, inputs)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, api, inputs, tuner)
        print(f"# batched: {out['batched']}", file=sys.stderr, flush=True)
    if not args.no_serving:
        out["serving"] = bench_serving(torch, inputs)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
