"""Autotuner: recursion depth (cutoff / levels) and MFMA tile shape per size class.

Section 3.4 derives the cutoff from an operation-count model (the naive method
wins below order 12 on the paper's CPU).  On MI355X the break-even is set by
MFMA rate against HBM bandwidth instead, so it is measured: for a size class
the tuner times each candidate (levels L = 0..Lmax of Strassen-Winograd with
the grouped schedule, L = 0 being the plain MFMA GEMM, crossed with a few
leaf tile shapes and, for L > 0, with and without the S/T passes overlapped
on a second stream, and (float32) the fused last-level kernel with its own
tiles) on the GPU with HIP events and keeps the fastest.

Choices are cached per (GPU architecture, dtype, size class) in a JSON file
(``tuning/<arch>.json`` next to this module) so that a process, a batch or a
server reuses them.  A size class is the (m, n, k) triple rounded to half
octaves.  Without a cached entry ``choose`` falls back to a rule of thumb
measured on MI355X: one level per halving while the leaf stays at or above
2048 (float32) / 4096 (split bfloat16), at most two levels.
"""
import json
import math
import os
import threading
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_DIR = os.path.join(HERE, "tuning")

_lock = threading.Lock()
_cache = {}


def size_class(m, n, k):
    def q(x):
        return round(2 * math.log2(max(int(x), 1))) / 2
    return (q(m), q(n), q(k))


def class_key(dtype, m, n, k):
    a, b, c = size_class(m, n, k)
    return f"{dtype}|{a:.1f}|{b:.1f}|{c:.1f}"


def _arch():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        pass
    return "gfx950"


def cache_path(arch=None):
    return os.path.join(CACHE_DIR, f"{arch or _arch()}.json")


def load_cache(arch=None):
    arch = arch or _arch()
    with _lock:
        if arch not in _cache:
            p = cache_path(arch)
            _cache[arch] = json.load(open(p)) if os.path.exists(p) else {}
        return _cache[arch]


def save_cache(arch=None):
    arch = arch or _arch()
    with _lock:
        os.makedirs(CACHE_DIR, exist_ok=True)
        tmp = cache_path(arch) + ".tmp"
        with open(tmp, "w") as f:
            json.dump(_cache.get(arch, {}), f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path(arch))


def rule_of_thumb(m, n, k, dtype):
    """Levels by the leaf-size rule; tile left to the planner."""
    leaf = 2048 if dtype != "bf16x3" else 4096
    L = 0
    while L < 2 and min(m, n, k) >> (L + 1) >= leaf:
        L += 1
    return {"levels": L, "tile": None, "cutoff": 1, "overlap": False, "leaf_u": False, "trans_b": False,
            "split_k": None, "source": "rule"}


def choose(m, n, k, dtype="f32"):
    """(levels, tile, cutoff) for C = A (m x k) B (k x n)."""
    entry = load_cache().get(class_key(dtype, m, n, k))
    if entry is not None:
        return dict(entry, source="tuned")
    return rule_of_thumb(m, n, k, dtype)


def options_at(m, n, k, dtype, levels):
    """The tuner's (tile, overlap, leaf_u, trans_b) for a recursion of exactly
    ``levels`` levels, or None when it has not measured that level count."""
    ch = choose(m, n, k, dtype)
    if ch.get("source") != "tuned":
        return None
    c = (ch.get("by_level") or {}).get(str(levels))
    if c is None:
        for c2 in (ch, ch.get("best_recursive") or {}):
            if c2.get("levels") == levels:
                c = c2
                break
    if c is None:
        return None
    return c.get("tile"), bool(c.get("overlap", False)), bool(c.get("leaf_u", False)), bool(c.get("trans_b", False))


def _time_plan(plan, A, B, C, reps, warmup):
    import ctypes

    import torch

    from . import _lib as L
    lib = L.load()
    s = torch.cuda.current_stream()
    ws = torch.empty(max(plan.ws_bytes, 256), dtype=torch.uint8, device=A.device)
    for _ in range(warmup):
        L.check(lib.mm_plan_execute(plan._ptr, A.data_ptr(), B.data_ptr(), C.data_ptr(), ws.data_ptr(),
                                    ws.numel(), s.cuda_stream))
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        e0[i].record(s)
        L.check(lib.mm_plan_execute(plan._ptr, A.data_ptr(), B.data_ptr(), C.data_ptr(), ws.data_ptr(),
                                    ws.numel(), s.cuda_stream))
        e1[i].record(s)
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in zip(e0, e1))
    return ts[len(ts) // 2]


TILES = {"f32": (None, 0, 3, 4, 8), "bf16x3": (None, 0, 1, 4, 6, 8), "f64": (None,)}
LEAF_U_TILES = (None, 0, 1, 2)  # tiles of the fused last-level kernel (float32)


def candidates(dtype, L_, tiles=None, k=None):
    """Option sets tried at L_ levels: dicts of tile, overlap, leaf_u,
    trans_b and split_k (the plain product's k split, when k allows it)."""
    def c(tile, overlap=False, leaf_u=False, trans_b=False, split_k=None):
        return dict(tile=tile, overlap=overlap, leaf_u=leaf_u, trans_b=trans_b, split_k=split_k)
    out = []
    for tile in (tiles or TILES.get(dtype, (None,))):
        for ov in ((False, True) if L_ else (False,)):
            out.append(c(tile, overlap=ov))
        if L_ and dtype == "f32":
            out.append(c(tile, trans_b=True))
    if L_ == 0 and dtype in ("f32", "bf16x3") and tiles is None and k is not None:
        out += [c(None, split_k=s) for s in SPLIT_K if k >= 64 * s]
    if L_ and dtype == "f32" and tiles is None:
        out += [c(tile, leaf_u=True) for tile in LEAF_U_TILES]
    return out


# k splits tried for the plain product (they pay when C has few tiles)
SPLIT_K = (2, 4, 8)


# An option (overlap, fused last level) is chosen only when it beats the
# plans without options by more than this fraction: differences smaller than
# the run-to-run spread of the timings are not evidence.
OPTION_MARGIN = 0.01


def tune(m, n, k, dtype="f32", max_levels=3, reps=5, warmup=2, tiles=None, save=True, verbose=False, rounds=5):
    """Measure the candidates for this size class and cache the fastest."""
    import numpy as np
    import torch

    from . import api, inputs
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ndt = np.float64 if dtype == "f64" else np.float32
    A_np, B_np = inputs.pair("uniform", m, n, k, 0, ndt)
    A = torch.from_numpy(A_np).cuda()
    B = torch.from_numpy(B_np).cuda()
    C = torch.empty((m, n), dtype=tdt, device="cuda")
    # every candidate is timed in several interleaved rounds (after the GPU
    # has run for a while), so clock drift does not favour whichever
    # candidate happens to run first; the median of the rounds decides
    cands = []
    for L_ in range(0, max_levels + 1):
        if L_ > 0 and min(m, n, k) >> L_ < 64:
            break
        for opt in candidates(dtype, L_, tiles, k):
            algo = "naive" if L_ == 0 else "winograd"
            key = (L_, opt["tile"], opt["overlap"], opt["leaf_u"], opt["trans_b"], opt["split_k"])
            try:
                p = api.Plan(algo, "grouped" if L_ else "auto", m, n, k, cutoff=1, levels=L_, dtype=dtype, **opt)
            except Exception as e:  # an unsupported candidate is skipped
                if verbose:
                    print(f"  skip L={L_} {opt}: {e}")
                continue
            cands.append((key, p))
    if not cands:
        raise RuntimeError("no tuning candidate")
    warm_until = time.perf_counter() + 0.1
    while time.perf_counter() < warm_until:
        _time_plan(cands[0][1], A, B, C, 1, 1)
    times = {key: [] for key, _ in cands}
    for _ in range(rounds):
        for key, p in cands:
            times[key].append(_time_plan(p, A, B, C, reps, warmup))
    results = []
    for key, ts in times.items():
        t = sorted(ts)[len(ts) // 2]
        results.append((t,) + key)
        if verbose:
            L_, tile, ov, lu, tb, sk = key
            print(f"  {dtype} {m}x{n}x{k} L={L_} tile={tile} overlap={int(ov)} leaf_u={int(lu)} trans_b={int(tb)} "
                  f"split_k={sk}: {t:.3f} ms {2.0 * m * n * k / t / 1e9:.1f} TFLOP/s", flush=True)
    def score(r):
        return r[0] * (1.0 + OPTION_MARGIN if (r[3] or r[4] or r[5] or r[6]) else 1.0)

    t, L_, tile, ov, lu, tb, sk = min(results, key=score)
    leaf = min(m, n, k) >> L_
    # the cutoff that stops the recursion after L_ halvings: the leaf order
    entry = {"levels": L_, "tile": tile, "overlap": ov, "leaf_u": lu, "trans_b": tb, "split_k": sk,
             "cutoff": leaf if L_ else min(m, n, k),
             "ms": round(t, 4), "tflops": round(2.0 * m * n * k / t / 1e9, 2),
             "shape": [m, n, k]}
    # the fastest recursive candidate too (for callers that ask for a
    # recursion, and to report how close the recursion comes to the plain
    # product when it does not win)
    plain = [r for r in results if r[1] == 0]
    if plain:
        t0, _, tile0, _, _, _, sk0 = min(plain, key=score)
        entry["best_plain"] = {"levels": 0, "tile": tile0, "split_k": sk0, "ms": round(t0, 4),
                               "tflops": round(2.0 * m * n * k / t0 / 1e9, 2)}
    rec = [r for r in results if r[1] > 0]
    if rec:
        t2, L2, tile2, ov2, lu2, tb2, _ = min(rec, key=score)
        entry["best_recursive"] = {"levels": L2, "tile": tile2, "overlap": ov2, "leaf_u": lu2, "trans_b": tb2,
                                   "ms": round(t2, 4), "tflops": round(2.0 * m * n * k / t2 / 1e9, 2)}
        # the fastest options at every level count measured (for callers
        # that fix the levels)
        by_level = {}
        for lv in sorted({r[1] for r in rec}):
            t3, _, tile3, ov3, lu3, tb3, _ = min((r for r in rec if r[1] == lv), key=score)
            by_level[str(lv)] = {"tile": tile3, "overlap": ov3, "leaf_u": lu3, "trans_b": tb3,
                                 "ms": round(t3, 4), "tflops": round(2.0 * m * n * k / t3 / 1e9, 2)}
        entry["by_level"] = by_level
    arch = _arch()
    load_cache(arch)[class_key(dtype, m, n, k)] = entry
    if save:
        save_cache(arch)
    return entry


# ---------------------------------------------------------------------------
# Batches: levels per size class, measured in the batch itself
# ---------------------------------------------------------------------------
# In a batch the GPU is already full of leaf products, so whether a
# recursion level pays for a problem depends on the batch, not on the
# problem alone.  The tuner measures the batched workload (512 products,
# m, n, k log-uniform in [64, 2048]) as one batched plan and, class by
# class (largest share of the flops first), keeps the level count that
# makes the whole batch fastest.  The library reads the result
# (tuning/<arch>_batched.txt: "dtype class levels") whenever a batch is
# given no levels.

def batched_class(m, n, k):
    """Size class of a batched product: its volume-equivalent order
    (m n k)^(1/3) rounded to half octaves (as the library computes it)."""
    return math.floor(2.0 * math.log2(max(m * n * k, 1)) / 3.0 + 0.5) / 2.0


def batch_table_path(arch=None):
    return os.path.join(CACHE_DIR, f"{arch or _arch()}_batched.txt")


def tune_batched(count=512, seed=7, dtype="f32", max_levels=2, reps=10, rounds=3, margin=0.01, save=True,
                 verbose=False, out=None):
    import torch

    from . import api, inputs
    shapes = inputs.batched_shapes(count, seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    As, Bs, Cs = [], [], []
    for (m, n, k) in shapes:
        As.append(torch.rand((m, k), generator=g, device="cuda") * 2 - 1)
        Bs.append(torch.rand((k, n), generator=g, device="cuda") * 2 - 1)
        Cs.append(torch.empty((m, n), device="cuda"))
    cls = [batched_class(*s) for s in shapes]
    flops = {}
    for (m, n, k), c in zip(shapes, cls):
        flops[c] = flops.get(c, 0.0) + 2.0 * m * n * k
    classes = sorted(flops, key=lambda c: -flops[c])
    choice = {c: 0 for c in classes}
    s = torch.cuda.current_stream()

    def time_levels(lv):
        plan = api.BatchedPlan(As, Bs, Cs, cutoff=[1] * count, levels=lv, graph=True)
        for _ in range(3):
            plan()
        ts = []
        for _ in range(rounds):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                plan()
            e1.record(s)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / reps)
        return sorted(ts)[len(ts) // 2]

    total = sum(flops.values())
    base = time_levels([0] * count)
    if verbose:
        print(f"batched all L=0: {base:.4f} ms {total / base / 1e9:.1f} TFLOP/s", flush=True)
    for c in classes:
        best_t, best_l = None, 0
        for L_ in range(0, max_levels + 1):
            if L_ and any(min(sh) >> L_ < 16 for sh, cc in zip(shapes, cls) if cc == c):
                break                   # leaves of fewer than 16 rows: not worth a level
            lv = [L_ if cc == c else choice[cc] for cc in cls]
            t = time_levels(lv)
            if verbose:
                print(f"  class {c:.1f} ({flops[c] / total:.1%} of the flops) L={L_}: {t:.4f} ms "
                      f"{total / t / 1e9:.1f} TFLOP/s", flush=True)
            if best_t is None or t < best_t * (1.0 - margin):
                best_t, best_l = t, L_
        choice[c] = best_l
    lines = ["# levels per size class of batched float32 products, measured on the batched workload",
             f"# ({count} products, m, n, k log-uniform in [64, 2048], seed {seed}) as one batched plan;",
             "# class = round(2 log2 (m n k)^(1/3)) / 2.  Columns: dtype class levels"]
    lines += [f"{dtype} {c:.1f} {choice[c]}" for c in sorted(choice)]
    text = "\n".join(lines) + "\n"
    if save:
        os.makedirs(CACHE_DIR, exist_ok=True)
        with open(batch_table_path(), "w") as f:
            f.write(text)
    if out:
        with open(out, "w") as f:
            f.write(text)
    return choice


def main(argv=None):
    """Tune square size classes: python -m paper_2309_00628_amd.tuner --n 1024,4096 --dtype f32"""
    import argparse
    import shutil
    ap = argparse.ArgumentParser(description="measure and cache recursion levels / tile per size class")
    ap.add_argument("--n", default="256,362,512,724,1024,1448,2048,2896,3000,4096,5793,8192")
    ap.add_argument("--dtype", default="f32,bf16x3")
    ap.add_argument("--max-levels", type=int, default=3)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--copy-to", default=None, help="also copy the cache file here")
    ap.add_argument("--batched", action="store_true",
                    help="tune the levels per size class of the batched workload instead")
    args = ap.parse_args(argv)
    if args.batched:
        ch = tune_batched(verbose=True, out=args.copy_to)
        print({f"{c:.1f}": l for c, l in sorted(ch.items())}, flush=True)
        return
    for dt in args.dtype.split(","):
        for n in [int(x) for x in args.n.split(",")]:
            e = tune(n, n, n, dt, max_levels=args.max_levels, reps=args.reps, verbose=True)
            print(f"{dt} n={n}: levels={e['levels']} tile={e['tile']} overlap={e['overlap']} "
                  f"leaf_u={e['leaf_u']} trans_b={e['trans_b']} split_k={e.get('split_k')} {e['tflops']} TFLOP/s",
                  flush=True)
    if args.copy_to:
        shutil.copy(cache_path(), args.copy_to)


if __name__ == "__main__":
    main()
