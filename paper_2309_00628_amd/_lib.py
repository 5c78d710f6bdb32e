"""ctypes binding of libmm.so: the same entry points as include/mm.h.

Argument marshalling only: every step of a product runs in the library's HIP
kernels.  There is no fallback of any kind; if the library is missing or does
not load, every call raises.

torch is imported before the library is loaded so that the process has one
HIP runtime: libmm.so needs libamdhip64.so.7, and the dynamic loader then
reuses the copy torch already mapped.  Streams and device pointers obtained
from torch are therefore valid in the library.
"""
import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

# mm.h enums
MM_F64, MM_F32, MM_BF16X3_REFINED = 0, 1, 2
MM_ALGO_NAIVE, MM_ALGO_STRASSEN, MM_ALGO_WINOGRAD = 0, 1, 2
MM_SCHED_TWO_TEMP, MM_SCHED_IN_PLACE, MM_SCHED_GROUPED, MM_SCHED_DFS3, MM_SCHED_AUTO = 0, 1, 2, 3, 4
MM_PLAN_GRAPH = 1
MM_PLAN_FUSE = 2
MM_PLAN_OVERLAP = 4
MM_PLAN_LEAF_U = 8
MM_PLAN_SPLIT_PASS = 16
MM_PLAN_ACCUMULATE = 32
MM_PLAN_PEEL = 64
MM_PLAN_TRANS_B = 128
MM_PLAN_UNROLL_BASE = 0x100000
MM_PLAN_PERSISTENT = 0x200000
MM_PLAN_LEVEL_PASSES = 0x400000


def plan_split_k(s):
    """MM_PLAN_SPLIT_K(s) flag bits (0 when s is None or 1: no split)."""
    return 0 if not s or s <= 1 else (int(s) & 0xF) << 16


def plan_pad(mult):
    """MM_PLAN_PAD(q) flag bits for padding to a multiple of ``mult`` (a
    power of two; None or 1: no extra padding)."""
    if not mult or mult <= 1:
        return 0
    q = int(mult).bit_length() - 1
    if 1 << q != int(mult) or q > 15:
        raise ValueError("pad multiple must be a power of two up to 2^15")
    return q << 24


def plan_tile(c):
    """MM_PLAN_TILE(c) flag bits (0 when c is None: planner's choice)."""
    return 0 if c is None else ((int(c) + 1) << 8)

STATUS = {0: "MM_OK", 1: "MM_E_INVALID", 2: "MM_E_UNSUPPORTED", 3: "MM_E_WORKSPACE",
          4: "MM_E_ALIAS", 5: "MM_E_HIP", 6: "MM_E_NOMEM"}

ALGOS = {"naive": MM_ALGO_NAIVE, "strassen": MM_ALGO_STRASSEN, "winograd": MM_ALGO_WINOGRAD}
SCHEDS = {"two_temp": MM_SCHED_TWO_TEMP, "in_place": MM_SCHED_IN_PLACE,
          "grouped": MM_SCHED_GROUPED, "dfs3": MM_SCHED_DFS3, "auto": MM_SCHED_AUTO}
DTYPES = {"f64": MM_F64, "f32": MM_F32, "bf16x3": MM_BF16X3_REFINED}


class MMError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {msg}")


_lib = None
_lock = threading.Lock()

c_i64 = ctypes.c_int64
c_int = ctypes.c_int
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_intp = ctypes.POINTER(ctypes.c_int)
c_vpp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "mm_naive": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, c_vp]),
    "mm_strassen": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, c_int, c_int, c_vp]),
    "mm_winograd": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, c_int, c_int, c_vp]),
    "mm_winograd_noalloc": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, c_int, c_int, c_vp]),
    "mm_gemm_ex": (c_int, [c_int, c_int, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
                           c_int, c_int, c_int, c_vp, c_sz, c_vp]),
    "mm_workspace_size": (c_sz, [c_int, c_int, c_i64, c_i64, c_i64, c_int, c_int, c_int]),
    "mm_set_workspace": (c_int, [c_vp, c_sz, c_vp]),
    "mm_plan_create": (c_int, [c_int, c_int, c_i64, c_i64, c_i64, c_i64, c_i64, c_i64, c_int, c_int,
                               c_int, ctypes.c_uint, ctypes.POINTER(c_vp)]),
    "mm_plan_execute": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "mm_plan_info": (c_int, [c_vp, c_i64p, c_int]),
    "mm_plan_execute_beta": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, ctypes.c_double, c_vp]),
    "mm_plan_execute_timed": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp, c_vpp, c_int]),
    "mm_plan_op_kind": (c_int, [c_vp, c_int]),
    "mm_plan_describe": (c_sz, [c_vp, ctypes.c_char_p, c_sz]),
    "mm_plan_destroy": (c_int, [c_vp]),
    "mm_batched_plan_create": (c_int, [c_int, c_i64p, c_vpp, c_vpp, c_vpp, c_int, c_intp, c_intp,
                                       ctypes.c_uint, ctypes.POINTER(c_vp)]),
    "mm_batched": (c_int, [c_int, c_i64p, c_vpp, c_vpp, c_vpp, c_int, c_intp, c_intp, c_vp, c_sz,
                           c_vp]),
    "mm_describe": (c_sz, [c_int, c_int, c_i64, c_i64, c_i64, c_i64, c_i64, c_i64, c_int, c_int,
                           c_int, ctypes.c_uint, ctypes.c_char_p, c_sz, c_i64p, c_int]),
    "mm_batched_describe": (c_sz, [c_int, c_i64p, c_vpp, c_vpp, c_vpp, c_int, c_intp, c_intp,
                                   ctypes.c_uint, ctypes.c_char_p, c_sz, c_i64p, c_int]),
    "mm_batched_table": (c_sz, [c_int, c_i64p, c_vpp, c_vpp, c_vpp, c_int, c_intp, c_intp, ctypes.c_uint,
                                c_vp, c_sz]),
    "mm_batched_levels": (c_int, [c_int, c_i64p, c_int, c_intp, c_intp, c_intp]),
    "mm_tuning_source": (ctypes.c_char_p, []),
    "mm_plan_check": (c_int, [c_vp, c_vp]),
    "mm_last_error": (ctypes.c_char_p, []),
    "mm_version": (c_int, []),
}


def load():
    """Load libmm.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                                   "or python paper_2309_00628_amd/build.py")
            import torch  # noqa: F401  (one HIP runtime per process, see module docstring)
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def last_error():
    return load().mm_last_error().decode(errors="replace")


def check(status):
    if status != 0:
        raise MMError(status, last_error())
    return status


def describe(algo, sched, m, n, k, cutoff=1, levels=-1, dtype="f32", lda=None, ldb=None, ldc=None,
             fuse=False, overlap=False, leaf_u=False, split_pass=False, accumulate=False, tile=None,
             peel=False, trans_b=False, unroll_base=False, split_k=None, pad_to=None, level_passes=False):
    """Host-only plan listing and facts (no device needed)."""
    lib = load()
    lda = max(k, 1) if lda is None else lda
    ldb = max(n, 1) if ldb is None else ldb
    ldc = max(n, 1) if ldc is None else ldc
    info = (ctypes.c_int64 * NINFO)()
    args = (ALGOS.get(algo, algo), SCHEDS.get(sched, sched), m, n, k, lda, ldb, ldc, cutoff, levels,
            DTYPES.get(dtype, dtype), (MM_PLAN_FUSE if fuse else 0) | (MM_PLAN_OVERLAP if overlap else 0) |
            (MM_PLAN_LEAF_U if leaf_u else 0) | (MM_PLAN_SPLIT_PASS if split_pass else 0) |
            (MM_PLAN_ACCUMULATE if accumulate else 0) | (MM_PLAN_PEEL if peel else 0) |
            (MM_PLAN_TRANS_B if trans_b else 0) | (MM_PLAN_UNROLL_BASE if unroll_base else 0) | plan_split_k(split_k) |
            plan_tile(tile) | plan_pad(pad_to) | (MM_PLAN_LEVEL_PASSES if level_passes else 0))
    need = lib.mm_describe(*args, None, 0, info, NINFO)
    if need == 0:
        raise MMError(1, last_error())
    buf = ctypes.create_string_buffer(need + 1)
    lib.mm_describe(*args, buf, need + 1, info, NINFO)
    return buf.value.decode(), _info_dict(info)


def batched_levels(mnk, dtype="f32", cutoff=None, levels=None):
    """The level count each problem of a batch gets (mm_batched_levels;
    host only): None arrays as NULL (tuned levels per size class, cutoff 1)."""
    lib = load()
    cnt = len(mnk)
    flat = (ctypes.c_int64 * max(3 * cnt, 1))(*[v for t in mnk for v in t])
    cp = (c_int * cnt)(*cutoff) if cutoff is not None else None
    lp = (c_int * cnt)(*levels) if levels is not None else None
    out = (c_int * max(cnt, 1))()
    check(lib.mm_batched_levels(cnt, flat, DTYPES.get(dtype, dtype), cp, lp, out))
    return [int(out[i]) for i in range(cnt)]


def batched_table(mnk, addrs, dtype="f32", cutoff=None, levels=None, persistent=True):
    """Host-only: the bytes of a batched plan's device descriptor table."""
    lib = load()
    cnt = len(mnk)
    flat = (ctypes.c_int64 * max(3 * cnt, 1))(*[v for t in mnk for v in t])
    A = (c_vp * max(cnt, 1))(*[a for a, _, _ in addrs])
    B = (c_vp * max(cnt, 1))(*[b for _, b, _ in addrs])
    C = (c_vp * max(cnt, 1))(*[c for _, _, c in addrs])
    cp = (c_int * cnt)(*cutoff) if cutoff is not None else None
    lp = (c_int * cnt)(*levels) if levels is not None else None
    fl = MM_PLAN_PERSISTENT if persistent else 0
    need = lib.mm_batched_table(cnt, flat, A, B, C, DTYPES.get(dtype, dtype), cp, lp, fl, None, 0)
    if need == 0:
        raise MMError(1, last_error())
    buf = ctypes.create_string_buffer(need)
    lib.mm_batched_table(cnt, flat, A, B, C, DTYPES.get(dtype, dtype), cp, lp, fl, buf, need)
    return buf.raw


def tuning_source():
    """Path of the size-class table the library read ("" when none)."""
    return load().mm_tuning_source().decode()


def batched_describe(mnk, addrs, dtype="f32", cutoff=None, levels=None, persistent=False):
    """Host-only listing of a batched plan; ``addrs`` = [(a, b, c)] byte addresses."""
    lib = load()
    cnt = len(mnk)
    flat = (ctypes.c_int64 * (3 * cnt))(*[v for t in mnk for v in t])
    A = (c_vp * cnt)(*[a for a, _, _ in addrs])
    B = (c_vp * cnt)(*[b for _, b, _ in addrs])
    C = (c_vp * cnt)(*[c for _, _, c in addrs])
    cp = (c_int * cnt)(*cutoff) if cutoff is not None else None
    lp = (c_int * cnt)(*levels) if levels is not None else None
    info = (ctypes.c_int64 * NINFO)()
    fl = MM_PLAN_PERSISTENT if persistent else 0
    need = lib.mm_batched_describe(cnt, flat, A, B, C, DTYPES.get(dtype, dtype), cp, lp, fl, None, 0,
                                   info, NINFO)
    if need == 0:
        raise MMError(1, last_error())
    buf = ctypes.create_string_buffer(need + 1)
    lib.mm_batched_describe(cnt, flat, A, B, C, DTYPES.get(dtype, dtype), cp, lp, fl, buf, need + 1,
                            info, NINFO)
    return buf.value.decode(), _info_dict(info)


INFO_KEYS = ("ws_bytes", "levels", "M", "N", "K", "launches", "leaves", "sched", "leaf_rows", "fused",
             "leaf_u")
NINFO = len(INFO_KEYS)


def _info_dict(info):
    return {k: int(info[i]) for i, k in enumerate(INFO_KEYS)}
