"""torch-facing wrappers of libmm: device tensors in, device tensors out.

PyTorch supplies device memory (its caching allocator) and streams; every
arithmetic step runs in libmm's HIP kernels through the C ABI.  Nothing here
computes a product or falls back to another implementation.
"""
import ctypes
import threading

import torch

from . import _lib as L
from ._lib import MMError

_TORCH_DT = {torch.float64: "f64", torch.float32: "f32"}
_ESZ = {"f64": 8, "f32": 4, "bf16x3": 4}


def _resolve_dtype(t, dtype):
    if dtype is None:
        if t.dtype not in _TORCH_DT:
            raise TypeError(f"unsupported tensor dtype {t.dtype} (float32 or float64)")
        return _TORCH_DT[t.dtype]
    if dtype not in L.DTYPES:
        raise ValueError(f"unknown dtype {dtype!r}; one of {sorted(L.DTYPES)}")
    want = torch.float64 if dtype == "f64" else torch.float32
    if t.dtype != want:
        raise TypeError(f"dtype {dtype} needs {want} tensors, got {t.dtype}")
    return dtype


def _ld(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.numel() == 0:
        return max(t.shape[1], 1)
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be row-major with unit column stride")
    return t.stride(0)


def _stream(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return s


class Plan:
    """A built launch sequence for one product shape (mm_plan_create)."""

    def __init__(self, algo, sched, m, n, k, cutoff=1, levels=-1, dtype="f32", lda=None, ldb=None,
                 ldc=None, graph=False, device=None, tile=None, fuse=False, overlap=False, leaf_u=False,
                 split_pass=False, accumulate=False, peel=False, trans_b=False, unroll_base=False,
                 split_k=None, pad_to=None, level_passes=False):
        lib = L.load()
        self.algo, self.sched, self.dtype = algo, sched, dtype
        self.m, self.n, self.k = m, n, k
        self.lda = max(k, 1) if lda is None else lda
        self.ldb = max(n, 1) if ldb is None else ldb
        self.ldc = max(n, 1) if ldc is None else ldc
        self.device = (torch.device(device) if device is not None
                       else torch.device("cuda", torch.cuda.current_device()))
        self._ptr = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.mm_plan_create(L.ALGOS[algo], L.SCHEDS[sched], m, n, k, self.lda, self.ldb,
                                       self.ldc, cutoff, levels, L.DTYPES[dtype],
                                       (L.MM_PLAN_GRAPH if graph else 0) | L.plan_tile(tile) |
                                       (L.MM_PLAN_FUSE if fuse else 0) |
                                       (L.MM_PLAN_OVERLAP if overlap else 0) |
                                       (L.MM_PLAN_LEAF_U if leaf_u else 0) |
                                       (L.MM_PLAN_SPLIT_PASS if split_pass else 0) |
                                       (L.MM_PLAN_ACCUMULATE if accumulate else 0) |
                                       (L.MM_PLAN_PEEL if peel else 0) |
                                       (L.MM_PLAN_TRANS_B if trans_b else 0) |
                                       (L.MM_PLAN_UNROLL_BASE if unroll_base else 0) |
                                       L.plan_split_k(split_k) | L.plan_pad(pad_to) |
                                       (L.MM_PLAN_LEVEL_PASSES if level_passes else 0),
                                       ctypes.byref(self._ptr)))
        self.accumulate = accumulate
        info = (ctypes.c_int64 * L.NINFO)()
        lib.mm_plan_info(self._ptr, info, L.NINFO)
        self.info = L._info_dict(info)
        self.ws_bytes = self.info["ws_bytes"]

    def describe(self):
        lib = L.load()
        need = lib.mm_plan_describe(self._ptr, None, 0)
        buf = ctypes.create_string_buffer(need + 1)
        lib.mm_plan_describe(self._ptr, buf, need + 1)
        return buf.value.decode()

    def __call__(self, A, B, C, ws=None, stream=None, beta=None):
        """C = A @ B, or C = A @ B + beta * C for an accumulating plan
        (beta None means 1)."""
        s = _stream(stream, self.device)
        if self.ws_bytes and ws is None:
            ws = workspace(self.ws_bytes, self.device, s)
        wptr = ws.data_ptr() if ws is not None else None
        wbytes = ws.numel() * ws.element_size() if ws is not None else 0
        if self.accumulate:
            L.check(L.load().mm_plan_execute_beta(self._ptr, A.data_ptr(), B.data_ptr(), C.data_ptr(), wptr,
                                                  wbytes, 1.0 if beta is None else float(beta), s.cuda_stream))
        else:
            if beta is not None:
                raise ValueError("beta needs a plan created with accumulate=True")
            L.check(L.load().mm_plan_execute(self._ptr, A.data_ptr(), B.data_ptr(), C.data_ptr(), wptr,
                                             wbytes, s.cuda_stream))
        return C

    def __del__(self):
        try:
            if self._ptr:
                L.load().mm_plan_destroy(self._ptr)
                self._ptr = ctypes.c_void_p()
        except Exception:
            pass


_plans = {}
_plans_lock = threading.Lock()
_ws = {}


def workspace(nbytes, device, stream):
    """A device buffer of at least ``nbytes`` bytes reserved for ``stream``."""
    key = (str(device), stream.cuda_stream)
    cur = _ws.get(key)
    if cur is None or cur.numel() < nbytes:
        if cur is not None:
            cur.record_stream(stream)
        cur = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws[key] = cur
    return cur


def get_plan(algo, sched, m, n, k, cutoff, levels, dtype, lda, ldb, ldc, graph, device, tile=None,
             fuse=False, overlap=False, leaf_u=False, split_pass=False, accumulate=False, peel=False,
             trans_b=False, split_k=None):
    key = (str(device), algo, sched, m, n, k, cutoff, levels, dtype, lda, ldb, ldc, graph, tile, fuse,
           overlap, leaf_u, split_pass, accumulate, peel, trans_b, split_k)
    with _plans_lock:
        p = _plans.get(key)
        if p is None:
            p = Plan(algo, sched, m, n, k, cutoff, levels, dtype, lda, ldb, ldc, graph, device, tile, fuse,
                     overlap, leaf_u, split_pass, accumulate, peel, trans_b, split_k=split_k)
            _plans[key] = p
    return p


def mm(A, B, algo="winograd", sched="auto", cutoff=None, levels=None, dtype=None, out=None,
       graph=False, stream=None, clobber_inputs=False, tile=None, fuse=False, overlap=None, leaf_u=None,
       split_pass=False, beta=None, peel=False, trans_b=None, split_k=None):
    """C = A @ B on the GPU by ``algo`` in {"naive", "strassen", "winograd"}.

    ``cutoff`` / ``levels`` control the recursion as in mm.h; when both are
    None the autotuner's choice for this size class is used (levels and leaf
    tile shape).

    ``sched``: "auto", "grouped", "two_temp", "in_place" (Winograd) or
    "auto", "grouped", "dfs3" (Strassen).  ``dtype``: None (from the tensors), "f64", "f32" or
    "bf16x3" (float32 tensors, split-bfloat16 leaf products).  ``fuse`` /
    ``overlap`` / ``leaf_u``: MM_PLAN_FUSE / MM_PLAN_OVERLAP / MM_PLAN_LEAF_U
    (None: the autotuner's choice when it picks the recursion, else off);
    ``split_pass``: MM_PLAN_SPLIT_PASS.  ``beta`` (needs ``out``): the
    accumulating form out = A @ B + beta * out (MM_PLAN_ACCUMULATE).  ``peel``:
    MM_PLAN_PEEL (grouped schedule: thin products for ragged edges instead of
    zero padding).  ``trans_b``: MM_PLAN_TRANS_B (None: the autotuner's choice
    when it picks the recursion, else off).  ``split_k``: MM_PLAN_SPLIT_K for
    plain products (None: the autotuner's choice when it picks the levels).  The in-place
    schedule overwrites its operands, so unless ``clobber_inputs`` is set the
    wrapper hands it copies.
    """
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be device tensors")
    if A.device != B.device:
        raise ValueError("A and B are on different devices")
    dt = _resolve_dtype(A, dtype)
    _resolve_dtype(B, dt)
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {tuple(A.shape)} x {tuple(B.shape)}")
    m, k = A.shape
    n = B.shape[1]
    if sched == "in_place" and not clobber_inputs:
        A = A.contiguous().clone()
        B = B.contiguous().clone()
    lda, ldb = _ld(A, "A"), _ld(B, "B")
    if beta is not None and out is None:
        raise ValueError("beta needs out (the C that is accumulated into)")
    C = out if out is not None else torch.empty((m, n), dtype=A.dtype, device=A.device)
    if C.shape != (m, n) or C.dtype != A.dtype or C.device != A.device:
        raise ValueError("out has the wrong shape, dtype or device")
    ldc = _ld(C, "out")
    if m == 0 or n == 0:
        return C
    if cutoff is None and levels is None:
        if algo == "naive":
            cutoff, levels = 1, 0
            from . import tuner
            ch = tuner.choose(m, n, k, dt)
            bp = ch.get("best_plain") or (ch if ch.get("levels") == 0 else {})
            if tile is None:
                tile = bp.get("tile")
            if split_k is None:
                split_k = bp.get("split_k")
        else:
            from . import tuner
            ch = tuner.choose(m, n, k, dt)
            cutoff, levels = 1, ch["levels"]
            if tile is None:
                tile = ch["tile"]
            if overlap is None:
                overlap = bool(ch.get("overlap", False))
            if leaf_u is None:
                leaf_u = bool(ch.get("leaf_u", False))
            if trans_b is None:
                trans_b = bool(ch.get("trans_b", False))
            if split_k is None:
                split_k = ch.get("split_k")
    elif cutoff is None:
        cutoff = 1
    elif levels is None:
        levels = -1
    p = get_plan(algo, sched, m, n, k, cutoff, levels, dt, lda, ldb, ldc, graph, A.device, tile, fuse,
                 bool(overlap), bool(leaf_u), bool(split_pass), beta is not None, bool(peel), bool(trans_b),
                 split_k)
    with torch.cuda.device(A.device):
        p(A, B, C, stream=stream, beta=beta)
    return C


class BatchedPlan:
    """Independent products C_i = A_i B_i bound to fixed tensors
    (mm_batched_plan_create).  Run with ``plan()``; with ``graph=True`` the
    launch sequence is captured once and replayed.  ``levels=None``: each
    problem's tuned level count for its size class; ``persistent=True``
    (float32): the whole batch as one persistent launch."""

    def __init__(self, As, Bs, Cs, cutoff=None, levels=None, dtype=None, graph=True, tile=None,
                 persistent=False):
        lib = L.load()
        if not (len(As) == len(Bs) == len(Cs)):
            raise ValueError("As, Bs, Cs differ in length")
        cnt = len(As)
        dt = _resolve_dtype(As[0], dtype) if cnt else (dtype or "f32")
        self.device = As[0].device if cnt else torch.device("cuda", torch.cuda.current_device())
        mnk = []
        for a, b, c in zip(As, Bs, Cs):
            for t, nm in ((a, "A"), (b, "B"), (c, "C")):
                _resolve_dtype(t, dt)
                if not t.is_contiguous():
                    raise ValueError(f"batched {nm} must be contiguous")
            if a.shape[1] != b.shape[0] or c.shape != (a.shape[0], b.shape[1]):
                raise ValueError("batched shape mismatch")
            mnk.append((a.shape[0], b.shape[1], a.shape[1]))
        self.tensors = (list(As), list(Bs), list(Cs))  # keep the bound memory alive
        self.mnk = mnk
        flat = (ctypes.c_int64 * (3 * max(cnt, 1)))(*[v for t in mnk for v in t])
        Ap = (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in As])
        Bp = (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in Bs])
        Cp = (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in Cs])
        cp = (ctypes.c_int * cnt)(*cutoff) if cutoff is not None else None
        lp = (ctypes.c_int * cnt)(*levels) if levels is not None else None
        self._ptr = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.mm_batched_plan_create(cnt, flat, Ap, Bp, Cp, L.DTYPES[dt], cp, lp,
                                               (L.MM_PLAN_GRAPH if graph else 0) | L.plan_tile(tile) |
                                               (L.MM_PLAN_PERSISTENT if persistent else 0),
                                               ctypes.byref(self._ptr)))
        info = (ctypes.c_int64 * L.NINFO)()
        lib.mm_plan_info(self._ptr, info, L.NINFO)
        self.info = L._info_dict(info)
        self.ws_bytes = self.info["ws_bytes"]
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)

    def __call__(self, stream=None):
        s = _stream(stream, self.device)
        L.check(L.load().mm_plan_execute(self._ptr, None, None, None, self.ws.data_ptr(),
                                         self.ws.numel(), s.cuda_stream))
        return self.tensors[2]

    def check(self, stream=None):
        """Wait for ``stream`` and raise if a task of a persistent launch
        waited past its bound since the last check (mm_plan_check)."""
        s = _stream(stream, self.device)
        L.check(L.load().mm_plan_check(self._ptr, s.cuda_stream))

    def __del__(self):
        try:
            if self._ptr:
                L.load().mm_plan_destroy(self._ptr)
                self._ptr = ctypes.c_void_p()
        except Exception:
            pass
