"""Test-side simulator of libmm launch sequences (not the oracle).

``mm_describe`` lists a plan as text, one line per block operation and one
``LAUNCH`` line closing each kernel launch (tagged ``aux`` when it runs on
the plan's auxiliary stream, between ``FORK`` and ``JOIN`` lines).  This
module parses that listing and executes it on numpy buffers, doing per
block what the kernels do per element: reads outside a view's valid extent give zero, writes there are
dropped, element-wise recipes combine their inputs, GEMM descriptors form
a @ b and apply their epilogues, and WINO descriptors (a last Winograd level
in one kernel) form the seven products and write the four U combinations.  It also checks that no two operations of
one launch touch memory in a conflicting way (the kernels of one launch run
concurrently), and that launches on the two streams of a fork window never
touch memory the other stream writes, so a planner bug shows up as a hazard
even when the numbers happen to come out right.

Run on integer matrices, the simulated product must equal the oracle's
exactly.
"""
import numpy as np

EW_COPY, EW_ADD, EW_SUB, EW_WINO_S, EW_WINO_T, EW_WINO_U, EW_TT_U = range(7)
EW_IP_A, EW_IP_B, EW_IP_U, EW_DIST, EW_ZERO = 7, 8, 9, 10, 11
EW_SPLIT, EW_WINO_S_SPL, EW_WINO_T_SPL, EW_WINO_U_ACC, EW_AXPBY = 12, 13, 14, 15, 16
EW_STR_S, EW_STR_T, EW_STR_U, EW_STR_U_ACC = 17, 18, 19, 20
EW_WINO_T_TR = 21
EW_SUM, EW_SUM_ACC = 22, 23
EW2_S, EW2_T, EW2_U = 0, 1, 2
OK_TRANS = 9
GM_STORE, GM_ADD, GM_AXPBY = 1, 2, 3
MB_A, MB_B, MB_C, MB_WS, MB_ABS = 0, 1, 2, 3, 4


class View:
    __slots__ = ("base", "off", "ld", "rows", "cols", "vrows", "vcols")

    def __init__(self, fields):
        (self.base, self.off, self.ld, self.rows, self.cols, self.vrows, self.vcols) = fields

    def index(self, valid_only=True):
        r = self.vrows if valid_only else self.rows
        c = self.vcols if valid_only else self.cols
        return (self.off + np.arange(r, dtype=np.int64)[:, None] * self.ld
                + np.arange(c, dtype=np.int64)[None, :])


def spl_index(v, valid_only=True):
    """bfloat16 indices of the hi / lo / res slots of an SPL matrix view
    (rows x cols, chunks of 8 columns, 24 slots per chunk)."""
    r = v.vrows if valid_only else v.rows
    c = v.vcols if valid_only else v.cols
    k = np.arange(c, dtype=np.int64)
    base = (v.off + np.arange(r, dtype=np.int64)[:, None] * v.ld + (k // 8 * 24 + k % 8)[None, :])
    return base, base + 8, base + 16


def _spl_footprint(v):
    if v is None or not (v.vrows and v.vcols):
        return set()
    idx = np.concatenate([x.ravel() for x in spl_index(v)]) // 2  # 4-byte units
    return set(zip([v.base] * idx.size, idx.tolist()))


def _view(tok):
    if tok == "-":
        return None
    return View([int(x) for x in tok.split(":")])


def parse(text):
    """List of launches; each launch is ("EW"|"GEMM", [items], stream) with
    stream 0 (the caller's) or 1 (the plan's auxiliary stream), or a
    ("FORK"|"JOIN", [], 0) marker."""
    launches, cur = [], []
    for line in text.splitlines():
        if not line.strip():
            continue
        if line.startswith("PDEP"):
            continue      # dependency of a persistent batch's task (checked by the host tests)
        if line in ("FORK", "JOIN"):
            assert not cur, "fork/join inside a launch"
            launches.append((line, [], 0))
            continue
        if line.startswith("LAUNCH"):
            words = line.split()
            _, kind, cnt, _grid = words[:4]
            assert len(cur) == int(cnt), (line, len(cur))
            assert all(it[0] == kind for it in cur)
            if "fused" in words[4:]:
                for _, it in cur:
                    check_fused_preconditions(it)
            if "spl" in words[4:]:
                for _, it in cur:
                    it["spl"] = True
            launches.append((kind, cur, 1 if words[-1] == "aux" else 0))
            cur = []
            continue
        head, *rest = [s.strip() for s in line.split("|")]
        h = head.split()
        if h[0] == "BASE":
            a, b, c = [_view(t) for t in rest[0].split()]
            cur.append(("BASE", dict(order=int(h[1]), a=a, b=b, c=c)))
            continue
        if h[0] == "EW2":
            kind, rows, cols = map(int, h[1:])
            x = _view(rest[0].split()[0])
            top = [_view(t) for t in rest[1].split()]
            low = [_view(t) for t in rest[2].split()]
            per = 7 if kind == EW2_U else 4
            assert len(top) == 4 and len(low) == 7 * per
            cur.append(("EW2", dict(kind=kind, rows=rows, cols=cols, x=x, top=top,
                                    low=[low[per * q:per * q + per] for q in range(7)])))
            continue
        if h[0] == "TRANS":
            kind, rows, cols = map(int, h[1:])
            ins = [_view(t) for t in rest[0].split()]
            outs = [_view(t) for t in rest[1].split()]
            cur.append(("TRANS", dict(kind=kind, rows=rows, cols=cols, ins=ins, outs=outs)))
            continue
        if h[0] == "SPLIT":
            kind, rows, cols, mode = map(int, h[1:])
            ins = [_view(t) for t in rest[0].split()]
            outs = [_view(t) for t in rest[1].split()]
            cur.append(("SPLIT", dict(kind=kind, rows=rows, cols=cols, mode=mode, ins=ins, outs=outs)))
        elif h[0] == "WINO":
            m, n, k, acc, fused = map(int, h[1:])
            ops = [_view(t) for t in rest[0].split()]
            cs = [_view(t) for t in rest[1].split()]
            assert len(ops) == 14 and len(cs) == 4
            cur.append(("WINO", dict(m=m, n=n, k=k, acc=acc, fused=fused, a=ops[0::2], b=ops[1::2], c=cs)))
        elif h[0] == "EW":
            kind, rows, cols, m0, m1 = map(int, h[1:])
            ins = [_view(t) for t in rest[0].split()] if rest[0] else []
            outs = [_view(t) for t in rest[1].split()] if rest[1] else []
            cur.append(("EW", dict(kind=kind, rows=rows, cols=cols, mode=(m0, m1), ins=ins, outs=outs)))
        else:
            m, n, k, ak, bk = map(int, h[1:])
            a, b = [_view(t) for t in rest[0].split()]
            outs = []
            for tok in rest[1].split():
                f = tok.split(":")
                mode, sign = int(f[0]), int(f[1])
                c = View([int(x) for x in f[2:9]])
                d = None if f[9] == "-" else View([int(x) for x in f[9:16]])
                outs.append((mode, sign, c, d))
            cur.append(("GEMM", dict(m=m, n=n, k=k, a=a, b=b, outs=outs, ak=ak, bk=bk)))
    assert not cur, "listing ends inside a launch"
    check_streams(launches)
    return launches


def check_streams(launches):
    """Auxiliary-stream launches appear only between FORK and JOIN, windows do
    not nest, and no launch on one stream inside a window touches memory that
    a launch on the other stream writes (the two streams run concurrently)."""
    inside = False
    window = []
    for kind, items, stream in launches:
        if kind == "FORK":
            assert not inside, "nested fork"
            inside, window = True, []
        elif kind == "JOIN":
            assert inside, "join without fork"
            assert any(st == 1 for _, _, st in window), "empty auxiliary window"
            fp = {0: (set(), set()), 1: (set(), set())}
            for k2, it2, st in window:
                r, w = _launch_footprint(k2, it2)
                fp[st][0].update(r)
                fp[st][1].update(w)
            (r0, w0), (r1, w1) = fp[0], fp[1]
            assert not (w0 & w1), "both streams write the same memory"
            assert not (w0 & r1) and not (w1 & r0), "one stream writes what the other reads"
            inside = False
        else:
            assert inside or stream == 0, "auxiliary launch outside a fork window"
            if inside:
                window.append((kind, items, stream))
    assert not inside, "listing ends inside a fork window"


def _sub_view(v, sa, sc):
    """Sub-block (sa, sc) of the 2 x 2 split of view v."""
    r, c = v.rows // 2, v.cols // 2
    return View([v.base, v.off + sa * r * v.ld + sc * c, v.ld, r, c,
                 max(0, min(r, v.vrows - sa * r)), max(0, min(c, v.vcols - sc * c))])


def _ew2_written_top(it):
    """The parts of an EW2 pass's top views it writes: all of a U pass's C
    quadrants; three of the four sub-blocks of each upper-level sum (the one
    the lower level never reads plainly is skipped)."""
    if it["kind"] == EW2_U:
        return [(v, None, k) for k, v in enumerate(it["top"])]
    skip = (1, 0) if it["kind"] == EW2_S else (0, 1)
    return [(_sub_view(v, sa, sc), (sa, sc), k) for k, v in enumerate(it["top"]) for sa in (0, 1)
            for sc in (0, 1) if (sa, sc) != skip]


def _ew2_footprint(it):
    if it["kind"] == EW2_U:
        reads = set().union(*[_footprint(v) for row in it["low"] for v in row])
        writes = set().union(*[_footprint(v) for v in it["top"]])
    else:
        reads = _footprint(it["x"])
        writes = set().union(*[_footprint(v) for v, _, _ in _ew2_written_top(it)])
        writes |= set().union(*[_footprint(v) for row in it["low"] for v in row])
    return reads, writes


def _launch_footprint(kind, items):
    reads, writes = set(), set()
    for _, it in items:
        if kind == "EW2":
            r, w = _ew2_footprint(it)
            reads |= r
            writes |= w
        elif kind in ("EW", "TRANS"):
            for v in it["ins"]:
                reads |= _footprint(v)
            for v in it["outs"]:
                writes |= _footprint(v)
        elif kind == "BASE":
            reads |= _footprint(it["a"]) | _footprint(it["b"])
            writes |= _footprint(it["c"])
        elif kind == "WINO":
            for v in it["a"] + it["b"]:
                reads |= _footprint(v)
            for v in it["c"]:
                writes |= _footprint(v)
        elif kind == "SPLIT":
            for v in it["ins"]:
                reads |= _footprint(v)
            for v in it["outs"]:
                writes |= _spl_footprint(v)
        else:
            fp = _spl_footprint if it.get("spl") else _footprint
            reads |= fp(it["a"]) | fp(it["b"])
            for mode, sign, c, d in it["outs"]:
                writes |= _footprint(c)
                if d is not None and mode in (GM_ADD, GM_AXPBY):
                    reads |= _footprint(d)
    return reads, writes


def check_fused_preconditions(it, vec=4):
    """The fused loader reads every operand (or parent block) with 16-byte
    vector loads and no masks: offsets and leading dimensions must be
    multiples of the vector width and the blocks entirely valid."""
    for v in (it["a"], it["b"]):
        assert v.off % vec == 0 and v.ld % vec == 0, "fused operand not 16-byte aligned"
        assert v.vrows == v.rows and v.vcols == v.cols, "fused operand partially valid"
    for kind, v in ((it["ak"], it["a"]), (it["bk"], it["b"])):
        if kind:
            assert (v.cols // 2) % vec == 0 and v.rows % 2 == 0 and v.cols % 2 == 0


class Memory:
    def __init__(self, bufs):
        self.bufs = bufs  # base -> flat numpy array
        self.spl = {}     # base -> bfloat16 slots of SPL matrices (values kept exactly)

    def spl_read(self, v):
        out = np.zeros((v.rows, v.cols), dtype=self.dtype)
        if v.vrows and v.vcols:
            mem = self.spl[v.base]
            hi, lo, rs = spl_index(v)
            out[:v.vrows, :v.vcols] = mem[hi] + mem[lo] + mem[rs]
        return out

    def spl_write(self, v, val):
        # the simulator keeps each value whole in the hi slot
        mem = self.spl.setdefault(v.base, np.zeros(2 * len(self.bufs[v.base]), dtype=self.dtype))
        if v.vrows and v.vcols:
            hi, lo, rs = spl_index(v)
            mem[hi] = val[:v.vrows, :v.vcols]
            mem[lo] = 0
            mem[rs] = 0

    def read(self, v, shape=None):
        rows, cols = (v.rows, v.cols) if shape is None else shape
        out = np.zeros((rows, cols), dtype=self.dtype)
        r, c = min(v.vrows, rows), min(v.vcols, cols)
        if r and c:
            out[:r, :c] = self.bufs[v.base][v.index()[:r, :c]]
        return out

    def write(self, v, val):
        if v.vrows and v.vcols:
            self.bufs[v.base][v.index()] = val[:v.vrows, :v.vcols]

    @property
    def dtype(self):
        return next(iter(self.bufs.values())).dtype


def _recipe(kind, x, mode):
    if kind == EW_COPY:
        return [x[0]]
    if kind == EW_ADD:
        return [x[0] + x[1]]
    if kind == EW_SUB:
        return [x[0] - x[1]]
    if kind == EW_WINO_S:
        a11, a12, a21, a22 = x
        s1 = a21 + a22
        s2 = s1 - a11
        return [s1, s2, a11 - a21, a12 - s2]
    if kind == EW_WINO_T:
        b11, b12, b21, b22 = x
        t1 = b12 - b11
        t2 = b22 - t1
        return [t1, t2, b22 - b12, t2 - b21]
    if kind == EW_WINO_U:
        p1, p2, p3, p4, p5, p6, p7 = x
        u2 = p1 + p6
        u3 = u2 + p7
        return [p1 + p2, u2 + p5 + p3, u3 - p4, u3 + p5]
    if kind == EW_STR_S:
        a11, a12, a21, a22 = x
        return [a11 + a22, a21 + a22, a11 + a12, a21 - a11, a12 - a22]
    if kind == EW_STR_T:
        b11, b12, b21, b22 = x
        return [b11 + b22, b12 - b22, b21 - b11, b11 + b12, b21 + b22]
    if kind == EW_STR_U:
        p1, p2, p3, p4, p5, p6, p7 = x
        return [((p1 + p4) - p5) + p7, p3 + p5, p2 + p4, ((p1 + p3) - p2) + p6]
    if kind == EW_TT_U:
        xp, c11, c12, c21, c22 = x
        u2 = xp + c12
        u3 = u2 + c21
        return [u2 + c22 + c11, u3, u3 + c22]
    if kind == EW_IP_A:
        a11, a21, a22 = x
        return [a11 - a21, a21 + a22]
    if kind == EW_IP_B:
        b11, b12, b22 = x
        return [b12 - b11, b22 - b12]
    if kind == EW_IP_U:
        p1, p2, u2, p5, p7, p4 = x
        u3 = u2 + p7
        return [p1 + p2, u2 + p5, u3 - p4, u3 + p5]
    if kind == EW_DIST:
        z, d0, d1 = x
        out = []
        for md, d in zip(mode, (d0, d1)):
            if d is None:
                break
            out.append(z if md == 1 else (d + z if md == 2 else d - z))
        return out
    if kind == EW_ZERO:
        return [np.zeros_like(x[0]) if x else None]
    raise ValueError(kind)


def _footprint(v):
    if v is None or not (v.vrows and v.vcols):
        return set()
    return set(zip([v.base] * (v.vrows * v.vcols), v.index().ravel().tolist()))


def check_hazards(launch):
    """No operation of a launch writes what another one reads or writes, and
    a GEMM never writes its own operands (element-wise parts may read and
    write the same element in place)."""
    kind, items = launch[0], launch[1]
    reads, writes = [], []
    for _, it in items:
        if kind == "EW":
            r = set().union(*[_footprint(v) for v in it["ins"]]) if it["ins"] else set()
            w = set().union(*[_footprint(v) for v in it["outs"]])
            # in-place element-wise: an input element may be rewritten only at
            # the same (row, col) position of the block
            for v_in in it["ins"]:
                if v_in is None:
                    continue
                for v_out in it["outs"]:
                    if v_in.base != v_out.base:
                        continue
                    ii = v_in.index()
                    oi = v_out.index()
                    common = np.intersect1d(ii, oi)
                    if common.size:
                        pos_in = {int(x): p for p, x in enumerate(ii.ravel().tolist())}
                        pos_out = {int(x): p for p, x in enumerate(oi.ravel().tolist())}
                        ci = ii.shape[1]
                        co = oi.shape[1]
                        for x in common.tolist():
                            pi, po = pos_in[x], pos_out[x]
                            assert (pi // ci, pi % ci) == (po // co, po % co), "EW cross-element alias"
        elif kind == "EW2":
            r, w = _ew2_footprint(it)
            assert not (w & r), "EW2 writes its own inputs"
            outs = [v for v, _, _ in _ew2_written_top(it)] + ([] if it["kind"] == EW2_U else
                                                            [v for row in it["low"] for v in row])
            assert sum(len(_footprint(v)) for v in outs) == len(w), "EW2 outputs overlap"
            R, C = it["rows"], it["cols"]
            for v in it["top"]:
                assert (v.rows, v.cols) == (2 * R, 2 * C), "EW2 upper block of another shape"
            for row in it["low"]:
                for v in row:
                    assert (v.rows, v.cols) == (R, C), "EW2 lower block of another shape"
        elif kind == "BASE":
            r, w = _footprint(it["a"]) | _footprint(it["b"]), _footprint(it["c"])
            assert not (w & r), "BASE writes its own operands"
            for v in (it["a"], it["b"], it["c"]):
                assert v.rows == v.cols == it["order"], "BASE block of another order"
        elif kind == "TRANS":
            r, w = _launch_footprint("EW", [(kind, it)])
            assert sum(len(_footprint(v)) for v in it["outs"]) == len(w), "TRANS outputs overlap"
            assert not (w & r), "TRANS writes its own inputs"
            for v in it["outs"]:
                assert (v.rows, v.cols) == (it["cols"], it["rows"]), "TRANS output not transposed"
                assert v.off % 4 == 0 and v.ld % 4 == 0, "TRANS output rows not 16-byte aligned"
        elif kind == "SPLIT":
            r, w = _launch_footprint(kind, [(kind, it)])
            assert sum(len(_spl_footprint(v)) for v in it["outs"]) == len(w), "SPLIT outputs overlap"
            assert not (w & r), "SPLIT writes its own inputs"
        elif kind == "WINO":
            r, w = _launch_footprint(kind, [(kind, it)])
            fcs = [_footprint(v) for v in it["c"]]
            assert sum(len(f) for f in fcs) == len(w), "WINO output quadrants overlap"
            assert not (w & r), "WINO writes its own operands"
        else:
            fp = _spl_footprint if it.get("spl") else _footprint
            r = fp(it["a"]) | fp(it["b"])
            w = set()
            for mode, sign, c, d in it["outs"]:
                fc = _footprint(c)
                assert not (fc & r), "GEMM writes its own operand"
                assert not (fc & w), "GEMM outputs overlap"
                w |= fc
                if d is not None and mode in (GM_ADD, GM_AXPBY):
                    fd = _footprint(d)
                    if fd & fc:
                        assert d.off == c.off and d.ld == c.ld and d.base == c.base, \
                            "GEMM epilogue reads C elsewhere than it writes"
                    r |= fd - fc
        reads.append(r)
        writes.append(w)
    for i in range(len(items)):
        for j in range(len(items)):
            if i != j:
                assert not (writes[i] & writes[j]), f"{kind}: two operations write the same memory"
                assert not (writes[i] & reads[j]), f"{kind}: one operation writes what another reads"


def operand(M, kind):
    """Operand of a leaf product: the block itself, or the Winograd sum of
    its quadrants named by kind (1..4: S1..S4, 5..8: T1..T4)."""
    if kind == 0:
        return M
    if kind == OK_TRANS:  # the view holds the transpose of the operand
        return M.T
    r, c = M.shape[0] // 2, M.shape[1] // 2
    q11, q12, q21, q22 = M[:r, :c], M[:r, c:], M[r:, :c], M[r:, c:]
    if kind <= 4:
        s1 = q21 + q22
        s2 = s1 - q11
        return {1: s1, 2: s2, 3: q11 - q21, 4: q12 - s2}[kind]
    t1 = q12 - q11
    t2 = q22 - t1
    return {5: t1, 6: t2, 7: q22 - q12, 8: t2 - q21}[kind]


def unrolled_winograd(a, b):
    """The 22-operation form of Section 2.3 applied down to scalars (orders
    1, 2, 4, 8): what an unrolled base case computes."""
    n = a.shape[0]
    if n == 1:
        return a * b
    h = n // 2
    a11, a12, a21, a22 = a[:h, :h], a[:h, h:], a[h:, :h], a[h:, h:]
    b11, b12, b21, b22 = b[:h, :h], b[:h, h:], b[h:, :h], b[h:, h:]
    s1 = a21 + a22
    s2 = s1 - a11
    s3 = a11 - a21
    s4 = a12 - s2
    t1 = b12 - b11
    t2 = b22 - t1
    t3 = b22 - b12
    t4 = t2 - b21
    p = [unrolled_winograd(x, y) for x, y in ((a11, b11), (a12, b21), (s4, b22), (a22, t4), (s1, t1),
                                              (s2, t2), (s3, t3))]
    u2 = p[0] + p[5]
    u3 = u2 + p[6]
    c = np.empty_like(a)
    c[:h, :h] = p[0] + p[1]
    c[:h, h:] = (u2 + p[4]) + p[2]
    c[h:, :h] = u3 - p[3]
    c[h:, h:] = u3 + p[4]
    return c


def _quads(m):
    r, c = m.shape[0] // 2, m.shape[1] // 2
    return m[:r, :c], m[:r, c:], m[r:, :c], m[r:, c:]


def _ew2_run(mem, it):
    """Two recursion levels of Section 2.3's pre- or post-additions (an EW2
    part), level by level, as the two separate passes compute them."""
    outs = []
    if it["kind"] == EW2_U:
        def u(p):  # U1 U5 U6 U7 of P1..P7, assembled into one block
            u2 = p[0] + p[5]
            u3 = u2 + p[6]
            return np.block([[p[0] + p[1], (u2 + p[4]) + p[2]], [u3 - p[3], u3 + p[4]]])
        upper = [u([mem.read(v) for v in row]) for row in it["low"]]
        c = u(upper)
        for v, q in zip(it["top"], _quads(c)):
            outs.append((v, q))
        return outs
    x = mem.read(it["x"])
    q11, q12, q21, q22 = _quads(x)
    if it["kind"] == EW2_S:
        s1 = q21 + q22
        s2 = s1 - q11
        sums = [s1, s2, q11 - q21, q12 - s2]
        ops = [q11, q12, sums[3], q22, sums[0], sums[1], sums[2]]
    else:
        t1 = q12 - q11
        t2 = q22 - t1
        sums = [t1, t2, q22 - q12, t2 - q21]
        ops = [q11, q21, q22, sums[3], sums[0], sums[1], sums[2]]
    for v, (sa, sc), k in _ew2_written_top(it):
        outs.append((v, _quads(sums[k])[2 * sa + sc]))
    for o, row in zip(ops, it["low"]):
        o11, o12, o21, o22 = _quads(o)
        if it["kind"] == EW2_S:
            z1 = o21 + o22
            z2 = z1 - o11
            z = [z1, z2, o11 - o21, o12 - z2]
        else:
            z1 = o12 - o11
            z2 = o22 - z1
            z = [z1, z2, o22 - o12, z2 - o21]
        outs.extend(zip(row, z))
    return outs


def run(text, bufs, hazards=True, beta=1):
    mem = Memory(bufs)
    for launch in parse(text):
        kind, items = launch[0], launch[1]
        if kind in ("FORK", "JOIN"):
            continue
        if hazards:
            check_hazards(launch)
        results = []
        for _, it in items:
            if kind == "EW":
                x = [mem.read(v, (it["rows"], it["cols"])) if v is not None else None
                     for v in it["ins"]]
                if it["kind"] == EW_ZERO:
                    y = [np.zeros((it["rows"], it["cols"]), dtype=mem.dtype)]
                elif it["kind"] in (EW_WINO_U_ACC, EW_STR_U_ACC):
                    base = EW_WINO_U if it["kind"] == EW_WINO_U_ACC else EW_STR_U
                    u = _recipe(base, x[:7], it["mode"])
                    y = [beta * c + v for c, v in zip(x[7:], u)]
                elif it["kind"] == EW_AXPBY:
                    y = [beta * x[1] + x[0]]
                elif it["kind"] in (EW_SUM, EW_SUM_ACC):
                    npart = it["mode"][0]
                    s = x[0]
                    for v in x[1:npart]:
                        s = s + v
                    y = [beta * x[npart] + s if it["kind"] == EW_SUM_ACC else s]
                else:
                    y = _recipe(it["kind"], x, it["mode"])
                results.append(list(zip(it["outs"], y)))
            elif kind == "EW2":
                results.append(_ew2_run(mem, it))
            elif kind == "BASE":
                results.append([(it["c"], unrolled_winograd(mem.read(it["a"]), mem.read(it["b"])))])
            elif kind == "TRANS":
                x = [mem.read(v, (it["rows"], it["cols"])) for v in it["ins"]]
                assert it["kind"] == EW_WINO_T_TR
                b11, b12, b21, b22 = x
                t1 = b12 - b11
                t2 = b22 - t1
                y = [t1, t2, b22 - b12, t2 - b21, b11, b21, b22]
                results.append([(v, t.T) for v, t in zip(it["outs"], y)])
            elif kind == "SPLIT":
                x = [mem.read(v, (it["rows"], it["cols"])) for v in it["ins"]]
                if it["kind"] == EW_SPLIT:
                    y = [x[0]]
                elif it["kind"] == EW_WINO_S_SPL:
                    a11, a12, a21, a22 = x
                    s1 = a21 + a22
                    s2 = s1 - a11
                    y = [s1, s2, a11 - a21, a12 - s2, a11, a12, a22]
                else:
                    b11, b12, b21, b22 = x
                    t1 = b12 - b11
                    t2 = b22 - t1
                    y = [t1, t2, b22 - b12, t2 - b21, b11, b21, b22]
                if it["mode"]:
                    y = [t.T for t in y]
                results.append([("spl", v, t) for v, t in zip(it["outs"], y)])
            elif kind == "WINO":
                # fused: P3..P7 read the parent blocks and form S4, S1..S3 / T4, T1..T3
                ak, bk = ((0, 0, 4, 0, 1, 2, 3), (0, 0, 0, 8, 5, 6, 7)) if it["fused"] else ((0,) * 7, (0,) * 7)
                p = [operand(mem.read(a), ka) @ operand(mem.read(b), kb)
                     for a, b, ka, kb in zip(it["a"], it["b"], ak, bk)]
                u2 = p[0] + p[5]
                u3 = u2 + p[6]
                u4 = u2 + p[4]
                vals = [p[0] + p[1], u4 + p[2], u3 - p[3], u3 + p[4]]
                if it["acc"]:
                    vals = [beta * mem.read(c) + v for c, v in zip(it["c"], vals)]
                results.append(list(zip(it["c"], vals)))
            else:
                if it.get("spl"):
                    a = mem.spl_read(it["a"])
                    b = mem.spl_read(it["b"]).T
                else:
                    a = operand(mem.read(it["a"]), it["ak"])
                    b = operand(mem.read(it["b"]), it["bk"])
                acc = a @ b
                outs = []
                for mode, sign, c, d in it["outs"]:
                    if mode == GM_STORE:
                        val = sign * acc
                    elif mode == GM_AXPBY:
                        val = beta * mem.read(d) + sign * acc
                    else:
                        val = mem.read(d) + sign * acc
                    outs.append((c, val))
                results.append(outs)
        for outs in results:
            for o in outs:
                if o[0] == "spl":
                    mem.spl_write(o[1], o[2])
                else:
                    mem.write(*o)
    return mem
