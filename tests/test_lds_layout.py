"""LDS layouts of the MFMA tile loop (paper_2309_00628_amd/csrc/gemm_tile.h,
gemm_common.h) checked for bank conflicts on the host.

gfx950's LDS has 64 four-byte banks: a 16-byte access is served 16 lanes
per cycle, and those lanes hit distinct banks when their 16-byte slots are
distinct modulo 16 (rocprofv3's SQ_LDS_BANK_CONFLICT reads 0 for these
kernels).  The stores and the B reads are also free of conflicts in groups
of 8 lanes (an LDS serving 128 bytes per cycle); the A fragment reads are
not (two rows share a slot modulo 8), which this test records.
The slot formulas of the kernels are restated here (a_idx with the row XOR,
b_idx with swz_b, and the row layout of float32 B) and every access phase
of every instantiated tile shape is checked: the fragment reads of the K
loop and the register-path stores of edge tiles.  The kernels' bits are
checked on the GPU; this test pins only the address patterns.
"""
import pytest

# (T, BM, BN, BKC, WGM, WGN) of every GEMM / fused-U tile loop instantiation
F32_TILES = [(128, 128, 8, 4, 2), (256, 128, 8, 4, 2), (128, 256, 8, 2, 4), (256, 256, 8, 4, 2),
             (64, 128, 8, 2, 2), (128, 64, 8, 2, 2), (256, 128, 4, 2, 2), (128, 128, 4, 2, 2),
             (128, 128, 8, 2, 2), (64, 64, 8, 2, 2)]
F64_TILES = [(128, 128, 8, 2, 2), (128, 64, 8, 2, 2)]
MT = {"f32": dict(TM=32, KG=2, E=4), "f64": dict(TM=16, KG=4, E=2)}


def a_idx(row, kc, bkc):
    return row * bkc + (kc ^ ((row // (16 // bkc)) & (bkc - 1)))


def swz_b(col, e):
    if e == 4:
        return col ^ (((col >> 3) ^ (col >> 5)) & 3)
    return col ^ (((col >> 3) ^ (col >> 4)) & 1)


def b_idx(col, kc, bn, e):
    return kc * bn + swz_b(col, e)


def conflict_free(slots, width):
    """Slots of consecutive lanes: every aligned group of `width` lanes
    touches `width` distinct bank groups."""
    for g in range(0, len(slots), width):
        grp = [s % width for s in slots[g:g + width]]
        if len(set(grp)) != len(grp):
            return False
    return True


def tiles():
    for t in F32_TILES:
        yield ("f32",) + t
    for t in F64_TILES:
        yield ("f64",) + t


@pytest.mark.parametrize("dt,bm,bn,bkc,wgm,wgn", list(tiles()))
@pytest.mark.parametrize("width", [8, 16])
def test_a_fragment_reads_and_stores(dt, bm, bn, bkc, wgm, wgn, width):
    # the reads: 16 lanes per cycle; the stores: 8 or 16
    tm, kg = MT[dt]["TM"], MT[dt]["KG"]
    wm = bm // wgm
    nt = 64 * wgm * wgn
    # fragment reads: lane (g, t) of wave row wm0 reads row wm0 WM + a TM + t, chunk plane kb KG + g
    for wm0 in range(wgm):
        for a in range(wm // tm):
            for kb in range(bkc // kg):
                slots = [a_idx(wm0 * wm + a * tm + (l % tm), kb * kg + l // tm, bkc) for l in range(64)]
                assert len(set(slots)) == len(slots)
                assert conflict_free(slots, 16), (wm0, a, kb)
                if width == 8:
                    assert not conflict_free(slots, 8) or bkc < 8
    # register-path stores: thread q writes chunk (q / BKC, q % BKC)
    for i in range((bm * bkc + nt - 1) // nt):
        slots = [a_idx(q // bkc, q % bkc, bkc) for q in range(i * nt, min((i + 1) * nt, bm * bkc))]
        assert conflict_free(slots, width), i


@pytest.mark.parametrize("bm,bn,bkc,wgm,wgn", F64_TILES)
@pytest.mark.parametrize("width", [8, 16])
def test_k_chunked_b_float64(bm, bn, bkc, wgm, wgn, width):
    tm, kg, e = MT["f64"]["TM"], MT["f64"]["KG"], MT["f64"]["E"]
    wn = bn // wgn
    nt = 64 * wgm * wgn
    for wn0 in range(wgn):
        for b in range(wn // tm):
            for kb in range(bkc // kg):
                slots = [b_idx(wn0 * wn + b * tm + (l % tm), kb * kg + l // tm, bn, e) for l in range(64)]
                assert conflict_free(slots, width), (wn0, b, kb)
    # register-path stores: thread q holds the E x E block (kc, cb) and
    # writes column cb E + c for each c
    nblk = bkc * (bn // e)
    for i in range((nblk + nt - 1) // nt):
        qs = range(i * nt, min((i + 1) * nt, nblk))
        for c in range(e):
            slots = [b_idx((q % (bn // e)) * e + c, q // (bn // e), bn, e) for q in qs]
            assert conflict_free(slots, width), (i, c)


@pytest.mark.parametrize("bm,bn,bkc,wgm,wgn", F32_TILES)
def test_row_layout_b_float32(bm, bn, bkc, wgm, wgn):
    # float32 B as it lies in memory: lane (g, t) reads FN consecutive floats
    # of row (kb KG + g) E + s at column wn0 WN + FN t.  Every group of lanes
    # that the LDS serves together (128 bytes) must read one contiguous,
    # aligned 128-byte run, and the reads must stay inside the stage.
    tm, kg, e = MT["f32"]["TM"], MT["f32"]["KG"], MT["f32"]["E"]
    wn = bn // wgn
    fn = wn // tm
    assert fn in (1, 2, 4) and wn == fn * tm
    per_phase = 128 // (4 * fn)  # lanes per 128 bytes
    for wn0 in range(wgn):
        for kb in range(bkc // kg):
            for s in range(e):
                addr = [((kb * kg + l // tm) * e + s) * bn + wn0 * wn + fn * (l % tm) for l in range(64)]
                assert all(0 <= x and x + fn <= bkc * e * bn for x in addr)
                for p0 in range(0, 64, per_phase):
                    run = addr[p0:p0 + per_phase]
                    assert run == list(range(run[0], run[0] + fn * per_phase, fn)) and run[0] % 32 == 0
    # every output column of the tile is owned by exactly one (wave column, tile, lane)
    cols = sorted(wn0 * wn + fn * t + b for wn0 in range(wgn) for b in range(fn) for t in range(tm))
    assert cols == list(range(bn))
