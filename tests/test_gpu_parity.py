"""Parity of the HIP path with the oracle, through the C ABI (needs a GPU).

Every product is compared element by element with the oracle's double
triple loop on the same seeded inputs: exactly on integer inputs (where
every method is exact), within 1e-12 relative Frobenius error in float64 and
within 1e-5 in float32 (the stated target).  At the full sizes the oracle
computes a sample of rows, which it does exactly as it would in the full
product.
"""
import ctypes
import itertools

import numpy as np
import pytest

from paper_2309_00628_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_00628_amd import api as a
    return a


@pytest.fixture(scope="module")
def naive(oracle_built):
    from oracle import naive
    return naive


def rel_fro(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(np.asarray(got, dtype=np.float64) - ref)
    nr = np.linalg.norm(ref)
    return d / nr if nr else d


def gpu_mm(api, A, B, **kw):
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    Bt = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    C = api.mm(At, Bt, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()


SHAPES = [(1, 1, 1), (15, 16, 17), (64, 64, 64), (127, 129, 128), (375, 511, 512),
          (129, 257, 33), (1000, 1, 300), (1, 700, 2000), (257, 129, 1025), (130, 300, 7)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_naive_gemm_shapes(api, naive, dtype, m, n, k):
    A, B = inputs.pair("uniform", m, n, k, 3, dtype)
    print(f"naive {dtype.__name__} {m}x{n}x{k}", flush=True)
    got = gpu_mm(api, A, B, algo="naive")
    ref = naive.gemm(A, B)
    tol = 1e-13 if dtype == np.float64 else 2e-6
    assert rel_fro(got, ref) < tol


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("m,n,k", [(601, 603, 605), (1000, 1001, 640)])
def test_naive_gemm_unaligned_copies(api, naive, dtype, m, n, k):
    # rows that are not 16-byte multiples: the plan copies A and B into
    # aligned blocks first
    A, B = inputs.pair("uniform", m, n, k, 50, dtype)
    got = gpu_mm(api, A, B, algo="naive")
    tol = 1e-13 if dtype == np.float64 else 2e-6
    assert rel_fro(got, naive.gemm(A, B)) < tol


@pytest.mark.parametrize("m,n,k", [(1024, 768, 512), (600, 520, 300), (1100, 260, 1000)])
def test_every_float32_tile_configuration(api, naive, m, n, k):
    # each float32 tile shape (MM_PLAN_TILE 0 .. 8) of the plain product and
    # of a Winograd level: within tolerance of the oracle, and bitwise equal
    # to each other (every tile shape accumulates k in the same order)
    A, B = inputs.pair("uniform", m, n, k, 60, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = naive.gemm(A, B)
    for algo, levels in (("naive", 0), ("winograd", 1)):
        first = None
        for tile in range(9):
            print(f"tile {tile} {algo} {m}x{n}x{k}", flush=True)
            C = torch.full((m, n), float("nan"), device="cuda")
            if algo == "naive":
                api.mm(At, Bt, algo="naive", tile=tile, out=C)
            else:
                api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, tile=tile, out=C)
            torch.cuda.synchronize()
            assert rel_fro(C.cpu().numpy(), ref) < (2e-6 if levels == 0 else 1e-5), tile
            if first is None:
                first = C
            else:
                assert torch.equal(C, first), tile


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_naive_gemm_exact_on_integers(api, naive, dtype):
    A, B = inputs.pair("int", 300, 200, 250, 4, dtype)
    assert np.array_equal(gpu_mm(api, A, B, algo="naive").astype(np.float64), naive.gemm(A, B))


VARIANTS = [("naive", "auto"), ("strassen", "dfs3"), ("strassen", "grouped"), ("winograd", "two_temp"),
            ("winograd", "in_place"), ("winograd", "grouped")]


@pytest.mark.parametrize("n", [4, 8])
@pytest.mark.parametrize("cutoff", [1, 2, 4])
def test_integer_exact_small_fp64(api, naive, n, cutoff):
    for seed in range(3):
        A, B = inputs.pair("int", n, n, n, seed, np.float64)
        ref = naive.gemm(A, B)
        for algo, sched in VARIANTS:
            got = gpu_mm(api, A, B, algo=algo, sched=sched, cutoff=cutoff)
            assert np.array_equal(got, ref), (algo, sched, n, cutoff, seed)


def test_fp64_512_cutoff_64(api, naive):
    A, B = inputs.pair("uniform", 512, 512, 512, 0, np.float64)
    ref = naive.gemm(A, B)
    res = {}
    for algo, sched in VARIANTS:
        got = gpu_mm(api, A, B, algo=algo, sched=sched, cutoff=64)
        err = rel_fro(got, ref)
        print(f"fp64 512 {algo}/{sched}: {err:.3e}", flush=True)
        assert err < 1e-12, (algo, sched, err)
        res[(algo, sched)] = got
    # the three Winograd schedules do the same operations in the same order
    assert np.array_equal(res[("winograd", "two_temp")], res[("winograd", "in_place")])
    assert np.array_equal(res[("winograd", "two_temp")], res[("winograd", "grouped")])
    # and so do the two Strassen schedules
    assert np.array_equal(res[("strassen", "dfs3")], res[("strassen", "grouped")])


def test_fp64_512_integer_exact(api, naive):
    A, B = inputs.pair("int", 512, 512, 512, 5, np.float64)
    ref = naive.gemm(A, B)
    for algo, sched in VARIANTS:
        assert np.array_equal(gpu_mm(api, A, B, algo=algo, sched=sched, cutoff=64), ref), (algo, sched)


def test_fp32_integer_exact(api, naive):
    # entries in {-1, 0, 1}, 256 with two levels: every intermediate is an
    # integer below 2^24, so float32 arithmetic is exact
    A, B = inputs.pair("int", 256, 256, 256, 6, np.float32)
    A = np.clip(A, -1, 1)
    B = np.clip(B, -1, 1)
    ref = naive.gemm(A, B)
    for algo, sched in VARIANTS:
        got = gpu_mm(api, A, B, algo=algo, sched=sched, cutoff=1, levels=2)
        assert np.array_equal(got.astype(np.float64), ref), (algo, sched)


def test_fp32_schedules_bitwise(api):
    A, B = inputs.pair("uniform", 1024, 1024, 1024, 7, np.float32)
    outs = [gpu_mm(api, A, B, algo="winograd", sched=s, cutoff=1, levels=2)
            for s in ("two_temp", "in_place", "grouped")]
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])
    outs = [gpu_mm(api, A, B, algo="strassen", sched=s, cutoff=1, levels=2) for s in ("dfs3", "grouped")]
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("m,n,k,cutoff,levels", [(100, 60, 80, 8, -1), (1000, 777, 555, 1, 2),
                                                 (333, 333, 333, 1, 3), (96, 2000, 48, 1, 1)])
def test_padding_shapes_fp32(api, naive, m, n, k, cutoff, levels):
    A, B = inputs.pair("uniform", m, n, k, 8, np.float32)
    ref = naive.gemm(A, B)
    for algo, sched in [("winograd", "grouped"), ("winograd", "two_temp"), ("strassen", "dfs3"),
                        ("strassen", "grouped")]:
        got = gpu_mm(api, A, B, algo=algo, sched=sched, cutoff=cutoff, levels=levels)
        err = rel_fro(got, ref)
        assert err < 1e-5, (algo, sched, err)


def test_in_place_square_padded(api, naive):
    A, B = inputs.pair("uniform", 200, 200, 200, 9, np.float64)
    got = gpu_mm(api, A, B, algo="winograd", sched="in_place", cutoff=1, levels=3)
    assert rel_fro(got, naive.gemm(A, B)) < 1e-12


def test_leading_dimensions(api, naive):
    A, B = inputs.pair("uniform", 300, 260, 200, 10, np.float32)
    Aw = torch.zeros((300, 211), dtype=torch.float32, device="cuda")
    Bw = torch.zeros((200, 301), dtype=torch.float32, device="cuda")
    Cw = torch.full((300, 263), 7.0, dtype=torch.float32, device="cuda")
    Aw[:, :200] = torch.from_numpy(A)
    Bw[:, :260] = torch.from_numpy(B)
    for algo, sched in [("naive", "auto"), ("winograd", "grouped"), ("winograd", "two_temp")]:
        api.mm(Aw[:, :200], Bw[:, :260], algo=algo, sched=sched, cutoff=1, levels=2,
               out=Cw[:, :260])
        torch.cuda.synchronize()
        got = Cw.cpu().numpy()
        assert rel_fro(got[:, :260], naive.gemm(A, B)) < 1e-5
        assert np.all(got[:, 260:] == 7.0)   # nothing written outside C


@pytest.mark.parametrize("n", [4096, 3000])
def test_fp32_full_size_sampled_rows(api, naive, n):
    A, B = inputs.pair("uniform", n, n, n, 11, np.float32)
    rows = inputs.rng(12).choice(n, size=48, replace=False)
    rows = np.sort(np.concatenate([rows, [0, n - 1]]))
    ref = naive.gemm_rows(A, B, rows)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for algo, sched, lv in [("naive", "auto", 0), ("winograd", "grouped", 1), ("winograd", "grouped", 2),
                            ("winograd", "grouped", 3), ("winograd", "two_temp", 2),
                            ("strassen", "dfs3", 1), ("strassen", "grouped", 2)]:
        print(f"fp32 {n} {algo}/{sched} L={lv}", flush=True)
        C = api.mm(At, Bt, algo=algo, sched=sched, cutoff=1, levels=lv)
        torch.cuda.synchronize()
        err = rel_fro(C[torch.from_numpy(rows).cuda()].cpu().numpy(), ref)
        print(f"   rel err {err:.3e}", flush=True)
        assert err < 1e-5, (algo, sched, lv, err)


def test_degenerate_sizes(api):
    z = torch.zeros((0, 5), device="cuda")
    assert api.mm(z, torch.zeros((5, 3), device="cuda")).shape == (0, 3)
    A = torch.zeros((6, 0), device="cuda")
    B = torch.zeros((0, 4), device="cuda")
    C = torch.full((6, 4), 3.0, device="cuda")
    for algo in ("naive", "winograd", "strassen"):
        C.fill_(3.0)
        api.mm(A, B, algo=algo, out=C)
        torch.cuda.synchronize()
        assert torch.all(C == 0)


def test_error_paths(api):
    from paper_2309_00628_amd import _lib as L
    lib = L.load()
    A = torch.ones((64, 64), device="cuda")
    with pytest.raises(L.MMError) as e:
        api.mm(A, A, algo="winograd", out=A)
    assert e.value.name == "MM_E_ALIAS"
    with pytest.raises(L.MMError) as e:
        api.mm(torch.ones((64, 32), device="cuda"), torch.ones((32, 64), device="cuda"),
               algo="winograd", sched="in_place", cutoff=1, levels=1)
    assert e.value.name == "MM_E_UNSUPPORTED"
    B = torch.ones((64, 64), device="cuda")
    C = torch.empty((64, 64), device="cuda")
    need = lib.mm_workspace_size(2, 0, 64, 64, 64, 1, 2, 1)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    st = lib.mm_gemm_ex(2, 0, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, C.data_ptr(), 64, 1, 2, 1,
                        ws.data_ptr(), need - 4, s)
    assert L.STATUS[st] == "MM_E_WORKSPACE"
    st = lib.mm_gemm_ex(2, 0, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, C.data_ptr(), 64, 1, 2, 1,
                        ws.data_ptr(), need, s)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.all(C == 64)
    st = lib.mm_naive(-1, 4, 4, A.data_ptr(), B.data_ptr(), C.data_ptr(), 1, s)
    assert L.STATUS[st] == "MM_E_INVALID"


def test_short_forms_through_the_abi(api, naive):
    from paper_2309_00628_amd import _lib as L
    lib = L.load()
    A, B = inputs.pair("uniform", 384, 384, 384, 13, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((384, 384), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    ref = naive.gemm(A, B)
    for fn, args in [(lib.mm_naive, ()), (lib.mm_strassen, (64, -1)), (lib.mm_winograd, (64, -1))]:
        C.zero_()
        st = fn(384, 384, 384, At.data_ptr(), Bt.data_ptr(), C.data_ptr(), *args, L.MM_F32, s)
        assert st == 0, L.last_error()
        torch.cuda.synchronize()
        assert rel_fro(C.cpu().numpy(), ref) < 1e-5


def test_batched_matches_single(api, naive):
    shapes = inputs.batched_shapes(12, 14, lo=64, hi=512)
    As, Bs, Cs, refs = [], [], [], []
    for i, (m, n, k) in enumerate(shapes):
        A, B = inputs.pair("uniform", m, n, k, 20 + i, np.float32)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        Cs.append(torch.empty((m, n), device="cuda"))
        refs.append(naive.gemm(A, B))
    levels = [i % 3 for i in range(len(shapes))]
    plan = api.BatchedPlan(As, Bs, Cs, cutoff=[1] * len(shapes), levels=levels, graph=False)
    plan()
    torch.cuda.synchronize()
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        single = api.mm(A, B, algo="winograd", sched="grouped", cutoff=1, levels=levels[i])
        torch.cuda.synchronize()
        assert torch.equal(C, single), i
        assert rel_fro(C.cpu().numpy(), refs[i]) < 1e-5


def test_graph_replay_matches_eager(api):
    A, B = inputs.pair("uniform", 512, 512, 512, 15, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    eager = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=2)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        C = torch.empty_like(At)
        for rep in range(4):
            C.fill_(float("nan"))
            api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=2, out=C, graph=True,
                   stream=s)
            s.synchronize()
            junk = At @ Bt  # unrelated eager work between replays
            s.synchronize()
            assert torch.equal(C, eager), rep
            del junk


@pytest.mark.parametrize("m,n,k,levels", [(1024, 1024, 1024, 1), (1024, 1024, 1024, 2), (3000, 3000, 3000, 1),
                                          (1024, 768, 512, 2), (2048, 2048, 2048, 1), (3000, 3000, 3000, 3)])
def test_fused_loader_bitwise_equal_to_separate_pass(api, naive, m, n, k, levels):
    # the S/T sums formed in the leaf loader must give the same bits as the
    # separate pre-addition launch
    A, B = inputs.pair("uniform", m, n, k, 30, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Cf = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, fuse=True)
    Cu = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, fuse=False)
    torch.cuda.synchronize()
    p = api.get_plan("winograd", "grouped", m, n, k, 1, levels, "f32", k, n, n, False, At.device, None, True)  # fused
    assert p.info["fused"] == 1
    assert torch.equal(Cf, Cu)
    rows = np.arange(0, m, max(1, m // 16))
    assert rel_fro(Cf[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A, B, rows)) < 1e-5


def test_fused_plan_with_unaligned_operands_falls_back(api, naive):
    # A and B start 4 bytes past a 16-byte boundary: the fused loader's vector
    # loads would be misaligned, so the plan runs its unfused twin
    m = n = k = 512
    A, B = inputs.pair("uniform", m, n, k, 31, np.float32)
    Ab = torch.zeros(m * k + 1, device="cuda")
    Bb = torch.zeros(k * n + 1, device="cuda")
    Ab[1:] = torch.from_numpy(A.ravel())
    Bb[1:] = torch.from_numpy(B.ravel())
    At, Bt = Ab[1:].view(m, k), Bb[1:].view(k, n)
    assert At.data_ptr() % 16 != 0
    C = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=1, fuse=True)
    Ca = api.mm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), algo="winograd", sched="grouped",
                cutoff=1, levels=1, fuse=False)
    torch.cuda.synchronize()
    assert torch.equal(C, Ca)
    assert rel_fro(C.cpu().numpy(), naive.gemm(A, B)) < 1e-5


@pytest.mark.parametrize("m,n,k,levels", [(1024, 1024, 1024, 1), (2048, 2048, 2048, 2), (3000, 3000, 3000, 1),
                                          (1000, 777, 555, 2), (640, 384, 1152, 3)])
def test_overlapped_schedule_bitwise_equal_to_serial(api, naive, m, n, k, levels):
    # the S/T passes on the plan's auxiliary stream beside P1/P2 must give
    # the same bits as the serial launch order, on the default stream and on
    # a side stream, eagerly and from a replayed graph
    A, B = inputs.pair("uniform", m, n, k, 32, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    print(f"overlap {m}x{n}x{k} L={levels}", flush=True)
    serial = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels)
    over = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, overlap=True)
    torch.cuda.synchronize()
    p = api.get_plan("winograd", "grouped", m, n, k, 1, levels, "f32", k, n, n, False, At.device, overlap=True)
    assert "FORK" in p.describe()
    assert torch.equal(over, serial)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        C = torch.empty((m, n), device="cuda")
        for rep in range(3):
            C.fill_(float("nan"))
            api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, out=C, graph=rep > 0,
                   stream=s, overlap=True)
            s.synchronize()
            junk = At[:64] @ Bt  # unrelated eager work between replays
            s.synchronize()
            assert torch.equal(C, serial), rep
            del junk
    rows = np.arange(0, m, max(1, m // 16))
    assert rel_fro(over[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A, B, rows)) < 1e-5


def test_timed_execution_events_per_launch(api):
    # mm_plan_execute_timed records two events per launch on the stream the
    # launch runs on; the result equals an untimed run
    from paper_2309_00628_amd import _lib as L
    lib = L.load()
    m = n = k = 1024
    A, B = inputs.pair("uniform", m, n, k, 33, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    p = api.Plan("winograd", "grouped", m, n, k, cutoff=1, levels=2, overlap=True)
    ws = torch.empty(p.ws_bytes, dtype=torch.uint8, device="cuda")
    ref = torch.empty((m, n), device="cuda")
    p(At, Bt, ref, ws)
    nops = p.info["launches"]
    kinds = [lib.mm_plan_op_kind(p._ptr, j) for j in range(nops)]
    assert kinds[0] == 2 and 3 in kinds and any(x >= 8 for x in kinds)
    assert lib.mm_plan_op_kind(p._ptr, nops) == -1
    s = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nops)]
    for e in evs:
        e.record(s)
    torch.cuda.synchronize()
    arr = (ctypes.c_void_p * (2 * nops))(*[e.cuda_event for e in evs])
    C = torch.full((m, n), float("nan"), device="cuda")
    assert lib.mm_plan_execute_timed(p._ptr, At.data_ptr(), Bt.data_ptr(), C.data_ptr(), ws.data_ptr(),
                                     ws.numel(), s.cuda_stream, arr, 2 * nops - 1) == 1  # MM_E_INVALID
    L.check(lib.mm_plan_execute_timed(p._ptr, At.data_ptr(), Bt.data_ptr(), C.data_ptr(), ws.data_ptr(),
                                      ws.numel(), s.cuda_stream, arr, 2 * nops))
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
    durs = [evs[2 * j].elapsed_time(evs[2 * j + 1]) for j in range(nops)]
    assert all(d >= 0 for d in durs)
    assert evs[0].elapsed_time(evs[-1]) >= max(durs) * 0.99


@pytest.mark.parametrize("m,n,k,levels", [(1024, 1024, 1024, 1), (2048, 2048, 2048, 2), (3000, 3000, 3000, 1),
                                          (1000, 777, 555, 2), (640, 384, 1152, 3), (130, 70, 90, 1)])
def test_leaf_u_bitwise_equal_to_separate_u_pass(api, naive, m, n, k, levels):
    # the last level's products and U combinations formed in registers must
    # give the same bits as storing the products and running the U pass, for
    # every tile configuration of the fused kernel
    A, B = inputs.pair("uniform", m, n, k, 34, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    print(f"leaf_u {m}x{n}x{k} L={levels}", flush=True)
    ref = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, leaf_u=False)
    for tile in (None, 0, 1, 2):
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, leaf_u=True, tile=tile, out=C)
        torch.cuda.synchronize()
        p = api.get_plan("winograd", "grouped", m, n, k, 1, levels, "f32", k, n, n, False, At.device, tile,
                         leaf_u=True)
        assert p.info["leaf_u"] == 1
        assert torch.equal(C, ref), tile
    rows = np.arange(0, m, max(1, m // 16))
    assert rel_fro(ref[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A, B, rows)) < 1e-5


@pytest.mark.parametrize("m,n,k,levels", [(1024, 1024, 1024, 1), (2048, 2048, 2048, 2), (3000, 3000, 3000, 1),
                                          (640, 384, 1152, 3), (128, 96, 64, 1)])
def test_zero_temporary_level_bitwise(api, naive, m, n, k, levels):
    # LEAF_U with FUSE: S/T formed in the loader of the fused last level,
    # bitwise equal to the separate passes for every tile configuration
    A, B = inputs.pair("uniform", m, n, k, 51, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    print(f"zero-temp {m}x{n}x{k} L={levels}", flush=True)
    ref = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, leaf_u=False)
    for tile in (None, 0, 1, 2):
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, leaf_u=True, fuse=True,
               tile=tile, out=C)
        torch.cuda.synchronize()
        p = api.get_plan("winograd", "grouped", m, n, k, 1, levels, "f32", k, n, n, False, At.device, tile,
                         fuse=True, leaf_u=True)
        assert p.info["leaf_u"] == 1 and p.info["fused"] == 1
        assert torch.equal(C, ref), tile
    rows = np.arange(0, m, max(1, m // 16))
    assert rel_fro(ref[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A, B, rows)) < 1e-5
    # accumulating, and through an unaligned A (the plan then runs its unfused twin)
    C0 = torch.from_numpy(inputs.uniform((m, n), 52, dtype=np.float32)).cuda()
    want = ref + 0.5 * C0
    C = C0.clone()
    api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, leaf_u=True, fuse=True, out=C,
           beta=0.5)
    torch.cuda.synchronize()
    assert torch.equal(C, api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels,
                                 leaf_u=False, out=C0.clone(), beta=0.5))
    assert rel_fro(C.cpu().numpy(), want.cpu().numpy().astype(np.float64)) < 1e-6
    Abuf = torch.empty(m * k + 1, device="cuda")
    Au = Abuf[1:].view(m, k)
    Au.copy_(At)
    C = api.mm(Au, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, leaf_u=True, fuse=True)
    torch.cuda.synchronize()
    assert torch.equal(C, ref)


def test_leaf_u_integer_exact_and_strided(api, naive):
    # integer inputs: exact; operands inside larger row-major buffers
    m, n, k = 384, 320, 256
    Ai = inputs.integers((m, k), 35).astype(np.float32)
    Bi = inputs.integers((k, n), 36).astype(np.float32)
    Abuf = torch.zeros((m, k + 12), device="cuda")
    Bbuf = torch.zeros((k, n + 4), device="cuda")
    Abuf[:, :k] = torch.from_numpy(Ai).cuda()
    Bbuf[:, :n] = torch.from_numpy(Bi).cuda()
    Cbuf = torch.full((m, n + 8), float("nan"), device="cuda")
    api.mm(Abuf[:, :k], Bbuf[:, :n], algo="winograd", sched="grouped", cutoff=1, levels=2, leaf_u=True,
           out=Cbuf[:, :n])
    torch.cuda.synchronize()
    got = Cbuf[:, :n].cpu().numpy()
    assert np.array_equal(got, naive.gemm(Ai.astype(np.float64), Bi.astype(np.float64)))
    assert torch.isnan(Cbuf[:, n:]).all()


ACC_GPU = [("naive", "auto", 300, 200, 100, 0, "f32", {}), ("naive", "auto", 257, 129, 65, 0, "f64", {}),
           ("winograd", "grouped", 1024, 768, 512, 2, "f32", {}),
           ("winograd", "grouped", 1000, 777, 555, 1, "f32", {"leaf_u": True}),
           ("winograd", "grouped", 512, 512, 512, 2, "f64", {}),
           ("winograd", "two_temp", 512, 256, 384, 2, "f32", {}),
           ("winograd", "in_place", 512, 256, 256, 1, "f32", {}),
           ("strassen", "dfs3", 384, 320, 256, 2, "f64", {}),
           ("winograd", "grouped", 1024, 1024, 1024, 2, "bf16x3", {}),
           ("naive", "auto", 640, 384, 200, 0, "bf16x3", {"split_pass": True}),
           ("strassen", "grouped", 640, 384, 512, 2, "f32", {}),
           ("winograd", "grouped", 1000, 777, 555, 2, "f32", {"peel": True}),
           ("strassen", "grouped", 301, 290, 257, 2, "f64", {"peel": True}),
           # edge tiles and a ragged k on the split-bf16 ring tiles and on the
           # float32 direct loop, each epilogue reading the C it adds to
           ("naive", "auto", 1000, 777, 520, 0, "bf16x3", {"tile": 6}),
           ("winograd", "grouped", 1000, 777, 555, 2, "bf16x3", {"tile": 0}),
           ("naive", "auto", 1000, 776, 512, 0, "f32", {"tile": 3})]


PEEL_GPU = [("winograd", 1000, 777, 555, 2, "f32"), ("winograd", 1200, 1300, 1100, 3, "f32"),
            ("winograd", 1023, 1025, 1027, 2, "f64"), ("strassen", 1000, 777, 555, 2, "f32"),
            ("winograd", 1030, 1100, 1050, 2, "bf16x3")]


@pytest.mark.parametrize("algo,m,n,k,levels,dt", PEEL_GPU)
def test_peeled_plans(api, naive, algo, m, n, k, levels, dt):
    # MM_PLAN_PEEL against the oracle, and exact on small integers
    npdt = np.float64 if dt == "f64" else np.float32
    print(f"peel {algo} {m}x{n}x{k} L={levels} {dt}", flush=True)
    A, B = inputs.pair("uniform", m, n, k, 46, npdt)
    got = gpu_mm(api, A, B, algo=algo, sched="grouped", cutoff=1, levels=levels, dtype=dt, peel=True)
    tol = 1e-12 if dt == "f64" else 1e-5
    assert rel_fro(got, naive.gemm(A, B)) < tol
    A, B = inputs.pair("int", m, n, k, 47, npdt)
    A, B = np.clip(A, -1, 1), np.clip(B, -1, 1)
    got = gpu_mm(api, A, B, algo=algo, sched="grouped", cutoff=1, levels=levels, dtype=dt, peel=True)
    assert np.array_equal(got.astype(np.float64), naive.gemm(A, B))


@pytest.mark.parametrize("algo,sched,m,n,k,levels,dt,opts", ACC_GPU)
def test_accumulating_form(api, naive, algo, sched, m, n, k, levels, dt, opts):
    # C <- A B + beta C against the oracle's A B plus beta C0 (float64); with
    # beta = 0 a C full of NaN must not leak into the result
    npdt = np.float64 if dt == "f64" else np.float32
    A, B = inputs.pair("uniform", m, n, k, 36, npdt)
    C0 = inputs.uniform((m, n), 37, dtype=npdt)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    AB = naive.gemm(A, B)
    tol = 1e-12 if dt == "f64" else 1e-5
    print(f"accumulate {algo} {sched} {m}x{n}x{k} L={levels} {dt} {opts}", flush=True)
    for beta in (1.5, -1.0, 0.0):
        C = torch.from_numpy(C0.copy()).cuda() if beta else torch.full((m, n), float("nan"), dtype=At.dtype,
                                                                        device="cuda")
        api.mm(At, Bt, algo=algo, sched=sched, cutoff=1, levels=levels, dtype=dt, out=C, beta=beta, **opts)
        torch.cuda.synchronize()
        want = AB + beta * C0.astype(np.float64)
        assert rel_fro(C.cpu().numpy(), want) < tol, beta


def test_accumulating_leaf_u_and_graph_bitwise(api):
    # the fused last level applies beta exactly as the separate U pass does,
    # and a graph captured per beta replays the eager result
    m = n = k = 1024
    A, B = inputs.pair("uniform", m, n, k, 38, np.float32)
    C0 = torch.from_numpy(inputs.uniform((m, n), 39, dtype=np.float32)).cuda()
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    outs = []
    for leaf_u in (False, True):
        C = C0.clone()
        api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=1, out=C, beta=0.75, leaf_u=leaf_u)
        outs.append(C)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    p = api.Plan("winograd", "grouped", m, n, k, cutoff=1, levels=2, graph=True, accumulate=True)
    ws = torch.empty(p.ws_bytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()  # graphs are captured on non-default streams
    for beta in (0.5, 2.0, 0.5):
        eager = C0.clone()
        api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=2, out=eager, beta=beta)
        C = C0.clone()
        torch.cuda.synchronize()
        p(At, Bt, C, ws, stream=s, beta=beta)
        s.synchronize()
        assert torch.equal(C, eager), beta
    with pytest.raises(ValueError):
        api.Plan("naive", "auto", 8, 8, 8)(At[:8, :8].contiguous(), Bt[:8, :8].contiguous(),
                                           torch.empty(8, 8, device="cuda"), beta=2.0)


@pytest.mark.parametrize("m,n,k,levels", [(1024, 1024, 1024, 1), (2048, 2048, 2048, 2), (3000, 3000, 3000, 1),
                                          (1000, 777, 555, 2), (640, 384, 1152, 3), (130, 70, 90, 1)])
def test_transposed_b_bitwise(api, naive, m, n, k, levels):
    # MM_PLAN_TRANS_B: the last level's B operands written transposed by the
    # transposing T pass and staged like A; bitwise equal to the default plan
    # for every tile configuration, accumulating too
    A, B = inputs.pair("uniform", m, n, k, 55, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    print(f"trans_b {m}x{n}x{k} L={levels}", flush=True)
    ref = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, trans_b=False)
    for tile in (None, 0, 1, 3, 4, 7):
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, trans_b=True, tile=tile, out=C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), tile
    rows = np.arange(0, m, max(1, m // 16))
    assert rel_fro(ref[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A, B, rows)) < 1e-5
    C0 = torch.from_numpy(inputs.uniform((m, n), 56, dtype=np.float32)).cuda()
    C1, C2 = C0.clone(), C0.clone()
    api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, trans_b=True, out=C1, beta=-0.5)
    api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, trans_b=False, out=C2, beta=-0.5)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_unrolled_base_case_bitwise(api, naive, dt):
    # leaves of order 8, 4 and 2 by the unrolled base case (win8x8, win4x4,
    # win2x2) give the bits of the plan recursing to scalar leaves (1x1 MFMA
    # products), i.e. of the plan with three, two and one more levels
    npdt = np.float64 if dt == "f64" else np.float32
    n = 64
    A, B = inputs.pair("uniform", n, n, n, 59, npdt)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=6)
    for lv in (3, 4, 5, 6):
        p = api.Plan("winograd", "grouped", n, n, n, cutoff=1, levels=lv, dtype=dt, unroll_base=True)
        assert "LAUNCH BASE" in p.describe()
        C = torch.full((n, n), float("nan"), dtype=At.dtype, device="cuda")
        ws = torch.empty(max(p.ws_bytes, 256), dtype=torch.uint8, device="cuda")
        p(At, Bt, C, ws)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), lv
    # six levels down to scalars: the error bound of the recursion grows
    # geometrically with the number of levels, so this deep plan gets one
    # more digit of slack than the two- and three-level plans
    err = rel_fro(ref.cpu().numpy(), naive.gemm(A, B))
    print(f"unrolled base {dt}: six-level error {err:.3e}", flush=True)
    assert err < (1e-11 if dt == "f64" else 1e-4)
    # ragged (virtual padding; leaves of order 4 and 8, i.e. five and six
    # levels down to scalars): against the oracle, the six-level case with
    # the deep plan's slack, and exact on integers
    for (m, n2, k), kind in itertools.product(((28, 30, 26), (60, 62, 58)), ("uniform", "int")):
        deep = m > 32
        tol = (1e-11 if deep else 1e-12) if dt == "f64" else (1e-4 if deep else 1e-5)
        A, B = inputs.pair(kind, m, n2, k, 60, npdt)
        got = gpu_mm(api, A, B, algo="winograd", sched="grouped", cutoff=1, levels=3, dtype=dt)
        p = api.get_plan("winograd", "grouped", m, n2, k, 1, 3, dt, k, n2, n2, False, torch.device("cuda"))
        At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        pb = api.Plan("winograd", "grouped", m, n2, k, cutoff=1, levels=3, dtype=dt, unroll_base=True)
        C = torch.empty((m, n2), dtype=At.dtype, device="cuda")
        ws = torch.empty(max(pb.ws_bytes, 256), dtype=torch.uint8, device="cuda")
        pb(At, Bt, C, ws)
        torch.cuda.synchronize()
        if kind == "int":
            assert np.array_equal(C.cpu().numpy().astype(np.float64), naive.gemm(A, B))
        else:
            assert rel_fro(C.cpu().numpy(), naive.gemm(A, B)) < tol
        del p, got


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16x3"])
@pytest.mark.parametrize("m,n,k,s", [(256, 256, 1024, 4), (300, 200, 777, 8), (512, 384, 2048, 2)])
def test_split_k_plain_product(api, naive, dt, m, n, k, s):
    # MM_PLAN_SPLIT_K against the oracle, exact on integers, accumulating
    npdt = np.float64 if dt == "f64" else np.float32
    tol = 1e-12 if dt == "f64" else 1e-5
    A, B = inputs.pair("uniform", m, n, k, 64, npdt)
    got = gpu_mm(api, A, B, algo="naive", dtype=dt, split_k=s)
    assert rel_fro(got, naive.gemm(A, B)) < tol
    Ai, Bi = inputs.pair("int", m, n, k, 65, npdt)
    assert np.array_equal(gpu_mm(api, Ai, Bi, algo="naive", dtype=dt, split_k=s).astype(np.float64),
                          naive.gemm(Ai, Bi))
    C0 = inputs.uniform((m, n), 66, dtype=npdt)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for beta in (0.5, 0.0):
        C = torch.from_numpy(C0.copy()).cuda() if beta else torch.full((m, n), float("nan"), dtype=At.dtype,
                                                                        device="cuda")
        api.mm(At, Bt, algo="naive", dtype=dt, split_k=s, out=C, beta=beta)
        torch.cuda.synchronize()
        assert rel_fro(C.cpu().numpy(), naive.gemm(A, B) + beta * C0.astype(np.float64)) < tol


@pytest.mark.parametrize("m,n,k,levels", [(1024, 1024, 1024, 1), (1000, 777, 555, 2)])
def test_option_combinations_bitwise(api, m, n, k, levels):
    # pairs of the grouped options that keep the bits give the bits of the
    # plain grouped plan
    import itertools
    A, B = inputs.pair("uniform", m, n, k, 70, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, overlap=False,
                 leaf_u=False, trans_b=False)
    for combo in itertools.combinations(("overlap", "leaf_u", "fuse", "trans_b"), 2):
        kw = dict(overlap=False, leaf_u=False, trans_b=False, fuse=False)
        kw.update({o: True for o in combo})
        C = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=levels, **kw)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), combo
