// Leaf products of the last Strassen-Winograd level with the operand sums
// fused into the tile loader (float32).
//
// In the 22-operation form (Section 2.3) the leaf products are
//   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4,
//   P5 = S1 T1,   P6 = S2 T2,   P7 = S3 T3,
// with S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2 and
// T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21.  Instead of
// writing S1..S4 and T1..T4 to HBM in a separate pass and reading them back,
// this kernel reads the quadrants of the parent block each S / T needs and
// forms the sum in registers while staging the LDS tile, in exactly the
// order above, so the result is bitwise the same as the unfused schedule.
// The pass over A and B (read 8 quarters, write 8) disappears; the GEMM reads
// up to four quadrant chunks per operand chunk instead (mostly from L2).
//
// The (S, T) combination of a product is uniform per workgroup; each of the
// six combinations gets its own branch-free main loop.  Loads of the next
// stage stay in flight during the MFMAs; the sums are formed when the stage
// is written to LDS.  Operands are aligned and entirely valid (the planner
// fuses only then); interior tiles load unmasked, edge tiles (when the leaf
// size is not a multiple of the tile) load whole chunks from a clamped
// address and zero them.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.h"
#include "gemm_common.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace gemm_detail;

typedef float f32x4v __attribute__((ext_vector_type(4)));

constexpr int E = 4;    // floats per 16-byte chunk
constexpr int TM = 32;  // v_mfma_f32_32x32x2_f32 tile edge
constexpr int KG = 2;

__device__ __forceinline__ f32x16 mfma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int row32(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

template <int BM, int BN, int BKC, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_fused_kernel(KernelBases kb,
                                                                    const GemmDesc* __restrict__ descs,
                                                                    int ndesc, int remap) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int BK = BKC * E;
  constexpr int NBLK_B = BKC * (BN / E);
  constexpr int NB = (NBLK_B + NT - 1) / NT;
  constexpr int NCH_A = BM * BKC;
  constexpr int NA = (NCH_A + NT - 1) / NT;
  constexpr int KB = BKC / KG;

  __shared__ f32x4v As[2][BKC][BM];
  __shared__ f32x4v Bs[2][BKC][BN];

  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const GemmDesc& D = descs[tr.desc];
  const int i0 = tr.i0, j0 = tr.j0;
  const MView av = D.a, bv = D.b;
  const float* __restrict__ Ap = resolve<float>(kb, av);
  const float* __restrict__ Bp = resolve<float>(kb, bv);
  const int64_t lda = av.ld, ldb = bv.ld;
  const int Mo = D.m, No = D.n, K = D.k;  // operand extents (a quadrant of the parent when fused)
  const int akind = D.kinds & 0xff, bkind = (D.kinds >> 8) & 0xff;
  // quadrant offsets in the parent blocks (order 11 12 21 22)
  const int64_t aq[4] = {0, K, (int64_t)Mo * lda, (int64_t)Mo * lda + K};
  const int64_t bq[4] = {0, No, (int64_t)K * ldb, (int64_t)K * ldb + No};
  const int ktiles = (K + BK - 1) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int g = lane / TM, t = lane % TM;

  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  auto run = [&](auto ak_tag, auto bk_tag, auto edge_tag) {
    constexpr int AK = decltype(ak_tag)::value, BKD = decltype(bk_tag)::value;
    constexpr bool EDGE = decltype(edge_tag)::value;
    constexpr int QA = kind_quads(AK), QB = kind_quads(BKD);
    constexpr int NQA = popc4(QA), NQB = popc4(QB);
    f32x4v ra[NA][NQA];
    f32x4v rb[NB][E][NQB];
    uint32_t amask = 0, bmask = 0;

    auto load_tile = [&](int kt) {
      const int k0 = kt * BK;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int q = tid + NT * i;
        if (NCH_A % NT != 0 && q >= NCH_A) break;
        const int row = q / BKC, kc = q % BKC;
        const int gr = i0 + row, gc = k0 + kc * E;
        const bool ok = !EDGE || (gr < Mo && gc < K);
        const int64_t off = ok ? (int64_t)gr * lda + gc : 0;
        int j = 0;
#pragma unroll
        for (int qd = 0; qd < 4; ++qd)
          if ((QA >> qd) & 1) ra[i][j++] = *reinterpret_cast<const f32x4v*>(Ap + off + aq[qd]);
        if (EDGE) amask = ok ? (amask | (1u << i)) : (amask & ~(1u << i));
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int q = tid + NT * i;
        if (NBLK_B % NT != 0 && q >= NBLK_B) break;
        const int kc = q / (BN / E), cb = q % (BN / E);
        const int gc = j0 + cb * E;
#pragma unroll
        for (int rr = 0; rr < E; ++rr) {
          const int gr = k0 + kc * E + rr;
          const bool ok = !EDGE || (gr < K && gc < No);
          const int64_t off = ok ? (int64_t)gr * ldb + gc : 0;
          int j = 0;
#pragma unroll
          for (int qd = 0; qd < 4; ++qd)
            if ((QB >> qd) & 1) rb[i][rr][j++] = *reinterpret_cast<const f32x4v*>(Bp + off + bq[qd]);
          if (EDGE) {
            const uint32_t bit = 1u << (i * E + rr);
            bmask = ok ? (bmask | bit) : (bmask & ~bit);
          }
        }
      }
    };

    auto store_tile = [&](int buf) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int q = tid + NT * i;
        if (NCH_A % NT != 0 && q >= NCH_A) break;
        const int row = q / BKC, kc = q % BKC;
        f32x4v v;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          float x[4] = {0.f, 0.f, 0.f, 0.f};
          int j = 0;
#pragma unroll
          for (int qd = 0; qd < 4; ++qd)
            if ((QA >> qd) & 1) x[qd] = ra[i][j++][e];
          v[e] = combine<AK>(x);
        }
        if (EDGE && !((amask >> i) & 1)) v = f32x4v{};
        As[buf][kc][swz_a<BKC>(row, kc)] = v;
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int q = tid + NT * i;
        if (NBLK_B % NT != 0 && q >= NBLK_B) break;
        const int kc = q / (BN / E), cb = q % (BN / E);
        float y[E][E];  // [k row][column]
#pragma unroll
        for (int rr = 0; rr < E; ++rr)
#pragma unroll
          for (int c = 0; c < E; ++c) {
            float x[4] = {0.f, 0.f, 0.f, 0.f};
            int j = 0;
#pragma unroll
            for (int qd = 0; qd < 4; ++qd)
              if ((QB >> qd) & 1) x[qd] = rb[i][rr][j++][c];
            const float s = combine<BKD>(x);
            y[rr][c] = (EDGE && !((bmask >> (i * E + rr)) & 1)) ? 0.f : s;
          }
#pragma unroll
        for (int c = 0; c < E; ++c) {
          f32x4v col;
#pragma unroll
          for (int rr = 0; rr < E; ++rr) col[rr] = y[rr][c];
          Bs[buf][kc][swz_b<E>(cb * E + c)] = col;
        }
      }
    };

    auto compute = [&](int buf, auto lo_tag, auto hi_tag) {
      constexpr int KLO = decltype(lo_tag)::value, KHI = decltype(hi_tag)::value;
#pragma unroll
      for (int kb2 = KLO; kb2 < KHI; ++kb2) {
        const int plane = kb2 * KG + g;
        f32x4v fa[FM], fb[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) fa[a] = As[buf][plane][swz_a<BKC>(wm * WM + a * TM + t, plane)];
#pragma unroll
        for (int b = 0; b < FN; ++b) fb[b] = Bs[buf][plane][swz_b<E>(wn * WN + b * TM + t)];
#pragma unroll
        for (int s = 0; s < E; ++s)
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) acc[a][b] = mfma(fa[a][s], fb[b][s], acc[a][b]);
      }
    };

    load_tile(0);
    store_tile(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      const bool more = kt + 1 < ktiles;
      if (more) load_tile(kt + 1);
      compute(buf, std::integral_constant<int, 0>{}, std::integral_constant<int, KB / 2>{});
      if (more) store_tile(buf ^ 1);
      compute(buf, std::integral_constant<int, KB / 2>{}, std::integral_constant<int, KB>{});
      __syncthreads();
    }
  };

  if (ktiles > 0) {
    const bool edge = (i0 + BM > Mo) || (j0 + BN > No) || (K % BK != 0);
    auto dispatch = [&](auto edge_tag) {
      typedef std::integral_constant<int, OK_PLAIN> P0;
      if (akind == OK_PLAIN && bkind == OK_PLAIN) run(P0{}, P0{}, edge_tag);
      else if (akind == OK_S4 && bkind == OK_PLAIN) run(std::integral_constant<int, OK_S4>{}, P0{}, edge_tag);
      else if (akind == OK_PLAIN && bkind == OK_T4) run(P0{}, std::integral_constant<int, OK_T4>{}, edge_tag);
      else if (akind == OK_S1) run(std::integral_constant<int, OK_S1>{}, std::integral_constant<int, OK_T1>{}, edge_tag);
      else if (akind == OK_S2) run(std::integral_constant<int, OK_S2>{}, std::integral_constant<int, OK_T2>{}, edge_tag);
      else run(std::integral_constant<int, OK_S3>{}, std::integral_constant<int, OK_T3>{}, edge_tag);
    };
    if (edge)
      dispatch(std::true_type{});
    else
      dispatch(std::false_type{});
  }

  store_outputs<float, TM, 16, FM, FN, WM, WN>(kb, D, i0, j0, wm, wn, lane, acc,
                                               [](int l, int r) { return row32(l, r); });
}

template <int BM, int BN, int BKC, int WGM, int WGN>
hipError_t launch_cfg(const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap, hipStream_t s) {
  hipLaunchKernelGGL((gemm_fused_kernel<BM, BN, BKC, WGM, WGN>), dim3(tiles), dim3(64 * WGM * WGN), 0, s, kb,
                     d, n, remap);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_fused(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap,
                             hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  switch (cfg) {
    case 3: return launch_cfg<256, 256, 4, 2, 2>(kb, d, n, tiles, remap, s);
    case 4: return launch_cfg<64, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
    default: return launch_cfg<128, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
  }
}

}  // namespace mm
