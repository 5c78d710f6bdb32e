// Leaf products: the naive method (Section 2.1) as a tiled MFMA GEMM for
// gfx950, in float32 (v_mfma_f32_32x32x2_f32) and float64
// (v_mfma_f64_16x16x4_f64).  The same kernel is mm_naive on a whole problem and
// the base case of every Strassen / Winograd recursion, and one launch can run
// a group of independent products (the seven products of a level, or many
// problems of a batch), so small leaves still fill the 256 compute units.
//
// Workgroup: a BM x BN tile of C split among WGM x WGN wave64s (several tile
// configurations are instantiated; the planner picks one per launch).  The K
// loop stages BM x BK and BK x BN tiles of A and B in LDS, double-buffered:
// the global loads of stage t+1 are in flight while the MFMAs consume stage
// t, one barrier per stage.
//
// LDS layout ("k-chunked"): a 16-byte chunk holds E consecutive k values
// (E = 4 floats / 2 doubles) of one row of A or one column of B, so every MFMA
// operand fetch is one ds_read_b128 that feeds E MFMAs.  Row (A) and column
// (B) indices are XOR-swizzled so that both the stores of the global tile and
// the fragment reads touch 16 distinct 16-byte bank groups per 16 lanes.
//
// Edges: operand reads outside a view's valid extent are zero (this is also
// how quadrants of a zero-padded matrix are read without a copy), and stores
// outside the output's valid extent are dropped.  Interior tiles take an
// unmasked vector path.
//
// Epilogue per output: C = s * acc or C = D + s * acc (s = +1 or -1).  The
// accumulator holds the product rounded exactly as it would be stored, so
// folding a following block addition into the epilogue gives the same bits
// as storing the product and adding it in a separate step.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.h"
#include "gemm_common.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace gemm_detail;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct MT;

// v_mfma_f32_32x32x2_f32: lanes 0-31 supply k = 0 and lanes 32-63 k = 1 of a
// 32 x 2 by 2 x 32 product; lane l holds A[l % 32][l / 32] and B[l / 32][l % 32].
// Result register r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
template <>
struct MT<float> {
  static constexpr int TM = 32;  // MFMA tile edge
  static constexpr int KG = 2;   // lane groups along k
  static constexpr int E = 4;    // elements per 16-byte chunk
  static constexpr int NACC = 16;
  typedef f32x16 acc_t;
  typedef f32x4 chunk_t;
  static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  }
};

// v_mfma_f64_16x16x4_f64: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// result register r of lane l is C[4 r + l / 16][l % 16] (rows interleaved
// across the four lane groups, unlike the float32 16x16 form).
template <>
struct MT<double> {
  static constexpr int TM = 16;
  static constexpr int KG = 4;
  static constexpr int E = 2;
  static constexpr int NACC = 4;
  typedef f64x4 acc_t;
  typedef f64x2 chunk_t;
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

constexpr int BKC_MAX = 8;

// BM x BN tile per workgroup, WGM x WGN waves (each (BM/WGM) x (BN/WGN)),
// BKC 16-byte chunks of k per LDS stage.
template <typename T, int BM, int BN, int BKC, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_kernel(KernelBases kb,
                                                              const GemmDesc* __restrict__ descs,
                                                              int ndesc, int remap) {
  typedef MT<T> M;
  typedef typename M::chunk_t chunk_t;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int E = M::E;
  constexpr int TM = M::TM;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int BK = BKC * E;
  constexpr int NBLK_B = BKC * (BN / E);      // E x E blocks of B per stage
  constexpr int NB = (NBLK_B + NT - 1) / NT;  // ... per thread
  constexpr int NCH_A = BM * BKC;             // chunks of A per stage
  constexpr int NA = (NCH_A + NT - 1) / NT;
  static_assert(FM >= 1 && FN >= 1 && WM % TM == 0 && WN % TM == 0, "wave tile");
  static_assert(BKC % M::KG == 0 && BKC <= BKC_MAX && 16 % BKC == 0, "k chunks");

  __shared__ chunk_t As[2][BKC][BM];
  __shared__ chunk_t Bs[2][BKC][BN];

  // ---- which problem and which tile -------------------------------------
  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const GemmDesc& D = descs[tr.desc];
  const int i0 = tr.i0, j0 = tr.j0;

  const MView av = D.a, bv = D.b;
  const T* __restrict__ Ap = resolve<T>(kb, av);
  const T* __restrict__ Bp = resolve<T>(kb, bv);
  const int64_t lda = av.ld, ldb = bv.ld;
  const bool avec = view_vec(kb, av), bvec = view_vec(kb, bv);
  const int K = D.k;
  const int ktiles = (K + BK - 1) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  // ---- global -> register staging ----------------------------------------
  chunk_t ra[NA];
  chunk_t rbk[NB][E];  // E rows (k) of E columns
  // LOAD_EDGE_VEC validity of each staged chunk, applied when the stage is
  // written to LDS (not right after the load, which would wait for it)
  uint32_t amask = 0, bmask = 0;

  // LOAD_FULL: the whole stage is inside both operands' valid extents and
  // every access is a 16-byte vector load (no masks, no branches, so the
  // loads of the next stage stay in flight while the MFMAs of this one run).
  // LOAD_EDGE_VEC: edge tile of aligned operands whose valid widths are
  // multiples of the chunk: whole chunks are in or out, selected without
  // branches.  Otherwise per-element masked loads.
  auto load_tile = [&](auto mode_tag, int kt) {
    constexpr int MODE = decltype(mode_tag)::value;
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gc = k0 + kc * E;
      const T* p = Ap + (int64_t)gr * lda + gc;
      if (MODE == LOAD_FULL) {
        ra[i] = *reinterpret_cast<const chunk_t*>(p);
      } else if (MODE == LOAD_EDGE_VEC) {
        // whole chunks are either valid or not: load from a valid address
        // and zero the invalid ones when storing, so the loop has no
        // data-dependent branches
        const bool ok = gr < av.vrows && gc < av.vcols;
        ra[i] = *reinterpret_cast<const chunk_t*>(ok ? p : Ap);
        amask = ok ? (amask | (1u << i)) : (amask & ~(1u << i));
      } else if (avec && gr < av.vrows && gc + E <= av.vcols) {
        ra[i] = *reinterpret_cast<const chunk_t*>(p);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
          ra[i][e] = (gr < av.vrows && gc + e < av.vcols) ? p[e] : T(0);
      }
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
        const T* p = Bp + (int64_t)gr * ldb + gc;
        if (MODE == LOAD_FULL) {
          rbk[i][rr] = *reinterpret_cast<const chunk_t*>(p);
        } else if (MODE == LOAD_EDGE_VEC) {
          const bool ok = gr < bv.vrows && gc < bv.vcols;
          rbk[i][rr] = *reinterpret_cast<const chunk_t*>(ok ? p : Bp);
          const uint32_t bit = 1u << (i * E + rr);
          bmask = ok ? (bmask | bit) : (bmask & ~bit);
        } else if (bvec && gr < bv.vrows && gc + E <= bv.vcols) {
          rbk[i][rr] = *reinterpret_cast<const chunk_t*>(p);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e)
            rbk[i][rr][e] = (gr < bv.vrows && gc + e < bv.vcols) ? p[e] : T(0);
        }
      }
    }
  };

  auto store_tile = [&](auto mode_tag, int buf) {
    constexpr int MODE = decltype(mode_tag)::value;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      As[buf][kc][swz_a<BKC>(row, kc)] =
          (MODE != LOAD_EDGE_VEC || ((amask >> i) & 1)) ? ra[i] : chunk_t{};
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      if (NBLK_B % NT != 0 && q >= NBLK_B) break;
      const int kc = q / (BN / E), cb = q % (BN / E);
#pragma unroll
      for (int c = 0; c < E; ++c) {
        chunk_t t;
#pragma unroll
        for (int rr = 0; rr < E; ++rr)
          t[rr] = (MODE != LOAD_EDGE_VEC || ((bmask >> (i * E + rr)) & 1)) ? rbk[i][rr][c] : T(0);
        Bs[buf][kc][swz_b<E>(cb * E + c)] = t;
      }
    }
  };

  typename M::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[a][b][r] = T(0);

  const int g = lane / TM, t = lane % TM;

  // MFMAs of k-blocks [kb_lo, kb_hi) of one LDS stage (a k-block is 8 k
  // values).  The fragments of k-block j+1 are read into a second register
  // set while the MFMAs of k-block j run.
  auto compute = [&](int buf, auto lo_tag, auto hi_tag) {
    constexpr int KLO = decltype(lo_tag)::value, KHI = decltype(hi_tag)::value;
    chunk_t fa[2][FM], fb[2][FN];
    auto read_frags = [&](int kb2, chunk_t (&xa)[FM], chunk_t (&xb)[FN]) {
      const int plane = kb2 * M::KG + g;
#pragma unroll
      for (int a = 0; a < FM; ++a) xa[a] = As[buf][plane][swz_a<BKC>(wm * WM + a * TM + t, plane)];
#pragma unroll
      for (int b = 0; b < FN; ++b) xb[b] = Bs[buf][plane][swz_b<E>(wn * WN + b * TM + t)];
    };
    read_frags(KLO, fa[0], fb[0]);
#pragma unroll
    for (int kb2 = KLO; kb2 < KHI; ++kb2) {
      const int cur = (kb2 - KLO) & 1;
      if (kb2 + 1 < KHI) read_frags(kb2 + 1, fa[cur ^ 1], fb[cur ^ 1]);
#pragma unroll
      for (int s = 0; s < E; ++s)
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) acc[a][b] = M::mfma(fa[cur][a][s], fb[cur][b][s], acc[a][b]);
    }
  };
  constexpr int KB = BKC / M::KG;
  constexpr int KMID = KB / 2;

  // Pipeline: the global loads of stage t+1 are issued first; the stage is
  // written to the other LDS buffer halfway through the MFMAs of stage t, so
  // the wait for those loads and the LDS writes overlap the second half of
  // the MFMAs; one barrier ends the stage.  Writing the other buffer is safe:
  // every wave finished reading it before the barrier that ended stage t-1,
  // and it is read again only after the barrier that ends stage t.
  auto main_loop = [&](auto mode_tag) {
    load_tile(mode_tag, 0);
    store_tile(mode_tag, 0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      const bool more = kt + 1 < ktiles;
      if (more) load_tile(mode_tag, kt + 1);
      compute(buf, std::integral_constant<int, 0>{}, std::integral_constant<int, KMID>{});
      if (more) store_tile(mode_tag, buf ^ 1);
      compute(buf, std::integral_constant<int, KMID>{}, std::integral_constant<int, KB>{});
      __syncthreads();
    }
  };

  if (ktiles > 0) {
    const bool interior = avec && bvec && (i0 + BM <= av.vrows) && (j0 + BN <= bv.vcols) &&
                          (K % BK == 0) && (K <= av.vcols) && (K <= bv.vrows);
    const bool edge_vec = avec && bvec && av.vrows > 0 && av.vcols > 0 && bv.vrows > 0 && bv.vcols > 0 &&
                          av.vcols % E == 0 && bv.vcols % E == 0;
    if (interior)
      main_loop(std::integral_constant<int, LOAD_FULL>{});
    else if (edge_vec)
      main_loop(std::integral_constant<int, LOAD_EDGE_VEC>{});
    else
      main_loop(std::integral_constant<int, LOAD_MASKED>{});
  }

  // ---- epilogue --------------------------------------------------------------
  store_outputs<T, TM, M::NACC, FM, FN, WM, WN>(kb, D, i0, j0, wm, wn, lane, acc,
                                                 [](int l, int r) { return M::row(l, r); });
}

template <typename T, int BM, int BN, int BKC, int WGM, int WGN>
hipError_t launch_cfg(const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap, hipStream_t s) {
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BKC, WGM, WGN>), dim3(tiles), dim3(64 * WGM * WGN), 0, s, kb,
                     d, n, remap);
  return hipGetLastError();
}

}  // namespace

GemmCfg gemm_cfg(int dtype, int cfg) {
  if (dtype == DT_BF16X3) return gemm_bf16x3_cfg(cfg);
  if (dtype == DT_F64) {
    switch (cfg) {
      case 5: return {128, 64};
      default: return {128, 128};
    }
  }
  switch (cfg) {
    case 1: return {256, 128};
    case 2: return {128, 256};
    case 3: return {256, 256};
    case 4: return {64, 128};
    case 5: return {128, 64};
    case 6: return {256, 128};
    case 7: return {128, 128};
    default: return {128, 128};
  }
}

hipError_t launch_gemm(int dtype, int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles,
                       int remap, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  if (dtype == DT_BF16X3) return launch_gemm_bf16x3(cfg, kb, d, n, tiles, remap, s);
  if (dtype == DT_F64) {
    switch (cfg) {
      case 5: return launch_cfg<double, 128, 64, 8, 2, 2>(kb, d, n, tiles, remap, s);
      default: return launch_cfg<double, 128, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
    }
  }
  switch (cfg) {
    case 1: return launch_cfg<float, 256, 128, 8, 4, 2>(kb, d, n, tiles, remap, s);
    case 2: return launch_cfg<float, 128, 256, 8, 2, 4>(kb, d, n, tiles, remap, s);
    case 3: return launch_cfg<float, 256, 256, 4, 2, 2>(kb, d, n, tiles, remap, s);
    case 4: return launch_cfg<float, 64, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
    case 5: return launch_cfg<float, 128, 64, 8, 2, 2>(kb, d, n, tiles, remap, s);
    case 6: return launch_cfg<float, 256, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
    case 7: return launch_cfg<float, 128, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
    default: return launch_cfg<float, 128, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
  }
}

}  // namespace mm
