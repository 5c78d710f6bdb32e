// Leaf products for float32 operands on bfloat16 matrix cores, with the
// split-precision refinement of the MM_BF16X3_REFINED dtype.
//
// Every float32 operand element x is split once, when its tile is staged in
// LDS, into three bfloat16 parts (round to nearest even at each step):
//   hi  = bf16(x)
//   lo  = bf16(x - hi)
//   res = bf16(x - hi - lo)
// Each difference is exact in float32: x - hi is a multiple of x's float32
// unit in the last place and at most half a bfloat16 unit of x, so it needs
// at most 16 significant bits, and (x - hi) - lo needs at most 8.  The
// residual is thus formed exactly in float32 registers: forming it in
// float64, as a refinement residual is usually formed, gives the same bits at
// twice the vector cost.  For |x| >= 2^-110 the residual is itself a
// bfloat16 number and x = hi + lo + res exactly; below that it falls into
// bfloat16's subnormal range and is rounded.  A product of two parts is exact in float32 (8 x 8
// significant bits), so v_mfma_f32_32x32x16_bf16 accumulates them in float32
// without extra rounding.  Per 16-wide k step each C tile receives the three
// leading products hi*hi + hi*lo + lo*hi and the one-step correction
// lo*lo + res*hi + hi*res, smallest first; the neglected terms (lo*res,
// res*lo, res*res) are below 2^-24 relative.  The result therefore carries
// float32-level error while every multiply runs at the bfloat16 MFMA rate.
//
// Structure as in the float32 kernel: grouped problems, XCD-aware tile order,
// LDS double buffering (three planes per operand: hi, lo, res), masked edge
// tiles and a branch-free interior loop.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.h"
#include "gemm_common.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace gemm_detail;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// v_mfma_f32_32x32x16_bf16: lanes 0-31 and 32-63 supply the two 8-wide k
// halves of a 32 x 16 by 16 x 32 product (lane l: row / column l % 32); the
// result layout is that of the other 32 x 32 MFMAs:
// register r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int row32(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Round a pair of floats to bfloat16 (nearest even) with one packed
// conversion; element 0 lands in the low half of the returned word.
__device__ __forceinline__ unsigned cvt_pair(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
// The two bfloat16 halves of a packed word as floats (exact: a bfloat16 is
// the top half of a float).
__device__ __forceinline__ float lo_half(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_half(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// Split 8 floats into their bfloat16 hi, lo and residual parts (both
// differences are exact, see above), two elements per conversion.
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo, bf16x8& rs) {
  u32x4 H, Lw, R;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const float x0 = x[2 * p], x1 = x[2 * p + 1];
    const unsigned h = cvt_pair(x0, x1);
    const float d0 = x0 - lo_half(h), d1 = x1 - hi_half(h);
    const unsigned l = cvt_pair(d0, d1);
    const float e0 = d0 - lo_half(l), e1 = d1 - hi_half(l);
    H[p] = h;
    Lw[p] = l;
    R[p] = cvt_pair(e0, e1);
  }
  hi = __builtin_bit_cast(bf16x8, H);
  lo = __builtin_bit_cast(bf16x8, Lw);
  rs = __builtin_bit_cast(bf16x8, R);
}

constexpr int KC = 8;  // k values per 16-byte chunk (bfloat16)
constexpr int EB = 2;  // B columns per staged block (one float2 per k row)

template <int BM, int BN, int BKC, int WGM, int WGN, bool LATE>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_bf16x3_kernel(KernelBases kb,
                                                                     const GemmDesc* __restrict__ descs,
                                                                     int ndesc, int remap) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int TM = 32;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int BK = BKC * KC;
  constexpr int NCH_A = BM * BKC;  // 8-float chunks of A per stage
  constexpr int NA = (NCH_A + NT - 1) / NT;
  constexpr int NBLK_B = BKC * (BN / EB);  // 8 x 2 blocks of B per stage
  constexpr int NB = (NBLK_B + NT - 1) / NT;
  static_assert(BKC % 2 == 0 && 16 % BKC == 0 && FM >= 1 && FN >= 1, "tile shape");

  __shared__ bf16x8 As[2][3][BKC][BM];
  __shared__ bf16x8 Bs[2][3][BKC][BN];

  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const GemmDesc& D = descs[tr.desc];
  const int i0 = tr.i0, j0 = tr.j0;
  const MView av = D.a, bv = D.b;
  const float* __restrict__ Ap = resolve<float>(kb, av);
  const float* __restrict__ Bp = resolve<float>(kb, bv);
  const int64_t lda = av.ld, ldb = bv.ld;
  const bool avec = view_vec(kb, av), bvec = view_vec(kb, bv);
  const int K = D.k;
  const int ktiles = (K + BK - 1) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  float ra[NA][8];
  float rb[NB][8][EB];
  // LOAD_EDGE_VEC validity, applied when the stage is split into LDS
  uint32_t amask = 0, bmask = 0;

  auto load_tile = [&](auto mode_tag, int kt) {
    constexpr int MODE = decltype(mode_tag)::value;
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gc = k0 + kc * KC;
      const float* p = Ap + (int64_t)gr * lda + gc;
      if (MODE == LOAD_EDGE_VEC) {
        // float4 halves are either valid or not (valid width % 4 == 0)
        const bool r_ok = gr < av.vrows;
        const bool ok0 = r_ok && gc < av.vcols, ok1 = r_ok && gc + 4 < av.vcols;
        const f32x4 u = *reinterpret_cast<const f32x4*>(ok0 ? p : Ap);
        const f32x4 w = *reinterpret_cast<const f32x4*>(ok1 ? p + 4 : Ap);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ra[i][e] = u[e];
          ra[i][4 + e] = w[e];
        }
        const uint32_t b0 = 1u << (2 * i), b1 = 1u << (2 * i + 1);
        amask = ok0 ? (amask | b0) : (amask & ~b0);
        amask = ok1 ? (amask | b1) : (amask & ~b1);
      } else if (MODE == LOAD_FULL || (avec && gr < av.vrows && gc + KC <= av.vcols)) {
        const f32x4 u = *reinterpret_cast<const f32x4*>(p);
        const f32x4 w = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ra[i][e] = u[e];
          ra[i][4 + e] = w[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KC; ++e) ra[i][e] = (gr < av.vrows && gc + e < av.vcols) ? p[e] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      if (NBLK_B % NT != 0 && q >= NBLK_B) break;
      const int kc = q / (BN / EB), cb = q % (BN / EB);
      const int gc = j0 + cb * EB;
#pragma unroll
      for (int rr = 0; rr < KC; ++rr) {
        const int gr = k0 + kc * KC + rr;
        const float* p = Bp + (int64_t)gr * ldb + gc;
        if (MODE == LOAD_EDGE_VEC) {
          const bool ok = gr < bv.vrows && gc < bv.vcols;
          const f32x2 u = *reinterpret_cast<const f32x2*>(ok ? p : Bp);
          rb[i][rr][0] = u[0];
          rb[i][rr][1] = u[1];
          const uint32_t bit = 1u << (i * KC + rr);
          bmask = ok ? (bmask | bit) : (bmask & ~bit);
        } else if (MODE == LOAD_FULL || (bvec && gr < bv.vrows && gc + EB <= bv.vcols)) {
          const f32x2 u = *reinterpret_cast<const f32x2*>(p);
          rb[i][rr][0] = u[0];
          rb[i][rr][1] = u[1];
        } else {
#pragma unroll
          for (int e = 0; e < EB; ++e) rb[i][rr][e] = (gr < bv.vrows && gc + e < bv.vcols) ? p[e] : 0.f;
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
      if (MODE == LOAD_EDGE_VEC) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (!((amask >> (2 * i + e / 4)) & 1)) ra[i][e] = 0.f;
      }
      bf16x8 h, l, r;
      split8(ra[i], h, l, r);
      const int sr = swz_a<BKC>(row, kc);
      As[buf][0][kc][sr] = h;
      As[buf][1][kc][sr] = l;
      As[buf][2][kc][sr] = r;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      if (NBLK_B % NT != 0 && q >= NBLK_B) break;
      const int kc = q / (BN / EB), cb = q % (BN / EB);
#pragma unroll
      for (int c = 0; c < EB; ++c) {
        float col[8];
#pragma unroll
        for (int rr = 0; rr < KC; ++rr)
          col[rr] = (MODE != LOAD_EDGE_VEC || ((bmask >> (i * KC + rr)) & 1)) ? rb[i][rr][c] : 0.f;
        bf16x8 h, l, r;
        split8(col, h, l, r);
        const int sc = swz_b<EB>(cb * EB + c);
        Bs[buf][0][kc][sc] = h;
        Bs[buf][1][kc][sc] = l;
        Bs[buf][2][kc][sc] = r;
      }
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int g = lane / TM, t = lane % TM;

  // MFMAs of k-steps [ks_lo, ks_hi) (16 k values each).  The six products
  // of a tile are issued in the refinement order (smallest first); tiles of
  // one product type are interleaved so consecutive MFMAs are independent.
  auto compute = [&](int buf, int ks_lo, int ks_hi) {
#pragma unroll
    for (int ks = ks_lo; ks < ks_hi; ++ks) {
      const int plane = 2 * ks + g;
      bf16x8 fb[3][FN];
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int b = 0; b < FN; ++b) fb[p][b] = Bs[buf][p][plane][swz_b<EB>(wn * WN + b * TM + t)];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        bf16x8 fa[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) fa[p] = As[buf][p][plane][swz_a<BKC>(wm * WM + a * TM + t, plane)];
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[1], fb[1][b], acc[a][b]);  // lo  * lo
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[2], fb[0][b], acc[a][b]);  // res * hi
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[0], fb[2][b], acc[a][b]);  // hi  * res
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[1], fb[0][b], acc[a][b]);  // lo  * hi
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[0], fb[1][b], acc[a][b]);  // hi  * lo
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[0], fb[0][b], acc[a][b]);  // hi  * hi
      }
    }
  };

  // The next stage is split into the other LDS buffer halfway through this
  // stage's MFMAs, or (LATE) after all of them, which gives its global loads
  // a whole stage to arrive (safe with two buffers: it was last read before
  // the previous barrier and is read after the next one).
  auto main_loop = [&](auto mode_tag) {
    load_tile(mode_tag, 0);
    store_tile(mode_tag, 0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      const bool more = kt + 1 < ktiles;
      if (more) load_tile(mode_tag, kt + 1);
      if constexpr (LATE) {
        compute(buf, 0, BKC / 2);
        if (more) store_tile(mode_tag, buf ^ 1);
      } else {
        compute(buf, 0, BKC / 4);
        if (more) store_tile(mode_tag, buf ^ 1);
        compute(buf, BKC / 4, BKC / 2);
      }
      __syncthreads();
    }
  };

  if (ktiles > 0) {
    const bool interior = avec && bvec && (i0 + BM <= av.vrows) && (j0 + BN <= bv.vcols) &&
                          (K % BK == 0) && (K <= av.vcols) && (K <= bv.vrows);
    const bool edge_vec = avec && bvec && av.vrows > 0 && av.vcols > 0 && bv.vrows > 0 && bv.vcols > 0 &&
                          av.vcols % 4 == 0 && bv.vcols % EB == 0;
    if (interior)
      main_loop(std::integral_constant<int, LOAD_FULL>{});
    else if (edge_vec)
      main_loop(std::integral_constant<int, LOAD_EDGE_VEC>{});
    else
      main_loop(std::integral_constant<int, LOAD_MASKED>{});
  }

  // (the checked epilogue: this kernel has no registers to spare)
  store_outputs<float, TM, 16, FM, FN, WM, WN, false, false>(kb, D, i0, j0, wm, wn, lane, acc,
                                                             [](int l, int r) { return row32(l, r); });
}

// f(integral_constant<int, I>) for I = I0 .. N-1, unrolled by construction
// (a loop whose body indexes register arrays must not be left rolled).
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// The same products on a 256 x 256 tile with eight waves (two per SIMD, each
// 128 x 64; also instantiated as 128 x 128 with four waves of 64 x 64, two
// workgroups per CU), software-pipelined over a ring of three LDS stages of
// 16 k (one MFMA k-step; 48 MFMAs per wave and stage on the large tile).
// Each thread stages one 8-float chunk of A and one 8-row column of B per
// stage, so the split work is the same in every wave.  During stage t:
//  * the registers hold the raw float32 data of stage t+2 (loaded during
//    stage t-1); it is split into hi, lo and residual and stored to the
//    third LDS buffer between the MFMAs of the first two rows of 32 x 32
//    tiles, after which the loads of stage t+3 are issued into the same
//    registers (buffer loads: per-lane 32-bit offsets fixed for the whole
//    loop, the stage's position in scalar registers);
//  * the buffer of stage t+1 was written during stage t-1 and published by
//    the barrier that began stage t, so each wave reads stage t+1's B
//    fragments and first-row A fragments during the last row of MFMAs, and
//    the barrier that ends the stage (a wait for this wave's LDS accesses,
//    not for the global loads in flight) is followed by MFMAs at once;
//  * the A fragments of the next row are read during the current row.
// The last three stages are peeled (no loads, then no split).  A k that is
// not a multiple of 16 is bounds-checked in its last stage; tiles at a
// matrix edge read clamped rows and columns (see the offsets below), or,
// where that is not allowed, run the ring with branch-free bounds-checked
// loads; products of fewer than three stages take a one-buffer loop.  The
// six products of a tile are issued in the order of the kernel above: the
// same bits.
template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_bf16r_kernel(KernelBases kb,
                                                                    const GemmDesc* __restrict__ descs,
                                                                    int ndesc, int remap) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int TM = 32;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int BKC = 2;
  constexpr int BK = BKC * KC;
  constexpr int NCH_A = BM * BKC;   // 8-float chunks of A per stage
  constexpr int NA = NCH_A / NT;
  constexpr int NBLK_B = BKC * BN;  // 8 x 1 columns of B per stage
  constexpr int NB = NBLK_B / NT;
  constexpr int NPART = NA + NB;    // split calls per thread and stage
  static_assert(NCH_A % NT == 0 && NBLK_B % NT == 0 && NA >= 1 && NB >= 1, "whole chunks per thread");
  static_assert(FM >= 2 && FM % 2 == 0, "rows of MFMA tiles in pairs (A fragments alternate)");

  __shared__ bf16x8 As[3][3][BKC][BM];
  __shared__ bf16x8 Bs[3][3][BKC][BN];

  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const GemmDesc& D = descs[tr.desc];
  const int i0 = tr.i0, j0 = tr.j0;
  const MView av = D.a, bv = D.b;
  const float* __restrict__ Ap = resolve<float>(kb, av);
  const float* __restrict__ Bp = resolve<float>(kb, bv);
  const int64_t lda = av.ld, ldb = bv.ld;
  const bool avec = view_vec(kb, av);
  const int K = D.k;
  const int ktiles = (K + BK - 1) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int g = lane / TM, t = lane % TM;

  float sa[NA][8];  // staged A chunks of one stage
  float sb[NB][8];  // staged B columns of one stage

  // buffer-load offsets: bytes from the stage's first element (A row i0,
  // column k0; B row k0, column j0); they fit in 32 bits for leading
  // dimensions below 2^21 (checked with the interior test).  In a tile at a
  // matrix edge, rows of A past its valid rows and columns of B past its
  // valid columns are read as copies of the last valid one: an output
  // element depends only on its own row of A and column of B, so these
  // reach only outputs past the edge, which are not stored (checked below).
  const int rlast = min(BM, av.vrows - i0) - 1, clast = min(BN, bv.vcols - j0) - 1;
  uint32_t oa[NA], ob[NB];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int q = tid + NT * i;
    oa[i] = (uint32_t)((min(q / BKC, rlast) * lda + (q % BKC) * KC) * (int64_t)sizeof(float));
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int q = tid + NT * i;
    ob[i] = (uint32_t)(((q / BN) * KC * ldb + min(q % BN, clast)) * (int64_t)sizeof(float));
  }
  const uint32_t brow = (uint32_t)(ldb * (int64_t)sizeof(float));
  auto rsrc = [](const float* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, -1, 0x00020000);
  };
  auto load_full = [&](int kt) {
    const int64_t k0 = (int64_t)kt * BK;
    const __amdgpu_buffer_rsrc_t ra = rsrc(Ap + (int64_t)i0 * lda + k0);
    const __amdgpu_buffer_rsrc_t rb = rsrc(Bp + k0 * ldb + j0);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const f32x4 u = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, oa[i], 0, 0));
      const f32x4 w = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, oa[i] + 16, 0, 0));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        sa[i][e] = u[e];
        sa[i][4 + e] = w[e];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int rr = 0; rr < KC; ++rr)
        sb[i][rr] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, ob[i], rr * brow, 0));
  };
  auto load_masked = [&](int kt) {
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gc = k0 + kc * KC;
      const float* p = Ap + (int64_t)gr * lda + gc;
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[i][e] = (gr < av.vrows && gc + e < av.vcols) ? p[e] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      const int kc = q / BN, cb = q % BN;
      const int gc = j0 + cb;
#pragma unroll
      for (int rr = 0; rr < KC; ++rr) {
        const int gr = k0 + kc * KC + rr;
        sb[i][rr] = (gr < bv.vrows && gc < bv.vcols) ? Bp[(int64_t)gr * ldb + gc] : 0.f;
      }
    }
  };
  // Stage kt of a tile at a matrix edge, without branches: every load reads
  // a valid element (indices clamped into the operand) and is replaced by
  // zero past the edges (the values of load_masked).
  auto load_edge = [&](int kt) {
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gc = k0 + kc * KC;
      const bool rok = gr < av.vrows;
      const float* p = Ap + (int64_t)(rok ? gr : 0) * lda;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool ok = rok && gc + e < av.vcols;
        const float v = p[ok ? gc + e : 0];
        sa[i][e] = ok ? v : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      const int kc = q / BN, cb = q % BN;
      const int gc = j0 + cb;
      const bool cok = gc < bv.vcols;
#pragma unroll
      for (int rr = 0; rr < KC; ++rr) {
        const int gr = k0 + kc * KC + rr;
        const bool ok = cok && gr < bv.vrows;
        const float v = Bp[(int64_t)(ok ? gr : 0) * ldb + (ok ? gc : 0)];
        sb[i][rr] = ok ? v : 0.f;
      }
    }
  };
  // Split call j (0 .. NPART - 1: the A chunks, then the B columns) of the
  // staged stage into LDS buffer buf.
  auto split_part = [&](int buf, int j) {
    bf16x8 h, l, r;
    if (j < NA) {
      const int q = tid + NT * j;
      const int row = q / BKC, kc = q % BKC;
      split8(sa[j], h, l, r);
      const int sr = swz_a<BKC>(row, kc);
      As[buf][0][kc][sr] = h;
      As[buf][1][kc][sr] = l;
      As[buf][2][kc][sr] = r;
    } else {
      const int q = tid + NT * (j - NA);
      const int kc = q / BN, cb = q % BN;
      split8(sb[j - NA], h, l, r);
      const int sc = swz_b<EB>(cb);
      Bs[buf][0][kc][sc] = h;
      Bs[buf][1][kc][sc] = l;
      Bs[buf][2][kc][sc] = r;
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  bf16x8 fb[3][FN], nfb[3][FN], fa[2][3];
  auto read_b = [&](int buf, bf16x8 (&x)[3][FN]) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int b = 0; b < FN; ++b) x[p][b] = Bs[buf][p][g][swz_b<EB>(wn * WN + b * TM + t)];
  };
  auto read_a = [&](int buf, int a, bf16x8 (&x)[3]) {
#pragma unroll
    for (int p = 0; p < 3; ++p) x[p] = As[buf][p][g][swz_a<BKC>(wm * WM + a * TM + t, g)];
  };
  // LDS accesses of this wave done, then the workgroup barrier (the global
  // loads in flight are not waited for: vmcnt left at its maximum)
  auto lds_barrier = [&]() {
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  // With k not a multiple of 16 the last stage is loaded with bounds checks
  // (zeros past k, as in the one-buffer loop: the same bits).
  const bool ragged = K % BK != 0;
  auto load_last = [&](int kt) {
    if (ragged)
      load_masked(kt);
    else
      load_full(kt);
  };

  // Stage kt from buffer kt % 3 (its B fragments and first-row A fragments
  // in registers).  SPLIT: the staged stage kt+2 goes into buffer (kt+2) % 3
  // between the first FM/2 rows; LOAD (1, or 2 when stage kt+3 is the last):
  // then stage kt+3 is loaded into the staging registers; NEXT: the last row
  // also reads stage kt+1's fragments.
  auto stage = [&](auto split_tag, auto load_tag, auto next_tag, int kt) __attribute__((always_inline)) {
    constexpr bool SPLIT = decltype(split_tag)::value;
    constexpr int LOAD = decltype(load_tag)::value;
    constexpr bool NEXT = decltype(next_tag)::value;
    const int buf = kt % 3, nbuf = (kt + 1) % 3, sbuf = (kt + 2) % 3;
    static_for<0, FM>([&](auto a_tag) {
      constexpr int a = decltype(a_tag)::value;
      constexpr int ca = a & 1;
      __builtin_amdgcn_sched_barrier(0);
      if (a + 1 < FM) {
        read_a(buf, a + 1, fa[ca ^ 1]);
      } else if (NEXT) {
        read_a(nbuf, 0, fa[ca ^ 1]);
        read_b(nbuf, nfb);
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[ca][1], fb[1][b], acc[a][b]);  // lo  * lo
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[ca][2], fb[0][b], acc[a][b]);  // res * hi
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[ca][0], fb[2][b], acc[a][b]);  // hi  * res
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[ca][1], fb[0][b], acc[a][b]);  // lo  * hi
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[ca][0], fb[1][b], acc[a][b]);  // hi  * lo
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[ca][0], fb[0][b], acc[a][b]);  // hi  * hi
      if constexpr (SPLIT) {
#pragma unroll
        for (int j = 0; j < NPART; ++j)
          if (j * (FM / 2) / NPART == a) split_part(sbuf, j);
      }
      if constexpr (LOAD == 1) {
        if (a == FM / 2 - 1) load_full(kt + 3);
      } else if constexpr (LOAD == 2) {
        if (a == FM / 2 - 1) load_last(kt + 3);
      } else if constexpr (LOAD == 3) {
        if (a == FM / 2 - 1) load_edge(kt + 3);
      }
      // one MFMA, then a share of the row's other work: an LDS read of the
      // next fragments, six vector instructions of the split, its LDS
      // stores and the global loads (measured 2 % faster than leaving the
      // order to the compiler, which gathers the reads before the barrier)
#pragma unroll
      for (int i = 0; i < 6 * FN; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
        __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // global load
      }
      __builtin_amdgcn_sched_barrier(0);
    });
    if constexpr (NEXT) {
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int b = 0; b < FN; ++b) fb[p][b] = nfb[p][b];
    }
  };
  typedef std::integral_constant<bool, true> yes;
  typedef std::integral_constant<bool, false> no;
  typedef std::integral_constant<int, 0> load_none;

  // The ring over all stages.  Tiles inside both operands (16-byte rows, k
  // within them, leading dimensions that fit the 32-bit offsets) load with
  // buffer loads (the last stage bounds-checked when k is ragged); tiles at
  // a matrix edge run the same loop with bounds-checked loads (zeros past
  // the edges, as in the one-buffer loop).
  auto ring = [&](auto masked_tag) __attribute__((always_inline)) {
    constexpr bool MASKED = decltype(masked_tag)::value;
    typedef std::integral_constant<int, MASKED ? 3 : 1> load_next;
    typedef std::integral_constant<int, MASKED ? 3 : 2> load_final;
    auto first = [&](int kt) __attribute__((always_inline)) {
      if constexpr (MASKED)
        load_edge(kt);
      else if (kt == ktiles - 1)
        load_last(kt);
      else
        load_full(kt);
    };
    first(0);
#pragma unroll
    for (int j = 0; j < NPART; ++j) split_part(0, j);
    first(1);
#pragma unroll
    for (int j = 0; j < NPART; ++j) split_part(1, j);
    first(2);
    lds_barrier();
    read_b(0, fb);
    read_a(0, 0, fa[0]);
    int kt = 0;
    for (; kt + 4 < ktiles; ++kt) {
      stage(yes{}, load_next{}, yes{}, kt);
      lds_barrier();
    }
    if (kt + 3 < ktiles) {  // kt = ktiles - 4: loads the last stage
      stage(yes{}, load_final{}, yes{}, kt);
      lds_barrier();
      ++kt;
    }
    stage(yes{}, load_none{}, yes{}, kt);  // kt = ktiles - 3
    lds_barrier();
    stage(no{}, load_none{}, yes{}, kt + 1);
    lds_barrier();
    stage(no{}, load_none{}, no{}, kt + 2);
  };

  // The buffer-load loop: A in 16-byte chunks, k within both operands,
  // offsets in 32 bits, and at a matrix edge every stored output inside the
  // operands' valid rows and columns (outputs past A's valid rows would be
  // zero rows of the padded product, not copies).
  bool edge_ok = rlast >= 0 && clast >= 0;
  for (int o = 0; o < D.nout; ++o)
    edge_ok = edge_ok && D.out[o].c.vrows <= av.vrows && D.out[o].c.vcols <= bv.vcols;
  const bool interior = avec && (K <= av.vcols) && (K <= bv.vrows) && lda < (int64_t(1) << 21) &&
                        ldb < (int64_t(1) << 21) &&
                        (((i0 + BM <= av.vrows) && (j0 + BN <= bv.vcols)) || edge_ok);
  if (ktiles >= 3) {
    if (interior)
      ring(no{});
    else
      ring(yes{});
  } else if (ktiles > 0) {
    for (int kt = 0; kt < ktiles; ++kt) {
      load_masked(kt);
#pragma unroll
      for (int j = 0; j < NPART; ++j) split_part(0, j);
      __syncthreads();
      read_b(0, fb);
      read_a(0, 0, fa[0]);
      stage(no{}, load_none{}, no{}, 0);
      __syncthreads();
    }
  }

  // (the epilogue's interior path only on the 256 x 256 tile: it would take the
  // 128 x 128 tile past the registers of two workgroups per CU)
  store_outputs<float, TM, 16, FM, FN, WM, WN, false, (BM == 256)>(kb, D, i0, j0, wm, wn, lane, acc,
                                                                    [](int l, int r) { return row32(l, r); });
}

// The same products from operands already split by the split pass (SPL
// layout, desc.h): a is the m x k A operand, b the n x k transpose of the B
// operand, each a run of 48-byte chunks (hi, lo, res of 8 consecutive k).
// Staging a tile is three 16-byte loads per chunk and three LDS stores, with
// no conversion work; the LDS layout, the MFMA sequence and the order of the
// six products are those of the kernel above, so both give the same bits.
template <int BM, int BN, int BKC, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_bf16s_kernel(KernelBases kb,
                                                                    const GemmDesc* __restrict__ descs,
                                                                    int ndesc, int remap) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int TM = 32;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int BK = BKC * KC;
  constexpr int NCH_A = BM * BKC, NA = (NCH_A + NT - 1) / NT;
  constexpr int NCH_B = BN * BKC, NB = (NCH_B + NT - 1) / NT;
  static_assert(BKC % 2 == 0 && 16 % BKC == 0 && FM >= 1 && FN >= 1, "tile shape");

  __shared__ bf16x8 As[2][3][BKC][BM];
  __shared__ bf16x8 Bs[2][3][BKC][BN];

  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const GemmDesc& D = descs[tr.desc];
  const int i0 = tr.i0, j0 = tr.j0;
  const MView av = D.a, bv = D.b;
  auto spl = [&](const MView& v) {
    char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
    return reinterpret_cast<const __bf16*>(b) + v.off;
  };
  const __bf16* __restrict__ Ap = spl(av);
  const __bf16* __restrict__ Bp = spl(bv);
  const int64_t lda = av.ld, ldb = bv.ld;
  const int K = D.k;
  const int ktiles = (K + BK - 1) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  bf16x8 ra[NA][3], rb[NB][3];

  // FULL: the stage lies inside both operands; otherwise rows past the valid
  // extent and chunks past the k extent read as zero.
  auto load_tile = [&](auto full_tag, int kt) {
    constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gq = kt * BKC + kc;
      const bf16x8* p = reinterpret_cast<const bf16x8*>(Ap + (int64_t)gr * lda + 24 * (int64_t)gq);
      const bool ok = FULL || (gr < av.vrows && 8 * gq < av.vcols);
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) ra[i][pl] = ok ? p[pl] : bf16x8{};
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      if (NCH_B % NT != 0 && q >= NCH_B) break;
      const int col = q / BKC, kc = q % BKC;
      const int gc = j0 + col, gq = kt * BKC + kc;
      const bf16x8* p = reinterpret_cast<const bf16x8*>(Bp + (int64_t)gc * ldb + 24 * (int64_t)gq);
      const bool ok = FULL || (gc < bv.vrows && 8 * gq < bv.vcols);
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) rb[i][pl] = ok ? p[pl] : bf16x8{};
    }
  };

  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      const int sr = swz_a<BKC>(row, kc);
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) As[buf][pl][kc][sr] = ra[i][pl];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      if (NCH_B % NT != 0 && q >= NCH_B) break;
      const int col = q / BKC, kc = q % BKC;
      const int sc = swz_a<BKC>(col, kc);
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) Bs[buf][pl][kc][sc] = rb[i][pl];
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int g = lane / TM, t = lane % TM;

  // MFMAs of k-step ks (16 k values) for tile rows [a_lo, a_hi) with the B
  // fragments fb of that step.  The six products of a tile are issued in
  // the refinement order (smallest first); tiles of one product type are
  // interleaved so consecutive MFMAs are independent.
  auto read_fb = [&](int buf, int ks, bf16x8 (&fb)[3][FN]) {
    const int plane = 2 * ks + g;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int b = 0; b < FN; ++b) fb[p][b] = Bs[buf][p][plane][swz_a<BKC>(wn * WN + b * TM + t, plane)];
  };
  auto compute = [&](int buf, int ks, int a_lo, int a_hi, const bf16x8 (&fb)[3][FN]) {
    const int plane = 2 * ks + g;
#pragma unroll
    for (int a = a_lo; a < a_hi; ++a) {
      bf16x8 fa[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) fa[p] = As[buf][p][plane][swz_a<BKC>(wm * WM + a * TM + t, plane)];
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[1], fb[1][b], acc[a][b]);  // lo  * lo
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[2], fb[0][b], acc[a][b]);  // res * hi
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[0], fb[2][b], acc[a][b]);  // hi  * res
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[1], fb[0][b], acc[a][b]);  // lo  * hi
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[0], fb[1][b], acc[a][b]);  // hi  * lo
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[0], fb[0][b], acc[a][b]);  // hi  * hi
    }
  };

  // The next stage is written to the other LDS buffer in the middle of this
  // stage's MFMAs: after the first k-step when a stage has two, else after
  // the first half of the tile rows.
  auto main_loop = [&](auto full_tag) {
    load_tile(full_tag, 0);
    store_tile(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      const bool more = kt + 1 < ktiles;
      if (more) load_tile(full_tag, kt + 1);
      bf16x8 fb[3][FN];
      if constexpr (BKC == 2) {
        read_fb(buf, 0, fb);
        compute(buf, 0, 0, FM / 2, fb);
        if (more) store_tile(buf ^ 1);
        compute(buf, 0, FM / 2, FM, fb);
      } else {
#pragma unroll
        for (int ks = 0; ks < BKC / 4; ++ks) {
          read_fb(buf, ks, fb);
          compute(buf, ks, 0, FM, fb);
        }
        if (more) store_tile(buf ^ 1);
#pragma unroll
        for (int ks = BKC / 4; ks < BKC / 2; ++ks) {
          read_fb(buf, ks, fb);
          compute(buf, ks, 0, FM, fb);
        }
      }
      __syncthreads();
    }
  };

  if (ktiles > 0) {
    const bool interior = (i0 + BM <= av.vrows) && (j0 + BN <= bv.vrows) && (K % BK == 0) &&
                          (K <= av.vcols) && (K <= bv.vcols);
    if (interior)
      main_loop(std::integral_constant<bool, true>{});
    else
      main_loop(std::integral_constant<bool, false>{});
  }

  // (the checked epilogue: its interior path costs the smaller tiles a wave per SIMD)
  store_outputs<float, TM, 16, FM, FN, WM, WN, false, false>(kb, D, i0, j0, wm, wn, lane, acc,
                                                             [](int l, int r) { return row32(l, r); });
}

template <int BM, int BN, int BKC, int WGM, int WGN>
hipError_t launch_spl(const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap, hipStream_t s) {
  hipLaunchKernelGGL((gemm_bf16s_kernel<BM, BN, BKC, WGM, WGN>), dim3(tiles), dim3(64 * WGM * WGN), 0, s, kb,
                     d, n, remap);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN>
hipError_t launch_ring(const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap, hipStream_t s) {
  hipLaunchKernelGGL((gemm_bf16r_kernel<BM, BN, WGM, WGN>), dim3(tiles), dim3(64 * WGM * WGN), 0, s, kb, d, n,
                     remap);
  return hipGetLastError();
}

template <int BM, int BN, int BKC, int WGM, int WGN, bool LATE = false>
hipError_t launch_cfg(const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap, hipStream_t s) {
  hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, BN, BKC, WGM, WGN, LATE>), dim3(tiles), dim3(64 * WGM * WGN), 0, s,
                     kb, d, n, remap);
  return hipGetLastError();
}

}  // namespace

bool gemm_bf16x3_available() { return true; }

GemmCfg gemm_bf16s_cfg(int cfg) {
  switch (cfg) {
    case 1: return {256, 128};
    case 3: return {256, 256};
    case 4: return {64, 128};
    case 5: return {256, 128};
    case 6: return {256, 256};
    default: return {128, 128};
  }
}

GemmCfg gemm_bf16x3_cfg(int cfg) {
  switch (cfg) {
    case 1: return {256, 128};
    case 3: return {256, 256};
    case 4: return {64, 128};
    case 6: return {256, 256};
    case 8: return {64, 64};
    default: return {128, 128};
  }
}

hipError_t launch_gemm_bf16x3(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles,
                              int remap, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  switch (cfg) {
    // 256x128 (eight waves, two per SIMD) writes the next stage after all of
    // this stage's MFMAs (measured 2-3% faster at n = 8192); the four-wave
    // tiles write it halfway
    case 1: return launch_cfg<256, 128, 4, 4, 2, true>(kb, d, n, tiles, remap, s);
    case 3: return launch_cfg<256, 256, 2, 4, 2, true>(kb, d, n, tiles, remap, s);
    case 4: return launch_cfg<64, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
    // eight waves of 128 x 64, split pipelined under the MFMAs, three LDS
    // stages
    case 6: return launch_ring<256, 256, 2, 4>(kb, d, n, tiles, remap, s);
    // small products: one 32x32 tile per wave
    case 8: return launch_cfg<64, 64, 4, 2, 2>(kb, d, n, tiles, remap, s);
    // 128x128: four waves of 64 x 64 on the same three-stage ring (two
    // workgroups per CU)
    default: return launch_ring<128, 128, 2, 2>(kb, d, n, tiles, remap, s);
  }
}

hipError_t launch_gemm_bf16s(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles,
                             int remap, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  switch (cfg) {
    case 1: return launch_spl<256, 128, 4, 4, 2>(kb, d, n, tiles, remap, s);
    case 3: return launch_spl<256, 256, 2, 2, 2>(kb, d, n, tiles, remap, s);
    case 4: return launch_spl<64, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
    case 5: return launch_spl<256, 128, 2, 2, 2>(kb, d, n, tiles, remap, s);
    case 6: return launch_spl<256, 256, 2, 4, 2>(kb, d, n, tiles, remap, s);
    default: return launch_spl<128, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
  }
}

}  // namespace mm
