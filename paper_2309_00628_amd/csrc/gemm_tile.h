// The K loop of one output tile of a leaf product on the MFMA units, shared
// by the GEMM kernels that accumulate products tile by tile: the plain /
// grouped leaf-product kernel and the kernel that forms a Winograd level's
// seven products and their U combinations in registers.
//
// Workgroup: a BM x BN tile of C split among WGM x WGN wave64s.  The K loop
// stages BM x BK and BK x BN tiles of A and B in LDS, double-buffered: the
// global loads of stage t+1 are in flight while the MFMAs consume stage t,
// one barrier per stage.
//
// LDS layout ("k-chunked"): a 16-byte chunk holds E consecutive k values
// (E = 4 floats / 2 doubles) of one row of A or one column of B, so every MFMA
// operand fetch is one ds_read_b128 that feeds E MFMAs.  Row (A) and column
// (B) indices are XOR-swizzled so that both the stores of the global tile and
// the fragment reads touch 16 distinct 16-byte bank groups per 16 lanes.
// float32 B (unless given transposed) is instead staged as it lies in
// memory, with the columns of each wave's MFMA tiles interleaved so that
// one read of FN consecutive floats feeds FN MFMAs (see nat_b below).
//
// Edges: operand reads outside a view's valid extent are zero (this is also
// how quadrants of a zero-padded matrix are read without a copy).  Interior
// tiles take an unmasked vector path.
//
// Operand sums: an operand may be one of the Strassen-Winograd sums S1..S4 /
// T1..T4 of Section 2.3 of a parent block's quadrants; the loader then
// reads the quadrants it needs and forms the sum, in the order of Section
// 2.3, when the stage is written to LDS (the same bits as a separate pass).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.h"
#include "gemm_common.h"

namespace mm {
namespace gemm_detail {

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


// One operand of a tile product: element (r, c) at p[r * ld + c], zero
// outside [0, vrows) x [0, vcols); vec: p and ld allow 16-byte loads.  For an
// operand sum p is the parent block's first element, (vrows, vcols) the
// extent of one (entirely valid) quadrant and q[i] the offset of quadrant i
// (order 11 12 21 22); a plain operand has q[0] = 0.
template <typename T>
struct Operand {
  const T* __restrict__ p;
  int64_t ld;
  int vrows, vcols;
  bool vec;
  int64_t q[4];
};

template <typename T>
__device__ __forceinline__ Operand<T> operand(const KernelBases& kb, const MView& v) {
  return Operand<T>{resolve<T>(kb, v), v.ld, v.vrows, v.vcols, view_vec(kb, v), {0, 0, 0, 0}};
}

// The sums of the quadrants of parent block v, each quadrant rows x cols.
template <typename T>
__device__ __forceinline__ Operand<T> operand_sum(const KernelBases& kb, const MView& v, int rows, int cols) {
  const int64_t r = (int64_t)rows * v.ld;
  return Operand<T>{resolve<T>(kb, v), v.ld, rows, cols, view_vec(kb, v), {0, cols, r, r + cols}};
}

// BM x BN tile per workgroup, WGM x WGN waves (each (BM/WGM) x (BN/WGN)),
// BKC 16-byte chunks of k per LDS stage.
template <typename T, int BM, int BN, int BKC, int WGM, int WGN>
struct TileLoop {
  typedef MT<T> M;
  typedef typename M::chunk_t chunk_t;
  typedef typename M::acc_t acc_t;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int E = M::E;
  static constexpr int TM = M::TM;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / TM, FN = WN / TM;
  static constexpr int BK = BKC * E;
  static constexpr int NBLK_B = BKC * (BN / E);      // E x E blocks of B per stage
  static constexpr int NB = (NBLK_B + NT - 1) / NT;  // ... per thread
  static constexpr int NCH_A = BM * BKC;             // chunks of A per stage
  static constexpr int NA = (NCH_A + NT - 1) / NT;
  static constexpr int KB = BKC / M::KG;             // k-blocks per stage
  static constexpr int KMID = KB / 2;
  static_assert(FM >= 1 && FN >= 1 && WM % TM == 0 && WN % TM == 0, "wave tile");
  static_assert(BKC % M::KG == 0 && BKC <= BKC_MAX && 16 % BKC == 0, "k chunks");
  static_assert(NA * E <= 64 && NB * E * E <= 64, "one validity bit per staged element");

  // A is staged row by row (BKC chunks per row, see a_idx); B as BKC planes
  // of BN column chunks (b_idx), or, when it is given transposed (OK_TRANS),
  // column by column like A.
  static constexpr int NCH_B = BN * BKC;             // chunks of B per stage
  static constexpr int NBT = (NCH_B + NT - 1) / NT;  // ... per thread (transposed B)
  static_assert(NBT <= NB * E && NBT * E <= 64, "staging of a transposed B");
  struct Smem {
    chunk_t As[2][BM * BKC];
    chunk_t Bs[2][BKC * BN];
  };
  static __device__ __forceinline__ int b_idx(int col, int kc) { return kc * BN + swz_b<E>(col); }

  // float32 B that is not given transposed is staged as it lies in memory
  // ("natural": BK rows of BN consecutive columns, no swizzle), and the
  // columns of a wave's FN MFMA tiles are interleaved: lane t of tile b
  // computes column FN t + b of the wave's WN columns, so one LDS read of FN
  // consecutive floats of a row of B feeds the lane's FN tiles.  B then needs
  // no transposition on the way into LDS (interior stages load straight into
  // it), and every k pairing of the MFMAs is that of the k-chunked layout,
  // so the products keep their bits.
  static constexpr bool NATF = std::is_same<T, float>::value;
  template <int KB2>
  static constexpr bool nat_b() { return NATF && KB2 != OK_TRANS; }
  static_assert(!NATF || FN == 1 || FN == 2 || FN == 4, "natural B: FN floats per LDS read");
  // column (within the tile) of lane t's outputs in MFMA tile b of wave
  // column wn, for B given transposed or not
  template <bool BT>
  static __device__ __forceinline__ int out_col(int wn, int b, int t) {
    return wn * WN + ((NATF && !BT) ? FN * t + b : b * TM + t);
  }

  // LDS slot of chunk kc of tile row `row`: the chunks of a row are contiguous
  // and their order is XOR-ed with bits of the row above log2(16 / BKC), so
  // 16 consecutive rows at one chunk position (a fragment read) and 16
  // consecutive chunks of the stores both fall in 16 distinct bank groups.
  static __device__ __forceinline__ int a_idx(int row, int kc) {
    return row * BKC + (kc ^ ((row / (16 / BKC)) & (BKC - 1)));
  }

  // Interior stages of a plain A load straight into LDS (global_load_lds,
  // 16 bytes per lane, 64 consecutive slots per wave instruction), with no
  // register staging or LDS stores; the lane that fills slot p loads the
  // chunk that a_idx places there.
  static constexpr bool DMA_A = NCH_A % NT == 0;
  static constexpr bool DMA_B = NCH_B % NT == 0;  // (transposed or natural B)
  // R rows (of A, or of a transposed B when IS_B) at r0 of the operand,
  // chunks of k0 + [0, BK), into LDS buffer buf in a_idx order.
  template <int R, bool IS_B>
  static __device__ __forceinline__ void dma_rows(Smem& sm, int buf, const Operand<T>& X, int r0, int k0) {
    constexpr int PER = (R * BKC) / NT;  // instructions per thread
    // (the wave index in a scalar register: the LDS destinations, M0, are
    // then computed without vector instructions)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int base = (wave * PER + i) * 64;
      const int p = base + lane;
      const int row = p / BKC, slot = p % BKC;
      const int kc = slot ^ ((row / (16 / BKC)) & (BKC - 1));
      const T* src = X.p + (int64_t)(r0 + row) * X.ld + k0 + kc * E;
      if (IS_B)
        __builtin_amdgcn_global_load_lds(src, &sm.Bs[buf][base], 16, 0, 0);
      else
        __builtin_amdgcn_global_load_lds(src, &sm.As[buf][base], 16, 0, 0);
    }
  }
  static __device__ __forceinline__ void dma_a(Smem& sm, int buf, const Operand<T>& A, int i0, int kt) {
    dma_rows<BM, false>(sm, buf, A, i0, kt * BK);
  }
  static __device__ __forceinline__ void dma_b(Smem& sm, int buf, const Operand<T>& B, int j0, int kt) {
    if constexpr (DMA_B) dma_rows<BN, true>(sm, buf, B, j0, kt * BK);
  }
  // Natural B (plain, interior stages): BK rows of BN columns at (kt BK, j0),
  // 16 bytes per lane in LDS order.
  static __device__ __forceinline__ void dma_bn(Smem& sm, int buf, const Operand<T>& B, int j0, int kt) {
    if constexpr (DMA_B) {
      constexpr int PER = NCH_B / NT;
      constexpr int CPR = BN / E;  // chunks per row
      const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int k0 = kt * BK;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int base = (wave * PER + i) * 64;
        const int p = base + lane;
        const T* src = B.p + (int64_t)(k0 + p / CPR) * B.ld + j0 + (p % CPR) * E;
        __builtin_amdgcn_global_load_lds(src, &sm.Bs[buf][base], 16, 0, 0);
      }
    }
  }

  typedef acc_t Acc[FM][FN];

  static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) acc[a][b][r] = T(0);
  }

  // Global -> register staging of stage kt (KA / KB2: operand kinds of A
  // and B, one staged chunk per quadrant a sum reads).
  // LOAD_FULL: the whole stage is inside both operands' valid extents and
  // every access is a 16-byte vector load (no masks, no branches, so the
  // loads of the next stage stay in flight while the MFMAs of this one run).
  // LOAD_EDGE_VEC: edge tile of aligned operands whose valid widths are
  // multiples of the chunk: whole chunks are in or out, selected without
  // branches (the validity is applied when the stage is written to LDS, not
  // right after the load, which would wait for it).  LOAD_MASKED: one load
  // per element, from the element itself when it is valid and from the
  // operand's first element otherwise, with the validity applied at the LDS
  // write in the same way (the operands are nonempty: see product).
  template <int MODE, int KA, int KB2>
  static __device__ __forceinline__ void load_tile(const Operand<T>& A, const Operand<T>& B, int i0, int j0,
                                                   int kt, chunk_t (&ra)[NA][popc4(kind_quads(KA))],
                                                   chunk_t (&rbk)[NB][E][popc4(kind_quads(KB2))],
                                                   uint64_t& amask, uint64_t& bmask) {
    constexpr int QA = kind_quads(KA), NQA = popc4(QA);
    constexpr int QB = kind_quads(KB2), NQB = popc4(QB);
    constexpr bool A_IN_REGS = !(MODE == LOAD_FULL && KA == OK_PLAIN && DMA_A);
    const int tid = threadIdx.x;
    const int k0 = kt * BK;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (!A_IN_REGS) break;
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gc = k0 + kc * E;
      const T* p = A.p + (int64_t)gr * A.ld + gc;
      if (MODE == LOAD_FULL) {
#pragma unroll
        for (int j = 0; j < NQA; ++j) ra[i][j] = *reinterpret_cast<const chunk_t*>(p + A.q[nth_quad(QA, j)]);
      } else if (MODE == LOAD_EDGE_VEC) {
        const bool ok = gr < A.vrows && gc < A.vcols;
        const T* s = ok ? p : A.p;
#pragma unroll
        for (int j = 0; j < NQA; ++j) ra[i][j] = *reinterpret_cast<const chunk_t*>(s + A.q[nth_quad(QA, j)]);
        const uint64_t bit = 1ull << i;
        amask = ok ? (amask | bit) : (amask & ~bit);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool ok = gr < A.vrows && gc + e < A.vcols;
          const T* s = ok ? p + e : A.p;
#pragma unroll
          for (int j = 0; j < NQA; ++j) ra[i][j][e] = s[A.q[nth_quad(QA, j)]];
          const uint64_t bit = 1ull << (i * E + e);
          amask = ok ? (amask | bit) : (amask & ~bit);
        }
      }
    }
    if constexpr (nat_b<KB2>()) {
      // natural B: chunk cc (E columns) of row `row` (one k) of the stage
      if (MODE == LOAD_FULL && KB2 == OK_PLAIN && DMA_B) return;  // loaded straight into LDS
      constexpr int CPR = BN / E;
#pragma unroll
      for (int i = 0; i < NBT; ++i) {
        const int q = tid + NT * i;
        if (NCH_B % NT != 0 && q >= NCH_B) break;
        const int row = q / CPR, cc = q % CPR;
        const int gr = k0 + row, gc = j0 + cc * E;
        const T* p = B.p + (int64_t)gr * B.ld + gc;
        chunk_t (&dst)[NQB] = rbk[i / E][i % E];
        if (MODE == LOAD_FULL) {
#pragma unroll
          for (int j = 0; j < NQB; ++j) dst[j] = *reinterpret_cast<const chunk_t*>(p + B.q[nth_quad(QB, j)]);
        } else if (MODE == LOAD_EDGE_VEC) {
          const bool ok = gr < B.vrows && gc < B.vcols;
          const T* src = ok ? p : B.p;
#pragma unroll
          for (int j = 0; j < NQB; ++j) dst[j] = *reinterpret_cast<const chunk_t*>(src + B.q[nth_quad(QB, j)]);
          const uint64_t bit = 1ull << i;
          bmask = ok ? (bmask | bit) : (bmask & ~bit);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const bool ok = gr < B.vrows && gc + e < B.vcols;
            const T* src = ok ? p + e : B.p;
#pragma unroll
            for (int j = 0; j < NQB; ++j) dst[j][e] = src[B.q[nth_quad(QB, j)]];
            const uint64_t bit = 1ull << (i * E + e);
            bmask = ok ? (bmask | bit) : (bmask & ~bit);
          }
        }
      }
      return;
    }
    if constexpr (KB2 == OK_TRANS) {
      // B given transposed: chunk kc of row `col` of B^T (one column of B)
      if (MODE == LOAD_FULL && DMA_B) return;  // loaded straight into LDS
#pragma unroll
      for (int i = 0; i < NBT; ++i) {
        const int q = tid + NT * i;
        if (NCH_B % NT != 0 && q >= NCH_B) break;
        const int col = q / BKC, kc = q % BKC;
        const int gr = j0 + col, gc = k0 + kc * E;
        const T* p = B.p + (int64_t)gr * B.ld + gc;
        chunk_t& dst = rbk[i / E][i % E][0];
        if (MODE == LOAD_FULL) {
          dst = *reinterpret_cast<const chunk_t*>(p);
        } else if (MODE == LOAD_EDGE_VEC) {
          const bool ok = gr < B.vrows && gc < B.vcols;
          dst = *reinterpret_cast<const chunk_t*>(ok ? p : B.p);
          const uint64_t bit = 1ull << i;
          bmask = ok ? (bmask | bit) : (bmask & ~bit);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const bool ok = gr < B.vrows && gc + e < B.vcols;
            dst[e] = *(ok ? p + e : B.p);
            const uint64_t bit = 1ull << (i * E + e);
            bmask = ok ? (bmask | bit) : (bmask & ~bit);
          }
        }
      }
      return;
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
        const T* p = B.p + (int64_t)gr * B.ld + gc;
        if (MODE == LOAD_FULL) {
#pragma unroll
          for (int j = 0; j < NQB; ++j)
            rbk[i][rr][j] = *reinterpret_cast<const chunk_t*>(p + B.q[nth_quad(QB, j)]);
        } else if (MODE == LOAD_EDGE_VEC) {
          const bool ok = gr < B.vrows && gc < B.vcols;
          const T* s = ok ? p : B.p;
#pragma unroll
          for (int j = 0; j < NQB; ++j)
            rbk[i][rr][j] = *reinterpret_cast<const chunk_t*>(s + B.q[nth_quad(QB, j)]);
          const uint64_t bit = 1ull << (i * E + rr);
          bmask = ok ? (bmask | bit) : (bmask & ~bit);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const bool ok = gr < B.vrows && gc + e < B.vcols;
            const T* s = ok ? p + e : B.p;
#pragma unroll
            for (int j = 0; j < NQB; ++j) rbk[i][rr][j][e] = s[B.q[nth_quad(QB, j)]];
            const uint64_t bit = 1ull << ((i * E + rr) * E + e);
            bmask = ok ? (bmask | bit) : (bmask & ~bit);
          }
        }
      }
    }
  }

  template <int MODE, int KA, int KB2>
  static __device__ __forceinline__ void store_tile(Smem& sm, int buf,
                                                    const chunk_t (&ra)[NA][popc4(kind_quads(KA))],
                                                    const chunk_t (&rbk)[NB][E][popc4(kind_quads(KB2))],
                                                    uint64_t amask, uint64_t bmask) {
    constexpr int QA = kind_quads(KA), NQA = popc4(QA);
    constexpr int QB = kind_quads(KB2), NQB = popc4(QB);
    constexpr bool A_IN_REGS = !(MODE == LOAD_FULL && KA == OK_PLAIN && DMA_A);
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (!A_IN_REGS) break;
      const int q = tid + NT * i;
      if (NCH_A % NT != 0 && q >= NCH_A) break;
      const int row = q / BKC, kc = q % BKC;
      chunk_t v;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        T x[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < NQA; ++j) x[nth_quad(QA, j)] = ra[i][j][e];
        v[e] = combine<KA>(x);
      }
      if (MODE == LOAD_EDGE_VEC) {
        if (!((amask >> i) & 1)) v = chunk_t{};
      } else if (MODE == LOAD_MASKED) {
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (!((amask >> (i * E + e)) & 1)) v[e] = T(0);
      }
      sm.As[buf][a_idx(row, kc)] = v;
    }
    if constexpr (nat_b<KB2>()) {
      if (MODE == LOAD_FULL && KB2 == OK_PLAIN && DMA_B) return;
#pragma unroll
      for (int i = 0; i < NBT; ++i) {
        const int q = tid + NT * i;
        if (NCH_B % NT != 0 && q >= NCH_B) break;
        chunk_t v;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          T x[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int j = 0; j < NQB; ++j) x[nth_quad(QB, j)] = rbk[i / E][i % E][j][e];
          v[e] = combine<KB2>(x);
        }
        if (MODE == LOAD_EDGE_VEC) {
          if (!((bmask >> i) & 1)) v = chunk_t{};
        } else if (MODE == LOAD_MASKED) {
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (!((bmask >> (i * E + e)) & 1)) v[e] = T(0);
        }
        sm.Bs[buf][q] = v;
      }
      return;
    }
    if constexpr (KB2 == OK_TRANS) {
      if (MODE == LOAD_FULL && DMA_B) return;
#pragma unroll
      for (int i = 0; i < NBT; ++i) {
        const int q = tid + NT * i;
        if (NCH_B % NT != 0 && q >= NCH_B) break;
        const int col = q / BKC, kc = q % BKC;
        chunk_t v = rbk[i / E][i % E][0];
        if (MODE == LOAD_EDGE_VEC) {
          if (!((bmask >> i) & 1)) v = chunk_t{};
        } else if (MODE == LOAD_MASKED) {
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (!((bmask >> (i * E + e)) & 1)) v[e] = T(0);
        }
        sm.Bs[buf][a_idx(col, kc)] = v;
      }
      return;
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
        for (int rr = 0; rr < E; ++rr) {
          T x[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int j = 0; j < NQB; ++j) x[nth_quad(QB, j)] = rbk[i][rr][j][c];
          bool ok = true;
          if (MODE == LOAD_EDGE_VEC) ok = (bmask >> (i * E + rr)) & 1;
          if (MODE == LOAD_MASKED) ok = (bmask >> ((i * E + rr) * E + c)) & 1;
          t[rr] = ok ? combine<KB2>(x) : T(0);
        }
        sm.Bs[buf][b_idx(cb * E + c, kc)] = t;
      }
    }
  }

  // MFMAs of k-blocks [KLO, KHI) of one LDS stage (a k-block is KG * E k
  // values).  The fragments of k-block j+1 are read into a second register
  // set while the MFMAs of k-block j run.
  template <int KLO, int KHI, bool BTL>
  static __device__ __forceinline__ void compute(const Smem& sm, int buf, Acc& acc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int g = lane / TM, t = lane % TM;
    if constexpr (NATF && !BTL) {
      // natural B: step s of k-block kb2 reads row (kb2 KG + g) E + s of the
      // stage, FN consecutive columns (the lane's column in each of its FN
      // tiles); the k pairing is that of the k-chunked A fragments
      typedef FVec<(NATF ? FN : 1)> FV;
      typedef typename FV::type bv_t;
      const float* Bf = reinterpret_cast<const float*>(&sm.Bs[buf][0]) + wn * WN + FN * t;
      chunk_t fa[2][FM];
      bv_t fb[2][E];
      auto read_frags = [&](int kb2, chunk_t (&xa)[FM], bv_t (&xb)[E]) {
        const int plane = kb2 * M::KG + g;
#pragma unroll
        for (int a = 0; a < FM; ++a) xa[a] = sm.As[buf][a_idx(wm * WM + a * TM + t, plane)];
#pragma unroll
        for (int s = 0; s < E; ++s) xb[s] = *reinterpret_cast<const bv_t*>(Bf + (plane * E + s) * BN);
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
            for (int b = 0; b < FN; ++b) acc[a][b] = M::mfma(fa[cur][a][s], FV::get(fb[cur][s], b), acc[a][b]);
      }
      return;
    }
    chunk_t fa[2][FM], fb[2][FN];
    auto read_frags = [&](int kb2, chunk_t (&xa)[FM], chunk_t (&xb)[FN]) {
      const int plane = kb2 * M::KG + g;
#pragma unroll
      for (int a = 0; a < FM; ++a) xa[a] = sm.As[buf][a_idx(wm * WM + a * TM + t, plane)];
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int col = wn * WN + b * TM + t;
        xb[b] = sm.Bs[buf][BTL ? a_idx(col, plane) : b_idx(col, plane)];
      }
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
  }

  // Interior tiles whose operands both load straight into LDS (plain A,
  // float32 B as it lies in memory).  Two LDS stages of BK k values.  An MFMA
  // step is one k value of every MFMA tile of the wave (FM x FN MFMAs); a
  // stage holds KB * E steps.  The fragments of step i+1 are read while the
  // MFMAs of step i run (two register sets, alternating with the step; A's
  // chunk covers the E steps of a k-block, B's read one step).  The loads of
  // stage t+1 are issued two per step during the first steps of stage t,
  // between MFMAs (issued together right after the barrier they held the
  // waves up at their issue); they go into the buffer freed by the barrier of
  // stage t-1.  The barrier that hands a stage over sits before the stage's
  // last step, once every wave holds that step's fragments and its own loads
  // of the next stage have landed; the next stage's first fragments are read
  // while the last MFMAs of this one run.  No wave waits for LDS with an
  // empty matrix pipeline.  The same MFMAs in the same order as the other
  // loops: the bits do not change.
  //
  // The loads are buffer loads (a resource over the stage's first element,
  // 32-bit per-lane byte offsets fixed for the whole loop): the compiler then
  // counts the fragment reads exactly (with the global form it waits for
  // every outstanding LDS read), and the per-stage address arithmetic is
  // scalar.  Row offsets must fit in 32 bits: leading dimensions below
  // kDirectLdMax.  The barrier is a bare s_barrier after an explicit wait.
  static constexpr int64_t kDirectLdMax = int64_t(1) << 21;
  static constexpr int DPA = BM * BKC / NT, DPB = BN * BKC / NT;  // loads per lane per stage
  // loads of the next stage issued per step: two measured best (one and
  // four lose 0.8 and 1.2 % in the loop at n = 8192)
  static constexpr int kLoadsPerStep = 2;
  // Whether operands of kinds KA, KB2 take this loop in interior tiles.
  template <int KA, int KB2>
  static constexpr bool direct_kind() {
    return KA == OK_PLAIN && KB2 == OK_PLAIN && NATF && DMA_A && DMA_B && KB % 2 == 0 && DPA + DPB < KB * E &&
           DPA * NT == BM * BKC && DPB * NT == BN * BKC;
  }
  static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const T* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, -1, 0x00020000);
  }
  static __device__ __forceinline__ __attribute__((address_space(3))) void* lds(const chunk_t* p) {
    return (__attribute__((address_space(3))) void*)(p);
  }
  static __device__ __forceinline__ void bare_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  }
  // rlast / clast: the last row of A and the last 16-byte column chunk of B
  // the tile may read (a tile at a matrix edge reads the rows and chunks
  // past them as copies of these; see product).
  // kvalid: k past which A's columns and B's rows are zero (a k that is not
  // a multiple of BK, but of E): the last two stages load through a checked
  // copy of the stage that skips the chunks past it and zeroes their LDS
  // slots instead (they lie past the operands, so they are never read).
  static __device__ __forceinline__ void main_loop_direct(Smem& sm, const Operand<T>& A, const Operand<T>& B,
                                                          int i0, int j0, int ktiles, Acc& acc,
                                                          int rlast = BM - 1, int clast = BN / E - 1,
                                                          int kvalid = 0x7fffffff) {
    static_assert(direct_kind<OK_PLAIN, OK_PLAIN>(),
                  "float32, whole loads per lane, even k-blocks per stage, a stage's loads spread over all but "
                  "its last step");
    constexpr int STEPS = KB * E;
    constexpr int CPR = BN / E;
    typedef FVec<FN> FV;
    typedef typename FV::type bv_t;
    // the wave index in a scalar register: the LDS destinations of the
    // direct loads (M0) are then computed without vector instructions
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / WGN, wn = wave % WGN;
    const int g = lane / TM, t = lane % TM;
    // byte offsets of this lane's chunks in a stage (A in a_idx order, B as
    // it lies in memory), from the stage's first element
    uint32_t oa[DPA], ob[DPB];
#pragma unroll
    for (int i = 0; i < DPA; ++i) {
      const int p = (wave * DPA + i) * 64 + lane;
      const int row = p / BKC, slot = p % BKC;
      const int kc = slot ^ ((row / (16 / BKC)) & (BKC - 1));
      oa[i] = (uint32_t)(((int64_t)min(row, rlast) * A.ld + kc * E) * (int64_t)sizeof(T));
    }
#pragma unroll
    for (int i = 0; i < DPB; ++i) {
      const int p = (wave * DPB + i) * 64 + lane;
      ob[i] = (uint32_t)(((int64_t)(p / CPR) * B.ld + min(p % CPR, clast) * E) * (int64_t)sizeof(T));
    }
    // load i (0 <= i < DPA + DPB: A's first) of this lane's share of stage
    // kt, into LDS buffer kt & 1
    auto load_part = [&](int kt, int i) {
      const int buf = kt & 1;
      if (i < DPA) {
        const __amdgpu_buffer_rsrc_t ra = rsrc(A.p + (int64_t)i0 * A.ld + (int64_t)kt * BK);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, lds(&sm.As[buf][(wave * DPA + i) * 64]), 16, oa[i], 0, 0, 0);
      } else {
        const int j = i - DPA;
        const __amdgpu_buffer_rsrc_t rb = rsrc(B.p + (int64_t)kt * BK * B.ld + j0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, lds(&sm.Bs[buf][(wave * DPB + j) * 64]), 16, ob[j], 0, 0, 0);
      }
    };
    // load_part, with the chunks at or past kvalid zeroed in LDS instead of
    // loaded
    auto load_part_checked = [&](int kt, int i) __attribute__((always_inline)) {
      const int buf = kt & 1;
      if (i < DPA) {
        const int p = (wave * DPA + i) * 64 + lane;
        const int row = p / BKC, slot = p % BKC;
        const int kc = slot ^ ((row / (16 / BKC)) & (BKC - 1));
        if (kt * BK + kc * E < kvalid) {
          const __amdgpu_buffer_rsrc_t ra = rsrc(A.p + (int64_t)i0 * A.ld + (int64_t)kt * BK);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, lds(&sm.As[buf][(wave * DPA + i) * 64]), 16, oa[i], 0, 0,
                                                   0);
        } else {
          sm.As[buf][p] = chunk_t{};
        }
      } else {
        const int j = i - DPA;
        const int p = (wave * DPB + j) * 64 + lane;
        if (kt * BK + p / CPR < kvalid) {
          const __amdgpu_buffer_rsrc_t rb = rsrc(B.p + (int64_t)kt * BK * B.ld + j0);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, lds(&sm.Bs[buf][(wave * DPB + j) * 64]), 16, ob[j], 0, 0,
                                                   0);
        } else {
          sm.Bs[buf][p] = chunk_t{};
        }
      }
    };
    chunk_t fa[2][FM];
    bv_t fb[2];
    auto read_a = [&](int buf, int kb2, chunk_t (&xa)[FM]) {
      const int plane = kb2 * M::KG + g;
#pragma unroll
      for (int a = 0; a < FM; ++a) xa[a] = sm.As[buf][a_idx(wm * WM + a * TM + t, plane)];
    };
    auto read_b = [&](int buf, int step, bv_t& xb) {
      const int plane = (step / E) * M::KG + g;
      const float* Bf = reinterpret_cast<const float*>(&sm.Bs[buf][0]) + wn * WN + FN * t;
      xb = *reinterpret_cast<const bv_t*>(Bf + (plane * E + step % E) * BN);
    };
#pragma unroll
    for (int i = 0; i < DPA + DPB; ++i) {
      if (ktiles == 1)
        load_part_checked(0, i);
      else
        load_part(0, i);
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's part of stage 0 has landed
    bare_barrier();
    read_a(0, 0, fa[0]);
    read_b(0, 0, fb[0]);
    // stage kt; CHECKED: its loads of stage kt+1 go through load_part_checked
    auto stage = [&](int kt, auto checked_tag) __attribute__((always_inline)) {
      constexpr bool CHECKED = decltype(checked_tag)::value;
      const int buf = kt & 1;
      const bool more = kt + 1 < ktiles;
#pragma unroll
      for (int step = 0; step < STEPS; ++step) {
        const int kb2 = step / E, s = step % E;
        const int ca = kb2 & 1, cb = step & 1;
        // MFMAs [m0, m1) of this step, in the order of the other loops
        auto mfmas = [&](int m0, int m1) {
#pragma unroll
          for (int m = m0; m < m1; ++m)
            acc[m / FN][m % FN] = M::mfma(fa[ca][m / FN][s], FV::get(fb[cb], m % FN), acc[m / FN][m % FN]);
        };
        if (step + 1 < STEPS) {
          if (s == E - 1) read_a(buf, kb2 + 1, fa[ca ^ 1]);
          read_b(buf, step + 1, fb[cb ^ 1]);
          __builtin_amdgcn_sched_barrier(0);
          if (step * kLoadsPerStep < DPA + DPB) {
            // kLoadsPerStep loads of stage kt+1 per step
            mfmas(0, (FM * FN) / 2);
            __builtin_amdgcn_sched_barrier(0);
            if (more) {
#pragma unroll
              for (int j = 0; j < kLoadsPerStep; ++j)
                if (step * kLoadsPerStep + j < DPA + DPB) {
                  if constexpr (CHECKED)
                    load_part_checked(kt + 1, step * kLoadsPerStep + j);
                  else
                    load_part(kt + 1, step * kLoadsPerStep + j);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            mfmas((FM * FN) / 2, FM * FN);
          } else {
            mfmas(0, FM * FN);
          }
        } else {
          // this step's fragments read, stage kt+1 landed (this wave's part)
          __builtin_amdgcn_s_waitcnt(0);
          bare_barrier();
          // half of the step's MFMAs first, so the matrix core has work while
          // the next stage's first fragments are read
          mfmas(0, (FM * FN) / 2);
          __builtin_amdgcn_sched_barrier(0);
          if (more) {
            read_a(buf ^ 1, 0, fa[ca ^ 1]);
            read_b(buf ^ 1, 0, fb[cb ^ 1]);
          }
          __builtin_amdgcn_sched_barrier(0);
          mfmas((FM * FN) / 2, FM * FN);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    typedef std::integral_constant<bool, false> plain_loads;
    typedef std::integral_constant<bool, true> checked_loads;
    int kt = 0;
    for (; kt + 2 < ktiles; ++kt) stage(kt, plain_loads{});
    for (; kt < ktiles; ++kt) stage(kt, checked_loads{});  // loads the last stage
    // Every wave read its last fragments before the last stage's barrier,
    // and no load is in flight: the LDS may be reused at once.
  }

  // Pipeline: the global loads of stage t+1 are issued first; the stage is
  // written to the other LDS buffer halfway through the MFMAs of stage t, so
  // the wait for those loads and the LDS writes overlap the second half of
  // the MFMAs; one barrier ends the stage.  Writing the other buffer is safe:
  // every wave finished reading it before the barrier that ended stage t-1,
  // and it is read again only after the barrier that ends stage t.  The loop
  // ends with a barrier, so the next product may reuse the LDS at once.
  template <int MODE, int KA, int KB2>
  static __device__ __forceinline__ void main_loop(Smem& sm, const Operand<T>& A, const Operand<T>& B, int i0,
                                                   int j0, int ktiles, Acc& acc) {
    if constexpr (MODE == LOAD_FULL && direct_kind<KA, KB2>()) {
      if (A.ld < kDirectLdMax && B.ld < kDirectLdMax) {
        main_loop_direct(sm, A, B, i0, j0, ktiles, acc);
        return;
      }
    }
    chunk_t ra[NA][popc4(kind_quads(KA))];
    chunk_t rbk[NB][E][popc4(kind_quads(KB2))];  // E rows (k) of E columns, per quadrant
    uint64_t amask = 0, bmask = 0;
    constexpr bool BTL = KB2 == OK_TRANS;
    constexpr bool DMA = MODE == LOAD_FULL && KA == OK_PLAIN && DMA_A;
    constexpr bool DMAB = MODE == LOAD_FULL && BTL && DMA_B;
    constexpr bool DMABN = MODE == LOAD_FULL && nat_b<KB2>() && KB2 == OK_PLAIN && DMA_B;
    if (DMA) dma_a(sm, 0, A, i0, 0);
    if (DMAB) dma_b(sm, 0, B, j0, 0);
    if (DMABN) dma_bn(sm, 0, B, j0, 0);
    load_tile<MODE, KA, KB2>(A, B, i0, j0, 0, ra, rbk, amask, bmask);
    store_tile<MODE, KA, KB2>(sm, 0, ra, rbk, amask, bmask);
    if (DMA || DMAB || DMABN) __builtin_amdgcn_s_waitcnt(0);  // the LDS writes of this wave's direct loads are done
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      const bool more = kt + 1 < ktiles;
      if (more) {
        if (DMA) dma_a(sm, buf ^ 1, A, i0, kt + 1);
        if (DMAB) dma_b(sm, buf ^ 1, B, j0, kt + 1);
        if (DMABN) dma_bn(sm, buf ^ 1, B, j0, kt + 1);
        load_tile<MODE, KA, KB2>(A, B, i0, j0, kt + 1, ra, rbk, amask, bmask);
      }
      compute<0, KMID, BTL>(sm, buf, acc);
      if (more) store_tile<MODE, KA, KB2>(sm, buf ^ 1, ra, rbk, amask, bmask);
      compute<KMID, KB, BTL>(sm, buf, acc);
      if (DMA || DMAB || DMABN) __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }

  // acc += A[i0 : i0 + BM, 0 : K] B[0 : K, j0 : j0 + BN] (A and B of kinds KA, KB2).
  // clamp_ok: the caller stores no output row past A's valid rows and no
  // output column past B's valid columns.  A tile at a matrix edge may then
  // take the direct loop, reading the rows of A and the column chunks of B
  // past the edge as copies of the last valid ones: an output depends only
  // on its own row of A and column of B, so the copies reach only outputs
  // that are not stored (B's valid width a multiple of E, so that no chunk
  // straddles the edge).
  template <int KA = OK_PLAIN, int KB2 = OK_PLAIN>
  static __device__ __forceinline__ void product(Smem& sm, const Operand<T>& A, const Operand<T>& B, int i0,
                                                 int j0, int K, Acc& acc, bool clamp_ok = false) {
    const int ktiles = (K + BK - 1) / BK;
    if (ktiles <= 0) return;
    // an operand with no valid element is zero: nothing to add (and the
    // loaders may then read its first element)
    if (A.vrows <= 0 || A.vcols <= 0 || B.vrows <= 0 || B.vcols <= 0) return;
    // extents of B along n and k (a transposed B holds n rows of k)
    constexpr bool BTL = KB2 == OK_TRANS;
    const int bn = BTL ? B.vrows : B.vcols, bk = BTL ? B.vcols : B.vrows;
    const bool interior = A.vec && B.vec && (i0 + BM <= A.vrows) && (j0 + BN <= bn) && (K % BK == 0) &&
                          (K <= A.vcols) && (K <= bk);
    const bool edge_vec = A.vec && B.vec && A.vrows > 0 && A.vcols > 0 && B.vrows > 0 && B.vcols > 0 &&
                          A.vcols % E == 0 && B.vcols % E == 0;
    // The direct loop also takes a k that is a multiple of E but not of BK
    // (the chunks past k zeroed in LDS, see main_loop_direct).
    if constexpr (direct_kind<KA, KB2>()) {
      const bool mn_in = (i0 + BM <= A.vrows) && (j0 + BN <= bn);
      if (!interior && (mn_in || (clamp_ok && i0 < A.vrows && j0 < bn && B.vcols % E == 0)) && A.vec && B.vec &&
          K % E == 0 && (K <= A.vcols) && (K <= bk) && A.ld < kDirectLdMax && B.ld < kDirectLdMax) {
        main_loop_direct(sm, A, B, i0, j0, ktiles, acc, min(BM, A.vrows - i0) - 1, min(BN, bn - j0) / E - 1, K);
        return;
      }
    }
    if (interior)
      main_loop<LOAD_FULL, KA, KB2>(sm, A, B, i0, j0, ktiles, acc);
    else if (edge_vec)
      main_loop<LOAD_EDGE_VEC, KA, KB2>(sm, A, B, i0, j0, ktiles, acc);
    else
      main_loop<LOAD_MASKED, KA, KB2>(sm, A, B, i0, j0, ktiles, acc);
  }
};

}  // namespace gemm_detail
}  // namespace mm
