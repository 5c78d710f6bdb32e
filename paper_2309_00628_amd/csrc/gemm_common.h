// Device helpers shared by the MFMA GEMM kernels: operand addressing, the
// problem / tile lookup of a grouped launch, LDS swizzles and the epilogue.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.h"

namespace mm {
namespace gemm_detail {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T* resolve(const KernelBases& kb, const MView& v) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<T*>(b) + v.off;
}

__device__ __forceinline__ bool view_vec(const KernelBases& kb, const MView& v) {
  return v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
}

// LDS swizzles (16-byte chunks).  gfx950's LDS serves a 128-bit access 16
// lanes per cycle (64 banks); the tile stores and the fragment reads of
// every instantiated tile shape touch 16 distinct bank groups per 16 lanes
// (tests/test_lds_layout.py checks every float32 and float64 tile shape;
// rocprofv3's SQ_LDS_BANK_CONFLICT reads 0 for these kernels):
// A: a store phase covers 16/BKC consecutive rows x BKC chunks; the row is
//    XOR-ed with kc ^ (row mod (16/BKC)) * BKC, a permutation within each
//    aligned group of 16 rows, so the 32 consecutive rows a fragment read
//    touches stay distinct.
// B (k-chunked, float64 and split-bfloat16): 8 consecutive lanes store
//    columns E*cb + c of 8 consecutive cb; the low bits are XOR-ed with a
//    function of column bits 3 and up, so each group of 8 (and 16) lanes
//    lands in distinct chunk slots, and reads of 32 consecutive columns
//    remain a permutation within aligned groups.  float32 B is staged as it
//    lies in memory (gemm_tile.h): its reads are contiguous runs.
template <int BKC>
__device__ __forceinline__ int swz_a(int row, int kc) {
  return row ^ ((kc ^ ((row % (16 / BKC)) * BKC)) & 15);
}
template <int E>
__device__ __forceinline__ int swz_b(int col) {
  if (E == 4) return col ^ (((col >> 3) ^ (col >> 5)) & 3);
  return col ^ (((col >> 3) ^ (col >> 4)) & 1);
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Workgroups are dealt to the 8 XCDs round-robin (b % 8).  Give each XCD a
  // contiguous range of tiles so that tiles sharing A rows / B columns share
  // that XCD's L2.
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// Quadrants read by each operand kind (bit q: quadrant q, order 11 12 21 22).
__host__ __device__ constexpr int kind_quads(int kind) {
  switch (kind) {
    case OK_S1: return 0b1100;  // A21 A22
    case OK_S2: return 0b1101;  // A11 A21 A22
    case OK_S3: return 0b0101;  // A11 A21
    case OK_S4: return 0b1111;
    case OK_T1: return 0b0011;  // B11 B12
    case OK_T2: return 0b1011;  // B11 B12 B22
    case OK_T3: return 0b1010;  // B12 B22
    case OK_T4: return 0b1111;
    default: return 0b0001;     // the view itself
  }
}
__host__ __device__ constexpr int popc4(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1); }
// The j-th quadrant (in order 11 12 21 22) of a quadrant mask.
__host__ __device__ constexpr int nth_quad(int mask, int j) {
  for (int q = 0; q < 4; ++q)
    if ((mask >> q) & 1) {
      if (j == 0) return q;
      --j;
    }
  return 0;
}

// The operand sum of kind KIND from the loaded quadrant values (indexed by
// quadrant, only the needed ones are read), in the order of Section 2.3.
template <int KIND, typename T>
__device__ __forceinline__ T combine(const T (&q)[4]) {
  if (KIND == OK_S1) return q[2] + q[3];
  if (KIND == OK_S2) return (q[2] + q[3]) - q[0];
  if (KIND == OK_S3) return q[0] - q[2];
  if (KIND == OK_S4) return q[1] - ((q[2] + q[3]) - q[0]);
  if (KIND == OK_T1) return q[1] - q[0];
  if (KIND == OK_T2) return q[3] - (q[1] - q[0]);
  if (KIND == OK_T3) return q[3] - q[1];
  if (KIND == OK_T4) return (q[3] - (q[1] - q[0])) - q[2];
  return q[0];
}

// N consecutive floats accessed as one vector (N = 1, 2, 4).
template <int N>
struct FVec {
  typedef float type __attribute__((ext_vector_type(N)));
  static __device__ __forceinline__ float get(const type& v, int i) { return v[i]; }
  static __device__ __forceinline__ void set(type& v, int i, float x) { v[i] = x; }
};
template <>
struct FVec<1> {
  typedef float type;
  static __device__ __forceinline__ float get(float v, int) { return v; }
  static __device__ __forceinline__ void set(float& v, int, float x) { v = x; }
};

// Store the N values x of one lane at p (N consecutive columns of one row,
// ncols of them inside the valid extent), out = x or fma(ds, d, x) with d
// read at q; vector accesses when vec (p, q 4N-byte aligned) and all N are valid.
template <int N>
__device__ __forceinline__ void store_group(float* p, const float* q, bool add, float ds, const float (&x)[N],
                                            int ncols, bool vec) {
  typedef FVec<N> FV;
  if (vec && ncols >= N) {
    typename FV::type v, d;
    if (add) d = *reinterpret_cast<const typename FV::type*>(q);
#pragma unroll
    for (int b = 0; b < N; ++b) FV::set(v, b, add ? fma(ds, FV::get(d, b), x[b]) : x[b]);
    *reinterpret_cast<typename FV::type*>(p) = v;
  } else {
#pragma unroll
    for (int b = 0; b < N; ++b)
      if (b < ncols) p[b] = add ? fma(ds, q[b], x[b]) : x[b];
  }
}

// Operand load modes of a tile's K loop (see the kernels).
enum LoadMode : int { LOAD_FULL = 0, LOAD_EDGE_VEC = 1, LOAD_MASKED = 2 };

struct TileRef {
  int desc;    // problem index in the launch
  int i0, j0;  // first row / column of the C tile
};

// Which problem of a grouped launch this workgroup serves, and which tile.
// Tiles of one problem are visited in groups of 8 tile-rows so that
// workgroups running at the same time share A rows and B columns.
// With remap == 0 (launches of unequal problems, sorted longest first) the
// hardware's round-robin spreads every run of 8 consecutive tiles over the
// 8 XCDs, which balances the XCDs and starts the longest tiles first.
// Tile lt (counted from the problem's first tile) of a problem with
// tiles_m x tiles_n tiles: groups of 8 tile-rows, column by column.
template <int BM, int BN>
__device__ __forceinline__ TileRef tile_in_problem(int desc, int lt, int tiles_m, int tiles_n) {
  constexpr int GROUP = 8;
  const int per_group = GROUP * tiles_n;
  const int gid = lt / per_group;
  const int first_m = gid * GROUP;
  const int gsz = min(tiles_m - first_m, GROUP);
  const int tm = first_m + (lt - gid * per_group) % gsz;
  const int tn = (lt - gid * per_group) / gsz;
  return TileRef{desc, tm * BM, tn * BN};
}

template <int BM, int BN, typename Desc>
__device__ __forceinline__ TileRef locate_tile(const Desc* __restrict__ descs, int ndesc, int remap) {
  const int rb = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_start <= rb) lo = mid; else hi = mid - 1;
  }
  const Desc& D = descs[lo];
  return tile_in_problem<BM, BN>(lo, rb - D.tile_start, D.tiles_m, D.tiles_n);
}

// Raw buffer stores of the epilogue's interior path: a resource over a
// base address (no range limit), a per-lane byte offset and a scalar one.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, -1, 0x00020000);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void buf_store(float x, __amdgpu_buffer_rsrc_t r, int v, int s) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 0);
}
__device__ __forceinline__ void buf_store(double x, __amdgpu_buffer_rsrc_t r, int v, int s) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, 0);
}

// N consecutive floats of one row at byte offsets (v, s) of rc: one vector
// store when the view allows 16-byte accesses (VEC).  A store of more than
// 8 bytes takes its whole offset in the vector register and a constant
// scalar offset: a vector instruction that overwrites the data registers
// of such a store right after it needs a wait state, which the compiler
// inserts for that form (and for global stores) but not when the scalar
// offset is a register, where gfx950 needs it as well (measured: the first
// dword of such stores was sometimes the overwritten value).
template <int N, bool VEC>
__device__ __forceinline__ void buf_store_group(__amdgpu_buffer_rsrc_t rc, int v, int s, const float (&x)[N]) {
  typedef FVec<N> FV;
  if constexpr (VEC && N == 4) {
    typename FV::type y;
#pragma unroll
    for (int b = 0; b < N; ++b) FV::set(y, b, x[b]);
    int vs = v + s;
    asm("" : "+v"(vs));  // (opaque: the compiler would move s back to the scalar offset)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, y), rc, vs, 0, 0);
  } else if constexpr (VEC && N == 2) {
    typename FV::type y;
#pragma unroll
    for (int b = 0; b < N; ++b) FV::set(y, b, x[b]);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, y), rc, v, s, 0);
  } else {
    // (the single stores may be merged into one wide store: the same
    // constant scalar offset)
    int vs = v + s;
    asm("" : "+v"(vs));
#pragma unroll
    for (int b = 0; b < N; ++b) buf_store(x[b], rc, vs + 4 * b, 0);
  }
}

// Epilogue: every output of the descriptor gets C = s * acc, C = D + s * acc
// or C = beta * D + s * acc at the positions this lane owns.  ROW(lane, r)
// gives the row (within an MFMA tile of edge TM) of accumulator register r;
// lane t of tile b holds column b TM + t of the wave's columns, or FN t + b
// with PERM (the interleaved columns of a tile loop that stages B as it lies
// in memory).  Every MFMA layout used puts register r of lane l on row
// ROW(l, 0) + ROW(0, r): a lane part and a part fixed at compile time.
template <typename T, int TM, int NACC, int FM, int FN, int WM, int WN, bool PERM = false, bool FAST = true,
          typename Acc, typename RowFn>
__device__ __forceinline__ void store_outputs(const KernelBases& kb, const GemmDesc& D, int i0, int j0,
                                              int wm, int wn, int lane, const Acc (&acc)[FM][FN],
                                              RowFn rowfn) {
  const int t = lane % TM;
  const int lr = rowfn(lane, 0);     // the lane's row in every MFMA tile, less ROW(0, r)
  const int lc = PERM ? FN * t : t;  // the lane's first column among the wave's
  // the wave's first row and column (uniform over the wave: in scalar
  // registers, so that the fast path's row addresses stay scalar)
  const int r0 = FAST ? __builtin_amdgcn_readfirstlane(i0 + wm * WM) : i0 + wm * WM;
  const int c0 = FAST ? __builtin_amdgcn_readfirstlane(j0 + wn * WN) : j0 + wn * WN;
  const int nout = D.nout;
  for (int o = 0; o < nout; ++o) {
    const MView cv = D.out[o].c;
    const MView dv = D.out[o].d;
    const int mode = D.out[o].mode;
    const T sg = T(D.out[o].sign);
    T* __restrict__ Cp = resolve<T>(kb, cv);
    const T beta = T(kb.beta);
    // d is read for GM_ADD, and for GM_AXPBY unless beta == 0
    const bool add = mode == GM_ADD || (mode == GM_AXPBY && kb.beta != 0.0);
    const T dscale = mode == GM_AXPBY ? beta : T(1);
    const T* Dp = add ? resolve<T>(kb, dv) : nullptr;
    const int64_t ldc = cv.ld, ldd = add ? dv.ld : 0;
    const int crows = cv.vrows, ccols = cv.vcols;
    const bool vec = PERM && view_vec(kb, cv) && (!add || view_vec(kb, dv));
    // Plain stores of a wave whose FM TM x FN TM outputs all lie inside C:
    // no per-element checks, and buffer stores over the wave's first
    // output with the lane's byte offset (computed once) and each row's
    // offset in a scalar register, so a store costs no vector address
    // arithmetic (the 64-bit row arithmetic of the checked loops below costs
    // more vector instructions than the stores themselves).  Offsets are
    // 32-bit: the leading dimension is bounded accordingly.  The same values
    // go to the same places as in the checked loops.  Tiles whose
    // accumulators take more than 128 registers per lane keep the checked
    // loops (there the extra registers of this path spill), as do callers
    // passing FAST = false.
    constexpr int64_t kMaxLd = (int64_t(1) << 31) / (FM * TM * (int64_t)sizeof(T));
    constexpr bool kFast = FAST && FM * FN * NACC * sizeof(T) / 4 <= 128;
    if (kFast && !add && r0 + FM * TM <= crows && c0 + FN * TM <= ccols && ldc < kMaxLd) {
      const __amdgpu_buffer_rsrc_t rc = buf_rsrc(Cp + (int64_t)r0 * ldc + c0);
      const int cl = (int)(((int64_t)lr * ldc + lc) * (int64_t)sizeof(T));
      auto rows = [&](auto vec_tag) __attribute__((always_inline)) {
        constexpr bool VEC = decltype(vec_tag)::value;
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int r = 0; r < NACC; ++r) {
            const int sc = (int)((a * TM + rowfn(0, r)) * ldc * (int64_t)sizeof(T));
            if constexpr (PERM) {
              float x[FN];
#pragma unroll
              for (int b = 0; b < FN; ++b) x[b] = sg * acc[a][b][r];
              buf_store_group<FN, VEC>(rc, cl, sc, x);
            } else {
#pragma unroll
              for (int b = 0; b < FN; ++b) buf_store(T(sg * acc[a][b][r]), rc, cl + b * TM * (int)sizeof(T), sc);
            }
          }
      };
      if (vec)
        rows(std::integral_constant<bool, true>{});
      else
        rows(std::integral_constant<bool, false>{});
      continue;
    }
    if constexpr (PERM) {
      // the lane's FN tiles hold FN consecutive columns of each row: one
      // vector store (and load of D) per row
      const int col0 = c0 + lc;
      if (col0 >= ccols) continue;
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int r = 0; r < NACC; ++r) {
          const int row = r0 + a * TM + rowfn(lane, r);
          if (row >= crows) continue;
          float x[FN];
#pragma unroll
          for (int b = 0; b < FN; ++b) x[b] = sg * acc[a][b][r];
          store_group<FN>(Cp + (int64_t)row * ldc + col0, add ? Dp + (int64_t)row * ldd + col0 : nullptr, add,
                          dscale, x, ccols - col0, vec);
        }
      continue;
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int col = c0 + b * TM + t;
        const int rbase = r0 + a * TM;
        T* cpt = Cp + (int64_t)rbase * ldc + col;
        const T* dpt = add ? Dp + (int64_t)rbase * ldd + col : nullptr;
#pragma unroll
        for (int r = 0; r < NACC; ++r) {
          const int rr = rowfn(lane, r);
          if (rbase + rr < crows && col < ccols) {
            const T v = sg * acc[a][b][r];
            // one rounding: the same as the element-wise accumulating recipes
            cpt[(int64_t)rr * ldc] = add ? fma(dscale, dpt[(int64_t)rr * ldd], v) : v;
          }
        }
      }
  }
}

}  // namespace gemm_detail
}  // namespace mm
