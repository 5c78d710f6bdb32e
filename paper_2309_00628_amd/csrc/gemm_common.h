// Device helpers shared by the MFMA GEMM kernels: operand addressing, the
// problem / tile lookup of a grouped launch, LDS swizzles and the epilogue.
#pragma once
#include <hip/hip_runtime.h>

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

// LDS swizzles.  A: the 16 lanes of a store phase cover 16/BKC consecutive
// rows x BKC chunks; XOR-ing the row by (16/BKC) * kc spreads them over 16
// bank groups.  B: 16 lanes store columns E*cb + c for 16 consecutive cb;
// XOR-ing the low bits with (col / 16) mod E does the same.  Fragment reads
// (16 consecutive rows or columns of one chunk plane) stay conflict-free
// because both swizzles permute within aligned groups of 16.
template <int BKC>
__device__ __forceinline__ int swz_a(int row, int kc) { return row ^ ((16 / BKC) * kc); }
template <int E>
__device__ __forceinline__ int swz_b(int col) { return col ^ ((col >> 4) & (E - 1)); }

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Workgroups are dealt to the 8 XCDs round-robin (b % 8).  Give each XCD a
  // contiguous range of tiles so that tiles sharing A rows / B columns share
  // that XCD's L2.
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

struct TileRef {
  int desc;    // problem index in the launch
  int i0, j0;  // first row / column of the C tile
};

// Which problem of a grouped launch this workgroup serves, and which tile.
// Tiles of one problem are visited in groups of 8 tile-rows so that
// workgroups running at the same time share A rows and B columns.
template <int BM, int BN>
__device__ __forceinline__ TileRef locate_tile(const GemmDesc* __restrict__ descs, int ndesc) {
  const int rb = xcd_remap(blockIdx.x, gridDim.x);
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_start <= rb) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& D = descs[lo];
  const int lt = rb - D.tile_start;
  const int tiles_m = D.tiles_m, tiles_n = D.tiles_n;
  constexpr int GROUP = 8;
  const int per_group = GROUP * tiles_n;
  const int gid = lt / per_group;
  const int first_m = gid * GROUP;
  const int gsz = min(tiles_m - first_m, GROUP);
  const int tm = first_m + (lt - gid * per_group) % gsz;
  const int tn = (lt - gid * per_group) / gsz;
  return TileRef{lo, tm * BM, tn * BN};
}

// Epilogue: every output of the descriptor gets C = s * acc or
// C = D + s * acc at the positions this lane owns.  ROW(lane, r) gives the
// row (within an MFMA tile of edge TM) of accumulator register r.
template <typename T, int TM, int NACC, int FM, int FN, int WM, int WN, typename Acc, typename RowFn>
__device__ __forceinline__ void store_outputs(const KernelBases& kb, const GemmDesc& D, int i0, int j0,
                                              int wm, int wn, int lane, const Acc (&acc)[FM][FN],
                                              RowFn rowfn) {
  const int t = lane % TM;
  const int nout = D.nout;
  for (int o = 0; o < nout; ++o) {
    const MView cv = D.out[o].c;
    const MView dv = D.out[o].d;
    const int mode = D.out[o].mode;
    const T sg = T(D.out[o].sign);
    T* __restrict__ Cp = resolve<T>(kb, cv);
    const bool add = mode == GM_ADD;
    const T* Dp = add ? resolve<T>(kb, dv) : nullptr;
    const int64_t ldc = cv.ld, ldd = add ? dv.ld : 0;
    const int crows = cv.vrows, ccols = cv.vcols;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int col = j0 + wn * WN + b * TM + t;
        const int rbase = i0 + wm * WM + a * TM;
        T* cpt = Cp + (int64_t)rbase * ldc + col;
        const T* dpt = add ? Dp + (int64_t)rbase * ldd + col : nullptr;
#pragma unroll
        for (int r = 0; r < NACC; ++r) {
          const int rr = rowfn(lane, r);
          if (rbase + rr < crows && col < ccols) {
            const T v = sg * acc[a][b][r];
            cpt[(int64_t)rr * ldc] = add ? dpt[(int64_t)rr * ldd] + v : v;
          }
        }
      }
  }
}

}  // namespace gemm_detail
}  // namespace mm
