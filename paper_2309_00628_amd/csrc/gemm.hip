// Leaf products: the naive method (Section 2.1) as a tiled MFMA GEMM for
// gfx950, in float32 (v_mfma_f32_32x32x2_f32) and float64
// (v_mfma_f64_16x16x4_f64).  The same kernel is mm_naive on a whole problem and
// the base case of every Strassen / Winograd recursion, and one launch can run
// a group of independent products (the seven products of a level, or many
// problems of a batch), so small leaves still fill the 256 compute units.
//
// Each workgroup computes one BM x BN tile of one problem with the
// double-buffered LDS K loop of gemm_tile.h (several tile configurations are
// instantiated; the planner picks one per launch).  Stores outside the
// output's valid extent are dropped.
//
// Epilogue per output: C = s * acc or C = D + s * acc (s = +1 or -1).  The
// accumulator holds the product rounded exactly as it would be stored, so
// folding a following block addition into the epilogue gives the same bits
// as storing the product and adding it in a separate step.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "gemm_common.h"
#include "gemm_tile.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace gemm_detail;

// BT: every problem's B view holds B transposed (OK_TRANS).
template <typename T, int BM, int BN, int BKC, int WGM, int WGN, bool BT>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_kernel(KernelBases kb,
                                                              const GemmDesc* __restrict__ descs,
                                                              int ndesc, int remap) {
  typedef TileLoop<T, BM, BN, BKC, WGM, WGN> TL;
  typedef MT<T> M;
  __shared__ typename TL::Smem sm;

  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const GemmDesc& D = descs[tr.desc];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  typename TL::Acc acc;
  TL::zero(acc);
  // edge tiles may read past the operands' valid extents when no output
  // stores there (TileLoop::product)
  bool clamp_ok = !BT;
  for (int o = 0; o < D.nout; ++o)
    clamp_ok = clamp_ok && D.out[o].c.vrows <= D.a.vrows && D.out[o].c.vcols <= D.b.vcols;
  TL::template product<OK_PLAIN, BT ? OK_TRANS : OK_PLAIN>(sm, operand<T>(kb, D.a), operand<T>(kb, D.b), tr.i0,
                                                         tr.j0, D.k, acc, clamp_ok);

  // (the epilogue's interior path costs the smaller tiles a wave per SIMD)
  store_outputs<T, TL::TM, M::NACC, TL::FM, TL::FN, TL::WM, TL::WN, TL::NATF && !BT, (BM >= 128 && BN >= 128)>(
      kb, D, tr.i0, tr.j0, wave / WGN, wave % WGN, lane, acc, [](int l, int r) { return M::row(l, r); });
}

template <typename T, int BM, int BN, int BKC, int WGM, int WGN, bool BT = false>
hipError_t launch_cfg(const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap, hipStream_t s) {
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BKC, WGM, WGN, BT>), dim3(tiles), dim3(64 * WGM * WGN), 0, s, kb,
                     d, n, remap);
  return hipGetLastError();
}

// float32 with B transposed in memory
hipError_t launch_f32_bt(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap,
                         hipStream_t s) {
  switch (cfg) {
    case 1: return launch_cfg<float, 256, 128, 8, 4, 2, true>(kb, d, n, tiles, remap, s);
    case 2: return launch_cfg<float, 128, 256, 8, 2, 4, true>(kb, d, n, tiles, remap, s);
    case 3: return launch_cfg<float, 256, 256, 8, 4, 2, true>(kb, d, n, tiles, remap, s);
    case 4: return launch_cfg<float, 64, 128, 8, 2, 2, true>(kb, d, n, tiles, remap, s);
    case 5: return launch_cfg<float, 128, 64, 8, 2, 2, true>(kb, d, n, tiles, remap, s);
    case 6: return launch_cfg<float, 256, 128, 4, 2, 2, true>(kb, d, n, tiles, remap, s);
    case 7: return launch_cfg<float, 128, 128, 4, 2, 2, true>(kb, d, n, tiles, remap, s);
    case 8: return launch_cfg<float, 64, 64, 8, 2, 2, true>(kb, d, n, tiles, remap, s);
    default: return launch_cfg<float, 128, 128, 8, 4, 2, true>(kb, d, n, tiles, remap, s);
  }
}

}  // namespace

GemmCfg gemm_cfg(int dtype, int cfg) {
  if (dtype == DT_BF16X3) return gemm_bf16x3_cfg(cfg);
  if (dtype == DT_BF16X3_SPL) return gemm_bf16s_cfg(cfg);
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
    case 8: return {64, 64};
    default: return {128, 128};
  }
}

hipError_t launch_gemm(int dtype, int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles,
                       int remap, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  if (dtype == DT_BF16X3) return launch_gemm_bf16x3(cfg, kb, d, n, tiles, remap, s);
  if (dtype == DT_BF16X3_SPL) return launch_gemm_bf16s(cfg, kb, d, n, tiles, remap, s);
  if (dtype == DT_F32_BT) return launch_f32_bt(cfg, kb, d, n, tiles, remap, s);
  if (dtype == DT_F64) {
    switch (cfg) {
      case 5: return launch_cfg<double, 128, 64, 8, 2, 2>(kb, d, n, tiles, remap, s);
      default: return launch_cfg<double, 128, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
    }
  }
  switch (cfg) {
    case 1: return launch_cfg<float, 256, 128, 8, 4, 2>(kb, d, n, tiles, remap, s);
    case 2: return launch_cfg<float, 128, 256, 8, 2, 4>(kb, d, n, tiles, remap, s);
    // 256x256 with eight waves (two per SIMD, each 64x128): while one wave
    // of a SIMD waits for memory the other keeps the matrix core busy
    case 3: return launch_cfg<float, 256, 256, 8, 4, 2>(kb, d, n, tiles, remap, s);
    case 4: return launch_cfg<float, 64, 128, 8, 2, 2>(kb, d, n, tiles, remap, s);
    case 5: return launch_cfg<float, 128, 64, 8, 2, 2>(kb, d, n, tiles, remap, s);
    case 6: return launch_cfg<float, 256, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
    case 7: return launch_cfg<float, 128, 128, 4, 2, 2>(kb, d, n, tiles, remap, s);
    // 64x64 with four waves (each 32x32): products too small to give the
    // larger tiles a workgroup per compute unit
    case 8: return launch_cfg<float, 64, 64, 8, 2, 2>(kb, d, n, tiles, remap, s);

    default: return launch_cfg<float, 128, 128, 8, 4, 2>(kb, d, n, tiles, remap, s);
  }
}

}  // namespace mm
