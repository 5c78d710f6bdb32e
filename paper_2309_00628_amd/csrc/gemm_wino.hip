// The last level of a Strassen-Winograd recursion in one launch: each
// workgroup computes one BM x BN tile of the four output quadrants of one
// subproblem by running the seven leaf products of Section 2.3 on that tile
// one after another (float32 MFMA, the K loop of gemm_tile.h) and forming
// the U combinations in registers:
//   U1 = P1 + P2 -> C11,  U2 = P1 + P6,  U3 = U2 + P7,  U4 = U2 + P5,
//   U5 = U4 + P3 -> C12,  U6 = U3 - P4 -> C21,  U7 = U3 + P5 -> C22.
// No product is written to memory, so the seven product stores and the
// separate U pass (seven reads and four writes of a quadrant) disappear.
// The products are ordered so that at most three tile accumulators are
// live; every sum is rounded in the order of the separate U pass, so the
// result has the same bits as the three-step path (products, then U).
//
// FUSED: the operands S1..S4 and T1..T4 are also formed in the tile loader
// from the quadrants of the subproblem's A and B blocks (gemm_tile.h), so
// the level runs with no temporaries at all: A and B are read, the four C
// quadrants written, nothing else touches memory.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "gemm_common.h"
#include "gemm_tile.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace gemm_detail;

// Operand kinds of P1 .. P7 when the sums are formed in the loader:
// P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
// P6 = S2 T2, P7 = S3 T3.
__host__ __device__ constexpr int wino_akind(int p) {
  return p == 2 ? OK_S4 : p == 4 ? OK_S1 : p == 5 ? OK_S2 : p == 6 ? OK_S3 : OK_PLAIN;
}
__host__ __device__ constexpr int wino_bkind(int p) {
  return p == 3 ? OK_T4 : p == 4 ? OK_T1 : p == 5 ? OK_T2 : p == 6 ? OK_T3 : OK_PLAIN;
}

template <int P>
using PIdx = std::integral_constant<int, P>;

template <int BM, int BN, int BKC, int WGM, int WGN, bool FUSED>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_wino_kernel(KernelBases kb,
                                                                   const WinoLeafDesc* __restrict__ descs,
                                                                   int ndesc, int remap) {
  typedef TileLoop<float, BM, BN, BKC, WGM, WGN> TL;
  typedef MT<float> M;
  typedef typename TL::Acc Acc;
  constexpr int FM = TL::FM, FN = TL::FN, TM = TL::TM;
  __shared__ typename TL::Smem sm;

  const TileRef tr = locate_tile<BM, BN>(descs, ndesc, remap);
  const WinoLeafDesc& D = descs[tr.desc];
  const int i0 = tr.i0, j0 = tr.j0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  // a[p], b[p]: the operands of P(p+1); with FUSED, the parent block for a sum
  auto prod = [&](auto ptag, Acc& acc) {
    constexpr int p = decltype(ptag)::value;
    constexpr int ka = FUSED ? wino_akind(p) : OK_PLAIN;
    constexpr int kb2 = FUSED ? wino_bkind(p) : OK_PLAIN;
    TL::zero(acc);
    const Operand<float> A =
        ka == OK_PLAIN ? operand<float>(kb, D.a[p]) : operand_sum<float>(kb, D.a[p], D.m, D.k);
    const Operand<float> B =
        kb2 == OK_PLAIN ? operand<float>(kb, D.b[p]) : operand_sum<float>(kb, D.b[p], D.k, D.n);
    TL::template product<ka, kb2>(sm, A, B, i0, j0, D.k, acc);
  };
  // v(a, b) gives the 16 values of MFMA tile (a, b) this lane stores; an
  // accumulating top level stores fma(beta, Cold, v) instead.
  const bool accum = D.acc && kb.beta != 0.0;
  const float beta = (float)kb.beta;
  // (the lane's FN tiles hold FN consecutive columns of each row: one vector
  // access per row)
  auto store = [&](const MView& cv, auto v) {
    float* __restrict__ Cp = resolve<float>(kb, cv);
    const int t = lane % TM;
    const int col0 = j0 + TL::template out_col<false>(wn, 0, t);
    if (col0 >= cv.vcols) return;
    const bool vec = view_vec(kb, cv);
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      typename M::acc_t x[FN];
#pragma unroll
      for (int b = 0; b < FN; ++b) x[b] = v(a, b);
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) {
        const int row = i0 + wm * TL::WM + a * TM + M::row(lane, r);
        if (row >= cv.vrows) continue;
        float y[FN];
#pragma unroll
        for (int b = 0; b < FN; ++b) y[b] = x[b][r];
        float* p = Cp + (int64_t)row * cv.ld + col0;
        store_group<FN>(p, p, accum, beta, y, cv.vcols - col0, vec);
      }
    }
  };
  auto add_to = [](Acc& x, const Acc& y) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) x[a][b] = x[a][b] + y[a][b];
  };

  Acc X, Y, Z;
  prod(PIdx<0>{}, X);                                            // P1
  prod(PIdx<1>{}, Y);                                            // P2
  store(D.c[0], [&](int a, int b) { return X[a][b] + Y[a][b]; });  // C11 = U1
  prod(PIdx<5>{}, Y);                                            // P6
  add_to(X, Y);                                                  // X = U2
  prod(PIdx<6>{}, Y);                                            // P7
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) Y[a][b] = X[a][b] + Y[a][b];    // Y = U3
  prod(PIdx<4>{}, Z);                                            // P5
  store(D.c[3], [&](int a, int b) { return Y[a][b] + Z[a][b]; });  // C22 = U7
  add_to(X, Z);                                                  // X = U4
  prod(PIdx<2>{}, Z);                                            // P3
  add_to(X, Z);                                                  // X = U5
  store(D.c[1], [&](int a, int b) { return X[a][b]; });          // C12
  prod(PIdx<3>{}, Z);                                            // P4
  store(D.c[2], [&](int a, int b) { return Y[a][b] - Z[a][b]; });  // C21 = U6
}

template <int BM, int BN, int BKC, int WGM, int WGN>
hipError_t launch_cfg(int fused, const KernelBases& kb, const WinoLeafDesc* d, int n, int tiles, int remap,
                      hipStream_t s) {
  if (fused)
    hipLaunchKernelGGL((gemm_wino_kernel<BM, BN, BKC, WGM, WGN, true>), dim3(tiles), dim3(64 * WGM * WGN), 0, s,
                       kb, d, n, remap);
  else
    hipLaunchKernelGGL((gemm_wino_kernel<BM, BN, BKC, WGM, WGN, false>), dim3(tiles), dim3(64 * WGM * WGN), 0, s,
                       kb, d, n, remap);
  return hipGetLastError();
}

}  // namespace

GemmCfg gemm_wino_cfg(int cfg) {
  switch (cfg) {
    case 2: return {64, 128};
    default: return {128, 128};
  }
}

hipError_t launch_gemm_wino(int cfg, int fused, const KernelBases& kb, const WinoLeafDesc* d, int n, int tiles,
                            int remap, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  switch (cfg) {
    case 1: return launch_cfg<128, 128, 8, 4, 2>(fused, kb, d, n, tiles, remap, s);
    case 2: return launch_cfg<64, 128, 8, 2, 2>(fused, kb, d, n, tiles, remap, s);
    default: return launch_cfg<128, 128, 8, 2, 2>(fused, kb, d, n, tiles, remap, s);
  }
}

}  // namespace mm
