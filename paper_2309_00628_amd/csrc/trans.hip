// Transposing element-wise passes (float32): the outputs hold the transpose
// of what the element-wise recipe computes, so that a leaf product can stage
// its B operand in 16-byte chunks along k, exactly as it stages A (OK_TRANS).
//
// EW_WINO_T_TR forms T1..T4 of Section 2.3 from the four B quadrants of a
// last-level block (in the order of the element-wise T recipe: the same
// bits) and also writes B11, B21 and B22, the plain B operands of P1, P2
// and P3, transposed.
//
// A block covers 64 rows (k) x 64 columns (n) of the inputs, staged in LDS
// with one padding column (conflict-free reads down a column); a thread then
// produces 4 consecutive k of one column per pass, so the 16 lanes that share
// a column write 256 contiguous bytes of that output row with one 16-byte
// store each.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "kernels.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;  // rows (k) and columns (n) of a block
constexpr int kIn = 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float* fptr(const KernelBases& kb, const MView& v) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<float*>(b) + v.off;
}

__global__ __launch_bounds__(kThreads) void trans_kernel(KernelBases kb, const EwPart* __restrict__ parts,
                                                         int nparts) {
  __shared__ float sh[kIn][kTile][kTile + 1];
  const int b = blockIdx.x;
  int lo = 0, hi = nparts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (parts[mid].blk_start <= b) lo = mid; else hi = mid - 1;
  }
  const EwPart& P = parts[lo];
  const int tid = threadIdx.x;
  const int lb = b - P.blk_start;
  const int bpr = (P.cols + kTile - 1) / kTile;
  const int r0 = (lb / bpr) * kTile, c0 = (lb % bpr) * kTile;  // input orientation: rows k, columns n

  // stage: 64 x 64 of every input, zero outside its valid extent
#pragma unroll
  for (int i = 0; i < kIn; ++i) {
    const MView& v = P.in[i];
    const float* base = fptr(kb, v);
    const bool vec = v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
#pragma unroll
    for (int it = 0; it < (kTile * kTile / 4) / kThreads; ++it) {
      const int item = tid + it * kThreads;
      const int rr = item / (kTile / 4), cc = (item % (kTile / 4)) * 4;
      const int gr = r0 + rr, gc = c0 + cc;
      const float* p = base + (int64_t)gr * v.ld + gc;
      float t[4];
      if (gr < v.vrows && vec && gc + 4 <= v.vcols) {
        const f32x4 u = *reinterpret_cast<const f32x4*>(p);
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = u[e];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (gr < v.vrows && gc + e < v.vcols) ? p[e] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) sh[i][rr][cc + e] = t[e];
    }
  }
  __syncthreads();

  const int kq = tid % 16;  // 4 consecutive k: kq * 4 .. kq * 4 + 3
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int c = tid / 16 + 16 * g;  // column (n) of this pass
    const int orow = c0 + c;          // output row
    const int k = kq * 4;
    const int ocol = r0 + k;
    if (orow >= P.cols || ocol >= P.rows) continue;
    f32x4 y[kEwMaxOut];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float b11 = sh[0][k + e][c], b12 = sh[1][k + e][c], b21 = sh[2][k + e][c], b22 = sh[3][k + e][c];
      const float t1 = b12 - b11;
      const float t2 = b22 - t1;
      y[0][e] = t1;
      y[1][e] = t2;
      y[2][e] = b22 - b12;
      y[3][e] = t2 - b21;
      y[4][e] = b11;
      y[5][e] = b21;
      y[6][e] = b22;
    }
#pragma unroll
    for (int o = 0; o < kEwMaxOut; ++o) {
      if (o >= P.nout) break;
      const MView& v = P.out[o];  // a workspace block of P.cols x P.rows (transposed), 16-byte rows
      float* q = fptr(kb, v) + (int64_t)orow * v.ld + ocol;
      if (ocol + 4 <= v.cols) {
        *reinterpret_cast<f32x4*>(q) = y[o];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (ocol + e < v.cols) q[e] = y[o][e];
      }
    }
  }
}

}  // namespace

int trans_blocks(int rows, int cols) {
  if (rows <= 0 || cols <= 0) return 0;
  return ((rows + kTile - 1) / kTile) * ((cols + kTile - 1) / kTile);
}

hipError_t launch_trans(const KernelBases& kb, const EwPart* dparts, int nparts, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(trans_kernel, dim3(blocks), dim3(kThreads), 0, s, kb, dparts, nparts);
  return hipGetLastError();
}

}  // namespace mm
