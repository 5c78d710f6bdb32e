// Split passes of the refined split-bfloat16 leaves: float32 blocks in, the
// split bfloat16 layout (hi, lo, res per element; see desc.h) out.  Each
// element is split exactly once here, in a pass that is bound by HBM
// bandwidth, instead of once per tile that stages it inside the leaf
// kernel (which repeats the split for every tile row or column that reads
// the element).
//
// Recipes: EW_SPLIT copies one block; EW_WINO_S_SPL forms S1..S4 of
// Section 2.3 from the four A quadrants of a last-level subproblem and also
// splits A11, A12 and A22 (the operands of P1, P2 and P4); EW_WINO_T_SPL does
// the same for T1..T4 and B11, B21, B22 (P1, P2, P3), storing every output
// transposed so that the leaf kernel reads B as columns of 8 consecutive k.
// The sums are rounded in float32 in the order of the element-wise S/T
// recipes.
//
// Non-transposed parts: a block covers 64 rows x 64 columns; a thread reads 8
// consecutive floats of a row from each input and writes one 48-byte chunk
// per output.  Transposed parts: a block stages 32 rows x 64 columns of each
// input in LDS and a thread then gathers 8 consecutive rows of one column.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "kernels.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kRowsN = 64, kColsN = 64;  // non-transposed block: 64 x 64 (8 chunks per row)
constexpr int kRowsT = 32, kColsT = 64;  // transposed block (input orientation)
constexpr int kIn = 4;                   // inputs of the split recipes

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// hi = bf16(x), lo = bf16(x - hi), res = bf16(x - hi - lo), the residual
// formed in float64 (both differences are exact, so float32 would give the
// same bits; here the arithmetic is free next to the memory traffic).
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo, bf16x8& rs) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    const float hf = (float)h;
    const __bf16 l = (__bf16)(x[e] - hf);
    const double r = ((double)x[e] - (double)hf) - (double)(float)l;
    hi[e] = h;
    lo[e] = l;
    rs[e] = (__bf16)(float)r;
  }
}

__device__ __forceinline__ float* fptr(const KernelBases& kb, const MView& v) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<float*>(b) + v.off;
}
__device__ __forceinline__ bf16x8* sptr(const KernelBases& kb, const MView& v, int64_t r, int q) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<bf16x8*>(reinterpret_cast<__bf16*>(b) + v.off + r * v.ld + 24 * (int64_t)q);
}

// The outputs of a recipe at one element from its inputs x[0..nin).
__device__ __forceinline__ int recipe(int kind, const float (&x)[kIn], float (&y)[kEwMaxOut]) {
  switch (kind) {
    case EW_WINO_S_SPL: {  // x = A11 A12 A21 A22
      const float s1 = x[2] + x[3];
      const float s2 = s1 - x[0];
      const float s3 = x[0] - x[2];
      const float s4 = x[1] - s2;
      y[0] = s1; y[1] = s2; y[2] = s3; y[3] = s4; y[4] = x[0]; y[5] = x[1]; y[6] = x[3];
      return 7;
    }
    case EW_WINO_T_SPL: {  // x = B11 B12 B21 B22
      const float t1 = x[1] - x[0];
      const float t2 = x[3] - t1;
      const float t3 = x[3] - x[1];
      const float t4 = t2 - x[2];
      y[0] = t1; y[1] = t2; y[2] = t3; y[3] = t4; y[4] = x[0]; y[5] = x[2]; y[6] = x[3];
      return 7;
    }
    default:  // EW_SPLIT
      y[0] = x[0];
      return 1;
  }
}

// Split the 8 values of each output and store them as chunk (row, q) of the
// output's SPL matrix when that chunk lies inside it.
__device__ __forceinline__ void emit(const KernelBases& kb, const EwPart& P, int row, int q,
                                     const float (&y)[kEwMaxOut][8]) {
#pragma unroll
  for (int o = 0; o < kEwMaxOut; ++o) {
    if (o >= P.nout) break;
    const MView& v = P.out[o];
    if (row >= v.rows || 8 * q >= v.cols) continue;
    bf16x8 h, l, r;
    split8(y[o], h, l, r);
    bf16x8* p = sptr(kb, v, row, q);
    p[0] = h;
    p[1] = l;
    p[2] = r;
  }
}

__global__ __launch_bounds__(kThreads) void split_kernel(KernelBases kb, const EwPart* __restrict__ parts,
                                                         int nparts) {
  __shared__ float sh[kIn][kRowsT][kColsT + 1];
  const int b = blockIdx.x;
  int lo = 0, hi = nparts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (parts[mid].blk_start <= b) lo = mid; else hi = mid - 1;
  }
  const EwPart& P = parts[lo];
  const int nin = P.nin;
  const int tid = threadIdx.x;
  const int lb = b - P.blk_start;

  if (P.mode[0] == 0) {
    const int nqb = (P.cols + 7) / 8;                // chunks per row
    const int bpr = (nqb + 7) / 8;                   // blocks per row band
    const int r0 = (lb / bpr) * kRowsN, q0 = (lb % bpr) * 8;
#pragma unroll
    for (int it = 0; it < (kRowsN * 8) / kThreads; ++it) {
      const int item = tid + it * kThreads;
      const int row = r0 + item / 8, q = q0 + item % 8;
      if (row >= P.rows || q >= nqb) continue;
      float x[kIn][8];
#pragma unroll
      for (int i = 0; i < kIn; ++i) {
        if (i >= nin) break;
        const MView& v = P.in[i];
        const int c0 = 8 * q;
        const float* p = fptr(kb, v) + (int64_t)row * v.ld + c0;
        const bool vec = v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
        if (row < v.vrows && vec && c0 + 8 <= v.vcols) {
          const f32x4 u = *reinterpret_cast<const f32x4*>(p);
          const f32x4 w = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            x[i][e] = u[e];
            x[i][4 + e] = w[e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) x[i][e] = (row < v.vrows && c0 + e < v.vcols) ? p[e] : 0.f;
        }
      }
      float y[kEwMaxOut][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float xe[kIn], ye[kEwMaxOut];
#pragma unroll
        for (int i = 0; i < kIn; ++i) xe[i] = i < nin ? x[i][e] : 0.f;
        recipe(P.kind, xe, ye);
#pragma unroll
        for (int o = 0; o < kEwMaxOut; ++o) y[o][e] = ye[o];
      }
      emit(kb, P, row, q, y);
    }
    return;
  }

  // Transposed: stage rows [r0, r0 + 32) x columns [c0, c0 + 64) of each
  // input, then each thread gathers 8 rows of one column.
  const int bpr = (P.cols + kColsT - 1) / kColsT;
  const int r0 = (lb / bpr) * kRowsT, c0 = (lb % bpr) * kColsT;
#pragma unroll
  for (int i = 0; i < kIn; ++i) {
    if (i >= nin) break;
    const MView& v = P.in[i];
    const float* base = fptr(kb, v);
    const bool vec = v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
#pragma unroll
    for (int it = 0; it < (kRowsT * kColsT / 4) / kThreads; ++it) {
      const int item = tid + it * kThreads;
      const int rr = item / (kColsT / 4), cc = (item % (kColsT / 4)) * 4;
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
  const int c = tid % kColsT, ql = tid / kColsT;  // column, chunk of 8 rows in the block
  const int col = c0 + c;
  if (col >= P.cols || r0 + 8 * ql >= P.rows) return;
  float y[kEwMaxOut][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float xe[kIn], ye[kEwMaxOut];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xe[i] = i < nin ? sh[i][8 * ql + e][c] : 0.f;
    recipe(P.kind, xe, ye);
#pragma unroll
    for (int o = 0; o < kEwMaxOut; ++o) y[o][e] = ye[o];
  }
  emit(kb, P, col, r0 / 8 + ql, y);
}

}  // namespace

int split_blocks(int rows, int cols, int transposed) {
  if (rows <= 0 || cols <= 0) return 0;
  if (transposed) return ((rows + kRowsT - 1) / kRowsT) * ((cols + kColsT - 1) / kColsT);
  const int nq = (cols + 7) / 8;
  return ((rows + kRowsN - 1) / kRowsN) * ((nq + 7) / 8);
}

hipError_t launch_split(const KernelBases& kb, const EwPart* dparts, int nparts, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_kernel, dim3(blocks), dim3(kThreads), 0, s, kb, dparts, nparts);
  return hipGetLastError();
}

}  // namespace mm
