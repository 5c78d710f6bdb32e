// Unrolled base cases of the Strassen-Winograd recursion (the paper's
// win2x2, win4x4 and win8x8 of Section 3): each thread computes one small
// leaf product C = A B (order S = 1, 2, 4 or 8) in registers by the
// 22-operation form of Section 2.3, unrolled down to scalars (S = 4: two
// levels, the seven 2 x 2 products each unrolled once more; S = 8: three
// levels, 343 scalar products, held partly in scratch: the 8 x 8 case is for
// completeness and exactness, not speed).  The sums and products are taken in the order the grouped schedule
// uses level by level, so a plan whose leaves are of order S gives the same
// bits as the plan with log2(S) more levels and scalar leaves.
//
// Operand elements outside a view's valid extent read as zero; only the
// valid part of C is written.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "kernels.h"

// Every product and sum is rounded on its own, as the separate passes and
// MFMA tiles of the recursion round them: no multiply-add contraction.
#pragma clang fp contract(off)

namespace mm {

namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ T* ptr(const KernelBases& kb, const MView& v) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<T*>(b) + v.off;
}

// C = A B for S x S blocks held in registers.
template <typename T, int S>
struct Wino {
  static __device__ __forceinline__ void mul(const T (&a)[S][S], const T (&b)[S][S], T (&c)[S][S]) {
    constexpr int H = S / 2;
    T s1[H][H], s2[H][H], s3[H][H], s4[H][H], t1[H][H], t2[H][H], t3[H][H], t4[H][H];
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const T a11 = a[i][j], a12 = a[i][j + H], a21 = a[i + H][j], a22 = a[i + H][j + H];
        const T b11 = b[i][j], b12 = b[i][j + H], b21 = b[i + H][j], b22 = b[i + H][j + H];
        s1[i][j] = a21 + a22;
        s2[i][j] = s1[i][j] - a11;
        s3[i][j] = a11 - a21;
        s4[i][j] = a12 - s2[i][j];
        t1[i][j] = b12 - b11;
        t2[i][j] = b22 - t1[i][j];
        t3[i][j] = b22 - b12;
        t4[i][j] = t2[i][j] - b21;
      }
    T a11[H][H], a12[H][H], a22[H][H], b11[H][H], b21[H][H], b22[H][H];
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int j = 0; j < H; ++j) {
        a11[i][j] = a[i][j];
        a12[i][j] = a[i][j + H];
        a22[i][j] = a[i + H][j + H];
        b11[i][j] = b[i][j];
        b21[i][j] = b[i + H][j];
        b22[i][j] = b[i + H][j + H];
      }
    T p1[H][H], p2[H][H], p3[H][H], p4[H][H], p5[H][H], p6[H][H], p7[H][H];
    Wino<T, H>::mul(a11, b11, p1);
    Wino<T, H>::mul(a12, b21, p2);
    Wino<T, H>::mul(s4, b22, p3);
    Wino<T, H>::mul(a22, t4, p4);
    Wino<T, H>::mul(s1, t1, p5);
    Wino<T, H>::mul(s2, t2, p6);
    Wino<T, H>::mul(s3, t3, p7);
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const T u2 = p1[i][j] + p6[i][j];
        const T u3 = u2 + p7[i][j];
        c[i][j] = p1[i][j] + p2[i][j];
        c[i][j + H] = (u2 + p5[i][j]) + p3[i][j];
        c[i + H][j] = u3 - p4[i][j];
        c[i + H][j + H] = u3 + p5[i][j];
      }
  }
};

template <typename T>
struct Wino<T, 1> {
  static __device__ __forceinline__ void mul(const T (&a)[1][1], const T (&b)[1][1], T (&c)[1][1]) {
    c[0][0] = a[0][0] * b[0][0];
  }
};

template <typename T, int S>
__global__ __launch_bounds__(kThreads) void base_kernel(KernelBases kb, const BaseDesc* __restrict__ d, int count) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= count) return;
  const BaseDesc& D = d[i];
  const T* A = ptr<T>(kb, D.a);
  const T* B = ptr<T>(kb, D.b);
  T* C = ptr<T>(kb, D.c);
  T a[S][S], b[S][S], c[S][S];
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int q = 0; q < S; ++q) {
      a[r][q] = (r < D.a.vrows && q < D.a.vcols) ? A[(int64_t)r * D.a.ld + q] : T(0);
      b[r][q] = (r < D.b.vrows && q < D.b.vcols) ? B[(int64_t)r * D.b.ld + q] : T(0);
    }
  Wino<T, S>::mul(a, b, c);
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (r < D.c.vrows && q < D.c.vcols) C[(int64_t)r * D.c.ld + q] = c[r][q];
}

template <typename T>
hipError_t launch_t(int s, const KernelBases& kb, const BaseDesc* d, int count, int blocks, hipStream_t st) {
  switch (s) {
    case 1: hipLaunchKernelGGL((base_kernel<T, 1>), dim3(blocks), dim3(kThreads), 0, st, kb, d, count); break;
    case 2: hipLaunchKernelGGL((base_kernel<T, 2>), dim3(blocks), dim3(kThreads), 0, st, kb, d, count); break;
    case 8: hipLaunchKernelGGL((base_kernel<T, 8>), dim3(blocks), dim3(kThreads), 0, st, kb, d, count); break;
    default: hipLaunchKernelGGL((base_kernel<T, 4>), dim3(blocks), dim3(kThreads), 0, st, kb, d, count); break;
  }
  return hipGetLastError();
}

}  // namespace

int base_blocks(int count) { return count <= 0 ? 0 : (count + kThreads - 1) / kThreads; }

hipError_t launch_base(int dtype, int s, const KernelBases& kb, const BaseDesc* d, int count, int blocks,
                       hipStream_t st) {
  if (blocks <= 0) return hipSuccess;
  return dtype == DT_F64 ? launch_t<double>(s, kb, d, count, blocks, st) : launch_t<float>(s, kb, d, count, blocks, st);
}

}  // namespace mm
