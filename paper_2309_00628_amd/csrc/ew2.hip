// Two recursion levels of Section 2.3's pre- or post-additions in one pass
// (desc.h: Ew2Part).  At two levels of the grouped schedule the separate
// passes move every element of the upper level's sums and products through
// HBM twice (written by one pass, read by the next); here they stay in
// registers.  Per n x n float32 product at the top two levels the S/T side
// moves 3.5 n^2 elements instead of 5.5 n^2 (A read once; the upper sums
// written only where the lower level reads them plainly, and the lower
// sums), the U side 4.06 n^2 instead of 7.56 n^2 (the 49 lower products read
// once, C written once).
//
// One thread per position of the lower-level grid (a 16-byte chunk of each
// block, or one element when a part's views are not 16-byte aligned); the
// formulas and their order are those of the element-wise passes, so the
// results are bitwise the same.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "kernels.h"

namespace mm {

namespace {

constexpr int kThreads2 = 256;

template <typename T, int V>
struct VT {
  typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VT<T, 1> {
  typedef T type;
};

template <typename T>
__device__ __forceinline__ T* at(const KernelBases& kb, const MView& v, int64_t r, int64_t c) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<T*>(b) + v.off + r * v.ld + c;
}

template <typename T, int V>
__device__ __forceinline__ typename VT<T, V>::type ld(const T* p) {
  return *reinterpret_cast<const typename VT<T, V>::type*>(p);
}
template <typename T, int V>
__device__ __forceinline__ typename VT<T, V>::type ld_nt(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const typename VT<T, V>::type*>(p));
}
template <typename T, int V>
__device__ __forceinline__ void st(T* p, const typename VT<T, V>::type& x) {
  *reinterpret_cast<typename VT<T, V>::type*>(p) = x;
}

// EW2_S / EW2_T at position (r, c) of the lower-level grid.
template <typename T, int V, bool IS_S>
__device__ __forceinline__ void pass_st(const KernelBases& kb, const Ew2Part& P, int r, int c) {
  typedef typename VT<T, V>::type vt;
  const int R = P.rows, C = P.cols;
  // x[a][b]: the parent block at row a R + r, column b C + c (a = 2 qa + sa,
  // b = 2 qc + sc: sub-block (sa, sc) of the upper quadrant (qa, qc))
  vt x[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) x[a][b] = ld<T, V>(at<T>(kb, P.x, (int64_t)a * R + r, (int64_t)b * C + c));
  // the seven operands of the upper level's products at the four sub-blocks
  vt op[7][2][2];
#pragma unroll
  for (int sa = 0; sa < 2; ++sa)
#pragma unroll
    for (int sc = 0; sc < 2; ++sc) {
      const vt q11 = x[sa][sc], q12 = x[sa][2 + sc], q21 = x[2 + sa][sc], q22 = x[2 + sa][2 + sc];
      vt y[4];
      if (IS_S) {  // S1..S4 of A11 A12 A21 A22
        y[0] = q21 + q22;
        y[1] = y[0] - q11;
        y[2] = q11 - q21;
        y[3] = q12 - y[1];
        op[0][sa][sc] = q11;
        op[1][sa][sc] = q12;
        op[2][sa][sc] = y[3];
        op[3][sa][sc] = q22;
      } else {  // T1..T4 of B11 B12 B21 B22
        y[0] = q12 - q11;
        y[1] = q22 - y[0];
        y[2] = q22 - q12;
        y[3] = y[1] - q21;
        op[0][sa][sc] = q11;
        op[1][sa][sc] = q21;
        op[2][sa][sc] = q22;
        op[3][sa][sc] = y[3];
      }
      op[4][sa][sc] = y[0];
      op[5][sa][sc] = y[1];
      op[6][sa][sc] = y[2];
      // the sub-block the lower level never reads plainly is not stored
      const bool unread = IS_S ? (sa == 1 && sc == 0) : (sa == 0 && sc == 1);
      if (!unread) {
#pragma unroll
        for (int k = 0; k < 4; ++k) st<T, V>(at<T>(kb, P.top[k], (int64_t)sa * R + r, (int64_t)sc * C + c), y[k]);
      }
    }
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    const vt v11 = op[o][0][0], v12 = op[o][0][1], v21 = op[o][1][0], v22 = op[o][1][1];
    vt z[4];
    if (IS_S) {
      z[0] = v21 + v22;
      z[1] = z[0] - v11;
      z[2] = v11 - v21;
      z[3] = v12 - z[1];
    } else {
      z[0] = v12 - v11;
      z[1] = v22 - z[0];
      z[2] = v22 - v12;
      z[3] = z[1] - v21;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) st<T, V>(at<T>(kb, P.low[o][k], r, c), z[k]);
  }
}

// EW2_U at position (r, c) of the lower-level grid.
template <typename T, int V>
__device__ __forceinline__ void pass_u(const KernelBases& kb, const Ew2Part& P, int r, int c) {
  typedef typename VT<T, V>::type vt;
  const int R = P.rows, C = P.cols;
  // upper-level product q at its four sub-blocks, from its seven lower
  // products: U1 U5 U6 U7 (Section 2.3)
  auto product = [&](int q, vt (&pq)[2][2]) {
    vt p[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) p[i] = ld_nt<T, V>(at<T>(kb, P.low[q][i], r, c));
    const vt u1 = p[0] + p[1];
    const vt u2 = p[0] + p[5];
    const vt u3 = u2 + p[6];
    const vt u4 = u2 + p[4];
    pq[0][0] = u1;
    pq[0][1] = u4 + p[2];
    pq[1][0] = u3 - p[3];
    pq[1][1] = u3 + p[4];
  };
  auto put = [&](int k, const vt (&y)[2][2]) {
#pragma unroll
    for (int sa = 0; sa < 2; ++sa)
#pragma unroll
      for (int sc = 0; sc < 2; ++sc)
        st<T, V>(at<T>(kb, P.top[k], (int64_t)sa * R + r, (int64_t)sc * C + c), y[sa][sc]);
  };
  // the upper level's U in the order of the element-wise pass, consuming the
  // products one at a time: U1 = P1 + P2, U2 = P1 + P6, U3 = U2 + P7,
  // U4 = U2 + P5, U7 = U3 + P5, U5 = U4 + P3, U6 = U3 - P4
  vt p1[2][2], px[2][2], u2[2][2], u3[2][2], u4[2][2], y[2][2];
  product(0, p1);
  product(1, px);
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i / 2][i % 2] = p1[i / 2][i % 2] + px[i / 2][i % 2];
  put(0, y);
  product(5, px);
#pragma unroll
  for (int i = 0; i < 4; ++i) u2[i / 2][i % 2] = p1[i / 2][i % 2] + px[i / 2][i % 2];
  product(6, px);
#pragma unroll
  for (int i = 0; i < 4; ++i) u3[i / 2][i % 2] = u2[i / 2][i % 2] + px[i / 2][i % 2];
  product(4, px);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    u4[i / 2][i % 2] = u2[i / 2][i % 2] + px[i / 2][i % 2];
    y[i / 2][i % 2] = u3[i / 2][i % 2] + px[i / 2][i % 2];
  }
  put(3, y);
  product(2, px);
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i / 2][i % 2] = u4[i / 2][i % 2] + px[i / 2][i % 2];
  put(1, y);
  product(3, px);
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i / 2][i % 2] = u3[i / 2][i % 2] - px[i / 2][i % 2];
  put(2, y);
}

// Whether every view of a part allows 16-byte accesses at chunk positions.
template <typename T>
__device__ __forceinline__ bool part_vec(const KernelBases& kb, const Ew2Part& P) {
  constexpr int V = 16 / sizeof(T);
  auto good = [&](const MView& v) {
    return v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
  };
  bool ok = P.cols % V == 0;
  if (P.kind == EW2_U) {
    for (int q = 0; q < 7; ++q)
      for (int i = 0; i < 7; ++i) ok = ok && good(P.low[q][i]);
  } else {
    ok = ok && good(P.x);
    for (int o = 0; o < 7; ++o)
      for (int k = 0; k < 4; ++k) ok = ok && good(P.low[o][k]);
  }
  for (int k = 0; k < 4; ++k) ok = ok && good(P.top[k]);
  return ok;
}

template <typename T, int V>
__device__ __forceinline__ void run_part(const KernelBases& kb, const Ew2Part& P, int lb) {
  const int cpr = P.cols / V;
  const int64_t q = (int64_t)lb * kThreads2 + threadIdx.x;
  if (q >= (int64_t)P.rows * cpr) return;
  const int r = (int)(q / cpr), c = (int)(q - (int64_t)r * cpr) * V;
  if (P.kind == EW2_S)
    pass_st<T, V, true>(kb, P, r, c);
  else if (P.kind == EW2_T)
    pass_st<T, V, false>(kb, P, r, c);
  else
    pass_u<T, V>(kb, P, r, c);
}

// A part's blocks are counted for its 16-byte positions; with a view not
// 16-byte aligned each block covers V times as many single elements in V
// rounds.
template <typename T>
__global__ __launch_bounds__(kThreads2) void ew2_kernel(KernelBases kb, const Ew2Part* __restrict__ parts,
                                                        int nparts) {
  constexpr int V = 16 / sizeof(T);
  const int b = blockIdx.x;
  int lo = 0, hi = nparts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (parts[mid].blk_start <= b) lo = mid; else hi = mid - 1;
  }
  const Ew2Part& P = parts[lo];
  const int lb = b - P.blk_start;
  if (part_vec<T>(kb, P)) {
    run_part<T, V>(kb, P, lb);
  } else {
    for (int i = 0; i < V; ++i) run_part<T, 1>(kb, P, lb * V + i);
  }
}

}  // namespace

int ew2_blocks(int rows, int cols, int dtype) {
  const int V = dtype == DT_F64 ? 2 : 4;
  const int64_t pos = (int64_t)rows * ((cols + V - 1) / V);
  return (int)((pos + kThreads2 - 1) / kThreads2);
}

hipError_t launch_ew2(int dtype, const KernelBases& kb, const Ew2Part* dparts, int nparts, int blocks,
                      hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (dtype == DT_F64)
    hipLaunchKernelGGL(ew2_kernel<double>, dim3(blocks), dim3(kThreads2), 0, s, kb, dparts, nparts);
  else
    hipLaunchKernelGGL(ew2_kernel<float>, dim3(blocks), dim3(kThreads2), 0, s, kb, dparts, nparts);
  return hipGetLastError();
}

}  // namespace mm
