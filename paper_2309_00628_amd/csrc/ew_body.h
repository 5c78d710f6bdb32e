// The element-wise block operations of the recursion levels: the
// pre-additions (S, T), post-additions (U, C) and copies.  They move data and
// do one add or subtract per output element, so they are bound by HBM
// bandwidth: every thread handles 16-byte chunks of each operand with one
// vector load or store (4 floats or 2 doubles), rows of a block map to
// consecutive threads, and all outputs of a fused step are produced from one
// read of its inputs.
//
// ew_block processes one block of kThreads * kItems chunks of one part with
// kThreads threads; the element-wise kernel (one block per workgroup) and
// the persistent batched kernel (several blocks per task) both run it.
#pragma once
#include <hip/hip_runtime.h>

#include "desc.h"

namespace mm {
namespace ew_detail {

constexpr int kThreads = 256;
constexpr int kItems = 2;  // chunks per thread
constexpr int kOut = 5;    // outputs of the element-wise recipes of this kernel
static_assert(kOut <= kEwMaxOut, "outputs");

template <typename T>
struct VecT;
template <>
struct VecT<float> {
  static constexpr int N = 4;
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct VecT<double> {
  static constexpr int N = 2;
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename T>
__device__ inline T* resolve(const KernelBases& kb, const MView& v) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<T*>(b) + v.off;
}

template <typename T, int V>
__device__ inline void load_chunk(const KernelBases& kb, const MView& v, int r, int c0, bool vec,
                                  T (&x)[V]) {
  if (r >= v.vrows || c0 >= v.vcols) {
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = T(0);
    return;
  }
  const T* p = resolve<T>(kb, v) + (int64_t)r * v.ld + c0;
  if (vec && c0 + V <= v.vcols) {
    typename VecT<T>::type t = *reinterpret_cast<const typename VecT<T>::type*>(p);
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = t[e];
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = (c0 + e < v.vcols) ? p[e] : T(0);
  }
}

template <typename T, int V>
__device__ inline void store_chunk(const KernelBases& kb, const MView& v, int r, int c0, bool vec,
                                   const T (&x)[V]) {
  if (r >= v.vrows || c0 >= v.vcols) return;
  T* p = resolve<T>(kb, v) + (int64_t)r * v.ld + c0;
  if (vec && c0 + V <= v.vcols) {
    typename VecT<T>::type t;
#pragma unroll
    for (int e = 0; e < V; ++e) t[e] = x[e];
    *reinterpret_cast<typename VecT<T>::type*>(p) = t;
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (c0 + e < v.vcols) p[e] = x[e];
  }
}

// Fast path of the Winograd passes (S / T / U of Section 2.3) and of
// Strassen's (Section 2.2) over blocks whose every input and output is
// entirely valid and 16-byte aligned: no bounds checks, and the loads of all
// of a thread's chunks are issued before its first store (the stores could
// otherwise alias later loads, which would serialise the chunks).  The arithmetic is that of the
// general path, in the same order.  Measured (n = 4096 and 8192): S/T
// passes at 5.2-5.5 TB/s (4.6-5.0 in the general path), U passes at
// 5.6-6.1 TB/s (4.6-5.1).
template <typename T, int KIND>
__device__ __forceinline__ void pass_fast(const KernelBases& kb, const EwPart& P, int64_t first, int64_t total,
                                          int cpr) {
  constexpr int V = VecT<T>::N;
  constexpr bool U = KIND == EW_WINO_U || KIND == EW_STR_U;
  constexpr int NIN = U ? 7 : 4;
  constexpr int NOUT = (KIND == EW_STR_S || KIND == EW_STR_T) ? 5 : 4;
  typedef typename VecT<T>::type vt;
  const T* ip[NIN];
  T* op[NOUT];
#pragma unroll
  for (int i = 0; i < NIN; ++i) ip[i] = resolve<T>(kb, P.in[i]);
#pragma unroll
  for (int o = 0; o < NOUT; ++o) op[o] = resolve<T>(kb, P.out[o]);
  vt x[kItems][NIN];
  int64_t at_in[kItems][NIN], at_out[kItems][NOUT];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t q = min(first + (int64_t)it * kThreads, total - 1);
    const int r = (int)(q / cpr);
    const int c0 = (int)(q - (int64_t)r * cpr) * V;
#pragma unroll
    for (int i = 0; i < NIN; ++i) at_in[it][i] = (int64_t)r * P.in[i].ld + c0;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) at_out[it][o] = (int64_t)r * P.out[o].ld + c0;
  }
  // The products are read once (nontemporal: measured 10-15 % faster U
  // passes); A and B quadrants are read again by the leaf products.
#pragma unroll
  for (int it = 0; it < kItems; ++it)
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
      const vt* src = reinterpret_cast<const vt*>(ip[i] + at_in[it][i]);
      x[it][i] = U ? __builtin_nontemporal_load(src) : *src;
    }
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    if (first + (int64_t)it * kThreads >= total) break;
    vt y[NOUT];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if (KIND == EW_WINO_S) {  // x = A11 A12 A21 A22
        const T s1 = x[it][2][e] + x[it][3][e];
        const T s2 = s1 - x[it][0][e];
        const T s3 = x[it][0][e] - x[it][2][e];
        const T s4 = x[it][1][e] - s2;
        y[0][e] = s1; y[1][e] = s2; y[2][e] = s3; y[3][e] = s4;
      } else if (KIND == EW_WINO_T) {  // x = B11 B12 B21 B22
        const T t1 = x[it][1][e] - x[it][0][e];
        const T t2 = x[it][3][e] - t1;
        const T t3 = x[it][3][e] - x[it][1][e];
        const T t4 = t2 - x[it][2][e];
        y[0][e] = t1; y[1][e] = t2; y[2][e] = t3; y[3][e] = t4;
      } else if (KIND == EW_STR_S) {  // x = A11 A12 A21 A22
        y[0][e] = x[it][0][e] + x[it][3][e];
        y[1][e] = x[it][2][e] + x[it][3][e];
        y[2][e] = x[it][0][e] + x[it][1][e];
        y[3][e] = x[it][2][e] - x[it][0][e];
        y[4][e] = x[it][1][e] - x[it][3][e];
      } else if (KIND == EW_STR_T) {  // x = B11 B12 B21 B22
        y[0][e] = x[it][0][e] + x[it][3][e];
        y[1][e] = x[it][1][e] - x[it][3][e];
        y[2][e] = x[it][2][e] - x[it][0][e];
        y[3][e] = x[it][0][e] + x[it][1][e];
        y[4][e] = x[it][2][e] + x[it][3][e];
      } else if (KIND == EW_STR_U) {  // x = P1..P7
        y[0][e] = ((x[it][0][e] + x[it][3][e]) - x[it][4][e]) + x[it][6][e];
        y[1][e] = x[it][2][e] + x[it][4][e];
        y[2][e] = x[it][1][e] + x[it][3][e];
        y[3][e] = ((x[it][0][e] + x[it][2][e]) - x[it][1][e]) + x[it][5][e];
      } else {  // x = P1..P7
        const T u1 = x[it][0][e] + x[it][1][e];
        const T u2 = x[it][0][e] + x[it][5][e];
        const T u3 = u2 + x[it][6][e];
        const T u4 = u2 + x[it][4][e];
        const T u5 = u4 + x[it][2][e];
        const T u6 = u3 - x[it][3][e];
        const T u7 = u3 + x[it][4][e];
        y[0][e] = u1; y[1][e] = u5; y[2][e] = u6; y[3][e] = u7;
      }
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) *reinterpret_cast<vt*>(op[o] + at_out[it][o]) = y[o];
  }
}

// Every input and output of part P covers its rows x cols entirely, in
// whole aligned 16-byte chunks.
template <typename T>
__device__ __forceinline__ bool part_full(const KernelBases& kb, const EwPart& P) {
  constexpr int V = VecT<T>::N;
  bool ok = P.cols % V == 0;
  auto good = [&](const MView& v) {
    return v.vrows >= P.rows && v.vcols >= P.cols && v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
  };
  for (int i = 0; i < P.nin; ++i) ok = ok && good(P.in[i]);
  for (int o = 0; o < P.nout; ++o) ok = ok && good(P.out[o]);
  return ok;
}

// Block lb (counted from the part's first block) of part P, processed by
// thread tid of kThreads.  No barrier inside.
template <typename T>
__device__ __forceinline__ void ew_block(const KernelBases& kb, const EwPart& P, int lb, int tid) {
  constexpr int V = VecT<T>::N;
  const int kind = P.kind, nout = P.nout;
  // with beta == 0 the old C (the trailing inputs of the accumulating
  // recipes) is not read
  const bool drop_c = kb.beta == 0.0 && (kind == EW_WINO_U_ACC || kind == EW_STR_U_ACC || kind == EW_AXPBY ||
                                         kind == EW_SUM_ACC);
  const int nin = drop_c ? (kind == EW_AXPBY ? 1 : (kind == EW_SUM_ACC ? P.mode[0] : 7)) : P.nin;
  const T beta = drop_c ? T(0) : T(kb.beta);
  bool vec = true;
  for (int i = 0; i < nin; ++i)
    vec = vec && (P.in[i].base == MB_NONE ||
                  (P.in[i].vec && (P.in[i].base == MB_ABS || ((kb.aligned >> P.in[i].base) & 1))));
  for (int o = 0; o < nout; ++o)
    vec = vec && P.out[o].vec && (P.out[o].base == MB_ABS || ((kb.aligned >> P.out[o].base) & 1));
  const int cpr = (P.cols + V - 1) / V;
  const int64_t total = (int64_t)P.rows * cpr;
  const int64_t first = (int64_t)lb * (kThreads * kItems) + tid;
  if ((kind == EW_WINO_S || kind == EW_WINO_T || kind == EW_WINO_U || kind == EW_STR_S || kind == EW_STR_T ||
       kind == EW_STR_U) &&
      first < total && part_full<T>(kb, P)) {
    switch (kind) {
      case EW_WINO_S: pass_fast<T, EW_WINO_S>(kb, P, first, total, cpr); break;
      case EW_WINO_T: pass_fast<T, EW_WINO_T>(kb, P, first, total, cpr); break;
      case EW_WINO_U: pass_fast<T, EW_WINO_U>(kb, P, first, total, cpr); break;
      case EW_STR_S: pass_fast<T, EW_STR_S>(kb, P, first, total, cpr); break;
      case EW_STR_T: pass_fast<T, EW_STR_T>(kb, P, first, total, cpr); break;
      default: pass_fast<T, EW_STR_U>(kb, P, first, total, cpr); break;
    }
    return;
  }

  for (int it = 0; it < kItems; ++it) {
    const int64_t q = first + (int64_t)it * kThreads;
    if (q >= total) break;
    const int r = (int)(q / cpr);
    const int c0 = (int)(q - (int64_t)r * cpr) * V;
    T x[kEwMaxIn][V];
    T y[kOut][V];
#pragma unroll
    for (int i = 0; i < kEwMaxIn; ++i) {
      if (i < nin)
        load_chunk<T, V>(kb, P.in[i], r, c0, vec, x[i]);
      else
#pragma unroll
        for (int e = 0; e < V; ++e) x[i][e] = T(0);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      switch (kind) {
        case EW_COPY: y[0][e] = x[0][e]; break;
        case EW_ADD: y[0][e] = x[0][e] + x[1][e]; break;
        case EW_SUB: y[0][e] = x[0][e] - x[1][e]; break;
        case EW_WINO_S: {  // x = A11 A12 A21 A22
          const T s1 = x[2][e] + x[3][e];
          const T s2 = s1 - x[0][e];
          const T s3 = x[0][e] - x[2][e];
          const T s4 = x[1][e] - s2;
          y[0][e] = s1; y[1][e] = s2; y[2][e] = s3; y[3][e] = s4;
          break;
        }
        case EW_WINO_T: {  // x = B11 B12 B21 B22
          const T t1 = x[1][e] - x[0][e];
          const T t2 = x[3][e] - t1;
          const T t3 = x[3][e] - x[1][e];
          const T t4 = t2 - x[2][e];
          y[0][e] = t1; y[1][e] = t2; y[2][e] = t3; y[3][e] = t4;
          break;
        }
        case EW_WINO_U: {  // x = P1..P7
          const T u1 = x[0][e] + x[1][e];
          const T u2 = x[0][e] + x[5][e];
          const T u3 = u2 + x[6][e];
          const T u4 = u2 + x[4][e];
          const T u5 = u4 + x[2][e];
          const T u6 = u3 - x[3][e];
          const T u7 = u3 + x[4][e];
          y[0][e] = u1; y[1][e] = u5; y[2][e] = u6; y[3][e] = u7;
          break;
        }
        case EW_TT_U: {  // x = X(P1) C11(P3) C12(P6) C21(P7) C22(P5)
          const T u2 = x[0][e] + x[2][e];
          const T u3 = u2 + x[3][e];
          const T u4 = u2 + x[4][e];
          const T u7 = u3 + x[4][e];
          const T u5 = u4 + x[1][e];
          y[0][e] = u5; y[1][e] = u3; y[2][e] = u7;
          break;
        }
        case EW_IP_A: {  // x = A11 A21 A22 ; y = S3 S1
          y[0][e] = x[0][e] - x[1][e];
          y[1][e] = x[1][e] + x[2][e];
          break;
        }
        case EW_IP_B: {  // x = B11 B12 B22 ; y = T1 T3
          y[0][e] = x[1][e] - x[0][e];
          y[1][e] = x[2][e] - x[1][e];
          break;
        }
        case EW_IP_U: {  // x = P1 P2 U2 P5 P7 P4 ; y = U1 U4 U6 U7
          const T u1 = x[0][e] + x[1][e];
          const T u4 = x[2][e] + x[3][e];
          const T u3 = x[2][e] + x[4][e];
          const T u6 = u3 - x[5][e];
          const T u7 = u3 + x[3][e];
          y[0][e] = u1; y[1][e] = u4; y[2][e] = u6; y[3][e] = u7;
          break;
        }
        case EW_WINO_U_ACC: {  // x = P1..P7 C11 C12 C21 C22
          const T u1 = x[0][e] + x[1][e];
          const T u2 = x[0][e] + x[5][e];
          const T u3 = u2 + x[6][e];
          const T u4 = u2 + x[4][e];
          const T u5 = u4 + x[2][e];
          const T u6 = u3 - x[3][e];
          const T u7 = u3 + x[4][e];
          y[0][e] = fma(beta, x[7][e], u1);
          y[1][e] = fma(beta, x[8][e], u5);
          y[2][e] = fma(beta, x[9][e], u6);
          y[3][e] = fma(beta, x[10][e], u7);
          break;
        }
        case EW_AXPBY: y[0][e] = fma(beta, x[1][e], x[0][e]); break;  // x = X C
        case EW_SUM:
        case EW_SUM_ACC: {  // x = X0 .. X(np-1) (C)
          const int np = P.mode[0];
          T s = x[0][e], c = T(0);
#pragma unroll
          for (int i = 1; i < kEwMaxIn; ++i) {
            if (i < np) s = s + x[i][e];
            if (i == np) c = x[i][e];
          }
          y[0][e] = kind == EW_SUM_ACC ? fma(beta, c, s) : s;
          break;
        }
        case EW_STR_S: {  // x = A11 A12 A21 A22
          y[0][e] = x[0][e] + x[3][e];
          y[1][e] = x[2][e] + x[3][e];
          y[2][e] = x[0][e] + x[1][e];
          y[3][e] = x[2][e] - x[0][e];
          y[4][e] = x[1][e] - x[3][e];
          break;
        }
        case EW_STR_T: {  // x = B11 B12 B21 B22
          y[0][e] = x[0][e] + x[3][e];
          y[1][e] = x[1][e] - x[3][e];
          y[2][e] = x[2][e] - x[0][e];
          y[3][e] = x[0][e] + x[1][e];
          y[4][e] = x[2][e] + x[3][e];
          break;
        }
        case EW_STR_U:
        case EW_STR_U_ACC: {  // x = P1..P7 (C11 C12 C21 C22)
          const T c11 = ((x[0][e] + x[3][e]) - x[4][e]) + x[6][e];
          const T c12 = x[2][e] + x[4][e];
          const T c21 = x[1][e] + x[3][e];
          const T c22 = ((x[0][e] + x[2][e]) - x[1][e]) + x[5][e];
          if (kind == EW_STR_U) {
            y[0][e] = c11; y[1][e] = c12; y[2][e] = c21; y[3][e] = c22;
          } else {
            y[0][e] = fma(beta, x[7][e], c11);
            y[1][e] = fma(beta, x[8][e], c12);
            y[2][e] = fma(beta, x[9][e], c21);
            y[3][e] = fma(beta, x[10][e], c22);
          }
          break;
        }
        case EW_DIST: {  // x = Z D0 D1
          for (int o = 0; o < 2; ++o) {
            const int md = P.mode[o];
            y[o][e] = md == 1 ? x[0][e] : (md == 2 ? x[1 + o][e] + x[0][e] : x[1 + o][e] - x[0][e]);
          }
          break;
        }
        default: y[0][e] = T(0); break;  // EW_ZERO
      }
    }
#pragma unroll
    for (int o = 0; o < kOut; ++o)
      if (o < nout) store_chunk<T, V>(kb, P.out[o], r, c0, vec, y[o]);
  }
}

}  // namespace ew_detail
}  // namespace mm
