// Leaf products: the naive method (Section 2.1) as a tiled MFMA GEMM for
// gfx950, in float32 (v_mfma_f32_32x32x2_f32) and float64
// (v_mfma_f64_16x16x4_f64).  The same kernel is mm_naive on a whole problem and
// the base case of every Strassen / Winograd recursion, and one launch can run
// a group of independent products (the seven products of a level, or many
// problems of a batch), so small leaves still fill the 256 compute units.
//
// Workgroup: 256 threads = 4 wave64s in a 2 x 2 arrangement, a 128 x 128 tile
// of C, each wave 64 x 64.  The K loop stages 128 x BK tiles of A and B in LDS
// (BK = 32 floats or 16 doubles), double-buffered: the global loads of tile
// t+1 are in flight while the MFMAs consume tile t, one barrier per step.
//
// LDS layout ("k-chunked"): a 16-byte chunk holds E consecutive k values
// (E = 4 floats / 2 doubles) of one row of A or one column of B, so every MFMA
// operand fetch is one ds_read_b128 that feeds E MFMAs.  Row (A) and column
// (B) indices are XOR-swizzled so that both the stores of the global tile and
// the fragment reads touch 16 distinct 16-byte bank groups per 16 lanes.
//
// Edges: operand reads outside a view's valid extent are zero (this is also
// how quadrants of a zero-padded matrix are read without a copy), and stores
// outside the output's valid extent are dropped.  Interior tiles take an
// unmasked vector path.
//
// Epilogue per output: C = s * acc or C = D + s * acc (s = +1 or -1).  The
// accumulator holds the product rounded exactly as it would be stored, so
// folding a following block addition into the epilogue gives the same bits
// as storing the product and adding it in a separate step.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "kernels.h"

namespace mm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
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

constexpr int BM = kGemmBM;
constexpr int BN = kGemmBN;
constexpr int BKC = 8;  // k-chunks per LDS tile
constexpr int NT = 256;
constexpr int WM = 64, WN = 64;  // wave tile

template <typename T>
__device__ __forceinline__ T* resolve(const KernelBases& kb, const MView& v) {
  char* b = v.base == MB_ABS ? nullptr : reinterpret_cast<char*>(kb.p[v.base]);
  return reinterpret_cast<T*>(b) + v.off;
}

__device__ __forceinline__ bool view_vec(const KernelBases& kb, const MView& v) {
  return v.vec && (v.base == MB_ABS || ((kb.aligned >> v.base) & 1));
}

// Column swizzle of B's LDS tile (and of A's rows, below).
template <int E>
__device__ __forceinline__ int swz_b(int col) { return col ^ ((col >> 4) & (E - 1)); }
__device__ __forceinline__ int swz_a(int row, int kc) { return row ^ (2 * kc); }

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Workgroups are dealt to the 8 XCDs round-robin (b % 8).  Give each XCD a
  // contiguous range of tiles so that tiles sharing A rows / B columns share
  // that XCD's L2.
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

template <typename T>
__global__ __launch_bounds__(NT) void gemm_kernel(KernelBases kb, const GemmDesc* __restrict__ descs,
                                                  int ndesc) {
  typedef MT<T> M;
  typedef typename M::chunk_t chunk_t;
  constexpr int E = M::E;
  constexpr int TM = M::TM;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int BK = BKC * E;
  constexpr int NB = BKC * (BN / E) / NT;  // E x E blocks of B per thread
  constexpr int NA = BM * BKC / NT;        // chunks of A per thread

  __shared__ chunk_t As[2][BKC][BM];
  __shared__ chunk_t Bs[2][BKC][BN];

  // ---- which problem and which tile -------------------------------------
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
  const int i0 = tm * BM, j0 = tn * BN;

  const MView av = D.a, bv = D.b;
  const T* __restrict__ Ap = resolve<T>(kb, av);
  const T* __restrict__ Bp = resolve<T>(kb, bv);
  const int64_t lda = av.ld, ldb = bv.ld;
  const bool avec = view_vec(kb, av), bvec = view_vec(kb, bv);
  const int K = D.k;
  const int ktiles = (K + BK - 1) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // ---- global -> register staging ----------------------------------------
  chunk_t ra[NA];
  chunk_t rbk[NB][E];  // E rows (k) of E columns

  auto load_tile = [&](int kt) {
    const int k0 = kt * BK;
    const bool afull = avec && (i0 + BM <= av.vrows) && (k0 + BK <= av.vcols);
    const bool bfull = bvec && (k0 + BK <= bv.vrows) && (j0 + BN <= bv.vcols);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      const int row = q / BKC, kc = q % BKC;
      const int gr = i0 + row, gc = k0 + kc * E;
      const T* p = Ap + (int64_t)gr * lda + gc;
      if (afull) {
        ra[i] = *reinterpret_cast<const chunk_t*>(p);
      } else if (avec && gr < av.vrows && gc + E <= av.vcols) {
        ra[i] = *reinterpret_cast<const chunk_t*>(p);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
          ra[i][e] = (gr < av.vrows && gc + e < av.vcols) ? p[e] : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      const int kc = q / (BN / E), cb = q % (BN / E);
      const int gc = j0 + cb * E;
#pragma unroll
      for (int rr = 0; rr < E; ++rr) {
        const int gr = k0 + kc * E + rr;
        const T* p = Bp + (int64_t)gr * ldb + gc;
        if (bfull) {
          rbk[i][rr] = *reinterpret_cast<const chunk_t*>(p);
        } else if (bvec && gr < bv.vrows && gc + E <= bv.vcols) {
          rbk[i][rr] = *reinterpret_cast<const chunk_t*>(p);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e)
            rbk[i][rr][e] = (gr < bv.vrows && gc + e < bv.vcols) ? p[e] : T(0);
        }
      }
    }
  };

  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + NT * i;
      const int row = q / BKC, kc = q % BKC;
      As[buf][kc][swz_a(row, kc)] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + NT * i;
      const int kc = q / (BN / E), cb = q % (BN / E);
#pragma unroll
      for (int c = 0; c < E; ++c) {
        chunk_t t;
#pragma unroll
        for (int rr = 0; rr < E; ++rr) t[rr] = rbk[i][rr][c];
        Bs[buf][kc][swz_b<E>(cb * E + c)] = t;
      }
    }
  };

  typename M::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[a][b][r] = T(0);

  const int g = lane / TM, t = lane % TM;

  if (ktiles > 0) {
    load_tile(0);
    store_tile(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < ktiles) load_tile(kt + 1);
#pragma unroll
      for (int kb2 = 0; kb2 < BKC / M::KG; ++kb2) {
        const int plane = kb2 * M::KG + g;
        chunk_t fa[FM], fb[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) fa[a] = As[buf][plane][swz_a(wm * WM + a * TM + t, plane)];
#pragma unroll
        for (int b = 0; b < FN; ++b) fb[b] = Bs[buf][plane][swz_b<E>(wn * WN + b * TM + t)];
#pragma unroll
        for (int s = 0; s < E; ++s)
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) acc[a][b] = M::mfma(fa[a][s], fb[b][s], acc[a][b]);
      }
      if (kt + 1 < ktiles) store_tile(buf ^ 1);
      __syncthreads();
    }
  }

  // ---- epilogue --------------------------------------------------------------
  for (int o = 0; o < D.nout; ++o) {
    const GemmOut& O = D.out[o];
    T* Cp = resolve<T>(kb, O.c);
    const int64_t ldc = O.c.ld;
    const bool add = O.mode == GM_ADD;
    const T* Dp = add ? resolve<T>(kb, O.d) : nullptr;
    const int64_t ldd = add ? O.d.ld : 0;
    const T sg = T(O.sign);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int col = j0 + wn * WN + b * TM + t;
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) {
          const int row = i0 + wm * WM + a * TM + M::row(lane, r);
          if (row < O.c.vrows && col < O.c.vcols) {
            const T v = sg * acc[a][b][r];
            Cp[(int64_t)row * ldc + col] = add ? Dp[(int64_t)row * ldd + col] + v : v;
          }
        }
      }
  }
}

}  // namespace

bool gemm_bf16x3_available() { return false; }

hipError_t launch_gemm(int dtype, const KernelBases& kb, const GemmDesc* ddescs, int ndesc, int tiles,
                       hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  if (dtype == DT_F64)
    hipLaunchKernelGGL(gemm_kernel<double>, dim3(tiles), dim3(NT), 0, s, kb, ddescs, ndesc);
  else
    hipLaunchKernelGGL(gemm_kernel<float>, dim3(tiles), dim3(NT), 0, s, kb, ddescs, ndesc);
  return hipGetLastError();
}

}  // namespace mm
