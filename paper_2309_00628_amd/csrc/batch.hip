// Persistent batched execution: every stage of every product of a batch
// (the S/T passes of each recursion level of Section 2.3, the leaf products
// of the naive method, the U passes) in ONE launch.  A fixed grid of
// workgroups, as many as fit on the GPU at once, takes tasks from a queue in
// order (desc.h: PersistHdr, PSeg, PDep): a run of element-wise blocks of
// one part, or one output tile of one leaf product.  A task that needs the
// results of an earlier stage of its problem waits on that stage's counter;
// a finished task adds one to its own stage's counter.
//
// Why the queue always drains: tasks are taken in queue order and every task
// depends only on tasks before it, so whenever some task is unfinished, the
// earliest unfinished one has all its inputs ready and is held by a running
// workgroup.  Every wait is also bounded (spin_limit polls, then the plan's
// error flag is set and the task proceeds), so a planner bug cannot hang the
// GPU.  The last workgroup to leave clears the counters for the next launch
// (so the kernel needs no memset node when captured in a hipGraph).
//
// Memory ordering: a producer's threads fence (device scope, release) before
// the barrier after which one thread adds to the counter; a consumer's
// thread polls the counter with device-scope atomic loads, and every thread
// fences (acquire) after the barrier that follows the poll.  Products and
// element-wise blocks compute exactly as in the separate kernels, so the
// batch gives the bits of the level-synchronous plan and of single products.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "ew_body.h"
#include "gemm_common.h"
#include "gemm_tile.h"
#include "kernels.h"

namespace mm {

namespace {

using namespace gemm_detail;

__device__ __forceinline__ int load_counter(int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last descriptor whose first task is at or before lt.
__device__ __forceinline__ int find_desc(const PDep* __restrict__ deps, int n, int lt) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (deps[mid].task_start <= lt) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int ew_part_blocks(const EwPart& P) {
  constexpr int V = 4;  // float32 chunks
  const int64_t chunks = (int64_t)P.rows * ((P.cols + V - 1) / V);
  constexpr int per = ew_detail::kThreads * ew_detail::kItems;
  return (int)((chunks + per - 1) / per);
}

template <int BM, int BN, int BKC, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void persist_kernel(KernelBases kb, const char* __restrict__ table,
                                                                 int* __restrict__ ctr, int spin_limit) {
  typedef TileLoop<float, BM, BN, BKC, WGM, WGN> TL;
  typedef MT<float> M;
  constexpr int NT = TL::NT;
  constexpr int EWT = ew_detail::kThreads;
  static_assert(NT % EWT == 0, "whole element-wise blocks per pass");
  constexpr int EWP = NT / EWT;  // element-wise blocks processed side by side
  __shared__ typename TL::Smem sm;
  __shared__ int s_task;
  const PersistHdr* __restrict__ H = reinterpret_cast<const PersistHdr*>(table);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int ntasks = H->ntasks, nseg = H->nseg;
  for (;;) {
    if (tid == 0) s_task = atomicAdd(&ctr[PC_HEAD], 1);
    __syncthreads();
    const int t = s_task;
    if (t >= ntasks) break;
    int si = 0;
    while (si + 1 < nseg && H->seg[si + 1].first <= t) ++si;
    const PSeg& S = H->seg[si];
    const int lt = t - S.first;
    const PDep* __restrict__ deps = reinterpret_cast<const PDep*>(table + S.dep_off);
    const int d = find_desc(deps, S.ndesc, lt);
    const PDep dep = deps[d];
    if (dep.wait >= 0) {
      if (tid == 0) {
        int* w = &ctr[PC_FIRST + dep.wait];
        for (int it = 0; load_counter(w) < dep.target; ++it) {
          if (it >= spin_limit) {
            atomicOr(&ctr[PC_ERROR], 1);
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
      }
      __syncthreads();
      __threadfence();  // acquire: the producers' stores are visible
    }
    if (S.kind == PT_GEMM) {
      const GemmDesc& D = reinterpret_cast<const GemmDesc*>(table + S.desc_off)[d];
      const TileRef tr = tile_in_problem<BM, BN>(d, lt - dep.task_start, D.tiles_m, D.tiles_n);
      typename TL::Acc acc;
      TL::zero(acc);
      TL::template product<OK_PLAIN, OK_PLAIN>(sm, operand<float>(kb, D.a), operand<float>(kb, D.b), tr.i0,
                                               tr.j0, D.k, acc);
      store_outputs<float, TL::TM, M::NACC, TL::FM, TL::FN, TL::WM, TL::WN, TL::NATF>(
          kb, D, tr.i0, tr.j0, wave / WGN, wave % WGN, lane, acc, [](int l, int r) { return M::row(l, r); });
    } else {
      const EwPart& P = reinterpret_cast<const EwPart*>(table + S.desc_off)[d];
      const int b0 = (lt - dep.task_start) * kPersistEwBlocks;
      const int b1 = min(b0 + kPersistEwBlocks, ew_part_blocks(P));
      for (int b = b0 + tid / EWT; b < b1; b += EWP) ew_detail::ew_block<float>(kb, P, b, tid % EWT);
    }
    if (dep.signal >= 0) {
      __threadfence();  // release: this task's stores
      __syncthreads();
      if (tid == 0) atomicAdd(&ctr[PC_FIRST + dep.signal], 1);
    } else {
      __syncthreads();  // every thread has read s_task before it is reused
    }
  }
  // Leave: the last workgroup out clears the counters for the next launch
  // (every other workgroup has made its last access to them).
  __shared__ int s_last;
  if (tid == 0) {
    __threadfence();
    s_last = atomicAdd(&ctr[PC_EXIT], 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    for (int i = tid; i < H->ncounters; i += NT)
      __hip_atomic_store(&ctr[PC_FIRST + i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (tid == 0) {
      __hip_atomic_store(&ctr[PC_HEAD], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctr[PC_EXIT], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int BM, int BN, int BKC, int WGM, int WGN>
hipError_t launch_cfg(const KernelBases& kb, const void* table, int* ctr, int grid, int spin, hipStream_t s) {
  hipLaunchKernelGGL((persist_kernel<BM, BN, BKC, WGM, WGN>), dim3(grid), dim3(64 * WGM * WGN), 0, s, kb,
                     (const char*)table, ctr, spin);
  return hipGetLastError();
}

template <int BM, int BN, int BKC, int WGM, int WGN>
int occupancy_cfg() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persist_kernel<BM, BN, BKC, WGM, WGN>, 64 * WGM * WGN, 0) !=
          hipSuccess ||
      n < 1) {
    (void)hipGetLastError();
    n = 1;
  }
  return n;
}

}  // namespace

// Tile configurations of the persistent kernel, numbered as the GEMM
// kernel's (MM_PLAN_TILE): 0 128x128 (8 waves), 4 64x128 (4 waves),
// 8 64x64 (4 waves).
bool persist_cfg_ok(int cfg) { return cfg == 0 || cfg == 4 || cfg == 8; }

int persist_occupancy(int cfg) {
  switch (cfg) {
    case 4: return occupancy_cfg<64, 128, 8, 2, 2>();
    case 8: return occupancy_cfg<64, 64, 8, 2, 2>();
    default: return occupancy_cfg<128, 128, 8, 4, 2>();
  }
}

hipError_t launch_persist(int cfg, const KernelBases& kb, const void* table, int* ctr, int grid, int spin,
                          hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (cfg) {
    case 4: return launch_cfg<64, 128, 8, 2, 2>(kb, table, ctr, grid, spin, s);
    case 8: return launch_cfg<64, 64, 8, 2, 2>(kb, table, ctr, grid, spin, s);
    default: return launch_cfg<128, 128, 8, 4, 2>(kb, table, ctr, grid, spin, s);
  }
}

}  // namespace mm
