// Host-side launch functions of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "desc.h"

namespace mm {

// Element types the kernels compute in (the public dtype codes of mm.h map
// onto these; the split-bfloat16 path keeps float32 buffers).
// DT_BF16X3_SPL: refined split-bfloat16 leaves whose operands were split by
// the split pass (SPL layout; B operands transposed).  DT_F32_BT: float32
// products whose B views hold B transposed (OK_TRANS).
enum KDtype : int { DT_F64 = 0, DT_F32 = 1, DT_BF16X3 = 2, DT_BF16X3_SPL = 3, DT_F32_BT = 4 };

// Tile configurations of the MFMA GEMM kernel (rows x cols of C per
// workgroup); the planner needs the geometry to count tiles.
struct GemmCfg {
  int bm, bn;
};
constexpr int kNumGemmCfg = 9;
GemmCfg gemm_cfg(int dtype, int cfg);

int ew_blocks(int rows, int cols, int dtype);
// Two recursion levels of pre- or post-additions in one pass (ew2.hip): the
// blocks of parts of rows x cols lower-level positions, and the launch.
int ew2_blocks(int rows, int cols, int dtype);
hipError_t launch_ew2(int dtype, const KernelBases& kb, const Ew2Part* dparts, int nparts, int blocks,
                      hipStream_t s);
hipError_t launch_ew(int dtype, const KernelBases& kb, const EwPart* dparts, int nparts, int blocks,
                     hipStream_t s);
bool gemm_bf16x3_available();
GemmCfg gemm_bf16x3_cfg(int cfg);
GemmCfg gemm_bf16s_cfg(int cfg);
hipError_t launch_gemm_bf16x3(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles,
                              int remap, hipStream_t s);
hipError_t launch_gemm_bf16s(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles,
                             int remap, hipStream_t s);
// Split passes (EW_SPLIT, EW_WINO_S_SPL, EW_WINO_T_SPL parts; rows x cols is
// the float32 input block, transposed = mode[0]).
// Unrolled base cases: count leaves of order s (1, 2, 4 or 8) in one launch.
int base_blocks(int count);
hipError_t launch_base(int dtype, int s, const KernelBases& kb, const BaseDesc* d, int count, int blocks,
                       hipStream_t st);
int trans_blocks(int rows, int cols);
hipError_t launch_trans(const KernelBases& kb, const EwPart* dparts, int nparts, int blocks, hipStream_t s);
int split_blocks(int rows, int cols, int transposed);
hipError_t launch_split(const KernelBases& kb, const EwPart* dparts, int nparts, int blocks, hipStream_t s);
// Float32 leaf products whose operands may be Winograd sums of parent
// quadrants (GemmDesc::kinds); aligned, fully valid operands only.
hipError_t launch_gemm_fused(int cfg, const KernelBases& kb, const GemmDesc* d, int n, int tiles, int remap,
                             hipStream_t s);
// Last-level Winograd subproblems: seven float32 products and their U
// combinations per output tile (WinoLeafDesc); cfg as gemm_wino_cfg.
constexpr int kNumWinoCfg = 3;
GemmCfg gemm_wino_cfg(int cfg);
hipError_t launch_gemm_wino(int cfg, int fused, const KernelBases& kb, const WinoLeafDesc* d, int n, int tiles, int remap,
                            hipStream_t s);
// Persistent batched plans (batch.hip): tile configurations 0, 4 and 8 of
// the float32 GEMM; workgroups per compute unit that fit at once; launch of
// the whole task queue (table: PersistHdr and its segments; ctr: the plan's
// counters; spin: polls before a wait gives up and flags the plan).
bool persist_cfg_ok(int cfg);
int persist_occupancy(int cfg);
hipError_t launch_persist(int cfg, const KernelBases& kb, const void* table, int* ctr, int grid, int spin,
                          hipStream_t s);
// remap: 1 = XCD-contiguous tile order (launches of equal problems),
// 0 = hardware round-robin (unequal problems, sorted longest first).
hipError_t launch_gemm(int dtype, int cfg, const KernelBases& kb, const GemmDesc* ddescs, int ndesc, int tiles,
                       int remap, hipStream_t s);

}  // namespace mm
