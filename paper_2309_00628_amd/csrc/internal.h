// Library-internal entry points shared between the host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

namespace mm {

// Record msg as the calling thread's last error and return code.
int set_error(int code, const char* msg);

// C = A B (contiguous operands) by (algo, sched) with no device allocation:
// the plan is built on the host (cached per shape and device), its
// descriptor table is copied with hipMemcpyAsync on `stream` to `table`
// (table_cap bytes of device memory) and its workspace is `ws` (ws_cap
// bytes).  MM_E_WORKSPACE, with nothing enqueued, when the table or the
// workspace does not fit; MM_E_UNSUPPORTED for schedules that need
// plan-owned streams.
int run_in_memory(int algo, int sched, int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C,
                  int cutoff, int levels, int dtype, void* table, size_t table_cap, void* ws, size_t ws_cap,
                  hipStream_t stream);

}  // namespace mm
