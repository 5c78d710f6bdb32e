/*
 * mm.h -- C ABI of libmm: C = A x B by the naive method, by Strassen's
 * recursion and by Strassen-Winograd, on AMD Instinct MI355X (gfx950).
 *
 * The operation (Section 2.1): given A (m x k) and B (k x n), compute
 * C (m x n) with c_ij = sum_p a_ip b_pj.  Strassen (Section 2.2) and
 * Strassen-Winograd (Section 2.3) reach the same C in exact arithmetic with
 * seven block products per level instead of eight; in floating point they
 * round differently, so results are compared by tolerance.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Layout     Row-major.  The short forms take contiguous matrices
 *            (lda = k, ldb = n, ldc = n); the _ex forms take leading
 *            dimensions in elements (ld >= row length).
 * Pointers   A, B, C and workspaces are DEVICE pointers on the current HIP
 *            device, owned by the caller, and must stay valid until the work
 *            enqueued on `stream` has completed.  Host pointers are never
 *            accepted.
 * dtype      MM_F64: double in, double out, double arithmetic.
 *            MM_F32: float in, float out, float MFMA products, float sums.
 *            MM_BF16X3_REFINED: float in and out; block sums in float; every
 *            leaf product splits each float operand x into bfloat16 parts
 *            x = hi + lo + res, multiplies the parts with bfloat16 MFMA
 *            into a float accumulator: three main products
 *            hi*hi + hi*lo + lo*hi plus one correction
 *            lo*lo + res*hi + hi*res.  The residual x - hi - lo is formed
 *            in float: both subtractions are exact there (x - hi fits in 16
 *            significant bits, x - hi - lo in 8), so it has the same bits a
 *            double residual would have.  Relative Frobenius error is about
 *            1e-6 on well-scaled inputs (float32 level).
 * Asynchrony Every call only enqueues work on `stream` (a hipStream_t; NULL
 *            is the legacy default stream) and returns.  Faults inside
 *            kernels surface at the caller's synchronisation.
 * Errors     Every call returns an mm_status; no exception crosses the ABI.
 *            mm_last_error() gives a message for the last non-OK status of
 *            the calling thread.
 * Sizes      m == 0 or n == 0: no-op, MM_OK.  k == 0: C is set to zero.
 *
 * Recursion control (cutoff, levels)
 * ---------------------------------
 * Section 3.4: the recursion stops and the naive method runs once the order
 * is at most the cutoff.  Here a level is added while (levels < 0 or the
 * number of levels so far < levels) and the smallest of ceil(m / 2^l),
 * ceil(n / 2^l), ceil(k / 2^l) is greater than max(cutoff, 1).  cutoff <= 1
 * is Algorithm 2's 1x1 base case.  At most MM_MAX_LEVELS levels are
 * allowed (MM_E_UNSUPPORTED beyond).  Dimensions that are not multiples of
 * 2^levels are zero-padded (Section 3.1): the grouped schedule pads virtually
 * (out-of-range reads are zero, no copy); the depth-first schedules copy A
 * and B into padded workspace buffers and copy the result back.
 */
#ifndef MM_H_
#define MM_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MM_MAX_LEVELS 6

typedef enum { MM_F64 = 0, MM_F32 = 1, MM_BF16X3_REFINED = 2 } mm_dtype;

/* Algorithms: Section 2.1 (naive), Section 2.2 (Strassen), Section 2.3
 * (Strassen-Winograd, the 22-operation block form). */
typedef enum { MM_ALGO_NAIVE = 0, MM_ALGO_STRASSEN = 1, MM_ALGO_WINOGRAD = 2 } mm_algo;

/* Schedules (the order of block operations and where each result lives).
 *  MM_SCHED_TWO_TEMP  Section 3.3, Table 2: depth-first, two temporaries
 *                     X ((m/2) x max(k,n)/2) and Y ((k/2) x (n/2)) per
 *                     level.  Winograd only.
 *  MM_SCHED_IN_PLACE  Section 3.3, Table 3: depth-first, no temporaries;
 *                     A and B are OVERWRITTEN (their contents are undefined
 *                     afterwards).  Winograd only; needs k == n <= m.
 *  MM_SCHED_GROUPED   Breadth-first (not in the paper): per level one fused
 *                     launch forms all S and T blocks, the 7^L leaf products
 *                     run as one grouped MFMA launch, and one fused launch per
 *                     level forms the U blocks.  More workspace, far fewer
 *                     launches, leaves fill the GPU.  Winograd and Strassen
 *                     (for Strassen: five A sums and five B sums per block,
 *                     and the C quadrants combined in the order of DFS3, so
 *                     the two Strassen schedules give the same bits).
 *  MM_SCHED_DFS3      Strassen, depth-first with three temporaries (the paper
 *                     gives no reduced-memory schedule for Strassen): X and Y
 *                     hold the operand sums, Z the product of a non-leaf level;
 *                     leaf products add themselves into their C quadrants.
 *  MM_SCHED_AUTO      GROUPED.
 * For MM_ALGO_NAIVE the schedule is ignored. */
typedef enum {
  MM_SCHED_TWO_TEMP = 0,
  MM_SCHED_IN_PLACE = 1,
  MM_SCHED_GROUPED = 2,
  MM_SCHED_DFS3 = 3,
  MM_SCHED_AUTO = 4
} mm_sched;

typedef enum {
  MM_OK = 0,
  MM_E_INVALID = 1,     /* bad argument: negative size, NULL pointer with nonzero size,
                           ld shorter than a row, unknown enum value */
  MM_E_UNSUPPORTED = 2, /* valid but not supported: schedule/algorithm mismatch, in-place
                           shape rule, too many levels, no GPU / wrong architecture */
  MM_E_WORKSPACE = 3,   /* workspace smaller than the plan needs */
  MM_E_ALIAS = 4,       /* C overlaps A or B */
  MM_E_HIP = 5,         /* a HIP runtime call failed at enqueue time */
  MM_E_NOMEM = 6        /* device allocation for plan metadata or a cached workspace failed */
} mm_status;

typedef struct mm_plan_s* mm_plan_t;

/* ---- short forms (contiguous operands) --------------------------------- */

/* The naive method (Section 2.1) as one MFMA GEMM.  Needs no workspace,
 * except when a leading dimension or width of A or B is not a multiple of
 * 16 bytes and the product is large (m, n, k >= 64, mnk >= 2^27): then both
 * are first copied into aligned blocks of a workspace obtained as for
 * mm_strassen. */
int mm_naive(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int dtype,
             hipStream_t stream);

/* Strassen (Section 2.2, Algorithm 2 with the cutoff of Section 3.4),
 * schedule MM_SCHED_AUTO.  Uses the workspace registered for `stream` with
 * mm_set_workspace, else a workspace the library allocates once per
 * (device, stream) and keeps (first call only; later calls allocate nothing
 * unless a larger size is needed). */
int mm_strassen(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int cutoff,
                int levels, int dtype, hipStream_t stream);

/* Strassen-Winograd (Section 2.3 with Section 3.4's cutoff), schedule
 * MM_SCHED_AUTO.  Workspace as for mm_strassen. */
int mm_winograd(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int cutoff,
                int levels, int dtype, hipStream_t stream);

/* ---- extended form ---------------------------------------------------- */

/* Any algorithm and schedule, leading dimensions, caller-provided workspace
 * (ws may be NULL when mm_workspace_size returns 0).  A and B are written
 * only by MM_SCHED_IN_PLACE. */
int mm_gemm_ex(int algo, int sched, int64_t m, int64_t n, int64_t k, void* A, int64_t lda, void* B,
               int64_t ldb, void* C, int64_t ldc, int cutoff, int levels, int dtype, void* ws,
               size_t ws_bytes, hipStream_t stream);

/* Workspace bytes mm_gemm_ex needs for these arguments (0 on invalid
 * arguments; see mm_last_error). */
size_t mm_workspace_size(int algo, int sched, int64_t m, int64_t n, int64_t k, int cutoff,
                         int levels, int dtype);

/* Register a caller-owned workspace for the short forms on `stream` (bytes 0
 * or ws NULL unregisters).  The library never frees it. */
int mm_set_workspace(void* ws, size_t bytes, hipStream_t stream);

/* ---- plans ------------------------------------------------------------ */

/* Flags for mm_plan_create. */
#define MM_PLAN_GRAPH 1u /* capture the launch sequence in a hipGraph per distinct
                            (A, B, C, workspace) address tuple and replay it */
#define MM_PLAN_FUSE 2u /* form the last level's S/T sums in the leaf GEMM's tile loader instead
                          of a separate pre-addition pass (float32, grouped schedule; results
                          are bitwise the same).  Off by default: on MI355X it doubles the
                          operand traffic into the CUs and measures slower. */
#define MM_PLAN_OVERLAP 4u /* grouped schedule: run the S/T pre-addition passes on an
                             auxiliary stream of the plan, concurrently with the leaf
                             products that read only blocks of A and B (P1 = A11 B11,
                             P2 = A12 B21 and their counterparts below); the leaves are then
                             split over two launches.  Results are bitwise the same as
                             without the flag; whether it is faster depends on the shape
                             and tile (the autotuner tries both). */
#define MM_PLAN_LEAF_U 8u /* Strassen-Winograd, grouped schedule, float32: run the last level
                            as one kernel in which each workgroup forms the seven products
                            (Section 2.3) of one output tile and their U combinations in
                            registers, so no product is stored and the last level's U pass
                            disappears.  Sums are rounded in the same order as the separate
                            U pass: results are bitwise the same.  Ignored for other dtypes
                            and schedules.  With MM_PLAN_FUSE as well, that kernel also forms
                            S1..S4 and T1..T4 in its tile loader (when every last-level block
                            is 16-byte aligned and has no padding): the last level then uses
                            no temporaries at all (a one-level product touches only A, B
                            and C; its workspace size still covers the unfused plan that runs
                            when A or B is not 16-byte aligned). */
#define MM_PLAN_SPLIT_PASS 16u /* MM_BF16X3_REFINED, grouped Winograd or plain product: split
                                 each float32 operand into its bfloat16 parts once, in a split
                                 pass (which also forms the last level's S/T sums), and run
                                 the leaves on the stored parts, instead of splitting every
                                 staged tile inside the leaf kernel (the default).  Both give
                                 the same bits; the stored parts move 1.5x the bytes of the
                                 float32 operands, and on MI355X the default measures faster. */
#define MM_PLAN_ACCUMULATE 32u /* the plan computes C <- A B + beta C, beta given per call by
                                 mm_plan_execute_beta (mm_plan_execute uses beta = 1).  With
                                 beta == 0 the old C is not read (it may hold anything).  The
                                 plain product and the grouped schedule apply beta in their
                                 last step (the GEMM epilogue or the top level's U pass, as
                                 fma(beta, Cold, x)); the depth-first schedules form A B in a
                                 workspace block of m x n (they use C as scratch) and add it
                                 in one more element-wise pass.  Not for batched plans. */
#define MM_PLAN_TRANS_B 128u /* Strassen-Winograd, grouped schedule, float32: the last level's
                               T pass writes T1..T4 and the B quadrants that are leaf operands
                               (B11, B21, B22) transposed, in one transposing pass, so the
                               leaf products stage B in 16-byte chunks along k exactly as they
                               stage A (straight from memory into LDS in interior tiles).
                               Results are bitwise the same; costs three more quarter-size
                               blocks of workspace and writes per last-level block.  The last
                               level's fused forms (MM_PLAN_LEAF_U, MM_PLAN_SPLIT_PASS) take
                               precedence; it takes precedence over MM_PLAN_FUSE. */
#define MM_PLAN_UNROLL_BASE 0x100000u /* Strassen-Winograd, grouped schedule, float32 / float64: when the
                                         leaves are of order 1, 2, 4 or 8 (the recursion run down to tiny
                                         blocks, as in Section 3's experiments with win2x2, win4x4 and
                                         win8x8), compute them with the unrolled base cases (one thread
                                         per leaf, the 22-operation form unrolled to scalars in
                                         registers) instead of MFMA tiles.  Gives the same bits as the
                                         plan with log2(order) more levels. */
#define MM_PLAN_PEEL 64u /* grouped schedule: instead of reading A, B and C as if zero-padded to
                           multiples of 2^L g, run the recursion on the largest leading block
                           whose sides are such multiples (pm x pk times pk x pn) and cover
                           the rest with one launch of thin products (dynamic peeling, the
                           alternative to padding that Section 3.1 mentions): C[:pm,:pn] +=
                           A[:pm,pk:] B[pk:,:pn], C[:pm,pn:] = A[:pm,:] B[:,pn:], C[pm:,:] =
                           A[pm:,:] B.  No effect when every side is already such a multiple
                           or when a side of the leading block would be empty. */
#define MM_PLAN_LEVEL_PASSES 0x400000u /* Strassen-Winograd, grouped schedule: one pre-addition
 * (S/T) and one post-addition (U) pass per recursion level.  By default two
 * consecutive levels whose blocks are entirely valid (no zero padding) and
 * split into whole 16-byte chunks share one pass each way, which keeps the
 * upper level's sums and products in registers instead of HBM (the same
 * bits); this flag asks for the level-by-level passes instead. */
#define MM_PLAN_PERSISTENT 0x200000u /* batched plans, MM_F32: run the whole batch -- the S/T passes of
                                       every recursion level, every leaf-product tile and the U passes
                                       of every problem -- as ONE launch of a persistent kernel whose
                                       workgroups (as many as fit on the GPU at once) take tasks from a
                                       queue in order; a task waits on a per-problem counter for the
                                       stage it needs (and gives up after a bounded number of polls,
                                       flagging the plan: see mm_plan_check).  Same results as the
                                       level-synchronous batched plan.  The plan owns a small counter
                                       buffer: its executions must not overlap (serialise them on one
                                       stream).  Other dtypes ignore the flag.  SWITCHED OFF on the
                                       device: its first run on MI355X hung and the cause is not yet
                                       found, so mm_batched_plan_create returns MM_E_UNSUPPORTED for it;
                                       the host-only calls (mm_batched_describe, mm_batched_table) still
                                       build it, for checking its task queue. */
/* Recursive plans: pad m, n and k up to multiples of 2^q as well as of 2^L
 * (q = 0 .. 15; 0: no extra padding).  For example MM_PLAN_PAD(7) takes
 * n = 3000 to 3072, giving leaves of 1536 / 768 / 384 (tile multiples)
 * instead of 1500 / 750 / 375 (Section 3.1 pads to a power of two; 3000 needs
 * no padding at all for up to three levels).  The grouped schedule pads
 * virtually (no copies); the depth-first schedules copy.  Ignored with
 * MM_PLAN_PEEL and for zero levels. */
#define MM_PLAN_PAD(q) (((unsigned)(q) & 0xfu) << 24)
/* Plain product (MM_ALGO_NAIVE, or a recursion of zero levels): split k into
 * s parts (2 .. 8, each a multiple of 64 long), run the s partial products
 * in one grouped launch into workspace blocks and sum them in order in one
 * element-wise pass (applying beta in accumulating plans).  For products
 * whose C has too few tiles to fill the 256 compute units; the sum order
 * differs from the unsplit product's, so the bits may differ too. */
#define MM_PLAN_SPLIT_K(s) (((unsigned)(s) & 0xfu) << 16)
/* Force the MFMA GEMM tile configuration c (0 .. 8) for every leaf launch
 * instead of the planner's choice.  float32: 0 128x128 (BK 32, 8 waves),
 * 1 256x128 (8 waves), 2 128x256 (8 waves), 3 256x256 (BK 32, 8 waves),
 * 4 64x128, 5 128x64, 6 256x128 (BK 16, 4 waves), 7 128x128 (BK 16,
 * 4 waves), 8 64x64 (BK 32, 4 waves); float64: 0 128x128, 5 128x64 (others fall back to 0);
 * MM_BF16X3_REFINED: 0 128x128 (4 waves, three LDS stages, two workgroups
 * per CU), 1 256x128 (8 waves), 3 256x256 (8 waves), 4 64x128, 6 256x256
 * (8 waves, three LDS stages, the split pipelined under the MFMAs), 8 64x64
 * (others fall back to 0), and with MM_PLAN_SPLIT_PASS 0, 1, 3
 * 256x256 (4 waves), 4, 5 256x128 (4 waves), 6 256x256 (8 waves).  With
 * MM_PLAN_LEAF_U in effect c picks the fused leaf-level kernel's tile
 * instead: 0 128x128 (4 waves), 1 128x128 (8 waves), 2 64x128 (4 waves). */
#define MM_PLAN_TILE(c) ((unsigned)((c) + 1) << 8)

/* Build (once) the launch sequence and device descriptor table of one
 * product shape on the current device.  The plan owns a small device table
 * (freed by mm_plan_destroy), with MM_PLAN_GRAPH its graphs, and, when its
 * schedule overlaps launches, one auxiliary stream (default priority) and
 * two events per caller stream it has run on. */
int mm_plan_create(int algo, int sched, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                   int64_t ldc, int cutoff, int levels, int dtype, unsigned flags, mm_plan_t* plan);

/* Enqueue the plan on `stream` for these operands.  No allocation. */
int mm_plan_execute(mm_plan_t plan, void* A, void* B, void* C, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* C <- A B + beta C for a plan created with MM_PLAN_ACCUMULATE (the
 * accumulating form C <- A B + beta C; beta finite).  Otherwise as
 * mm_plan_execute; MM_E_INVALID for other plans or a non-finite beta.  With
 * MM_PLAN_GRAPH a graph is captured per (A, B, C, ws, beta). */
int mm_plan_execute_beta(mm_plan_t plan, void* A, void* B, void* C, void* ws, size_t ws_bytes, double beta,
                         hipStream_t stream);

/* mm_plan_execute with timing: events[2i] and events[2i+1] (created by the
 * caller with hipEventCreate; nevents >= 2 * launches) are recorded before
 * and after launch i on the stream that launch runs on, so the caller can
 * read each launch's duration with hipEventElapsedTime after synchronising.
 * The whole product spans events[0] to events[2 * launches - 1].  Graph
 * capture is not used on this path. */
int mm_plan_execute_timed(mm_plan_t plan, void* A, void* B, void* C, void* ws, size_t ws_bytes,
                          hipStream_t stream, hipEvent_t* events, int nevents);

/* Kind of launch i of a plan: 0 element-wise block operations, 1 MFMA GEMM
 * group (leaf products), 2 fork to / 3 join of the plan's auxiliary stream,
 * 4 fused last Winograd level (MM_PLAN_LEAF_U), 5 split pass of the
 * split-bfloat16 leaves, 6 transposing pass (MM_PLAN_TRANS_B), 7 unrolled base
 * cases (MM_PLAN_UNROLL_BASE); plus 8 when
 * the launch runs on the auxiliary stream; 16 the persistent launch of a
 * whole batch (MM_PLAN_PERSISTENT); 18 (26 on the auxiliary stream) a pass
 * that forms two recursion levels' pre- or post-additions at once (see
 * MM_PLAN_LEVEL_PASSES); -1 if i is out of range. */
int mm_plan_op_kind(mm_plan_t plan, int i);

/* Plan facts: info[0] workspace bytes, [1] levels L, [2..4] padded m, n, k,
 * [5] kernel launches per execution, [6] leaf products, [7] schedule used,
 * [8] leaf edge (rows of a leaf block), [9] 1 if the last level's operand
 * sums are formed in the leaf loader, [10] 1 if the last level runs as the
 * fused products-and-U kernel.  Returns the number of entries written. */
int mm_plan_info(mm_plan_t plan, int64_t* info, int ninfo);

/* Human-readable listing of the launch sequence (one line per block
 * operation, "kind dst <- srcs" with block coordinates).  Returns the length
 * of the full text; writes at most len-1 characters and a NUL. */
size_t mm_plan_describe(mm_plan_t plan, char* buf, size_t len);

int mm_plan_destroy(mm_plan_t plan);

/* ---- batches ---------------------------------------------------------- */

/* A batch of independent products C_i = A_i x B_i (contiguous, one dtype),
 * mnk[3i .. 3i+2] = (m_i, n_i, k_i), each with its own cutoff and levels
 * (Section 3.4).  levels NULL: each problem's level count is the
 * autotuner's choice for its size class (see mm_batched_levels); cutoff
 * NULL: cutoff 1.  Without MM_PLAN_PERSISTENT problems are executed
 * level-synchronously: one launch per recursion stage for the whole batch
 * and one grouped MFMA launch for every leaf of every problem; with it (float32)
 * everything runs as one persistent launch.  The plan binds the operand
 * addresses. */
int mm_batched_plan_create(int count, const int64_t* mnk, void* const* A, void* const* B,
                           void* const* C, int dtype, const int* cutoff, const int* levels,
                           unsigned flags, mm_plan_t* plan);

/* The level count each problem of a batch gets (host only; no device
 * needed): given levels as given, NULL levels the size class's tuned count;
 * both then capped by the cutoff (NULL: 1) and the problem's shape.  A size
 * class is the volume-equivalent order v = (m n k)^(1/3) rounded to half
 * octaves; the table of tuned counts is read once per process from
 * tuning/gfx950_batched.txt next to the library (or $MM_TUNING_DIR), and
 * a dtype with no table takes one level per halving while the leaf's v
 * stays >= 2048 (4096 split bfloat16), at most two. */
int mm_batched_levels(int count, const int64_t* mnk, int dtype, const int* cutoff, const int* levels,
                      int* levels_out);

/* Path of the size-class table read by mm_batched_levels ("" when none was
 * found). */
const char* mm_tuning_source(void);

/* Persistent plans: wait for `stream`, then report (and clear) the flag a
 * task sets when it waits past its bound (MM_E_HIP: the results of the
 * executions since the last check are not reliable).  MM_OK for other
 * plans, without synchronising. */
int mm_plan_check(mm_plan_t plan, hipStream_t stream);

/* One-shot batch: builds (or fetches from a cache keyed by all arguments)
 * the level-synchronous batched plan and executes it with the workspace
 * given. */
int mm_batched(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
               int dtype, const int* cutoff, const int* levels, void* ws, size_t ws_bytes,
               hipStream_t stream);

/* ---- no device allocation --------------------------------------------- */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * library holds one static scratch array of MM_NOALLOC_SCRATCH_BYTES on each
 * GPU it runs on, from the load of its code object until the process ends. */
#define MM_NOALLOC_SCRATCH_BYTES (64u << 20)
#define MM_NOALLOC_TABLE_BYTES (4u << 20) /* of which: the plan's descriptor table */

/* mm_winograd without any device allocation: the Two Temp schedule (Section
 * 3.3, Table 2), its descriptor table and workspace in the static scratch
 * array of the current device (the table is copied there with an
 * asynchronous host-to-device copy on `stream` at every call).  Same
 * arguments, results within the float tolerance of mm_winograd's (bitwise
 * equal where both pad to the same blocks).  Returns MM_E_WORKSPACE, with
 * nothing enqueued, when the product's workspace exceeds
 * MM_NOALLOC_SCRATCH_BYTES - MM_NOALLOC_TABLE_BYTES (60 MiB: for example
 * float32 n <= 5400 with one level, n = 4096 with two) or its table exceeds
 * MM_NOALLOC_TABLE_BYTES.  Calls share the device's array and it keeps the
 * last call's contents (nothing in it needs to start at zero): calls that
 * overlap on one device, on different streams, race; serialise them on one
 * stream.  Allocates only host memory (the plan, on the first call of each
 * shape). */
int mm_winograd_noalloc(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int cutoff,
                        int levels, int dtype, hipStream_t stream);

/* ---- diagnostics ------------------------------------------------------ */

/* Host-only: build the plan mm_plan_create would build (same flags),
 * without touching a device, and return its listing as mm_plan_describe does (and its facts as
 * mm_plan_info does, when info is not NULL).  Returns 0 when the arguments
 * are rejected (see mm_last_error).  Lets the launch sequence be inspected
 * and checked on a machine with no GPU. */
size_t mm_describe(int algo, int sched, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                   int64_t ldc, int cutoff, int levels, int dtype, unsigned flags, char* buf, size_t len,
                   int64_t* info, int ninfo);

/* Host-only counterpart for mm_batched_plan_create.  The addresses are only
 * recorded (never dereferenced), so any values may be passed. */
size_t mm_batched_describe(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                           int dtype, const int* cutoff, const int* levels, unsigned flags, char* buf,
                           size_t len, int64_t* info, int ninfo);

/* Host-only: the device descriptor table of the batched plan
 * mm_batched_plan_create would build (same flags; for a persistent plan it
 * starts with the task queue's header, desc.h), copied into buf (up to len
 * bytes).  Returns its size, 0 when the arguments are rejected.  For
 * checking the task queue on a machine with no GPU. */
size_t mm_batched_table(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                        int dtype, const int* cutoff, const int* levels, unsigned flags, void* buf,
                        size_t len);

const char* mm_last_error(void);
int mm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MM_H_ */
