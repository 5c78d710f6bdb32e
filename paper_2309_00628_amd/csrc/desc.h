// Descriptors shared by the planner (host) and the kernels (device).
//
// A plan is a list of operations.  Each operation is one kernel launch that
// processes an array of descriptors stored in a device-resident table owned by
// the plan.  Descriptors address memory relative to the buffers of a call
// (A, B, C, workspace), so one plan serves every call with the same shape and
// the table is uploaded once, when the plan is built.
#pragma once
#include <stdint.h>

namespace mm {

enum Base : int32_t { MB_A = 0, MB_B = 1, MB_C = 2, MB_WS = 3, MB_ABS = 4, MB_NONE = 5 };
constexpr int kNumBases = 5;

// A rows x cols block of a row-major matrix.  Element (r, c) lives at
// base + off + r * ld + c.  Reads outside [0, vrows) x [0, vcols) return zero
// and writes there are dropped: this is how zero padding is applied without
// copying (the block is a quadrant of a conceptually padded matrix).
struct MView {
  int64_t off;
  int64_t ld;
  int32_t rows, cols;
  int32_t vrows, vcols;
  int32_t base;
  int32_t vec;  // off and ld are multiples of the 16-byte vector width
};

// Element-wise block recipes.  Each names the formulas of one fused step.
enum EwKind : int32_t {
  EW_COPY = 0,     // o0 = i0 (with zero fill where i0 is outside its valid extent)
  EW_ADD = 1,      // o0 = i0 + i1
  EW_SUB = 2,      // o0 = i0 - i1
  EW_WINO_S = 3,   // i = A11 A12 A21 A22 ; o = S1 S2 S3 S4        (Section 2.3)
  EW_WINO_T = 4,   // i = B11 B12 B21 B22 ; o = T1 T2 T3 T4        (Section 2.3)
  EW_WINO_U = 5,   // i = P1..P7 ; o = C11 C12 C21 C22 = U1 U5 U6 U7 (Section 2.3)
  EW_TT_U = 6,     // Table 2 operations 13-17: i = X(P1) C11(P3) C12(P6) C21(P7) C22(P5)
                   //                        o = C12(U5) C21(U3) C22(U7)
  EW_IP_A = 7,     // Table 3 operations 1-2: i = A11 A21 A22 ; o = C11(S3) A21(S1)
  EW_IP_B = 8,     // Table 3 operations 3-4: i = B11 B12 B22 ; o = C22(T1) B12(T3)
  EW_IP_U = 9,     // Table 3 operations 16-20: i = C11(P1) C12(P2) C22(U2) A11(P5) C21(P7) A21(P4)
                   //                          o = C11(U1) C12(U4) C21(U6) C22(U7)
  EW_DIST = 10,    // o_j = mode_j(d_j, z): i = Z D0 D1 ; mode 1: z, 2: d + z, 3: d - z
  EW_ZERO = 11,    // o0 = 0
  // Split recipes (split kernel): float32 inputs, outputs in the split
  // bfloat16 layout below; mode[0] = 1 stores each output transposed.
  EW_SPLIT = 12,       // o0 = split(i0)
  EW_WINO_S_SPL = 13,  // i = A11 A12 A21 A22 ; o = S1 S2 S3 S4 A11 A12 A22
  EW_WINO_T_SPL = 14,  // i = B11 B12 B21 B22 ; o = T1 T2 T3 T4 B11 B21 B22 (transposed)
  // Accumulating form C <- A B + beta C (beta from KernelBases, applied as
  // one fused multiply-add beta * Cold + x; with beta == 0 the old C is not
  // read):
  EW_WINO_U_ACC = 15,  // i = P1..P7 C11 C12 C21 C22 ; o = C11..C22 = beta Cij + (U1 U5 U6 U7)
  EW_AXPBY = 16,       // i = X C ; o0 = beta C + X
  // Strassen (Section 2.2), grouped schedule:
  EW_STR_S = 17,      // i = A11 A12 A21 A22 ; o = A11+A22, A21+A22, A11+A12, A21-A11, A12-A22
  EW_STR_T = 18,      // i = B11 B12 B21 B22 ; o = B11+B22, B12-B22, B21-B11, B11+B12, B21+B22
  EW_STR_U = 19,      // i = P1..P7 ; o = C11 = ((P1+P4)-P5)+P7, C12 = P3+P5, C21 = P2+P4,
                      //              C22 = ((P1+P3)-P2)+P6
  EW_STR_U_ACC = 20,  // i = P1..P7 C11 C12 C21 C22 ; o = fma(beta, Cij, EW_STR_U's Cij)
  // Transposing passes (trans kernel; every output holds the transpose):
  EW_WINO_T_TR = 21,  // i = B11 B12 B21 B22 ; o = T1' T2' T3' T4' B11' B21' B22' (T as EW_WINO_T)
  // Split-k plain products (mode[0] = number of partial products np):
  EW_SUM = 22,        // i = X0 .. X(np-1) ; o0 = ((X0 + X1) + X2) + ...
  EW_SUM_ACC = 23,    // i = X0 .. X(np-1) C ; o0 = fma(beta, C, EW_SUM's sum)
};

constexpr int kEwMaxIn = 11;
constexpr int kEwMaxOut = 7;

// Split bfloat16 layout ("SPL") of a float32 matrix X with R rows and Kc
// columns, as read by the split-operand leaf kernel: every element is
// x = hi + lo + res (three bfloat16 numbers), and each row holds chunks of 8
// consecutive columns, chunk q of row r being 48 bytes at bfloat16 index
// off + r * ld + 24 q: hi[8] lo[8] res[8].  An MView of an SPL matrix counts
// off and ld in bfloat16 elements (ld = 24 * ceil(Kc / 8) or more), rows = R
// and cols = Kc; columns past Kc inside the last chunk hold zeros.  The B
// operand of a product is stored transposed (R = its columns), so both
// operands of the leaf kernel are read as runs of 8 consecutive k.

struct EwPart {
  int32_t kind;
  int32_t nin, nout;
  int32_t rows, cols;
  int32_t blk_start;   // first block of this part in the launch
  int32_t mode[2];     // EW_DIST output modes
  MView in[kEwMaxIn];
  MView out[kEwMaxOut];
};

// Two consecutive recursion levels of Section 2.3's block form in one pass
// (grouped schedule, blocks entirely valid).  rows x cols is one block of
// the lower level (the position grid of the pass); the upper level's blocks
// are twice that, its parent block four times.
//  EW2_S (EW2_T): from the parent block X (quadrants A11 A12 A21 A22, or
//    B11 B12 B21 B22) the sums S1..S4 (T1..T4) of the upper level, kept in
//    registers and written in `top` only where the lower level reads them as
//    plain operands (quadrants 11, 12, 22 of an A-side sum; 11, 21, 22 of a
//    B-side sum), and, for each of the seven operands of the upper level's
//    products (A11 A12 S4 A22 S1 S2 S3, or B11 B21 B22 T4 T1 T2 T3), its own
//    sums S1..S4 (T1..T4), written in low[o][0..3].
//  EW2_U: from the 49 lower-level products (low[q][c]: product c of the
//    upper-level product q), each upper-level product's four quadrants
//    (U1 U5 U6 U7 of its seven, in registers), and from those the parent's
//    C11 C12 C21 C22 (top[0..3]).
// Per element the operations and their order are those of the two separate
// passes, so the results are bitwise the same.
enum Ew2Kind : int32_t { EW2_S = 0, EW2_T = 1, EW2_U = 2 };

struct Ew2Part {
  int32_t kind;
  int32_t rows, cols;
  int32_t blk_start;  // first block of this part in the launch
  MView x;            // EW2_S / EW2_T: the parent block (2 rows*2 x 2 cols*2)
  MView top[4];
  MView low[7][7];    // EW2_S / EW2_T use low[o][0..3]
};

// GEMM epilogue: out = sign * acc (store), out = d + sign * acc (add), or
// out = fma(beta, d, sign * acc) (axpby; beta from KernelBases, d not read
// when beta == 0).
enum GemmMode : int32_t { GM_NONE = 0, GM_STORE = 1, GM_ADD = 2, GM_AXPBY = 3 };

struct GemmOut {
  MView c;
  MView d;
  int32_t mode;
  int32_t sign;  // +1 or -1
};

// Operand kinds of a leaf product.  OK_PLAIN: the view is the operand.
// OK_S1..OK_S4 / OK_T1..OK_T4: the view is the parent block and the operand
// is the Winograd sum S_i of its A quadrants / T_i of its B quadrants
// (Section 2.3), formed while the tile is staged (fused loader).
// OK_TRANS (B only): the view holds the transpose of the operand (n x k, each
// row one column of B), so B is staged like A, in 16-byte chunks along k.
enum OperandKind : int32_t {
  OK_PLAIN = 0, OK_S1 = 1, OK_S2 = 2, OK_S3 = 3, OK_S4 = 4,
  OK_T1 = 5, OK_T2 = 6, OK_T3 = 7, OK_T4 = 8, OK_TRANS = 9
};

struct GemmDesc {
  MView a, b;
  int32_t m, n, k;     // operand extents: A operand m x k, B operand k x n
  int32_t tiles_m, tiles_n;
  int32_t tile_start;  // first tile of this problem in the launch
  int32_t nout;
  int32_t kinds;       // OperandKind of A (bits 0-7) and of B (bits 8-15)
  GemmOut out[2];
};

// One subproblem at the last level of a Winograd recursion, done by one
// launch that forms the seven leaf products and the U combinations of
// Section 2.3 tile by tile in registers (no product is stored):
//   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4,
//   P5 = S1 T1,   P6 = S2 T2,   P7 = S3 T3,
//   C11 = P1 + P2, C12 = U5, C21 = U6, C22 = U7.
// A leaf product C = A B of order 1, 2 or 4 computed in registers by the
// Strassen-Winograd formula of Section 2.3 unrolled down to scalars (the
// unrolled base cases of Section 3): one thread per leaf.
struct BaseDesc {
  MView a, b, c;
};

struct WinoLeafDesc {
  MView a[7], b[7];    // operands of P1 .. P7
  MView c[4];          // C11 C12 C21 C22
  int32_t m, n, k;     // product extents: operand A m x k, B k x n
  int32_t tiles_m, tiles_n;
  int32_t tile_start;  // first tile of this subproblem in the launch
  int32_t acc;         // 1: C = beta C + U (top level of an accumulating product)
};

// Persistent batched execution: a whole batch of products (every recursion
// stage of every problem) as one launch whose workgroups take tasks from a
// queue in order.  The tasks form segments: the S/T passes of each
// recursion level, then the leaf-product tiles, then the U passes of each
// level from the deepest up.  A task of an element-wise segment is a run of
// element-wise blocks of one part; a task of the GEMM segment is one output
// tile of one leaf product.  Dependencies are per problem and stage: a task
// waits until a counter has reached the number of tasks of the stage it
// needs, and signals its own stage's counter when done.  Every task depends
// only on tasks earlier in the queue, so the workgroup holding the earliest
// unfinished task never waits on an unfinished one: the queue drains.
enum PTaskKind : int32_t { PT_EW = 0, PT_GEMM = 1 };
constexpr int kPersistMaxSegs = 2 * 6 + 2;  // S/T and U per level (MM_MAX_LEVELS 6), leaves, zero fills
constexpr int kPersistEwBlocks = 8;         // element-wise blocks per task

struct PDep {
  int32_t wait;        // counter to wait for (-1: none)
  int32_t target;      // ... until it counts this many completed tasks
  int32_t signal;      // counter to increment per completed task (-1: none)
  int32_t task_start;  // first task (within its segment) of this descriptor
};

struct PSeg {
  int32_t kind;     // PTaskKind
  int32_t first;    // queue index of the segment's first task
  int32_t ntasks;
  int32_t ndesc;    // EwPart (PT_EW) or GemmDesc (PT_GEMM) entries
  int64_t desc_off; // byte offsets in the plan's table: descriptors ...
  int64_t dep_off;  // ... and one PDep per descriptor
};

struct PersistHdr {
  int32_t nseg, ntasks, ncounters, pad;
  PSeg seg[kPersistMaxSegs];
};

// Counters of a persistent plan (int32, device memory owned by the plan,
// zero between launches: the last workgroup to finish clears them).
enum PCounter : int32_t { PC_HEAD = 0, PC_EXIT = 1, PC_ERROR = 2, PC_FIRST = 4 };

struct KernelBases {
  void* p[kNumBases];
  int32_t aligned;  // bit b set: base b is 16-byte aligned
  double beta;      // C <- A B + beta C (accumulating plans; 1 otherwise)
};

}  // namespace mm
