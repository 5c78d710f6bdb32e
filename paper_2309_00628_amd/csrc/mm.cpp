// libmm host side: argument checking, the planner that turns a product
// (algorithm, schedule, shape, cutoff, levels) into a launch sequence, the
// executor, plan and workspace caches, hipGraph capture, and the C ABI.
//
// A plan is built once per shape.  The planner walks the recursion the way
// the chosen schedule orders it and records each block operation as a
// descriptor (element-wise parts for the additions, GEMM descriptors for the
// leaf products).  Descriptors address memory relative to the call's buffers
// (A, B, C, workspace) so the table is uploaded to the device once and every
// later execution is kernel launches only.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <list>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mm.h"
#include "desc.h"
#include "kernels.h"
#include "internal.h"

struct mm_plan_s;

namespace mm {

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

size_t elem_size(int dtype) { return dtype == MM_F64 ? 8 : 4; }
int kernel_dtype(int dtype) { return dtype == MM_F64 ? DT_F64 : (dtype == MM_F32 ? DT_F32 : DT_BF16X3); }
int ew_dtype(int dtype) { return dtype == MM_F64 ? DT_F64 : DT_F32; }

// OP_FORK: the auxiliary stream waits for the work enqueued so far on the
// main stream; OP_JOIN: the main stream waits for the auxiliary stream.
// OP_WINO: last-level Winograd subproblems, products and U combinations in
// one kernel (WinoLeafDesc).
// OP_SPLIT: split passes of the split-bfloat16 leaves (split kernel).
// OP_TRANS: element-wise passes with transposed outputs (trans kernel).
// OP_BASE: unrolled base cases, one leaf product per thread (BaseDesc).
enum OpType {
  OP_EW = 0, OP_GEMM = 1, OP_FORK = 2, OP_JOIN = 3, OP_WINO = 4, OP_SPLIT = 5, OP_TRANS = 6, OP_BASE = 7,
  OP_PERSIST = 16,  // a whole batch in one persistent launch (PersistHdr at the op's offset)
  OP_EW2 = 18       // two recursion levels of pre- or post-additions in one pass (Ew2Part)
};

struct OpRec {
  int type;
  int kdtype;
  size_t off;  // byte offset of the first descriptor in the table
  int count;   // descriptors
  int grid;    // workgroups
  int cfg;     // GEMM tile configuration
  int remap;   // GEMM: XCD-contiguous tile order
  int fused;   // GEMM: some operands are Winograd sums formed in the loader
  int stream;  // 0: the caller's stream, 1: the plan's auxiliary stream
};

}  // namespace

struct Plan {
  int algo = 0, sched = 0, dtype = 0;
  int64_t m = 0, n = 0, k = 0, lda = 0, ldb = 0, ldc = 0;
  int64_t M = 0, N = 0, K = 0;  // padded sizes
  int cutoff = 1, levels = 0, L = 0;
  int64_t leaf_rows = 0;
  int64_t leaves = 0;
  size_t ws_bytes = 0;
  bool batched = false;
  unsigned flags = 0;
  int tile_cfg = -1;  // forced GEMM tile configuration, -1: planner's choice
  bool fuse = false;  // fold the last level's S/T sums into the leaf loader
  bool overlap = false;  // run the S/T passes beside the products that do not need them
  bool leaf_u = false;   // last level: products and U combinations in one kernel (float32)
  bool wino = false;     // the plan has such a launch
  bool spl = false;      // split-bfloat16 leaves read operands split by a split pass
  bool accumulate = false;  // C <- A B + beta C (beta given per execution)
  bool peel = false;        // grouped: peel ragged rows / columns / k instead of padding
  bool level_passes = false; // grouped Winograd: one pre- and one post-addition pass per level
  bool trans_b = false;     // grouped Winograd float32: last-level B operands stored transposed
  bool unroll_base = false; // grouped Winograd: leaves of order 1, 2, 4, 8 by the unrolled base cases
  int split_k = 1;          // plain product: k split over this many partial products
  int64_t pad_mult = 1;     // recursive plans: pad m, n, k to multiples of this too (MM_PLAN_PAD)
  bool persistent = false;  // batched: one persistent launch (OP_PERSIST)
  int pcount = 0;           // ... its counters (besides PC_FIRST fixed ones)
  int pgrid = 0;            // ... its workgroups (as many as fit at once)
  int* dctr = nullptr;      // ... device counters, owned
  int64_t pm = 0, pn = 0, pk = 0;  // peeled: the leading block the recursion runs on
  bool has_aux = false;  // some launches go to the auxiliary stream
  struct Aux {
    hipStream_t main, aux;
    hipEvent_t fork, join;
  };
  std::list<Aux> aux;  // one auxiliary stream and event pair per caller stream
  std::mutex aux_mu;   // guards aux (enqueue may run while mu is held)
  bool fused = false;          // the plan has leaf products with fused operands
  bool fused_reads_ab = false;  // ... reading A or B directly (needs 16-byte aligned A, B)
  std::unique_ptr<Plan> unfused;  // same product without fusion, for unaligned A or B
  std::vector<OpRec> ops;
  std::vector<uint8_t> table;
  std::string text;
  void* dtable = nullptr;
  int device = -1;
  struct Graph {
    void *a, *b, *c, *ws;
    double beta;
    hipStream_t stream;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  std::mutex mu;
  ~Plan() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto& a : aux) {
      (void)hipStreamSynchronize(a.aux);
      (void)hipEventDestroy(a.fork);
      (void)hipEventDestroy(a.join);
      (void)hipStreamDestroy(a.aux);
    }
    if (dtable) (void)hipFree(dtable);
    if (dctr) (void)hipFree(dctr);
  }
};

namespace {

// Tile configuration for one GEMM launch (a group of independent products).
// Measured on MI355X (float32): 256x256 tiles (one workgroup per CU) reach
// the highest MFMA rate on large products but only when the launch fills
// whole waves of 256 workgroups; 128x128 tiles (two per CU) lose less to a
// partial last wave; 64x128 tiles keep small launches spread over more CUs.
int choose_gemm_cfg(int kdtype, const std::vector<GemmDesc>& group) {
  if (kdtype == DT_F64) return 0;
  if (kdtype == DT_F32_BT) kdtype = DT_F32;  // same tiles
  bool equal = true;
  for (const GemmDesc& g : group) equal = equal && g.m == group[0].m && g.n == group[0].n;
  if (!equal && kdtype == DT_F32 && group.size() > 1) {
    // Unequal problems: minimise the padded work (tile area x k) over the
    // measured per-tile MFMA efficiency of each shape.
    const int cand[5] = {0, 3, 4, 5, 8};
    const double eff[5] = {0.81, 0.87, 0.75, 0.72, 0.74};
    int best = 0;
    double best_cost = 1e300;
    for (int i = 0; i < 5; ++i) {
      const GemmCfg gc = gemm_cfg(kdtype, cand[i]);
      double work = 0;
      for (const GemmDesc& g : group)
        work += (double)ceil_div(g.m, gc.bm) * ceil_div(g.n, gc.bn) * gc.bm * gc.bn * (double)g.k;
      const double cost = work / eff[i];
      if (cost < best_cost) {
        best_cost = cost;
        best = cand[i];
      }
    }
    return best;
  }
  if (kdtype == DT_BF16X3 || kdtype == DT_BF16X3_SPL) {
    // eight-wave tiles (two waves per SIMD) hide the split's vector work
    // behind the MFMAs, and the 256x256 tile splits each element for half as
    // many tiles as 256x128; smaller launches keep more CUs busy with 64x128.
    int64_t t2x2 = 0, t256 = 0, t128 = 0, t64x128 = 0;
    for (const GemmDesc& g : group) {
      t2x2 += ceil_div(g.m, 256) * ceil_div(g.n, 256);
      t256 += ceil_div(g.m, 256) * ceil_div(g.n, 128);
      t128 += ceil_div(g.m, 128) * ceil_div(g.n, 128);
      t64x128 += ceil_div(g.m, 64) * ceil_div(g.n, 128);
    }
    if (kdtype == DT_BF16X3) {
      // the in-loader split's ring tiles (256x256 eight waves, 128x128 four
      // waves, both with three LDS stages and full-speed edge tiles):
      // measured best from half a round of 256x256 tiles up (n = 3000:
      // 329 us against 378 on 128x128 and 776 on the 256x128 tile), the
      // 128x128 ring below (n = 2048: 110 us against 159 and 221; n = 2560:
      // 206 us against 277 on 256x256); the 64-row tiles for small products
      // (n = 1024: 37 us on 64x64, 57 on the 128x128 ring)
      if (t2x2 >= 128) return 6;
      if (t128 >= 96) return 0;
      return t64x128 < 256 ? 8 : 4;
    }
    if (t256 >= 256) return 1;
    if (t128 >= 256) return 0;
    // (the in-loader split kernel also has 64x64 tiles for small products)
    return kdtype == DT_BF16X3 && t64x128 < 256 ? 8 : 4;
  }
  int64_t t256 = 0, t128 = 0, t64x128 = 0;
  for (const GemmDesc& g : group) {
    t256 += ceil_div(g.m, 256) * ceil_div(g.n, 256);
    t128 += ceil_div(g.m, 128) * ceil_div(g.n, 128);
    t64x128 += ceil_div(g.m, 64) * ceil_div(g.n, 128);
  }
  // whole rounds of 256 workgroups (one per CU) suit the eight-wave tiles
  if (t256 >= 1024 || (t256 >= 256 && t256 % 256 == 0)) return 3;
  if (t128 >= 2048 || (t128 >= 256 && t128 % 256 == 0)) return 0;
  // too few 64x128 tiles to give every CU one: 64x64 (measured at n = 512 ..
  // 1024: 1.4-1.7x the 64x128 tile)
  return t64x128 < 256 ? 8 : 4;
}

// ---------------------------------------------------------------------------
// Builder: records block operations while a schedule walks its recursion.
// ---------------------------------------------------------------------------
struct Builder {
  Plan& P;
  size_t esz;
  int64_t E;  // elements per 16-byte vector
  int64_t ws_top = 0, ws_peak = 0;
  std::vector<EwPart> ew;
  int ew_grid = 0;
  int cur_stream = 0;  // stream the next launches go to (0 main, 1 auxiliary)
  std::vector<GemmDesc> gm;
  std::vector<char> gm_fusable;  // descriptor satisfies the fused loader's preconditions
  std::vector<EwPart> tp;        // transposing passes of the current launch
  std::ostringstream ew_txt, tp_txt;  // listing lines of the pending element-wise / transposing parts
  std::vector<BaseDesc> bl;      // unrolled base cases of the current launch
  int bl_order = 0;
  int tp_grid = 0;
  std::vector<WinoLeafDesc> wl;  // last-level subproblems of the current launch
  bool wl_fused = false;         // ... whose S/T sums are formed in the loader
  std::vector<EwPart> sp;        // split parts of the current launch
  int sp_grid = 0;
  bool gm_spl = false;           // the pending GEMM descriptors read SPL operands
  int gm_grid = 0;
  std::vector<Ew2Part> e2;  // pending two-level passes
  int e2_grid = 0;
  std::ostringstream txt;

  explicit Builder(Plan& p) : P(p), esz(elem_size(p.dtype)), E(16 / (int64_t)elem_size(p.dtype)) {}

  MView view(int base, int64_t off, int64_t ld, int64_t rows, int64_t cols, int64_t vr, int64_t vc) {
    MView v;
    v.base = base;
    v.off = off;
    v.ld = ld;
    v.rows = (int32_t)rows;
    v.cols = (int32_t)cols;
    v.vrows = (int32_t)std::max<int64_t>(0, std::min(vr, rows));
    v.vcols = (int32_t)std::max<int64_t>(0, std::min(vc, cols));
    if (v.vrows == 0 || v.vcols == 0) v.vrows = v.vcols = 0;
    if (base == MB_ABS)
      v.vec = ((off * (int64_t)esz) % 16 == 0) && (ld % E == 0);
    else
      v.vec = (off % E == 0) && (ld % E == 0);
    return v;
  }
  MView none() {
    MView v;
    std::memset(&v, 0, sizeof v);
    v.base = MB_NONE;
    return v;
  }
  // Quadrant (qi, qj) of an even-sized block, with its valid extent clipped.
  MView quad(const MView& v, int qi, int qj) {
    const int64_t r = v.rows / 2, c = v.cols / 2;
    return view(v.base, v.off + qi * r * v.ld + qj * c, v.ld, r, c, (int64_t)v.vrows - qi * r,
                (int64_t)v.vcols - qj * c);
  }
  MView corner(const MView& v, int64_t rows, int64_t cols) {
    return view(v.base, v.off, v.ld, rows, cols, std::min<int64_t>(v.vrows, rows),
                std::min<int64_t>(v.vcols, cols));
  }
  // Temporaries of at least kGapFrom bytes are kGap bytes apart beyond their
  // 256-byte aligned slots.  Back to back, quarter blocks of 2^k bytes all
  // start at the same offset modulo 2^k, and the passes that stream dozens
  // of them at once (the two-level S/T pass writes 40 blocks per thread
  // position, the U pass reads 49) ran 3 % (S/T) and 6 % (U) slower at
  // n = 8192 than with a 4 KiB gap (gaps of 0.25 to 32 KiB measured: 4 KiB
  // fastest or tied).
  static constexpr int64_t kGap = 4096, kGapFrom = int64_t(1) << 20;
  MView temp(int64_t rows, int64_t cols) {
    const int64_t ld = std::max<int64_t>(round_up(std::max<int64_t>(cols, 1), E), 1);
    const int64_t off = ws_top;
    const int64_t n = round_up(rows * ld, 64);  // 256-byte aligned slots
    ws_top += n + (n * (int64_t)esz >= kGapFrom ? kGap / (int64_t)esz : 0);
    ws_peak = std::max(ws_peak, ws_top);
    return view(MB_WS, off, ld, rows, cols, rows, cols);
  }

  // An R x Kc matrix in the split bfloat16 layout (desc.h) in the workspace.
  MView spl_temp(int64_t R, int64_t Kc) {
    const int64_t nq = std::max<int64_t>((Kc + 7) / 8, 1);
    const int64_t off = ws_top;           // 4-byte units
    ws_top += round_up(R * 12 * nq, 64);  // 48 bytes per chunk
    ws_peak = std::max(ws_peak, ws_top);
    MView v;
    v.base = MB_WS;
    v.off = 2 * off;  // bfloat16 units
    v.ld = 24 * nq;
    v.rows = v.vrows = (int32_t)R;
    v.cols = v.vcols = (int32_t)Kc;
    v.vec = 1;
    return v;
  }

  static std::string vs(const MView& v) {
    std::ostringstream o;
    if (v.base == MB_NONE) return "-";
    o << v.base << ":" << v.off << ":" << v.ld << ":" << v.rows << ":" << v.cols << ":" << v.vrows
      << ":" << v.vcols;
    return o.str();
  }

  // ---- element-wise parts ------------------------------------------------
  void ew_part(int kind, int64_t rows, int64_t cols, std::initializer_list<MView> ins,
               std::initializer_list<MView> outs, int mode0 = 0, int mode1 = 0) {
    ew_parts(kind, rows, cols, std::vector<MView>(ins), std::vector<MView>(outs), mode0, mode1);
  }
  // An element-wise part (blk_start left 0) and its listing line.
  EwPart make_ew(int kind, int64_t rows, int64_t cols, const std::vector<MView>& ins,
                 const std::vector<MView>& outs, int mode0 = 0, int mode1 = 0) {
    EwPart p;
    std::memset(&p, 0, sizeof p);
    p.kind = kind;
    p.rows = (int32_t)rows;
    p.cols = (int32_t)cols;
    p.nin = (int32_t)ins.size();
    p.nout = (int32_t)outs.size();
    p.mode[0] = mode0;
    p.mode[1] = mode1;
    int i = 0;
    for (const auto& v : ins) p.in[i++] = v;
    for (; i < kEwMaxIn; ++i) p.in[i] = none();
    i = 0;
    for (const auto& v : outs) p.out[i++] = v;
    for (; i < kEwMaxOut; ++i) p.out[i] = none();
    return p;
  }
  static std::string ew_line(const EwPart& p) {
    std::ostringstream o;
    o << "EW " << p.kind << " " << p.rows << " " << p.cols << " " << p.mode[0] << " " << p.mode[1] << " |";
    for (int i = 0; i < p.nin; ++i) o << " " << vs(p.in[i]);
    o << " |";
    for (int i = 0; i < p.nout; ++i) o << " " << vs(p.out[i]);
    o << "\n";
    return o.str();
  }
  void ew_parts(int kind, int64_t rows, int64_t cols, const std::vector<MView>& ins,
                const std::vector<MView>& outs, int mode0 = 0, int mode1 = 0) {
    if (!e2.empty() || !gm.empty() || !wl.empty()) flush();
    EwPart p = make_ew(kind, rows, cols, ins, outs, mode0, mode1);
    const int blocks = ew_blocks((int)rows, (int)cols, ew_dtype(P.dtype));
    if (blocks == 0) return;
    p.blk_start = ew_grid;
    ew_grid += blocks;
    ew.push_back(p);
    ew_txt << ew_line(p);
  }

  // A two-level pre- or post-addition pass (desc.h, Ew2Part) over rows x
  // cols lower-level positions; low holds 7 x 4 (S, T) or 7 x 7 (U) views.
  void ew2_part(int kind, int64_t rows, int64_t cols, const MView& x, const MView (&top)[4],
                const std::vector<std::vector<MView>>& low) {
    if (!ew.empty() || !gm.empty() || !wl.empty() || !sp.empty() || !tp.empty() || !bl.empty()) flush();
    Ew2Part p;
    std::memset(&p, 0, sizeof p);
    p.kind = kind;
    p.rows = (int32_t)rows;
    p.cols = (int32_t)cols;
    p.x = kind == EW2_U ? none() : x;
    for (int k = 0; k < 4; ++k) p.top[k] = top[k];
    for (int q = 0; q < 7; ++q)
      for (int i = 0; i < 7; ++i) p.low[q][i] = i < (int)low[q].size() ? low[q][i] : none();
    const int blocks = ew2_blocks((int)rows, (int)cols, ew_dtype(P.dtype));
    if (blocks == 0) return;
    p.blk_start = e2_grid;
    e2_grid += blocks;
    e2.push_back(p);
    txt << "EW2 " << kind << " " << rows << " " << cols << " | " << vs(p.x) << " |";
    for (int k = 0; k < 4; ++k) txt << " " << vs(p.top[k]);
    txt << " |";
    for (int q = 0; q < 7; ++q)
      for (int i = 0; i < (kind == EW2_U ? 7 : 4); ++i) txt << " " << vs(p.low[q][i]);
    txt << "\n";
  }

  // GEMM epilogue outputs
  struct Out {
    MView c;
    int mode;
    int sign;
    MView d;
  };
  static Out store(const MView& c, int sign = 1) { return Out{c, GM_STORE, sign, MView{}}; }
  static Out add(const MView& c, const MView& d, int sign) { return Out{c, GM_ADD, sign, d}; }
  // c = beta c + acc (accumulating plans)
  static Out axpby(const MView& c) { return Out{c, GM_AXPBY, 1, c}; }

  // ---- split passes -------------------------------------------------------
  // rows x cols: the float32 input block; transposed: outputs hold its
  // transpose.
  void split_part(int kind, int64_t rows, int64_t cols, bool transposed, std::initializer_list<MView> ins,
                  std::initializer_list<MView> outs) {
    if (!e2.empty() || !ew.empty() || !gm.empty() || !wl.empty()) flush();
    EwPart p;
    std::memset(&p, 0, sizeof p);
    p.kind = kind;
    p.rows = (int32_t)rows;
    p.cols = (int32_t)cols;
    p.nin = (int32_t)ins.size();
    p.nout = (int32_t)outs.size();
    p.mode[0] = transposed ? 1 : 0;
    int i = 0;
    for (const auto& v : ins) p.in[i++] = v;
    for (; i < kEwMaxIn; ++i) p.in[i] = none();
    i = 0;
    for (const auto& v : outs) p.out[i++] = v;
    for (; i < kEwMaxOut; ++i) p.out[i] = none();
    const int blocks = split_blocks((int)rows, (int)cols, transposed ? 1 : 0);
    if (blocks == 0) return;
    p.blk_start = sp_grid;
    sp_grid += blocks;
    sp.push_back(p);
    txt << "SPLIT " << kind << " " << rows << " " << cols << " " << p.mode[0] << " |";
    for (const auto& v : ins) txt << " " << vs(v);
    txt << " |";
    for (const auto& v : outs) txt << " " << vs(v);
    txt << "\n";
  }

  // Leaf product c = a b of order s (1, 2 or 4) by the unrolled base case.
  void base(const MView& a, const MView& bop, const MView& c, int s) {
    if (!e2.empty() || !ew.empty() || !gm.empty() || !wl.empty() || !sp.empty() || !tp.empty() ||
        (!bl.empty() && bl_order != s))
      flush();
    bl_order = s;
    P.leaves += 1;
    bl.push_back(BaseDesc{a, bop, c});
    txt << "BASE " << s << " | " << vs(a) << " " << vs(bop) << " " << vs(c) << "\n";
  }

  // A transposing pass over rows x cols inputs; every output is a cols x rows
  // workspace block holding the transpose of the recipe's result.
  void trans_part(int kind, int64_t rows, int64_t cols, std::initializer_list<MView> ins,
                  std::initializer_list<MView> outs) {
    if (!e2.empty() || !gm.empty() || !wl.empty() || !sp.empty()) flush();
    EwPart p;
    std::memset(&p, 0, sizeof p);
    p.kind = kind;
    p.rows = (int32_t)rows;
    p.cols = (int32_t)cols;
    p.nin = (int32_t)ins.size();
    p.nout = (int32_t)outs.size();
    int i = 0;
    for (const auto& v : ins) p.in[i++] = v;
    for (; i < kEwMaxIn; ++i) p.in[i] = none();
    i = 0;
    for (const auto& v : outs) p.out[i++] = v;
    for (; i < kEwMaxOut; ++i) p.out[i] = none();
    const int blocks = trans_blocks((int)rows, (int)cols);
    if (blocks == 0) return;
    p.blk_start = tp_grid;
    tp_grid += blocks;
    tp.push_back(p);
    tp_txt << "TRANS " << kind << " " << rows << " " << cols << " |";
    for (const auto& v : ins) tp_txt << " " << vs(v);
    tp_txt << " |";
    for (const auto& v : outs) tp_txt << " " << vs(v);
    tp_txt << "\n";
  }

  // C = a b^T-stored: a is an m x k SPL matrix, bt the n x k SPL transpose of
  // the B operand.
  void gemm_spl(const MView& a, const MView& bt, std::initializer_list<Out> outs) {
    if (!e2.empty() || !ew.empty() || !sp.empty() || (!gm.empty() && !gm_spl)) flush();
    gm_spl = true;
    GemmDesc g;
    std::memset(&g, 0, sizeof g);
    g.a = a;
    g.b = bt;
    g.m = a.rows;
    g.k = a.cols;
    g.n = bt.rows;
    g.nout = (int32_t)outs.size();
    int i = 0;
    for (const auto& o : outs) {
      g.out[i].c = o.c;
      g.out[i].mode = o.mode;
      g.out[i].sign = o.sign;
      g.out[i].d = (o.mode == GM_ADD || o.mode == GM_AXPBY) ? o.d : none();
      ++i;
    }
    for (; i < 2; ++i) {
      g.out[i].c = none();
      g.out[i].d = none();
      g.out[i].mode = GM_NONE;
      g.out[i].sign = 1;
    }
    P.leaves += 1;
    if (g.m == 0 || g.n == 0) return;
    gm.push_back(g);
    gm_fusable.push_back(0);
  }

  // ---- leaf products -------------------------------------------------------

  // akind / bkind != OK_PLAIN: a / b is the parent block and the operand is
  // the Winograd sum of its quadrants (formed in the loader).
  // A leaf-product descriptor (tiles left 0), as gemm() records it.
  GemmDesc make_gemm(const MView& a, const MView& b, std::initializer_list<Out> outs) {
    GemmDesc g;
    std::memset(&g, 0, sizeof g);
    g.a = a;
    g.b = b;
    g.m = a.rows;
    g.k = a.cols;
    g.n = b.cols;
    g.nout = (int32_t)outs.size();
    int i = 0;
    for (const auto& o : outs) {
      g.out[i].c = o.c;
      g.out[i].mode = o.mode;
      g.out[i].sign = o.sign;
      g.out[i].d = (o.mode == GM_ADD || o.mode == GM_AXPBY) ? o.d : none();
      ++i;
    }
    for (; i < 2; ++i) {
      g.out[i].c = none();
      g.out[i].d = none();
      g.out[i].mode = GM_NONE;
      g.out[i].sign = 1;
    }
    return g;
  }
  static std::string gemm_line(const GemmDesc& g) {
    std::ostringstream o;
    o << "GEMM " << g.m << " " << g.n << " " << g.k << " " << (g.kinds & 0xff) << " " << (g.kinds >> 8) << " | "
      << vs(g.a) << " " << vs(g.b) << " |";
    for (int j = 0; j < g.nout; ++j)
      o << " " << g.out[j].mode << ":" << g.out[j].sign << ":" << vs(g.out[j].c) << ":" << vs(g.out[j].d);
    o << "\n";
    return o.str();
  }

  void gemm(const MView& a, const MView& b, std::initializer_list<Out> outs, int akind = OK_PLAIN,
            int bkind = OK_PLAIN, bool fusable = false) {
    if (!e2.empty() || !ew.empty() || !sp.empty() || gm_spl) flush();
    GemmDesc g;
    std::memset(&g, 0, sizeof g);
    g.a = a;
    g.b = b;
    g.m = akind == OK_PLAIN ? a.rows : a.rows / 2;
    g.k = akind == OK_PLAIN ? a.cols : a.cols / 2;
    g.n = bkind == OK_PLAIN ? b.cols : (bkind == OK_TRANS ? b.rows : b.cols / 2);
    g.kinds = akind | (bkind << 8);
    g.nout = (int32_t)outs.size();
    int i = 0;
    for (const auto& o : outs) {
      g.out[i].c = o.c;
      g.out[i].mode = o.mode;
      g.out[i].sign = o.sign;
      g.out[i].d = (o.mode == GM_ADD || o.mode == GM_AXPBY) ? o.d : none();
      ++i;
    }
    for (; i < 2; ++i) {
      g.out[i].c = none();
      g.out[i].d = none();
      g.out[i].mode = GM_NONE;
      g.out[i].sign = 1;
    }
    P.leaves += 1;
    if (g.m == 0 || g.n == 0) return;
    gm.push_back(g);
    gm_fusable.push_back(fusable ? 1 : 0);
  }

  // Close the current launch.
  // Start / end a section in which launches on the auxiliary stream run
  // concurrently with launches on the main stream.
  void fork() {
    flush();
    P.ops.push_back(OpRec{OP_FORK, 0, 0, 0, 0, 0, 0, 0, 0});
    txt << "FORK\n";
  }
  // Some launch since the last fork runs on the auxiliary stream.
  bool window_has_aux() const {
    for (size_t f = P.ops.size(); f > 0 && P.ops[f - 1].type != OP_FORK; --f)
      if (P.ops[f - 1].stream) return true;
    return false;
  }
  void join() {
    flush();
    if (!window_has_aux()) {
      size_t f = P.ops.size();
      while (P.ops[f - 1].type != OP_FORK) --f;
      // nothing runs on the auxiliary stream: drop the fork
      P.ops.erase(P.ops.begin() + (f - 1));
      std::string t = txt.str();
      const size_t at = t.rfind("FORK\n");
      t.erase(at, 5);
      txt.str(t);
      txt.seekp(0, std::ios_base::end);
      return;
    }
    P.ops.push_back(OpRec{OP_JOIN, 0, 0, 0, 0, 0, 0, 0, 0});
    P.has_aux = true;
    txt << "JOIN\n";
  }

  // One last-level Winograd subproblem C = A B: operands of P1 .. P7 (with
  // fused, the parent blocks A, B in place of S1..S4, T1..T4, whose sums the
  // loader forms) and the output quadrants.
  void wino(const MView (&a)[7], const MView (&bop)[7], const MView (&c)[4], int64_t m, int64_t n, int64_t k,
            bool acc = false, bool fused = false) {
    if (!e2.empty() || !ew.empty() || !gm.empty() || (!wl.empty() && wl_fused != fused)) flush();
    wl_fused = fused;
    WinoLeafDesc d;
    std::memset(&d, 0, sizeof d);
    for (int i = 0; i < 7; ++i) {
      d.a[i] = a[i];
      d.b[i] = bop[i];
    }
    for (int i = 0; i < 4; ++i) d.c[i] = c[i];
    d.m = (int32_t)m;
    d.n = (int32_t)n;
    d.k = (int32_t)k;
    d.acc = acc ? 1 : 0;
    P.leaves += 7;
    if (m == 0 || n == 0) return;
    wl.push_back(d);
  }

  void flush() {
    if (!e2.empty()) {
      OpRec r{OP_EW2, ew_dtype(P.dtype), P.table.size(), (int)e2.size(), e2_grid, 0, 0, 0, cur_stream};
      const size_t bytes = e2.size() * sizeof(Ew2Part);
      P.table.resize(round_up(P.table.size() + bytes, 256));
      std::memcpy(P.table.data() + r.off, e2.data(), bytes);
      P.ops.push_back(r);
      txt << "LAUNCH EW2 " << e2.size() << " " << e2_grid << (cur_stream ? " aux" : "") << "\n";
      e2.clear();
      e2_grid = 0;
    }
    if (!wl.empty()) emit_wino();
    if (!bl.empty()) {
      const int blocks = base_blocks((int)bl.size());
      OpRec r{OP_BASE, kernel_dtype(P.dtype), P.table.size(), (int)bl.size(), blocks, bl_order, 0, 0, cur_stream};
      const size_t bytes = bl.size() * sizeof(BaseDesc);
      P.table.resize(round_up(P.table.size() + bytes, 256));
      std::memcpy(P.table.data() + r.off, bl.data(), bytes);
      P.ops.push_back(r);
      txt << "LAUNCH BASE " << bl.size() << " " << blocks << " " << bl_order << (cur_stream ? " aux" : "") << "\n";
      bl.clear();
    }
    if (!sp.empty()) {
      OpRec r{OP_SPLIT, DT_BF16X3_SPL, P.table.size(), (int)sp.size(), sp_grid, 0, 0, 0, cur_stream};
      const size_t bytes = sp.size() * sizeof(EwPart);
      P.table.resize(round_up(P.table.size() + bytes, 256));
      std::memcpy(P.table.data() + r.off, sp.data(), bytes);
      P.ops.push_back(r);
      txt << "LAUNCH SPLIT " << sp.size() << " " << sp_grid << (cur_stream ? " aux" : "") << "\n";
      sp.clear();
      sp_grid = 0;
    }
    if (!ew.empty()) {
      OpRec r{OP_EW, ew_dtype(P.dtype), P.table.size(), (int)ew.size(), ew_grid, 0, 0, 0, cur_stream};
      const size_t bytes = ew.size() * sizeof(EwPart);
      P.table.resize(round_up(P.table.size() + bytes, 256));
      std::memcpy(P.table.data() + r.off, ew.data(), bytes);
      P.ops.push_back(r);
      txt << ew_txt.str();
      ew_txt.str("");
      txt << "LAUNCH EW " << ew.size() << " " << ew_grid << (cur_stream ? " aux" : "") << "\n";
      ew.clear();
      ew_grid = 0;
    }
    if (!tp.empty()) {
      OpRec r{OP_TRANS, DT_F32, P.table.size(), (int)tp.size(), tp_grid, 0, 0, 0, cur_stream};
      const size_t bytes = tp.size() * sizeof(EwPart);
      P.table.resize(round_up(P.table.size() + bytes, 256));
      std::memcpy(P.table.data() + r.off, tp.data(), bytes);
      P.ops.push_back(r);
      txt << tp_txt.str();
      tp_txt.str("");
      txt << "LAUNCH TRANS " << tp.size() << " " << tp_grid << (cur_stream ? " aux" : "") << "\n";
      tp.clear();
      tp_grid = 0;
    }
    if (!gm.empty()) {
      // Products with operand sums (and the plain products of the same
      // blocks) run in the fused kernel, products whose B is stored
      // transposed in the transposed-B kernel, everything else in the
      // regular one.
      auto sums = [](const GemmDesc& g) {
        const int ak = g.kinds & 0xff, bk = g.kinds >> 8;
        return (ak >= OK_S1 && ak <= OK_S4) || (bk >= OK_T1 && bk <= OK_T4);
      };
      bool any_fused = false, any_bt = false;
      for (const GemmDesc& g : gm) {
        any_fused = any_fused || sums(g);
        any_bt = any_bt || (g.kinds >> 8) == OK_TRANS;
      }
      if (any_fused) {
        std::vector<GemmDesc> f, r;
        for (size_t i = 0; i < gm.size(); ++i) (gm_fusable[i] ? f : r).push_back(gm[i]);
        gm.clear();
        gm_fusable.clear();
        emit_gemm(f, true);
        emit_gemm(r, false);
      } else if (any_bt) {
        std::vector<GemmDesc> t, r;
        for (const GemmDesc& g : gm) ((g.kinds >> 8) == OK_TRANS ? t : r).push_back(g);
        gm.clear();
        gm_fusable.clear();
        emit_gemm(t, false, true);
        emit_gemm(r, false);
      } else {
        emit_gemm(gm, false);
        gm.clear();
        gm_fusable.clear();
      }
      gm_grid = 0;
      gm_spl = false;
    }
  }

  void emit_wino() {
    int cfg = P.tile_cfg;
    if (cfg < 0) {
      int64_t t128 = 0;
      for (const WinoLeafDesc& d : wl) t128 += ceil_div(d.m, 128) * ceil_div(d.n, 128);
      cfg = t128 >= 256 ? 1 : 2;
    }
    const GemmCfg gc = gemm_wino_cfg(cfg);
    int grid = 0;
    for (WinoLeafDesc& d : wl) {
      d.tiles_m = (int32_t)ceil_div(d.m, gc.bm);
      d.tiles_n = (int32_t)ceil_div(d.n, gc.bn);
      d.tile_start = grid;
      grid += d.tiles_m * d.tiles_n;
      txt << "WINO " << d.m << " " << d.n << " " << d.k << " " << d.acc << " " << (wl_fused ? 1 : 0) << " |";
      for (int i = 0; i < 7; ++i) txt << " " << vs(d.a[i]) << " " << vs(d.b[i]);
      txt << " |";
      for (int i = 0; i < 4; ++i) txt << " " << vs(d.c[i]);
      txt << "\n";
    }
    OpRec r{OP_WINO, kernel_dtype(P.dtype), P.table.size(), (int)wl.size(), grid, cfg, 1, wl_fused ? 1 : 0,
            cur_stream};
    const size_t bytes = wl.size() * sizeof(WinoLeafDesc);
    P.table.resize(round_up(P.table.size() + bytes, 256));
    std::memcpy(P.table.data() + r.off, wl.data(), bytes);
    P.ops.push_back(r);
    txt << "LAUNCH WINO " << wl.size() << " " << grid << " " << cfg << (cur_stream ? " aux" : "") << "\n";
    wl.clear();
    P.wino = true;
    if (wl_fused) P.fused = true;
  }

  void emit_gemm(std::vector<GemmDesc>& group, bool fused, bool bt = false) {
    if (group.empty()) return;
    const int kd = gm_spl ? DT_BF16X3_SPL : (bt ? DT_F32_BT : kernel_dtype(P.dtype));
    // Unequal problems: longest (largest k) first, round-robin over XCDs.
    bool equal = true;
    for (const GemmDesc& g : group)
      equal = equal && g.m == group[0].m && g.n == group[0].n && g.k == group[0].k;
    if (!equal)
      std::stable_sort(group.begin(), group.end(), [](const GemmDesc& x, const GemmDesc& y) { return x.k > y.k; });
    int cfg = P.tile_cfg >= 0 ? P.tile_cfg : choose_gemm_cfg(kd, group);
    // the fused kernel has 256x256, 128x128 and 64x128 tiles; its 128x128
    // tile runs one wave per SIMD, so 64x128 is the default below 256x256
    if (fused && cfg != 3 && (cfg != 0 || P.tile_cfg < 0)) cfg = 4;
    if (P.tile_cfg < 0 && equal && !fused && (kd == DT_F32 || kd == DT_F32_BT) && (cfg == 0 || cfg == 3)) {
      const int p3 = split_for_rounds(group, 0.87, 0.84);
      if (p3 > 0 && p3 < (int)group.size()) {
        std::vector<GemmDesc> big(group.begin(), group.begin() + p3), small(group.begin() + p3, group.end());
        emit_gemm_cfg(big, false, 3, true, kd);
        emit_gemm_cfg(small, false, 0, true, kd);
        return;
      }
    }
    if (P.tile_cfg < 0 && equal && kd == DT_BF16X3 && cfg == 6) {
      // split-bfloat16: the 256x256 and 128x128 ring tiles (measured MFMA
      // fractions 0.53 to 0.56 and about 0.47)
      const int p6 = split_for_rounds(group, 0.55, 0.47, 2);
      if (p6 > 0 && p6 < (int)group.size()) {
        std::vector<GemmDesc> big(group.begin(), group.begin() + p6), small(group.begin() + p6, group.end());
        emit_gemm_cfg(big, false, 6, true, kd);
        emit_gemm_cfg(small, false, 0, true, kd);
        return;
      }
    }
    emit_gemm_cfg(group, fused, cfg, equal, kd);
  }

  // Equal problems on the large tiles: how many of them to give 256x256
  // tiles (one workgroup per CU), the rest 128x128 (w128 workgroups per CU:
  // float32 1, the split-bfloat16 ring 2), so that both launches fill whole
  // rounds.  Time model per problem class: rounds x tile work / measured
  // tile efficiency (e256 for 256x256, e128 for 128x128; float32: 0.87 and
  // 0.84), w128 tiles sharing a CU taking w128 times as long.  Returns the
  // count, or -1 when one tile shape for all is as good.
  static int split_for_rounds(const std::vector<GemmDesc>& group, double e256, double e128, int64_t w128 = 1) {
    const int64_t P = (int64_t)group.size();
    const int64_t m = group[0].m, n = group[0].n;
    const int64_t T3 = ceil_div(m, 256) * ceil_div(n, 256), T0 = ceil_div(m, 128) * ceil_div(n, 128);
    const double t3 = 256.0 * 256.0 / e256, t0 = 128.0 * 128.0 / e128;
    auto cost = [&](int64_t p) {
      return (double)ceil_div(p * T3, 256) * t3 + (double)ceil_div((P - p) * T0, 256 * w128) * t0 * (double)w128;
    };
    // (with w128 > 1 ties go to more 256x256 tiles: a partial round of
    // 128x128 tiles runs fewer workgroups per CU, faster than modelled)
    int64_t best = -1;
    double best_cost = 0.99 * std::min(cost(0), cost(P));
    for (int64_t i = 1; i < P; ++i) {
      const int64_t p = w128 > 1 ? P - i : i;
      if (cost(p) < best_cost) {
        best_cost = cost(p);
        best = p;
      }
    }
    return (int)best;
  }

  void emit_gemm_cfg(std::vector<GemmDesc>& group, bool fused, int cfg, bool equal, int kd) {
    const GemmCfg gc = gemm_cfg(kd, cfg);
    int grid = 0;
    for (GemmDesc& g : group) {
      g.tiles_m = (int32_t)ceil_div(g.m, gc.bm);
      g.tiles_n = (int32_t)ceil_div(g.n, gc.bn);
      g.tile_start = grid;
      grid += g.tiles_m * g.tiles_n;
    }
    for (const GemmDesc& g : group) txt << gemm_line(g);
    OpRec r{OP_GEMM, kd, P.table.size(), (int)group.size(), grid, cfg, equal ? 1 : 0, fused ? 1 : 0, cur_stream};
    const size_t bytes = group.size() * sizeof(GemmDesc);
    P.table.resize(round_up(P.table.size() + bytes, 256));
    std::memcpy(P.table.data() + r.off, group.data(), bytes);
    P.ops.push_back(r);
    txt << "LAUNCH GEMM " << group.size() << " " << grid << " " << cfg << (fused ? " fused" : "")
        << (gm_spl ? " spl" : "") << (kd == DT_F32_BT ? " bt" : "") << (cur_stream ? " aux" : "") << "\n";
    if (fused) P.fused = true;
  }
};

// ---------------------------------------------------------------------------
// Schedules
// ---------------------------------------------------------------------------

// Section 3.3, Table 2 (Two Temp Winograd), depth first.  C = A B.
void sched_two_temp(Builder& b, const MView& A, const MView& B, const MView& C, int depth) {
  const int L = b.P.L;
  if (depth == L) {
    b.gemm(A, B, {Builder::store(C)});
    b.flush();
    return;
  }
  const int64_t hm = A.rows / 2, hk = A.cols / 2, hn = B.cols / 2;
  const MView A11 = b.quad(A, 0, 0), A12 = b.quad(A, 0, 1), A21 = b.quad(A, 1, 0), A22 = b.quad(A, 1, 1);
  const MView B11 = b.quad(B, 0, 0), B12 = b.quad(B, 0, 1), B21 = b.quad(B, 1, 0), B22 = b.quad(B, 1, 1);
  const MView C11 = b.quad(C, 0, 0), C12 = b.quad(C, 0, 1), C21 = b.quad(C, 1, 0), C22 = b.quad(C, 1, 1);
  const int64_t mark = b.ws_top;
  const MView X = b.temp(hm, std::max(hk, hn));
  const MView Y = b.temp(hk, hn);
  const MView XS = b.corner(X, hm, hk), XP = b.corner(X, hm, hn);
  const bool leaf = depth + 1 == L;
  // 1, 2: S3 = A11 - A21 -> X ; T3 = B22 - B12 -> Y
  b.ew_part(EW_SUB, hm, hk, {A11, A21}, {XS});
  b.ew_part(EW_SUB, hk, hn, {B22, B12}, {Y});
  b.flush();
  // 3: P7 = S3 T3 -> C21
  sched_two_temp(b, XS, Y, C21, depth + 1);
  // 4, 5: S1 = A21 + A22 -> X ; T1 = B12 - B11 -> Y
  b.ew_part(EW_ADD, hm, hk, {A21, A22}, {XS});
  b.ew_part(EW_SUB, hk, hn, {B12, B11}, {Y});
  b.flush();
  // 6: P5 = S1 T1 -> C22
  sched_two_temp(b, XS, Y, C22, depth + 1);
  // 7, 8: S2 = S1 - A11 -> X ; T2 = B22 - T1 -> Y
  b.ew_part(EW_SUB, hm, hk, {XS, A11}, {XS});
  b.ew_part(EW_SUB, hk, hn, {B22, Y}, {Y});
  b.flush();
  // 9: P6 = S2 T2 -> C12
  sched_two_temp(b, XS, Y, C12, depth + 1);
  // 10: S4 = A12 - S2 -> X
  b.ew_part(EW_SUB, hm, hk, {A12, XS}, {XS});
  b.flush();
  // 11: P3 = S4 B22 -> C11
  sched_two_temp(b, XS, B22, C11, depth + 1);
  // 12: P1 = A11 B11 -> X
  sched_two_temp(b, A11, B11, XP, depth + 1);
  // 13-17: U2, U3, U4, U7, U5 (fused; same per-element order) ; 18: T4 = T2 - B21 -> Y
  b.ew_part(EW_TT_U, hm, hn, {XP, C11, C12, C21, C22}, {C12, C21, C22});
  b.ew_part(EW_SUB, hk, hn, {Y, B21}, {Y});
  b.flush();
  // 19, 20: P4 = A22 T4 -> C11 ; U6 = U3 - P4 -> C21
  if (leaf) {
    b.gemm(A22, Y, {Builder::add(C21, C21, -1)});
    b.flush();
  } else {
    sched_two_temp(b, A22, Y, C11, depth + 1);
    b.ew_part(EW_SUB, hm, hn, {C21, C11}, {C21});
    b.flush();
  }
  // 21, 22: P2 = A12 B21 -> C11 ; U1 = P1 + P2 -> C11
  if (leaf) {
    b.gemm(A12, B21, {Builder::add(C11, XP, +1)});
    b.flush();
  } else {
    sched_two_temp(b, A12, B21, C11, depth + 1);
    b.ew_part(EW_ADD, hm, hn, {XP, C11}, {C11});
    b.flush();
  }
  b.flush();
  b.ws_top = mark;
}

// Section 3.3, Table 3 (In-Place Winograd), depth first.  C = A B; A and B
// are overwritten.  Needs k == n <= m (slot sizes).
void sched_in_place(Builder& b, const MView& A, const MView& B, const MView& C, int depth) {
  const int L = b.P.L;
  if (depth == L) {
    b.gemm(A, B, {Builder::store(C)});
    b.flush();
    return;
  }
  const int64_t hm = A.rows / 2, hk = A.cols / 2, hn = B.cols / 2;
  const MView A11 = b.quad(A, 0, 0), A12 = b.quad(A, 0, 1), A21 = b.quad(A, 1, 0), A22 = b.quad(A, 1, 1);
  const MView B11 = b.quad(B, 0, 0), B12 = b.quad(B, 0, 1), B21 = b.quad(B, 1, 0), B22 = b.quad(B, 1, 1);
  const MView C11 = b.quad(C, 0, 0), C12 = b.quad(C, 0, 1), C21 = b.quad(C, 1, 0), C22 = b.quad(C, 1, 1);
  const MView S3 = b.corner(C11, hm, hk), T1 = b.corner(C22, hk, hn), S2 = b.corner(C12, hm, hk);
  const MView T4 = b.corner(C22, hk, hn);
  const MView P5 = b.corner(A11, hm, hn), P4 = b.corner(A21, hm, hn), P3 = b.corner(A12, hm, hn);
  const bool leaf = depth + 1 == L;
  // 1-4: S3 -> C11, S1 -> A21, T1 -> C22, T3 -> B12
  b.ew_part(EW_IP_A, hm, hk, {A11, A21, A22}, {S3, A21});
  b.ew_part(EW_IP_B, hk, hn, {B11, B12, B22}, {T1, B12});
  b.flush();
  // 5: P7 = S3 T3 -> C21
  sched_in_place(b, S3, B12, C21, depth + 1);
  // 6: S2 = S1 - A11 -> C12
  b.ew_part(EW_SUB, hm, hk, {A21, A11}, {S2});
  b.flush();
  // 7: P1 = A11 B11 -> C11
  sched_in_place(b, A11, B11, C11, depth + 1);
  // 8: T2 = B22 - T1 -> B11
  b.ew_part(EW_SUB, hk, hn, {B22, T1}, {B11});
  b.flush();
  // 9: P5 = S1 T1 -> A11
  sched_in_place(b, A21, T1, P5, depth + 1);
  // 10: T4 = T2 - B21 -> C22
  b.ew_part(EW_SUB, hk, hn, {B11, B21}, {T4});
  b.flush();
  // 11: P4 = A22 T4 -> A21
  sched_in_place(b, A22, T4, P4, depth + 1);
  // 12: S4 = A12 - S2 -> A22
  b.ew_part(EW_SUB, hm, hk, {A12, S2}, {A22});
  b.flush();
  // 13, 14: P6 = S2 T2 -> C22 ; U2 = P1 + P6 -> C22
  if (leaf) {
    b.gemm(S2, B11, {Builder::add(C22, C11, +1)});
    b.flush();
  } else {
    sched_in_place(b, S2, B11, C22, depth + 1);
    b.ew_part(EW_ADD, hm, hn, {C11, C22}, {C22});
    b.flush();
  }
  // 15: P2 = A12 B21 -> C12
  sched_in_place(b, A12, B21, C12, depth + 1);
  // 16-20: U1 -> C11, U4 -> C12, U3, U6 -> C21, U7 -> C22 (fused)
  b.ew_part(EW_IP_U, hm, hn, {C11, C12, C22, P5, C21, P4}, {C11, C12, C21, C22});
  b.flush();
  // 21, 22: P3 = S4 B22 -> A12 ; U5 = U4 + P3 -> C12
  if (leaf) {
    b.gemm(A22, B22, {Builder::add(C12, C12, +1)});
    b.flush();
  } else {
    sched_in_place(b, A22, B22, P3, depth + 1);
    b.ew_part(EW_ADD, hm, hn, {C12, P3}, {C12});
    b.flush();
  }
}

// Strassen (Section 2.2), depth first with three temporaries.  The products
// are taken in the order P1, P3, P2, P4, P5, P6, P7 so that every C quadrant
// is accumulated left to right exactly as the paper writes it:
// C11 = ((P1 + P4) - P5) + P7, C12 = P3 + P5, C21 = P2 + P4,
// C22 = ((P1 + P3) - P2) + P6.
void sched_strassen(Builder& b, const MView& A, const MView& B, const MView& C, int depth) {
  const int L = b.P.L;
  if (depth == L) {
    b.gemm(A, B, {Builder::store(C)});
    b.flush();
    return;
  }
  const int64_t hm = A.rows / 2, hk = A.cols / 2, hn = B.cols / 2;
  const MView A11 = b.quad(A, 0, 0), A12 = b.quad(A, 0, 1), A21 = b.quad(A, 1, 0), A22 = b.quad(A, 1, 1);
  const MView B11 = b.quad(B, 0, 0), B12 = b.quad(B, 0, 1), B21 = b.quad(B, 1, 0), B22 = b.quad(B, 1, 1);
  const MView C11 = b.quad(C, 0, 0), C12 = b.quad(C, 0, 1), C21 = b.quad(C, 1, 0), C22 = b.quad(C, 1, 1);
  const int64_t mark = b.ws_top;
  const MView X = b.temp(hm, hk);
  const MView Y = b.temp(hk, hn);
  const bool leaf = depth + 1 == L;
  const MView Z = leaf ? b.none() : b.temp(hm, hn);
  // mode: 1 = store, 2 = add, 3 = subtract
  auto product = [&](const MView& Aop, const MView& Bop, const MView& D0, int m0, const MView* D1, int m1) {
    if (leaf) {
      auto out = [&](const MView& d, int md) {
        return md == 1 ? Builder::store(d) : Builder::add(d, d, md == 2 ? +1 : -1);
      };
      if (D1)
        b.gemm(Aop, Bop, {out(D0, m0), out(*D1, m1)});
      else
        b.gemm(Aop, Bop, {out(D0, m0)});
      b.flush();
    } else {
      sched_strassen(b, Aop, Bop, Z, depth + 1);
      if (D1)
        b.ew_part(EW_DIST, hm, hn, {Z, D0, *D1}, {D0, *D1}, m0, m1);
      else
        b.ew_part(EW_DIST, hm, hn, {Z, D0, b.none()}, {D0}, m0, 0);
      b.flush();
    }
  };
  // P1 = (A11 + A22)(B11 + B22): C11 = P1, C22 = P1
  b.ew_part(EW_ADD, hm, hk, {A11, A22}, {X});
  b.ew_part(EW_ADD, hk, hn, {B11, B22}, {Y});
  b.flush();
  product(X, Y, C11, 1, &C22, 1);
  // P3 = A11 (B12 - B22): C12 = P3, C22 += P3
  b.ew_part(EW_SUB, hk, hn, {B12, B22}, {Y});
  b.flush();
  product(A11, Y, C12, 1, &C22, 2);
  // P2 = (A21 + A22) B11: C21 = P2, C22 -= P2
  b.ew_part(EW_ADD, hm, hk, {A21, A22}, {X});
  b.flush();
  product(X, B11, C21, 1, &C22, 3);
  // P4 = A22 (-B11 + B21): C11 += P4, C21 += P4
  b.ew_part(EW_SUB, hk, hn, {B21, B11}, {Y});
  b.flush();
  product(A22, Y, C11, 2, &C21, 2);
  // P5 = (A11 + A12) B22: C11 -= P5, C12 += P5
  b.ew_part(EW_ADD, hm, hk, {A11, A12}, {X});
  b.flush();
  product(X, B22, C11, 3, &C12, 2);
  // P6 = (-A11 + A21)(B11 + B12): C22 += P6
  b.ew_part(EW_SUB, hm, hk, {A21, A11}, {X});
  b.ew_part(EW_ADD, hk, hn, {B11, B12}, {Y});
  b.flush();
  product(X, Y, C22, 2, nullptr, 0);
  // P7 = (A12 - A22)(B21 + B22): C11 += P7
  b.ew_part(EW_SUB, hm, hk, {A12, A22}, {X});
  b.ew_part(EW_ADD, hk, hn, {B21, B22}, {Y});
  b.flush();
  product(X, Y, C11, 2, nullptr, 0);
  b.ws_top = mark;
}

// Breadth-first Winograd (the 22-operation form of Section 2.3 evaluated
// level by level): one launch forms S1..S4 and T1..T4 for every block of a
// level, one grouped launch runs all 7^L leaf products, and one launch per
// level forms U1, U5, U6, U7 into the C quadrants.  Per element the
// operations and their order are those of the block form, so the result is
// bitwise the same as the depth-first schedules with the same leaf kernel.
struct Sub {
  MView A, B, C;
  int akind = OK_PLAIN, bkind = OK_PLAIN;
  bool fusable = false;  // meets the fused loader's preconditions (aligned, fully valid)
  bool spl = false;      // A is an SPL matrix, B the SPL transpose of the B operand
};

// The last level's S/T sums can be formed in the leaf loader when both
// operand blocks are float32, entirely valid (no virtual padding) and every
// quadrant starts on a 16-byte boundary.
bool can_fuse(const Builder& b, const Sub& s) {
  if (!b.P.fuse || b.P.dtype != MM_F32) return false;
  const MView& A = s.A;
  const MView& B = s.B;
  if (A.vrows != A.rows || A.vcols != A.cols || B.vrows != B.rows || B.vcols != B.cols) return false;
  if (!A.vec || !B.vec) return false;
  if ((A.cols / 2) % b.E || (B.cols / 2) % b.E || A.rows < 2 || A.cols < 2 || B.cols < 2) return false;
  return true;
}

// With Strassen's algorithm (Section 2.2) the same level-by-level form
// applies: one launch per level forms the five A sums and five B sums of
// every block, the 7^L leaf products run as one grouped launch, and one launch
// per level forms the four C quadrants from P1..P7.  The sums and the order in
// which the products are combined are those of the depth-first Strassen
// schedule, so the two give the same bits.  The options that are particular
// to Winograd's operands (fused loader, leaf-side U, split pass, overlap of
// plain-operand products) do not apply and are ignored.
void sched_grouped(Builder& b, std::vector<Sub> subs) {
  const int L = b.P.L;
  const bool strassen = b.P.algo == MM_ALGO_STRASSEN;
  std::vector<std::vector<EwPart>> u_levels;  // recorded, emitted in reverse
  struct WinoSub {
    MView a[7], b[7], c[4];
    int64_t m, n, k;
    bool acc;
    bool fused;
  };
  std::vector<WinoSub> wl_pending;  // last-level subproblems (leaf_u)
  // The S/T passes run on the auxiliary stream while the leaf products whose
  // operands are plain blocks of A and B (P1 = A11 B11, P2 = A12 B21 at the
  // top level, and their counterparts below) run on the main stream.
  const bool leaf_u = b.P.leaf_u && L >= 1 && !strassen;
  const bool overlap_req = b.P.overlap && L >= 1 && !leaf_u && !b.P.spl && !strassen;
  if (overlap_req) {
    b.fork();
    b.cur_stream = 1;
  }
  // Pairs of levels (l, l + 1) whose pre-additions run as one two-level pass
  // (and post-additions too, except at the top of an accumulating plan):
  // the default form at both levels, every block entirely valid, sizes that
  // split into whole 16-byte chunks at the lower level (ew2.hip).
  const bool pairs_allowed = !strassen && !leaf_u && !b.P.spl && !b.P.trans_b && !b.P.fuse && !b.P.level_passes;
  auto pair_ok = [&](const std::vector<Sub>& v) {
    if (v.empty()) return false;
    for (const Sub& s : v) {
      const MView &A = s.A, &B = s.B, &C = s.C;
      if (s.akind != OK_PLAIN || s.bkind != OK_PLAIN || s.spl) return false;
      if (A.vrows != A.rows || A.vcols != A.cols || B.vrows != B.rows || B.vcols != B.cols ||
          C.vrows != C.rows || C.vcols != C.cols)
        return false;
      if (A.rows % 4 || A.cols % 4 || B.cols % 4 || (A.cols / 4) % b.E || (B.cols / 4) % b.E) return false;
    }
    return true;
  };
  std::vector<char> pair_top(std::max(L, 1), 0), upair_top(std::max(L, 1), 0);
  // upper level of a pair: its sums, kept for the pass that forms both levels
  std::vector<std::array<MView, 4>> up_s, up_t, lo_s, lo_t;
  std::vector<std::pair<MView, MView>> up_x;
  for (int l = 0; l < L; ++l) {
    const bool fuse_low = l > 0 && pair_top[l - 1];
    const bool fuse_top = pairs_allowed && !fuse_low && l + 1 < L && pair_ok(subs);
    pair_top[l] = fuse_top;
    upair_top[l] = fuse_top && !(l == 0 && b.P.accumulate);
    std::vector<Sub> next;
    next.reserve(subs.size() * 7);
    std::vector<std::array<MView, 11>> uargs;
    // fused last level with MM_PLAN_FUSE: no temporaries at all (every
    // subproblem must meet the fused loader's preconditions)
    bool leaf_fused = leaf_u && l == L - 1 && b.P.fuse;
    for (const Sub& s : subs) leaf_fused = leaf_fused && can_fuse(b, s);
    for (const Sub& s : subs) {
      const int64_t hm = s.A.rows / 2, hk = s.A.cols / 2, hn = s.B.cols / 2;
      if (strassen) {
        const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                    A22 = b.quad(s.A, 1, 1);
        const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                    B22 = b.quad(s.B, 1, 1);
        MView X[5], Y[5], Pt[7];
        for (auto& v : X) v = b.temp(hm, hk);
        for (auto& v : Y) v = b.temp(hk, hn);
        for (auto& v : Pt) v = b.temp(hm, hn);
        b.ew_part(EW_STR_S, hm, hk, {A11, A12, A21, A22}, {X[0], X[1], X[2], X[3], X[4]});
        b.ew_part(EW_STR_T, hk, hn, {B11, B12, B21, B22}, {Y[0], Y[1], Y[2], Y[3], Y[4]});
        next.push_back({X[0], Y[0], Pt[0]});  // P1 = (A11 + A22)(B11 + B22)
        next.push_back({X[1], B11, Pt[1]});   // P2 = (A21 + A22) B11
        next.push_back({A11, Y[1], Pt[2]});   // P3 = A11 (B12 - B22)
        next.push_back({A22, Y[2], Pt[3]});   // P4 = A22 (B21 - B11)
        next.push_back({X[2], B22, Pt[4]});   // P5 = (A11 + A12) B22
        next.push_back({X[3], Y[3], Pt[5]});  // P6 = (A21 - A11)(B11 + B12)
        next.push_back({X[4], Y[4], Pt[6]});  // P7 = (A12 - A22)(B21 + B22)
        uargs.push_back({Pt[0], Pt[1], Pt[2], Pt[3], Pt[4], Pt[5], Pt[6], b.quad(s.C, 0, 0),
                         b.quad(s.C, 0, 1), b.quad(s.C, 1, 0), b.quad(s.C, 1, 1)});
        continue;
      }
      if (leaf_fused) {
        // products, operand sums and U combinations of the last level in one kernel
        const MView C11 = b.quad(s.C, 0, 0), C12 = b.quad(s.C, 0, 1), C21 = b.quad(s.C, 1, 0),
                    C22 = b.quad(s.C, 1, 1);
        wl_pending.push_back({{b.quad(s.A, 0, 0), b.quad(s.A, 0, 1), s.A, b.quad(s.A, 1, 1), s.A, s.A, s.A},
                              {b.quad(s.B, 0, 0), b.quad(s.B, 1, 0), b.quad(s.B, 1, 1), s.B, s.B, s.B, s.B},
                              {C11, C12, C21, C22},
                              hm, hn, hk, l == 0 && b.P.accumulate, true});
        if (s.A.base == MB_A || s.A.base == MB_B || s.B.base == MB_A || s.B.base == MB_B)
          b.P.fused_reads_ab = true;
        continue;
      }
      if (l == L - 1 && leaf_u) {
        // products and U combinations of the last level in one kernel
        const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                    A22 = b.quad(s.A, 1, 1);
        const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                    B22 = b.quad(s.B, 1, 1);
        MView S[4], T[4];
        for (auto& v : S) v = b.temp(hm, hk);
        for (auto& v : T) v = b.temp(hk, hn);
        b.ew_part(EW_WINO_S, hm, hk, {A11, A12, A21, A22}, {S[0], S[1], S[2], S[3]});
        b.ew_part(EW_WINO_T, hk, hn, {B11, B12, B21, B22}, {T[0], T[1], T[2], T[3]});
        wl_pending.push_back({{A11, A12, S[3], A22, S[0], S[1], S[2]},
                              {B11, B21, B22, T[3], T[0], T[1], T[2]},
                              {b.quad(s.C, 0, 0), b.quad(s.C, 0, 1), b.quad(s.C, 1, 0), b.quad(s.C, 1, 1)},
                              hm, hn, hk, l == 0 && b.P.accumulate, false});
        continue;
      }
      if (l == L - 1 && b.P.spl) {  // (never with Strassen: handled above)
        // split-bfloat16 leaves: the split pass forms S1..S4 / T1..T4 and
        // splits the quadrants read as plain leaf operands
        const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                    A22 = b.quad(s.A, 1, 1);
        const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                    B22 = b.quad(s.B, 1, 1);
        MView S[4], T[4], Pt[7];
        for (auto& v : S) v = b.spl_temp(hm, hk);
        const MView a11 = b.spl_temp(hm, hk), a12 = b.spl_temp(hm, hk), a22 = b.spl_temp(hm, hk);
        for (auto& v : T) v = b.spl_temp(hn, hk);
        const MView b11 = b.spl_temp(hn, hk), b21 = b.spl_temp(hn, hk), b22 = b.spl_temp(hn, hk);
        for (auto& v : Pt) v = b.temp(hm, hn);
        b.split_part(EW_WINO_S_SPL, hm, hk, false, {A11, A12, A21, A22}, {S[0], S[1], S[2], S[3], a11, a12, a22});
        b.split_part(EW_WINO_T_SPL, hk, hn, true, {B11, B12, B21, B22}, {T[0], T[1], T[2], T[3], b11, b21, b22});
        auto leaf = [](const MView& x, const MView& y, const MView& c) {
          Sub r{x, y, c};
          r.spl = true;
          return r;
        };
        next.push_back(leaf(a11, b11, Pt[0]));
        next.push_back(leaf(a12, b21, Pt[1]));
        next.push_back(leaf(S[3], b22, Pt[2]));
        next.push_back(leaf(a22, T[3], Pt[3]));
        next.push_back(leaf(S[0], T[0], Pt[4]));
        next.push_back(leaf(S[1], T[1], Pt[5]));
        next.push_back(leaf(S[2], T[2], Pt[6]));
        uargs.push_back({Pt[0], Pt[1], Pt[2], Pt[3], Pt[4], Pt[5], Pt[6], b.quad(s.C, 0, 0),
                         b.quad(s.C, 0, 1), b.quad(s.C, 1, 0), b.quad(s.C, 1, 1)});
        continue;
      }
      if (l == L - 1 && b.P.trans_b) {
        // B side of the leaves stored transposed: T1..T4 and the plain B
        // quadrants come out of one transposing pass, and the leaves stage
        // B in k-chunks like A (straight into LDS in interior tiles)
        const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                    A22 = b.quad(s.A, 1, 1);
        const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                    B22 = b.quad(s.B, 1, 1);
        MView S[4], Tt[4], Pt[7];
        for (auto& v : S) v = b.temp(hm, hk);
        for (auto& v : Tt) v = b.temp(hn, hk);
        const MView b11 = b.temp(hn, hk), b21 = b.temp(hn, hk), b22 = b.temp(hn, hk);
        for (auto& v : Pt) v = b.temp(hm, hn);
        b.ew_part(EW_WINO_S, hm, hk, {A11, A12, A21, A22}, {S[0], S[1], S[2], S[3]});
        b.trans_part(EW_WINO_T_TR, hk, hn, {B11, B12, B21, B22}, {Tt[0], Tt[1], Tt[2], Tt[3], b11, b21, b22});
        auto leaf = [](const MView& x, const MView& y, const MView& c) {
          Sub r{x, y, c};
          r.bkind = OK_TRANS;
          return r;
        };
        next.push_back(leaf(A11, b11, Pt[0]));
        next.push_back(leaf(A12, b21, Pt[1]));
        next.push_back(leaf(S[3], b22, Pt[2]));
        next.push_back(leaf(A22, Tt[3], Pt[3]));
        next.push_back(leaf(S[0], Tt[0], Pt[4]));
        next.push_back(leaf(S[1], Tt[1], Pt[5]));
        next.push_back(leaf(S[2], Tt[2], Pt[6]));
        uargs.push_back({Pt[0], Pt[1], Pt[2], Pt[3], Pt[4], Pt[5], Pt[6], b.quad(s.C, 0, 0),
                         b.quad(s.C, 0, 1), b.quad(s.C, 1, 0), b.quad(s.C, 1, 1)});
        continue;
      }
      if (l == L - 1 && can_fuse(b, s)) {
        // leaf operands read straight from the quadrants (fused loader)
        MView Pt[7];
        for (auto& v : Pt) v = b.temp(hm, hn);
        next.push_back({b.quad(s.A, 0, 0), b.quad(s.B, 0, 0), Pt[0], OK_PLAIN, OK_PLAIN, true});
        next.push_back({b.quad(s.A, 0, 1), b.quad(s.B, 1, 0), Pt[1], OK_PLAIN, OK_PLAIN, true});
        next.push_back({s.A, b.quad(s.B, 1, 1), Pt[2], OK_S4, OK_PLAIN, true});
        next.push_back({b.quad(s.A, 1, 1), s.B, Pt[3], OK_PLAIN, OK_T4, true});
        next.push_back({s.A, s.B, Pt[4], OK_S1, OK_T1, true});
        next.push_back({s.A, s.B, Pt[5], OK_S2, OK_T2, true});
        next.push_back({s.A, s.B, Pt[6], OK_S3, OK_T3, true});
        if (s.A.base == MB_A || s.A.base == MB_B || s.B.base == MB_A || s.B.base == MB_B)
          b.P.fused_reads_ab = true;
        uargs.push_back({Pt[0], Pt[1], Pt[2], Pt[3], Pt[4], Pt[5], Pt[6], b.quad(s.C, 0, 0),
                         b.quad(s.C, 0, 1), b.quad(s.C, 1, 0), b.quad(s.C, 1, 1)});
        continue;
      }
      const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                  A22 = b.quad(s.A, 1, 1);
      const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                  B22 = b.quad(s.B, 1, 1);
      MView S[4], T[4], Pt[7];
      for (auto& v : S) v = b.temp(hm, hk);
      for (auto& v : T) v = b.temp(hk, hn);
      for (auto& v : Pt) v = b.temp(hm, hn);
      if (fuse_top) {
        up_s.push_back({S[0], S[1], S[2], S[3]});
        up_t.push_back({T[0], T[1], T[2], T[3]});
        up_x.push_back({s.A, s.B});
      } else if (fuse_low) {
        lo_s.push_back({S[0], S[1], S[2], S[3]});
        lo_t.push_back({T[0], T[1], T[2], T[3]});
      } else {
        b.ew_part(EW_WINO_S, hm, hk, {A11, A12, A21, A22}, {S[0], S[1], S[2], S[3]});
        b.ew_part(EW_WINO_T, hk, hn, {B11, B12, B21, B22}, {T[0], T[1], T[2], T[3]});
      }
      next.push_back({A11, B11, Pt[0]});
      next.push_back({A12, B21, Pt[1]});
      next.push_back({S[3], B22, Pt[2]});
      next.push_back({A22, T[3], Pt[3]});
      next.push_back({S[0], T[0], Pt[4]});
      next.push_back({S[1], T[1], Pt[5]});
      next.push_back({S[2], T[2], Pt[6]});
      uargs.push_back({Pt[0], Pt[1], Pt[2], Pt[3], Pt[4], Pt[5], Pt[6], b.quad(s.C, 0, 0),
                       b.quad(s.C, 0, 1), b.quad(s.C, 1, 0), b.quad(s.C, 1, 1)});
    }
    if (fuse_low) {
      // the pair's pre-additions: one part per upper-level block, the lower
      // level's sums of its seven operands (children 7 j .. 7 j + 6)
      for (size_t j = 0; j < up_x.size(); ++j) {
        std::vector<std::vector<MView>> ls(7), lt(7);
        for (int o = 0; o < 7; ++o) {
          ls[o].assign(lo_s[7 * j + o].begin(), lo_s[7 * j + o].end());
          lt[o].assign(lo_t[7 * j + o].begin(), lo_t[7 * j + o].end());
        }
        const MView &XA = up_x[j].first, &XB = up_x[j].second;
        MView ts[4], tt[4];
        for (int q = 0; q < 4; ++q) {
          ts[q] = up_s[j][q];
          tt[q] = up_t[j][q];
        }
        b.ew2_part(EW2_S, XA.rows / 4, XA.cols / 4, XA, ts, ls);
        b.ew2_part(EW2_T, XB.rows / 4, XB.cols / 4, XB, tt, lt);
      }
      up_s.clear();
      up_t.clear();
      up_x.clear();
      lo_s.clear();
      lo_t.clear();
    }
    b.flush();
    // U parts of this level are emitted after the deeper levels finish.
    u_levels.emplace_back();
    for (const auto& u : uargs) {
      EwPart p;
      std::memset(&p, 0, sizeof p);
      p.kind = strassen ? EW_STR_U : EW_WINO_U;
      p.rows = u[7].rows;
      p.cols = u[7].cols;
      p.nin = 7;
      p.nout = 4;
      for (int i = 0; i < 7; ++i) p.in[i] = u[i];
      for (int i = 0; i < 4; ++i) p.out[i] = u[7 + i];
      u_levels.back().push_back(p);
    }
    subs.swap(next);
  }
  b.flush();
  b.cur_stream = 0;
  for (const WinoSub& w : wl_pending) b.wino(w.a, w.b, w.c, w.m, w.n, w.k, w.acc, w.fused);
  b.flush();
  auto plain = [](const Sub& s) {
    return s.A.base != MB_WS && s.B.base != MB_WS && s.akind == OK_PLAIN && s.bkind == OK_PLAIN;
  };
  bool overlap = overlap_req;
  if (overlap && !b.window_has_aux()) {
    b.join();  // every S/T sum is formed in the leaf loader: nothing to overlap
    overlap = false;
  }
  if (overlap) {
    for (const Sub& s : subs)
      if (plain(s)) b.gemm(s.A, s.B, {Builder::store(s.C)}, s.akind, s.bkind, s.fusable);
    b.join();
  }
  // unrolled base cases for leaves of order 1, 2, 4 or 8 (all leaves of a
  // grouped level have the same order)
  int base_order = 0;
  if (b.P.unroll_base && !subs.empty()) {
    const int64_t o = subs[0].A.rows;
    base_order = (o == 1 || o == 2 || o == 4 || o == 8) ? (int)o : 0;
    for (const Sub& s : subs)
      if (s.A.rows != o || s.A.cols != o || s.B.cols != o || s.akind != OK_PLAIN || s.bkind != OK_PLAIN || s.spl)
        base_order = 0;
  }
  for (const Sub& s : subs) {
    if (overlap && plain(s)) continue;
    if (base_order)
      b.base(s.A, s.B, s.C, base_order);
    else if (s.spl)
      b.gemm_spl(s.A, s.B, {Builder::store(s.C)});
    else
      b.gemm(s.A, s.B, {Builder::store(s.C)}, s.akind, s.bkind, s.fusable);
  }
  b.flush();
  for (int l = L - 1; l >= 0; --l) {
    if (l > 0 && upair_top[l - 1]) continue;  // formed by the pair's two-level pass
    if (upair_top[l]) {
      // one part per upper-level block: its C quadrants from the 49 lower
      // products of its seven products
      const std::vector<EwPart>& up = u_levels[l];
      const std::vector<EwPart>& lo = u_levels[l + 1];
      for (size_t j = 0; j < up.size(); ++j) {
        std::vector<std::vector<MView>> low(7);
        for (int q = 0; q < 7; ++q) low[q].assign(lo[7 * j + q].in, lo[7 * j + q].in + 7);
        const MView top[4] = {up[j].out[0], up[j].out[1], up[j].out[2], up[j].out[3]};
        b.ew2_part(EW2_U, top[0].rows / 2, top[0].cols / 2, b.none(), top, low);
      }
      b.flush();
      continue;
    }
    for (const EwPart& p : u_levels[l]) {
      if (l == 0 && b.P.accumulate)  // C = beta C + U at the top level
        b.ew_part(strassen ? EW_STR_U_ACC : EW_WINO_U_ACC, p.rows, p.cols,
                  {p.in[0], p.in[1], p.in[2], p.in[3], p.in[4], p.in[5], p.in[6], p.out[0], p.out[1], p.out[2],
                   p.out[3]},
                  {p.out[0], p.out[1], p.out[2], p.out[3]});
      else
        b.ew_part(p.kind, p.rows, p.cols, {p.in[0], p.in[1], p.in[2], p.in[3], p.in[4], p.in[5], p.in[6]},
                  {p.out[0], p.out[1], p.out[2], p.out[3]});
    }
    b.flush();
  }
}

// ---------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------
int count_levels(int64_t m, int64_t n, int64_t k, int cutoff, int levels) {
  const int64_t c = std::max(cutoff, 1);
  int L = 0;
  while (levels < 0 || L < levels) {
    const int64_t d = (int64_t)1 << L;
    const int64_t mn = std::min(std::min(ceil_div(m, d), ceil_div(n, d)), ceil_div(k, d));
    if (mn <= c) break;
    ++L;
    if (L > 62) break;
  }
  return L;
}

bool bf16x3_available() { return gemm_bf16x3_available(); }

// ---------------------------------------------------------------------------
// Levels per size class for batches given no levels: Section 3.4 chooses
// the cutoff per size from a cost model; on the GPU the choice is measured
// by the autotuner (tuner.py --batched) and stored as a table.
//
// A size class is the product's volume-equivalent order v = (m n k)^(1/3)
// rounded to half octaves, round(2 log2 v) / 2.  The table is read once per
// process from <directory of libmm.so>/tuning/gfx950_batched.txt, or from
// $MM_TUNING_DIR/gfx950_batched.txt: lines "dtype class levels" (dtype
// f64, f32 or bf16x3), '#' starts a comment.  A class missing from the table
// takes the nearest class of its dtype that is there; with no entry for the
// dtype the rule is one level per halving while the leaf's v stays at or
// above 2048 (4096 for split bfloat16), at most two.  The count is then
// capped by the cutoff (count_levels).
// ---------------------------------------------------------------------------
struct ClassTable {
  std::map<std::string, std::map<double, int>> by_dtype;  // dtype name -> class -> levels
  std::string source;                                     // file read, empty when none
};

const char* dtype_name(int dtype) {
  return dtype == MM_F64 ? "f64" : (dtype == MM_F32 ? "f32" : "bf16x3");
}

std::string lib_dir() {
  Dl_info info;
  if (dladdr((void*)&mm_version, &info) && info.dli_fname) {
    std::string f(info.dli_fname);
    const size_t at = f.rfind('/');
    return at == std::string::npos ? std::string(".") : f.substr(0, at);
  }
  return ".";
}

const ClassTable& class_table() {
  static ClassTable t;
  static std::once_flag once;
  std::call_once(once, [] {
    const char* env = std::getenv("MM_TUNING_DIR");
    const std::string path = (env && *env ? std::string(env) : lib_dir() + "/tuning") + "/gfx950_batched.txt";
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
      char* hash = std::strchr(line, '#');
      if (hash) *hash = 0;
      char dt[32];
      double cls = 0;
      int lv = 0;
      if (std::sscanf(line, "%31s %lf %d", dt, &cls, &lv) == 3 && lv >= 0 && lv <= MM_MAX_LEVELS)
        t.by_dtype[dt][cls] = lv;
    }
    std::fclose(f);
    t.source = path;
  });
  return t;
}

double size_class(int64_t m, int64_t n, int64_t k) {
  if (m <= 0 || n <= 0 || k <= 0) return 0.0;
  // round(2 log2 v) / 2 with log2 v = log2(m n k) / 3 (halves rounded up)
  return std::floor(2.0 * std::log2((double)m * (double)n * (double)k) / 3.0 + 0.5) / 2.0;
}

int class_levels(int64_t m, int64_t n, int64_t k, int dtype) {
  const ClassTable& t = class_table();
  const double c = size_class(m, n, k);
  auto it = t.by_dtype.find(dtype_name(dtype));
  if (it != t.by_dtype.end() && !it->second.empty()) {
    int best = 0;
    double dist = 1e300;
    for (const auto& e : it->second)
      if (std::fabs(e.first - c) < dist) {
        dist = std::fabs(e.first - c);
        best = e.second;
      }
    return best;
  }
  // v / 2^(L+1) >= leaf, compared as m n k >= (leaf 2^(L+1))^3
  const double leaf = dtype == MM_BF16X3_REFINED ? 4096.0 : 2048.0;
  const double vol = (double)m * (double)n * (double)k;
  int L = 0;
  while (L < 2) {
    const double e = leaf * (double)((int64_t)2 << L);
    if (vol < e * e * e) break;
    ++L;
  }
  return L;
}

// The (cutoff, levels) of every problem of a batch: given arrays as given;
// a NULL cutoff array means cutoff 1, a NULL levels array the size class's
// tuned level count.
void resolve_batch(int count, const int64_t* mnk, int dtype, const int* cutoff, const int* levels,
                   std::vector<int>& cut, std::vector<int>& lev) {
  cut.assign(count, 1);
  lev.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    cut[i] = cutoff ? cutoff[i] : 1;
    lev[i] = levels ? levels[i] : class_levels(mnk[3 * i], mnk[3 * i + 1], mnk[3 * i + 2], dtype);
  }
}

int check_enums(int algo, int sched, int dtype) {
  if (dtype < MM_F64 || dtype > MM_BF16X3_REFINED) return fail(MM_E_INVALID, "unknown dtype");
  if (algo < MM_ALGO_NAIVE || algo > MM_ALGO_WINOGRAD) return fail(MM_E_INVALID, "unknown algorithm");
  if (sched < MM_SCHED_TWO_TEMP || sched > MM_SCHED_AUTO) return fail(MM_E_INVALID, "unknown schedule");
  return MM_OK;
}

int resolve_sched(int algo, int sched) {
  if (algo == MM_ALGO_NAIVE) return MM_SCHED_AUTO;
  if (sched == MM_SCHED_AUTO) return MM_SCHED_GROUPED;
  return sched;
}

// Build the launch sequence of one product into P (host side only).
int build_plan(Plan& P) {
  P.sched = resolve_sched(P.algo, P.sched);
  if (P.dtype == MM_BF16X3_REFINED && !bf16x3_available())
    return fail(MM_E_UNSUPPORTED, "split-bfloat16 leaves are not built into this library");
  if (P.algo == MM_ALGO_STRASSEN && P.sched != MM_SCHED_DFS3 && P.sched != MM_SCHED_GROUPED)
    return fail(MM_E_UNSUPPORTED, "Strassen supports the DFS3 and grouped schedules only");
  if (P.algo == MM_ALGO_WINOGRAD && P.sched == MM_SCHED_DFS3)
    return fail(MM_E_UNSUPPORTED, "DFS3 is a Strassen schedule");
  const int64_t m = P.m, n = P.n, k = P.k;
  P.L = (P.algo == MM_ALGO_NAIVE || m == 0 || n == 0 || k == 0)
            ? 0
            : count_levels(m, n, k, P.cutoff, P.levels);
  if (P.L > MM_MAX_LEVELS)
    return fail(MM_E_UNSUPPORTED, "recursion would need " + std::to_string(P.L) + " levels (max " +
                                      std::to_string(MM_MAX_LEVELS) + "); raise cutoff or set levels");
  Builder b(P);
  const int64_t step = (int64_t)1 << P.L;
  int64_t g = 1;
  if (P.sched == MM_SCHED_GROUPED && P.L > 0 && std::min(std::min(m, n), k) / step >= 32) g = b.E;
  const int64_t mult = std::max<int64_t>(step * g, P.pad_mult);
  P.M = round_up(m, mult);
  P.N = round_up(n, mult);
  P.K = round_up(k, mult);
  // Peeling: the recursion runs on the largest leading block whose sides are
  // multiples of 2^L g and thin products cover the rest (when every side of
  // that block is nonempty; otherwise the plan pads).
  P.pm = m / (step * g) * (step * g);
  P.pn = n / (step * g) * (step * g);
  P.pk = k / (step * g) * (step * g);
  const bool peel = P.peel && P.sched == MM_SCHED_GROUPED && P.L > 0 && P.pm > 0 && P.pn > 0 && P.pk > 0 &&
                    (P.pm != m || P.pn != n || P.pk != k);
  if (peel) {
    P.M = P.pm;
    P.N = P.pn;
    P.K = P.pk;
  }
  if (P.L == 0) {
    P.M = m;
    P.N = n;
    P.K = k;
  }
  P.leaf_rows = P.M >> P.L;
  if (P.sched == MM_SCHED_IN_PLACE && P.L > 0 && !(P.K == P.N && P.N <= P.M))
    return fail(MM_E_UNSUPPORTED, "in-place schedule needs k == n <= m");

  if (m == 0 || n == 0) {
    // nothing to do
  } else if (P.L == 0) {
    const MView A = b.view(MB_A, 0, P.lda, m, k, m, k);
    const MView B = b.view(MB_B, 0, P.ldb, k, n, k, n);
    const MView C = b.view(MB_C, 0, P.ldc, m, n, m, n);
    const Builder::Out out = P.accumulate ? Builder::axpby(C) : Builder::store(C);
    if (k == 0) {
      if (P.accumulate)  // C = beta C + 0
        b.ew_part(EW_AXPBY, m, n, {b.view(MB_C, 0, P.ldc, m, n, 0, 0), C}, {C});
      else
        b.ew_part(EW_ZERO, m, n, {}, {C});
    } else if (P.split_k > 1 && !P.spl && ceil_div(k, round_up(ceil_div(k, P.split_k), 64)) > 1) {
      // split k: the parts' partial products run in one grouped launch (the
      // whole GPU busy when C alone has few tiles), then one pass sums them
      // in order (and applies beta)
      const int64_t kc = round_up(ceil_div(k, P.split_k), 64);
      const int np = (int)ceil_div(k, kc);
      std::vector<MView> parts;
      for (int i = 0; i < np; ++i) {
        const int64_t k0 = i * kc, kl = std::min(kc, k - k0);
        const MView Pi = b.temp(m, n);
        parts.push_back(Pi);
        b.gemm(b.view(MB_A, k0, P.lda, m, kl, m, kl), b.view(MB_B, k0 * P.ldb, P.ldb, kl, n, kl, n),
               {Builder::store(Pi)});
      }
      b.flush();
      if (P.accumulate) parts.push_back(b.view(MB_C, 0, P.ldc, m, n, m, n));
      b.ew_parts(P.accumulate ? EW_SUM_ACC : EW_SUM, m, n, parts, std::vector<MView>{C}, np);
    } else if (P.dtype != MM_BF16X3_REFINED && (P.lda % b.E || P.ldb % b.E || k % b.E || n % b.E) &&
               m >= 64 && n >= 64 && k >= 64 && (double)m * n * k >= 134217728.0) {
      // Operands that cannot be read in 16-byte chunks (a leading dimension
      // or width not a multiple of 16 bytes) would put every tile on the
      // element-wise load path: copy them once into aligned blocks (k and n
      // rounded up, the extra k rows / columns zero) and run the GEMM on those.
      const int64_t k4 = round_up(k, b.E), n4 = round_up(n, b.E);
      const MView Ap = b.temp(m, k4), Bp = b.temp(k4, n4);
      b.ew_part(EW_COPY, m, k4, {b.view(MB_A, 0, P.lda, m, k4, m, k)}, {Ap});
      b.ew_part(EW_COPY, k4, n4, {b.view(MB_B, 0, P.ldb, k4, n4, k, n)}, {Bp});
      b.flush();
      b.gemm(Ap, Bp, {out});
    } else if (P.spl) {
      const MView As = b.spl_temp(m, k), Bt = b.spl_temp(n, k);
      b.split_part(EW_SPLIT, m, k, false, {A}, {As});
      b.split_part(EW_SPLIT, k, n, true, {B}, {Bt});
      b.flush();
      b.gemm_spl(As, Bt, {out});
    } else {
      b.gemm(A, B, {out});
    }
    b.flush();
  } else if (P.sched == MM_SCHED_GROUPED && peel) {
    // C[:pm, :pn] = A[:pm, :pk] B[:pk, :pn] by the recursion, then one
    // launch of thin products: C[:pm, :pn] += A[:pm, pk:] B[pk:, :pn],
    // C[:pm, pn:] = A[:pm, :] B[:, pn:] and C[pm:, :] = A[pm:, :] B
    // (beta C + ... for those two in accumulating plans; the recursion's
    // top-level combination applies beta to the leading block).
    const int64_t pm = P.pm, pn = P.pn, pk = P.pk;
    sched_grouped(b, {Sub{b.view(MB_A, 0, P.lda, pm, pk, pm, pk), b.view(MB_B, 0, P.ldb, pk, pn, pk, pn),
                          b.view(MB_C, 0, P.ldc, pm, pn, pm, pn)}});
    auto out = [&](const MView& c) { return P.accumulate ? Builder::axpby(c) : Builder::store(c); };
    if (pk < k) {
      const MView Cl = b.view(MB_C, 0, P.ldc, pm, pn, pm, pn);
      b.gemm(b.view(MB_A, pk, P.lda, pm, k - pk, pm, k - pk), b.view(MB_B, pk * P.ldb, P.ldb, k - pk, pn, k - pk, pn),
             {Builder::add(Cl, Cl, +1)});
    }
    if (pn < n)
      b.gemm(b.view(MB_A, 0, P.lda, pm, k, pm, k), b.view(MB_B, pn, P.ldb, k, n - pn, k, n - pn),
             {out(b.view(MB_C, pn, P.ldc, pm, n - pn, pm, n - pn))});
    if (pm < m)
      b.gemm(b.view(MB_A, pm * P.lda, P.lda, m - pm, k, m - pm, k), b.view(MB_B, 0, P.ldb, k, n, k, n),
             {out(b.view(MB_C, pm * P.ldc, P.ldc, m - pm, n, m - pm, n))});
    b.flush();
  } else if (P.sched == MM_SCHED_GROUPED) {
    const MView A = b.view(MB_A, 0, P.lda, P.M, P.K, m, k);
    const MView B = b.view(MB_B, 0, P.ldb, P.K, P.N, k, n);
    const MView C = b.view(MB_C, 0, P.ldc, P.M, P.N, m, n);
    sched_grouped(b, {Sub{A, B, C}});
  } else {
    // Depth-first schedules work on real buffers: pad by copying when needed.
    const bool pad = P.M != m || P.N != n || P.K != k;
    MView A = b.view(MB_A, 0, P.lda, m, k, m, k);
    MView B = b.view(MB_B, 0, P.ldb, k, n, k, n);
    MView C = b.view(MB_C, 0, P.ldc, m, n, m, n);
    MView Cw = C;
    // an accumulating depth-first plan forms the product in a temporary
    // (the schedules use C as scratch) and adds it to beta C at the end
    if (P.accumulate && !pad) Cw = b.temp(m, n);
    if (pad) {
      const MView Ap = b.temp(P.M, P.K), Bp = b.temp(P.K, P.N), Cp = b.temp(P.M, P.N);
      b.ew_part(EW_COPY, P.M, P.K, {b.view(MB_A, 0, P.lda, P.M, P.K, m, k)}, {Ap});
      b.ew_part(EW_COPY, P.K, P.N, {b.view(MB_B, 0, P.ldb, P.K, P.N, k, n)}, {Bp});
      b.flush();
      A = Ap;
      B = Bp;
      Cw = Cp;
    }
    if (P.sched == MM_SCHED_TWO_TEMP)
      sched_two_temp(b, A, B, Cw, 0);
    else if (P.sched == MM_SCHED_IN_PLACE)
      sched_in_place(b, A, B, Cw, 0);
    else
      sched_strassen(b, A, B, Cw, 0);
    if (P.accumulate) {
      b.ew_part(EW_AXPBY, m, n, {b.corner(Cw, m, n), C}, {C});
      b.flush();
    } else if (pad) {
      b.ew_part(EW_COPY, m, n, {b.corner(Cw, m, n)}, {C});
      b.flush();
    }
  }
  b.flush();
  P.ws_bytes = (size_t)b.ws_peak * b.esz;
  P.text = b.txt.str();
  return MM_OK;
}

// ---------------------------------------------------------------------------
// Devices, upload, execution
// ---------------------------------------------------------------------------
std::mutex g_dev_mu;
std::map<int, int> g_dev_ok;  // device -> MM_OK or error code

int check_device(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MM_E_UNSUPPORTED, "no HIP device available");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev_ok.find(dev);
  if (it == g_dev_ok.end()) {
    hipDeviceProp_t prop;
    int ok = MM_OK;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
      ok = MM_E_UNSUPPORTED;
    else if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      ok = MM_E_UNSUPPORTED;
    it = g_dev_ok.emplace(dev, ok).first;
  }
  if (it->second != MM_OK) return fail(MM_E_UNSUPPORTED, "device is not gfx950 (MI355X)");
  *dev_out = dev;
  return MM_OK;
}

int upload(Plan& P) {
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != MM_OK) return rc;
  P.device = dev;
  if (P.unfused) {
    rc = upload(*P.unfused);
    if (rc != MM_OK) return rc;
  }
  if (P.persistent) {
    // The persistent batched launch hung on its first run on MI355X (no
    // fault; every wait apparently ran to its bound) and the cause is not
    // known: it stays off the GPU until one is shown.  Its plans are still
    // built on the host (mm_batched_describe, mm_batched_table), where the
    // task queue is checked.
    return fail(MM_E_UNSUPPORTED, "the persistent batched launch is switched off (it hung on MI355X with "
                                  "the cause not yet found); use the level-synchronous batched plan");
    const size_t cb = (size_t)(PC_FIRST + P.pcount) * sizeof(int);
    if (hipMalloc((void**)&P.dctr, cb) != hipSuccess) {
      P.dctr = nullptr;
      (void)hipGetLastError();
      return fail(MM_E_NOMEM, "hipMalloc of the persistent plan's counters failed");
    }
    // zero once here; every launch leaves them zero again
    if (hipMemset(P.dctr, 0, cb) != hipSuccess) return fail(MM_E_HIP, "clearing the counters failed");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    P.pgrid = persist_occupancy(P.ops[0].cfg) * cus;
  }
  if (P.table.empty()) return MM_OK;
  if (hipMalloc(&P.dtable, P.table.size()) != hipSuccess) {
    P.dtable = nullptr;
    (void)hipGetLastError();
    return fail(MM_E_NOMEM, "hipMalloc of the plan's descriptor table failed");
  }
  if (hipMemcpy(P.dtable, P.table.data(), P.table.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MM_E_HIP, "upload of the plan's descriptor table failed");
  return MM_OK;
}

// The auxiliary stream and fork/join events of a plan for caller stream s
// (created on first use with that stream, default priority).
int aux_for(Plan& P, hipStream_t s, Plan::Aux** out) {
  std::lock_guard<std::mutex> lk(P.aux_mu);
  for (auto& a : P.aux)
    if (a.main == s) {
      *out = &a;
      return MM_OK;
    }
  Plan::Aux a{s, nullptr, nullptr, nullptr};
  if (hipStreamCreateWithFlags(&a.aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a.join, hipEventDisableTiming) != hipSuccess) {
    if (a.join) (void)hipEventDestroy(a.join);
    if (a.fork) (void)hipEventDestroy(a.fork);
    if (a.aux) (void)hipStreamDestroy(a.aux);
    return fail(MM_E_HIP, "could not create the plan's auxiliary stream");
  }
  P.aux.push_back(a);
  *out = &P.aux.back();
  return MM_OK;
}

// events (timed execution): events[2i] / events[2i+1] are recorded before /
// after launch i on the stream that launch runs on.
// Polls a persistent launch's task makes on a counter before it gives up
// and flags the plan (MM_PERSIST_SPIN_LIMIT overrides; tests lower it).
int persist_spin_limit() {
  static const int lim = [] {
    const char* e = std::getenv("MM_PERSIST_SPIN_LIMIT");
    const long v = e ? std::strtol(e, nullptr, 10) : 0;
    return v > 0 ? (int)std::min<long>(v, 1L << 30) : (1 << 22);
  }();
  return lim;
}

// table: the device copy of the plan's descriptor table to read (default:
// the one the plan uploaded).
int enqueue(Plan& P, void* A, void* B, void* C, void* ws, hipStream_t s, hipEvent_t* events = nullptr,
            double beta = 1.0, const void* table = nullptr) {
  const void* dtab = table ? table : P.dtable;
  KernelBases kb;
  kb.beta = beta;
  kb.p[MB_A] = A;
  kb.p[MB_B] = B;
  kb.p[MB_C] = C;
  kb.p[MB_WS] = ws;
  kb.p[MB_ABS] = nullptr;
  kb.aligned = 0;
  for (int i = 0; i < 4; ++i)
    if (((uintptr_t)kb.p[i] & 15) == 0) kb.aligned |= 1 << i;
  Plan::Aux* ax = nullptr;
  if (P.has_aux) {
    int rc = aux_for(P, s, &ax);
    if (rc != MM_OK) return rc;
  }
  int i = 0;
  for (const OpRec& op : P.ops) {
    const hipStream_t st = (op.stream && ax) ? ax->aux : s;
    if (events && hipEventRecord(events[2 * i], st) != hipSuccess) return fail(MM_E_HIP, "hipEventRecord failed");
    hipError_t e = hipSuccess;
    if (op.type == OP_FORK) {
      if (hipEventRecord(ax->fork, s) != hipSuccess || hipStreamWaitEvent(ax->aux, ax->fork, 0) != hipSuccess)
        return fail(MM_E_HIP, "fork to the auxiliary stream failed");
    } else if (op.type == OP_JOIN) {
      if (hipEventRecord(ax->join, ax->aux) != hipSuccess || hipStreamWaitEvent(s, ax->join, 0) != hipSuccess)
        return fail(MM_E_HIP, "join of the auxiliary stream failed");
    } else {
      const void* d = (const char*)dtab + op.off;
      if (op.type == OP_EW)
        e = launch_ew(op.kdtype, kb, (const EwPart*)d, op.count, op.grid, st);
      else if (op.type == OP_EW2)
        e = launch_ew2(op.kdtype, kb, (const Ew2Part*)d, op.count, op.grid, st);
      else if (op.type == OP_WINO)
        e = launch_gemm_wino(op.cfg, op.fused, kb, (const WinoLeafDesc*)d, op.count, op.grid, op.remap, st);
      else if (op.type == OP_SPLIT)
        e = launch_split(kb, (const EwPart*)d, op.count, op.grid, st);
      else if (op.type == OP_TRANS)
        e = launch_trans(kb, (const EwPart*)d, op.count, op.grid, st);
      else if (op.type == OP_BASE)
        e = launch_base(op.kdtype, op.cfg, kb, (const BaseDesc*)d, op.count, op.grid, st);
      else if (op.type == OP_PERSIST)
        e = launch_persist(op.cfg, kb, d, P.dctr, P.pgrid, persist_spin_limit(), st);
      else
        e = op.fused ? launch_gemm_fused(op.cfg, kb, (const GemmDesc*)d, op.count, op.grid, op.remap, st)
                     : launch_gemm(op.kdtype, op.cfg, kb, (const GemmDesc*)d, op.count, op.grid, op.remap, st);
    }
    if (e != hipSuccess) return fail(MM_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    if (events && hipEventRecord(events[2 * i + 1], st) != hipSuccess)
      return fail(MM_E_HIP, "hipEventRecord failed");
    ++i;
  }
  return MM_OK;
}

bool misaligned_ab(const void* A, const void* B) {
  return (((uintptr_t)A) & 15) || (((uintptr_t)B) & 15);
}

int execute(Plan& P, void* A, void* B, void* C, void* ws, size_t ws_bytes, hipStream_t s, double beta = 1.0) {
  if (P.fused_reads_ab && P.unfused && misaligned_ab(A, B))
    return execute(*P.unfused, A, B, C, ws, ws_bytes, s, beta);
  if (ws_bytes < P.ws_bytes || (P.ws_bytes > 0 && ws == nullptr))
    return fail(MM_E_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, plan needs " +
                                    std::to_string(P.ws_bytes));
  if (P.spl && P.ws_bytes > 0 && ((uintptr_t)ws & 15))
    return fail(MM_E_INVALID, "split-bfloat16 plans need a 16-byte aligned workspace");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != P.device)
    return fail(MM_E_INVALID, "plan was built for another device");
  if (P.ops.empty()) return MM_OK;
  if (!(P.flags & MM_PLAN_GRAPH) || s == nullptr) return enqueue(P, A, B, C, ws, s, nullptr, beta);
  std::lock_guard<std::mutex> lk(P.mu);
  for (auto& g : P.graphs)
    if (g.a == A && g.b == B && g.c == C && g.ws == ws && g.beta == beta) {
      if (hipGraphLaunch(g.exec, s) != hipSuccess) return fail(MM_E_HIP, "hipGraphLaunch failed");
      return MM_OK;
    }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(MM_E_HIP, "hipStreamBeginCapture failed");
  int rc = enqueue(P, A, B, C, ws, s, nullptr, beta);
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc != MM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess || !graph) return fail(MM_E_HIP, "hipStreamEndCapture failed");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MM_E_HIP, "hipGraphInstantiate failed");
  if (P.graphs.size() >= 8) {
    // Retire the oldest graph once the stream it last ran on has drained.
    (void)hipStreamSynchronize(P.graphs.front().stream);
    (void)hipGraphExecDestroy(P.graphs.front().exec);
    P.graphs.erase(P.graphs.begin());
  }
  P.graphs.push_back({A, B, C, ws, beta, s, exec});
  if (hipGraphLaunch(exec, s) != hipSuccess) return fail(MM_E_HIP, "hipGraphLaunch failed");
  return MM_OK;
}

// ---------------------------------------------------------------------------
// Argument checks
// ---------------------------------------------------------------------------
bool overlaps(const void* p, size_t pb, const void* q, size_t qb) {
  if (!p || !q || pb == 0 || qb == 0) return false;
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
  return a < b + qb && b < a + pb;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t esz) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((rows - 1) * ld + cols) * esz;
}

int check_args(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B, int64_t ldb,
               const void* C, int64_t ldc, int dtype) {
  if (m < 0 || n < 0 || k < 0) return fail(MM_E_INVALID, "negative dimension");
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX) return fail(MM_E_UNSUPPORTED, "dimension above 2^31-1");
  if (m == 0 || n == 0) return MM_OK;
  if (k > 0 && (!A || !B)) return fail(MM_E_INVALID, "NULL operand with nonzero size");
  if (!C) return fail(MM_E_INVALID, "NULL output with nonzero size");
  if ((k > 0 && lda < k) || (k > 0 && ldb < n) || ldc < n) return fail(MM_E_INVALID, "leading dimension shorter than a row");
  const size_t esz = elem_size(dtype);
  const size_t cb = span_bytes(m, n, ldc, esz);
  if (k > 0 && (overlaps(C, cb, A, span_bytes(m, k, lda, esz)) || overlaps(C, cb, B, span_bytes(k, n, ldb, esz))))
    return fail(MM_E_ALIAS, "C overlaps A or B");
  return MM_OK;
}

// ---------------------------------------------------------------------------
// Caches for the short forms and one-shot batches
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;
std::map<std::string, std::unique_ptr<Plan>> g_plans;
struct WsEntry {
  void* ptr = nullptr;
  size_t bytes = 0;
  bool owned = false;
};
std::map<std::pair<int, hipStream_t>, WsEntry> g_ws;

int make_plan(int algo, int sched, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc,
              int cutoff, int levels, int dtype, unsigned flags, std::unique_ptr<Plan>* out) {
  int rc = check_enums(algo, sched, dtype);
  if (rc != MM_OK) return rc;
  if (m < 0 || n < 0 || k < 0) return fail(MM_E_INVALID, "negative dimension");
  std::unique_ptr<Plan> P(new Plan);
  P->algo = algo;
  P->sched = sched;
  P->dtype = dtype;
  P->m = m;
  P->n = n;
  P->k = k;
  P->lda = lda;
  P->ldb = ldb;
  P->ldc = ldc;
  P->cutoff = cutoff;
  P->levels = levels;
  P->flags = flags;
  P->tile_cfg = (int)((flags >> 8) & 0xff) - 1;
  P->fuse = (flags & MM_PLAN_FUSE) != 0;
  P->overlap = (flags & MM_PLAN_OVERLAP) != 0;
  P->accumulate = (flags & MM_PLAN_ACCUMULATE) != 0;
  P->peel = (flags & MM_PLAN_PEEL) != 0;
  P->level_passes = (flags & MM_PLAN_LEVEL_PASSES) != 0;
  P->trans_b = (flags & MM_PLAN_TRANS_B) != 0 && dtype == MM_F32 && algo == MM_ALGO_WINOGRAD &&
               resolve_sched(algo, sched) == MM_SCHED_GROUPED;
  P->split_k = (int)((flags >> 16) & 0xf);
  P->pad_mult = (int64_t)1 << ((flags >> 24) & 0xf);
  if (P->split_k > 8) return fail(MM_E_INVALID, "MM_PLAN_SPLIT_K allows at most 8 parts");
  if (P->split_k < 1) P->split_k = 1;
  P->unroll_base = (flags & MM_PLAN_UNROLL_BASE) != 0 && dtype != MM_BF16X3_REFINED &&
                   algo == MM_ALGO_WINOGRAD && resolve_sched(algo, sched) == MM_SCHED_GROUPED;
  // the fused Winograd leaf level computes in float32 and replaces the
  // grouped schedule's last level; other dtypes and schedules ignore it
  P->leaf_u = (flags & MM_PLAN_LEAF_U) != 0 && dtype == MM_F32 && sched == MM_SCHED_GROUPED &&
              algo == MM_ALGO_WINOGRAD;
  // on request, split-bfloat16 leaves of the grouped schedule and of the
  // plain product read operands split once by a split pass
  const int rs = resolve_sched(algo, sched);
  P->spl = dtype == MM_BF16X3_REFINED && (flags & MM_PLAN_SPLIT_PASS) != 0 &&
           ((rs == MM_SCHED_GROUPED && algo == MM_ALGO_WINOGRAD) || algo == MM_ALGO_NAIVE);
  if (P->tile_cfg >= (P->leaf_u ? kNumWinoCfg : kNumGemmCfg))
    return fail(MM_E_INVALID, "unknown tile configuration");
  rc = build_plan(*P);
  if (rc != MM_OK) return rc;
  if (P->fused_reads_ab) {
    // A fused loader reads A and B with 16-byte vector loads; keep the
    // unfused plan for calls whose A or B is not 16-byte aligned.
    std::unique_ptr<Plan> U;
    rc = make_plan(algo, sched, m, n, k, lda, ldb, ldc, cutoff, levels, dtype, flags & ~MM_PLAN_FUSE, &U);
    if (rc != MM_OK) return rc;
    P->ws_bytes = std::max(P->ws_bytes, U->ws_bytes);
    P->unfused = std::move(U);
  }
  *out = std::move(P);
  return MM_OK;
}

int cached_plan(int algo, int sched, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc,
                int cutoff, int levels, int dtype, Plan** out) {
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != MM_OK) return rc;
  char key[256];
  std::snprintf(key, sizeof key, "%d|%d|%d|%lld|%lld|%lld|%lld|%lld|%lld|%d|%d|%d", dev, algo, sched,
                (long long)m, (long long)n, (long long)k, (long long)lda, (long long)ldb, (long long)ldc,
                cutoff, levels, dtype);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_plans.find(key);
  if (it == g_plans.end()) {
    std::unique_ptr<Plan> P;
    rc = make_plan(algo, sched, m, n, k, lda, ldb, ldc, cutoff, levels, dtype, 0, &P);
    if (rc != MM_OK) return rc;
    rc = upload(*P);
    if (rc != MM_OK) return rc;
    it = g_plans.emplace(key, std::move(P)).first;
  }
  *out = it->second.get();
  return MM_OK;
}

int stream_workspace(size_t need, hipStream_t s, void** ws) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MM_E_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  WsEntry& w = g_ws[{dev, s}];
  if (need == 0) {
    *ws = w.ptr;
    return MM_OK;
  }
  if (w.bytes < need) {
    if (!w.owned && w.ptr) return fail(MM_E_WORKSPACE, "registered workspace is smaller than the product needs");
    if (w.ptr) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    if (hipMalloc(&w.ptr, need) != hipSuccess) {
      w.ptr = nullptr;
      (void)hipGetLastError();
      return fail(MM_E_NOMEM, "could not allocate a workspace of " + std::to_string(need) + " bytes");
    }
    w.bytes = need;
    w.owned = true;
  }
  *ws = w.ptr;
  return MM_OK;
}

int short_form(int algo, int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int cutoff,
               int levels, int dtype, hipStream_t s) {
  int rc = check_enums(algo, MM_SCHED_AUTO, dtype);
  if (rc != MM_OK) return rc;
  rc = check_args(m, n, k, A, std::max<int64_t>(k, 1), B, std::max<int64_t>(n, 1), C, std::max<int64_t>(n, 1), dtype);
  if (rc != MM_OK) return rc;
  if (m == 0 || n == 0) return MM_OK;
  Plan* P = nullptr;
  rc = cached_plan(algo, MM_SCHED_AUTO, m, n, k, std::max<int64_t>(k, 1), std::max<int64_t>(n, 1),
                   std::max<int64_t>(n, 1), cutoff, levels, dtype, &P);
  if (rc != MM_OK) return rc;
  void* ws = nullptr;
  rc = stream_workspace(P->ws_bytes, s, &ws);
  if (rc != MM_OK) return rc;
  return execute(*P, (void*)A, (void*)B, C, ws, P->ws_bytes, s);
}

// Plans of the entry point that allocates nothing: host only (their table is
// copied into the caller's memory at every call), keyed like the short forms.
std::map<std::string, std::unique_ptr<Plan>> g_host_plans;

// ---------------------------------------------------------------------------
// Batches: every problem planned with the grouped schedule on absolute
// addresses, then merged stage by stage across problems.
// ---------------------------------------------------------------------------
int build_batched(Plan& P, int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                  const int* cutoff, const int* levels) {
  Builder b(P);
  const size_t esz = b.esz;
  struct Prob {
    int L;
    std::vector<std::vector<Sub>> subs;  // per level
    std::vector<std::vector<EwPart>> st, u;
  };
  std::vector<Prob> probs(count);
  int Lmax = 0;
  for (int i = 0; i < count; ++i)
    if (mnk[3 * i] < 0 || mnk[3 * i + 1] < 0 || mnk[3 * i + 2] < 0)
      return fail(MM_E_INVALID, "negative dimension in batch");
  std::vector<int> cut, lev;
  resolve_batch(count, mnk, P.dtype, cutoff, levels, cut, lev);
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    const int c = cut[i];
    const int lv = lev[i];
    int rc = check_args(m, n, k, A[i], std::max<int64_t>(k, 1), B[i], std::max<int64_t>(n, 1), C[i],
                        std::max<int64_t>(n, 1), P.dtype);
    if (rc != MM_OK) return rc;
    const int L = (m == 0 || n == 0 || k == 0) ? 0 : count_levels(m, n, k, c, lv);
    if (L > MM_MAX_LEVELS) return fail(MM_E_UNSUPPORTED, "too many levels in batch problem");
    probs[i].L = L;
    Lmax = std::max(Lmax, L);
  }
  // Stage l: S/T parts of every problem with more than l levels.
  std::vector<std::vector<Sub>> cur(count);
  std::vector<std::vector<std::array<MView, 11>>> uargs_by_level_prob;
  std::vector<std::vector<EwPart>> u_stage(Lmax);
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    if (m == 0 || n == 0) continue;
    const int L = probs[i].L;
    const int64_t step = (int64_t)1 << L;
    int64_t g = (L > 0 && std::min(std::min(m, n), k) / step >= 32) ? b.E : 1;
    const int64_t M = L ? round_up(m, step * g) : m, N = L ? round_up(n, step * g) : n,
                  K = L ? round_up(k, step * g) : k;
    const int64_t ka = std::max<int64_t>(k, 1), na = std::max<int64_t>(n, 1);
    cur[i].push_back({b.view(MB_ABS, (int64_t)((uintptr_t)A[i] / esz), ka, M, K, m, k),
                      b.view(MB_ABS, (int64_t)((uintptr_t)B[i] / esz), na, K, N, k, n),
                      b.view(MB_ABS, (int64_t)((uintptr_t)C[i] / esz), na, M, N, m, n)});
  }
  for (int l = 0; l < Lmax; ++l) {
    for (int i = 0; i < count; ++i) {
      if (probs[i].L <= l) continue;
      std::vector<Sub> next;
      for (const Sub& s : cur[i]) {
        const int64_t hm = s.A.rows / 2, hk = s.A.cols / 2, hn = s.B.cols / 2;
        const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                    A22 = b.quad(s.A, 1, 1);
        const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                    B22 = b.quad(s.B, 1, 1);
        MView S[4], T[4], Pt[7];
        for (auto& v : S) v = b.temp(hm, hk);
        for (auto& v : T) v = b.temp(hk, hn);
        for (auto& v : Pt) v = b.temp(hm, hn);
        b.ew_part(EW_WINO_S, hm, hk, {A11, A12, A21, A22}, {S[0], S[1], S[2], S[3]});
        b.ew_part(EW_WINO_T, hk, hn, {B11, B12, B21, B22}, {T[0], T[1], T[2], T[3]});
        next.push_back({A11, B11, Pt[0]});
        next.push_back({A12, B21, Pt[1]});
        next.push_back({S[3], B22, Pt[2]});
        next.push_back({A22, T[3], Pt[3]});
        next.push_back({S[0], T[0], Pt[4]});
        next.push_back({S[1], T[1], Pt[5]});
        next.push_back({S[2], T[2], Pt[6]});
        EwPart p;
        std::memset(&p, 0, sizeof p);
        p.kind = EW_WINO_U;
        p.rows = (int32_t)hm;
        p.cols = (int32_t)hn;
        p.nin = 7;
        p.nout = 4;
        for (int j = 0; j < 7; ++j) p.in[j] = Pt[j];
        p.out[0] = b.quad(s.C, 0, 0);
        p.out[1] = b.quad(s.C, 0, 1);
        p.out[2] = b.quad(s.C, 1, 0);
        p.out[3] = b.quad(s.C, 1, 1);
        u_stage[l].push_back(p);
      }
      cur[i].swap(next);
    }
    b.flush();
  }
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    if (m == 0 || n == 0) continue;
    for (const Sub& s : cur[i]) {
      if (k == 0)
        continue;
      b.gemm(s.A, s.B, {Builder::store(s.C)});
    }
  }
  b.flush();
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    if (m > 0 && n > 0 && k == 0) b.ew_part(EW_ZERO, m, n, {}, {cur[i][0].C});
  }
  b.flush();
  for (int l = Lmax - 1; l >= 0; --l) {
    for (const EwPart& p : u_stage[l])
      b.ew_part(EW_WINO_U, p.rows, p.cols, {p.in[0], p.in[1], p.in[2], p.in[3], p.in[4], p.in[5], p.in[6]},
                {p.out[0], p.out[1], p.out[2], p.out[3]});
    b.flush();
  }
  P.ws_bytes = (size_t)b.ws_peak * esz;
  P.text = b.txt.str();
  int64_t lmax = 0;
  for (auto& pr : probs) lmax = std::max<int64_t>(lmax, pr.L);
  P.L = (int)lmax;
  return MM_OK;
}

// Batches as ONE persistent launch (batch.hip, desc.h): the recursion of
// every problem as in build_batched (same blocks, same temporaries), laid
// out as a task queue: the S/T passes of level 0, 1, ..., the leaf-product
// tiles (longest k first), the U passes of the deepest level up to level 0.
// Each element-wise part and each leaf product carries its problem's
// dependency: S/T of level l waits for S/T of level l - 1, the leaves wait
// for the last S/T level, U of the deepest level waits for the leaves, U of
// level l for U of level l + 1.  Float32 only.
int build_batched_persistent(Plan& P, int count, const int64_t* mnk, void* const* A, void* const* B,
                             void* const* C, const int* cutoff, const int* levels) {
  Builder b(P);
  const size_t esz = b.esz;
  for (int i = 0; i < count; ++i)
    if (mnk[3 * i] < 0 || mnk[3 * i + 1] < 0 || mnk[3 * i + 2] < 0)
      return fail(MM_E_INVALID, "negative dimension in batch");
  std::vector<int> cut, lev;
  resolve_batch(count, mnk, P.dtype, cutoff, levels, cut, lev);
  std::vector<int> Ls(count, 0);
  int Lmax = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    int rc = check_args(m, n, k, A[i], std::max<int64_t>(k, 1), B[i], std::max<int64_t>(n, 1), C[i],
                        std::max<int64_t>(n, 1), P.dtype);
    if (rc != MM_OK) return rc;
    Ls[i] = (m == 0 || n == 0 || k == 0) ? 0 : count_levels(m, n, k, cut[i], lev[i]);
    if (Ls[i] > MM_MAX_LEVELS) return fail(MM_E_UNSUPPORTED, "too many levels in batch problem");
    Lmax = std::max(Lmax, Ls[i]);
  }
  // stage lists, each entry tagged with its problem
  std::vector<std::vector<std::pair<int, EwPart>>> st(Lmax), u(Lmax);
  std::vector<std::pair<int, EwPart>> zeros;
  std::vector<std::pair<int, GemmDesc>> leaves;
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    if (m == 0 || n == 0) continue;
    const int L = Ls[i];
    const int64_t step = (int64_t)1 << L;
    const int64_t g = (L > 0 && std::min(std::min(m, n), k) / step >= 32) ? b.E : 1;
    const int64_t M = L ? round_up(m, step * g) : m, N = L ? round_up(n, step * g) : n,
                  K = L ? round_up(k, step * g) : k;
    const int64_t ka = std::max<int64_t>(k, 1), na = std::max<int64_t>(n, 1);
    std::vector<Sub> cur{{b.view(MB_ABS, (int64_t)((uintptr_t)A[i] / esz), ka, M, K, m, k),
                          b.view(MB_ABS, (int64_t)((uintptr_t)B[i] / esz), na, K, N, k, n),
                          b.view(MB_ABS, (int64_t)((uintptr_t)C[i] / esz), na, M, N, m, n)}};
    if (k == 0) {
      zeros.push_back({i, b.make_ew(EW_ZERO, m, n, {}, {cur[0].C})});
      continue;
    }
    for (int l = 0; l < L; ++l) {
      std::vector<Sub> next;
      for (const Sub& s : cur) {
        const int64_t hm = s.A.rows / 2, hk = s.A.cols / 2, hn = s.B.cols / 2;
        const MView A11 = b.quad(s.A, 0, 0), A12 = b.quad(s.A, 0, 1), A21 = b.quad(s.A, 1, 0),
                    A22 = b.quad(s.A, 1, 1);
        const MView B11 = b.quad(s.B, 0, 0), B12 = b.quad(s.B, 0, 1), B21 = b.quad(s.B, 1, 0),
                    B22 = b.quad(s.B, 1, 1);
        MView S[4], T[4], Pt[7];
        for (auto& v : S) v = b.temp(hm, hk);
        for (auto& v : T) v = b.temp(hk, hn);
        for (auto& v : Pt) v = b.temp(hm, hn);
        st[l].push_back({i, b.make_ew(EW_WINO_S, hm, hk, {A11, A12, A21, A22}, {S[0], S[1], S[2], S[3]})});
        st[l].push_back({i, b.make_ew(EW_WINO_T, hk, hn, {B11, B12, B21, B22}, {T[0], T[1], T[2], T[3]})});
        next.push_back({A11, B11, Pt[0]});
        next.push_back({A12, B21, Pt[1]});
        next.push_back({S[3], B22, Pt[2]});
        next.push_back({A22, T[3], Pt[3]});
        next.push_back({S[0], T[0], Pt[4]});
        next.push_back({S[1], T[1], Pt[5]});
        next.push_back({S[2], T[2], Pt[6]});
        u[l].push_back({i, b.make_ew(EW_WINO_U, hm, hn, {Pt[0], Pt[1], Pt[2], Pt[3], Pt[4], Pt[5], Pt[6]},
                                     {b.quad(s.C, 0, 0), b.quad(s.C, 0, 1), b.quad(s.C, 1, 0),
                                      b.quad(s.C, 1, 1)})});
      }
      cur.swap(next);
    }
    for (const Sub& s : cur) {
      P.leaves += 1;
      GemmDesc gd = b.make_gemm(s.A, s.B, {Builder::store(s.C)});
      if (gd.m > 0 && gd.n > 0) leaves.push_back({i, gd});
    }
  }
  // tile configuration of the leaf products: the unequal-batch cost model
  // over the persistent kernel's tiles
  int cfg = P.tile_cfg;
  if (cfg < 0 || !persist_cfg_ok(cfg)) {
    const int cand[3] = {0, 4, 8};
    const double eff[3] = {0.81, 0.75, 0.74};
    double best_cost = 1e300;
    cfg = 0;
    for (int c = 0; c < 3; ++c) {
      const GemmCfg gc = gemm_cfg(DT_F32, cand[c]);
      double work = 0;
      for (const auto& e : leaves)
        work += (double)ceil_div(e.second.m, gc.bm) * ceil_div(e.second.n, gc.bn) * gc.bm * gc.bn * e.second.k;
      if (work / eff[c] < best_cost) {
        best_cost = work / eff[c];
        cfg = cand[c];
      }
    }
  }
  const GemmCfg gc = gemm_cfg(DT_F32, cfg);
  std::stable_sort(leaves.begin(), leaves.end(), [](const std::pair<int, GemmDesc>& x,
                                                    const std::pair<int, GemmDesc>& y) {
    return x.second.k > y.second.k;
  });
  // counters: per problem with levels, one per S/T level, one for the
  // leaves, one per U level above the top
  std::vector<std::vector<int>> c_st(count), c_u(count);
  std::vector<int> c_leaf(count, -1);
  int nctr = 0;
  for (int i = 0; i < count; ++i) {
    if (Ls[i] == 0) continue;
    for (int l = 0; l < Ls[i]; ++l) c_st[i].push_back(nctr++);
    c_leaf[i] = nctr++;
    c_u[i].assign(Ls[i], -1);
    for (int l = 1; l < Ls[i]; ++l) c_u[i][l] = nctr++;
  }
  // tasks per (problem, stage)
  auto ew_tasks = [](const EwPart& p) {
    return (int)ceil_div(ew_blocks(p.rows, p.cols, DT_F32), kPersistEwBlocks);
  };
  std::vector<std::vector<int>> n_st(count), n_u(count);
  std::vector<int> n_leaf(count, 0);
  for (int i = 0; i < count; ++i) {
    n_st[i].assign(Ls[i], 0);
    n_u[i].assign(Ls[i], 0);
  }
  for (int l = 0; l < Lmax; ++l) {
    for (const auto& e : st[l]) n_st[e.first][l] += ew_tasks(e.second);
    for (const auto& e : u[l]) n_u[e.first][l] += ew_tasks(e.second);
  }
  for (auto& e : leaves) {
    e.second.tiles_m = (int32_t)ceil_div(e.second.m, gc.bm);
    e.second.tiles_n = (int32_t)ceil_div(e.second.n, gc.bn);
    n_leaf[e.first] += e.second.tiles_m * e.second.tiles_n;
  }
  // segments
  PersistHdr hdr;
  std::memset(&hdr, 0, sizeof hdr);
  std::vector<uint8_t>& tab = P.table;
  tab.assign(round_up(sizeof(PersistHdr), 256), 0);
  int ntasks = 0;
  auto add_seg = [&](int kind, const std::vector<uint8_t>& descs, const std::vector<PDep>& deps, int nt) {
    if (deps.empty() || nt == 0) return;
    PSeg& sg = hdr.seg[hdr.nseg++];
    sg.kind = kind;
    sg.first = ntasks;
    sg.ntasks = nt;
    sg.ndesc = (int32_t)deps.size();
    sg.desc_off = (int64_t)tab.size();
    tab.insert(tab.end(), descs.begin(), descs.end());
    tab.resize(round_up(tab.size(), 256), 0);
    sg.dep_off = (int64_t)tab.size();
    const uint8_t* d = reinterpret_cast<const uint8_t*>(deps.data());
    tab.insert(tab.end(), d, d + deps.size() * sizeof(PDep));
    tab.resize(round_up(tab.size(), 256), 0);
    ntasks += nt;
  };
  auto ew_seg = [&](const std::vector<std::pair<int, EwPart>>& parts, auto dep_of) {
    std::vector<uint8_t> descs;
    std::vector<PDep> deps;
    int nt = 0;
    for (const auto& e : parts) {
      const int t = ew_tasks(e.second);
      if (t == 0) continue;
      PDep d = dep_of(e.first);
      d.task_start = nt;
      nt += t;
      const uint8_t* p = reinterpret_cast<const uint8_t*>(&e.second);
      descs.insert(descs.end(), p, p + sizeof(EwPart));
      deps.push_back(d);
      b.txt << Builder::ew_line(e.second);
      b.txt << "PDEP " << d.wait << " " << d.target << " " << d.signal << " " << d.task_start << " " << t << "\n";
    }
    add_seg(PT_EW, descs, deps, nt);
    if (nt) b.txt << "LAUNCH EW " << deps.size() << " " << nt << " persist\n";
  };
  for (int l = 0; l < Lmax; ++l) {
    std::vector<std::pair<int, EwPart>> parts = st[l];
    if (l == 0) parts.insert(parts.end(), zeros.begin(), zeros.end());
    ew_seg(parts, [&](int i) {
      if (Ls[i] == 0) return PDep{-1, 0, -1, 0};  // a zero fill
      return l == 0 ? PDep{-1, 0, c_st[i][0], 0} : PDep{c_st[i][l - 1], n_st[i][l - 1], c_st[i][l], 0};
    });
  }
  if (Lmax == 0) ew_seg(zeros, [](int) { return PDep{-1, 0, -1, 0}; });
  {
    std::vector<uint8_t> descs;
    std::vector<PDep> deps;
    int nt = 0;
    for (auto& e : leaves) {
      const int i = e.first;
      PDep d = Ls[i] ? PDep{c_st[i][Ls[i] - 1], n_st[i][Ls[i] - 1], c_leaf[i], nt} : PDep{-1, 0, -1, nt};
      e.second.tile_start = nt;
      nt += e.second.tiles_m * e.second.tiles_n;
      const uint8_t* p = reinterpret_cast<const uint8_t*>(&e.second);
      descs.insert(descs.end(), p, p + sizeof(GemmDesc));
      deps.push_back(d);
      b.txt << Builder::gemm_line(e.second);
      b.txt << "PDEP " << d.wait << " " << d.target << " " << d.signal << " " << d.task_start << " "
            << e.second.tiles_m * e.second.tiles_n << "\n";
    }
    add_seg(PT_GEMM, descs, deps, nt);
    if (nt) b.txt << "LAUNCH GEMM " << deps.size() << " " << nt << " " << cfg << " persist\n";
  }
  for (int l = Lmax - 1; l >= 0; --l)
    ew_seg(u[l], [&](int i) {
      const int L = Ls[i];
      const PDep w = l == L - 1 ? PDep{c_leaf[i], n_leaf[i], -1, 0} : PDep{c_u[i][l + 1], n_u[i][l + 1], -1, 0};
      return PDep{w.wait, w.target, l > 0 ? c_u[i][l] : -1, 0};
    });
  hdr.ntasks = ntasks;
  hdr.ncounters = nctr;
  std::memcpy(tab.data(), &hdr, sizeof hdr);
  P.ops.push_back(OpRec{OP_PERSIST, DT_F32, 0, ntasks, 0, cfg, 0, 0, 0});
  b.txt << "LAUNCH PERSIST 0 " << ntasks << " " << cfg << "\n";
  P.persistent = true;
  P.pcount = nctr;
  P.ws_bytes = (size_t)b.ws_peak * esz;
  P.text = b.txt.str();
  P.L = Lmax;
  return MM_OK;
}

// A batched plan: persistent (one launch) when asked for and float32,
// level-synchronous otherwise.
int build_batch_plan(Plan& P, int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                     const int* cutoff, const int* levels) {
  if ((P.flags & MM_PLAN_PERSISTENT) && P.dtype == MM_F32)
    return build_batched_persistent(P, count, mnk, A, B, C, cutoff, levels);
  return build_batched(P, count, mnk, A, B, C, cutoff, levels);
}

}  // namespace

int set_error(int code, const char* msg) { return fail(code, msg); }

int run_in_memory(int algo, int sched, int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C,
                  int cutoff, int levels, int dtype, void* table, size_t table_cap, void* ws, size_t ws_cap,
                  hipStream_t s) {
  int rc = check_enums(algo, sched, dtype);
  if (rc != MM_OK) return rc;
  const int64_t lda = std::max<int64_t>(k, 1), ldb = std::max<int64_t>(n, 1);
  rc = check_args(m, n, k, A, lda, B, ldb, C, ldb, dtype);
  if (rc != MM_OK) return rc;
  if (m == 0 || n == 0) return MM_OK;
  int dev = 0;
  rc = check_device(&dev);
  if (rc != MM_OK) return rc;
  char key[256];
  std::snprintf(key, sizeof key, "%d|%d|%d|%lld|%lld|%lld|%d|%d|%d", dev, algo, sched, (long long)m,
                (long long)n, (long long)k, cutoff, levels, dtype);
  Plan* P = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_host_plans.find(key);
    if (it == g_host_plans.end()) {
      std::unique_ptr<Plan> np;
      rc = make_plan(algo, sched, m, n, k, lda, ldb, ldb, cutoff, levels, dtype, 0, &np);
      if (rc != MM_OK) return rc;
      np->device = dev;
      it = g_host_plans.emplace(key, std::move(np)).first;
    }
    P = it->second.get();
  }
  if (P->has_aux || P->unfused) return fail(MM_E_UNSUPPORTED, "schedule needs plan-owned resources");
  if (P->table.size() > table_cap)
    return fail(MM_E_WORKSPACE, "descriptor table of " + std::to_string(P->table.size()) +
                                    " bytes exceeds the static scratch's table area of " +
                                    std::to_string(table_cap));
  if (P->ws_bytes > ws_cap)
    return fail(MM_E_WORKSPACE, "workspace of " + std::to_string(P->ws_bytes) +
                                    " bytes exceeds the static scratch's workspace area of " +
                                    std::to_string(ws_cap));
  if (P->ops.empty()) return MM_OK;
  if (!P->table.empty() &&
      hipMemcpyAsync(table, P->table.data(), P->table.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(MM_E_HIP, "copy of the descriptor table failed");
  return enqueue(*P, (void*)A, (void*)B, C, ws, s, nullptr, 1.0, table);
}

}  // namespace mm

struct mm_plan_s {
  std::unique_ptr<mm::Plan> p;
};

using namespace mm;

extern "C" {

const char* mm_last_error(void) { return g_err.c_str(); }

int mm_version(void) { return 1; }

int mm_naive(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int dtype,
             hipStream_t stream) {
  return short_form(MM_ALGO_NAIVE, m, n, k, A, B, C, 1, 0, dtype, stream);
}

int mm_strassen(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int cutoff,
                int levels, int dtype, hipStream_t stream) {
  return short_form(MM_ALGO_STRASSEN, m, n, k, A, B, C, cutoff, levels, dtype, stream);
}

int mm_winograd(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C, int cutoff,
                int levels, int dtype, hipStream_t stream) {
  return short_form(MM_ALGO_WINOGRAD, m, n, k, A, B, C, cutoff, levels, dtype, stream);
}

int mm_gemm_ex(int algo, int sched, int64_t m, int64_t n, int64_t k, void* A, int64_t lda, void* B,
               int64_t ldb, void* C, int64_t ldc, int cutoff, int levels, int dtype, void* ws,
               size_t ws_bytes, hipStream_t stream) {
  int rc = check_enums(algo, sched, dtype);
  if (rc != MM_OK) return rc;
  rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, dtype);
  if (rc != MM_OK) return rc;
  if (m == 0 || n == 0) return MM_OK;
  Plan* P = nullptr;
  rc = cached_plan(algo, sched, m, n, k, lda, ldb, ldc, cutoff, levels, dtype, &P);
  if (rc != MM_OK) return rc;
  return execute(*P, A, B, C, ws, ws_bytes, stream);
}

size_t mm_workspace_size(int algo, int sched, int64_t m, int64_t n, int64_t k, int cutoff, int levels,
                         int dtype) {
  std::unique_ptr<Plan> P;
  const int64_t lda = std::max<int64_t>(k, 1), ldb = std::max<int64_t>(n, 1);
  if (make_plan(algo, sched, m, n, k, lda, ldb, ldb, cutoff, levels, dtype, 0, &P) != MM_OK) return 0;
  return P->ws_bytes;
}

int mm_set_workspace(void* ws, size_t bytes, hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MM_E_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  WsEntry& w = g_ws[{dev, stream}];
  if (w.owned && w.ptr) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(w.ptr);
  }
  w.ptr = (ws && bytes) ? ws : nullptr;
  w.bytes = (ws && bytes) ? bytes : 0;
  w.owned = false;
  return MM_OK;
}

int mm_plan_create(int algo, int sched, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                   int64_t ldc, int cutoff, int levels, int dtype, unsigned flags, mm_plan_t* plan) {
  if (!plan) return fail(MM_E_INVALID, "NULL plan pointer");
  *plan = nullptr;
  if ((m > 0 && k > 0 && lda < k) || (k > 0 && n > 0 && ldb < n) || (m > 0 && n > 0 && ldc < n))
    return fail(MM_E_INVALID, "leading dimension shorter than a row");
  std::unique_ptr<Plan> P;
  int rc = make_plan(algo, sched, m, n, k, lda, ldb, ldc, cutoff, levels, dtype, flags, &P);
  if (rc != MM_OK) return rc;
  rc = upload(*P);
  if (rc != MM_OK) return rc;
  *plan = new mm_plan_s{std::move(P)};
  return MM_OK;
}

int mm_plan_execute(mm_plan_t plan, void* A, void* B, void* C, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
  if (!plan || !plan->p) return fail(MM_E_INVALID, "NULL plan");
  Plan& P = *plan->p;
  if (!P.batched) {
    int rc = check_args(P.m, P.n, P.k, A, P.lda, B, P.ldb, C, P.ldc, P.dtype);
    if (rc != MM_OK) return rc;
  }
  return execute(P, A, B, C, ws, ws_bytes, stream);
}

int mm_plan_execute_beta(mm_plan_t plan, void* A, void* B, void* C, void* ws, size_t ws_bytes, double beta,
                         hipStream_t stream) {
  if (!plan || !plan->p) return fail(MM_E_INVALID, "NULL plan");
  Plan& P = *plan->p;
  if (!P.accumulate) return fail(MM_E_INVALID, "plan was not created with MM_PLAN_ACCUMULATE");
  if (!std::isfinite(beta)) return fail(MM_E_INVALID, "beta must be finite");
  int rc = check_args(P.m, P.n, P.k, A, P.lda, B, P.ldb, C, P.ldc, P.dtype);
  if (rc != MM_OK) return rc;
  return execute(P, A, B, C, ws, ws_bytes, stream, beta);
}

int mm_plan_execute_timed(mm_plan_t plan, void* A, void* B, void* C, void* ws, size_t ws_bytes,
                          hipStream_t stream, hipEvent_t* events, int nevents) {
  if (!plan || !plan->p) return fail(MM_E_INVALID, "NULL plan");
  Plan& P = *plan->p;
  if (!events || nevents < 2 * (int)P.ops.size())
    return fail(MM_E_INVALID, "need two events per launch");
  if (!P.batched) {
    int rc = check_args(P.m, P.n, P.k, A, P.lda, B, P.ldb, C, P.ldc, P.dtype);
    if (rc != MM_OK) return rc;
  }
  if (ws_bytes < P.ws_bytes || (P.ws_bytes > 0 && ws == nullptr))
    return fail(MM_E_WORKSPACE, "workspace smaller than the plan needs");
  if (P.spl && P.ws_bytes > 0 && ((uintptr_t)ws & 15))
    return fail(MM_E_INVALID, "split-bfloat16 plans need a 16-byte aligned workspace");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != P.device)
    return fail(MM_E_INVALID, "plan was built for another device");
  if (P.fused_reads_ab && misaligned_ab(A, B))
    return fail(MM_E_UNSUPPORTED, "timed execution of a fused plan needs 16-byte aligned A and B");
  return enqueue(P, A, B, C, ws, stream, events);
}

int mm_plan_op_kind(mm_plan_t plan, int i) {
  if (!plan || !plan->p || i < 0 || i >= (int)plan->p->ops.size()) return -1;
  return plan->p->ops[i].type + 8 * plan->p->ops[i].stream;
}

int mm_plan_info(mm_plan_t plan, int64_t* info, int ninfo) {
  if (!plan || !plan->p || !info) return 0;
  const Plan& P = *plan->p;
  const int64_t v[11] = {(int64_t)P.ws_bytes, P.L, P.M, P.N, P.K, (int64_t)P.ops.size(), P.leaves, P.sched,
                         P.leaf_rows, P.fused ? 1 : 0, P.wino ? 1 : 0};
  const int cnt = std::min(ninfo, 11);
  for (int i = 0; i < cnt; ++i) info[i] = v[i];
  return cnt;
}

size_t mm_plan_describe(mm_plan_t plan, char* buf, size_t len) {
  if (!plan || !plan->p) return 0;
  const std::string& t = plan->p->text;
  if (buf && len) {
    const size_t c = std::min(len - 1, t.size());
    std::memcpy(buf, t.data(), c);
    buf[c] = 0;
  }
  return t.size();
}

int mm_plan_destroy(mm_plan_t plan) {
  delete plan;
  return MM_OK;
}

size_t mm_describe(int algo, int sched, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                   int64_t ldc, int cutoff, int levels, int dtype, unsigned flags, char* buf, size_t len,
                   int64_t* info, int ninfo) {
  std::unique_ptr<Plan> P;
  if (make_plan(algo, sched, m, n, k, lda, ldb, ldc, cutoff, levels, dtype, flags, &P) != MM_OK) return 0;
  mm_plan_s tmp{std::move(P)};
  if (info) mm_plan_info(&tmp, info, ninfo);
  const size_t r = mm_plan_describe(&tmp, buf, len);
  return r ? r : 1;
}

size_t mm_batched_describe(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                           int dtype, const int* cutoff, const int* levels, unsigned flags, char* buf,
                           size_t len, int64_t* info, int ninfo) {
  if (count < 0 || (count > 0 && (!mnk || !A || !B || !C))) return 0;
  if (check_enums(MM_ALGO_WINOGRAD, MM_SCHED_GROUPED, dtype) != MM_OK) return 0;
  std::unique_ptr<Plan> P(new Plan);
  P->algo = MM_ALGO_WINOGRAD;
  P->sched = MM_SCHED_GROUPED;
  P->dtype = dtype;
  P->batched = true;
  P->flags = flags;
  P->tile_cfg = (int)((flags >> 8) & 0xff) - 1;
  if (build_batch_plan(*P, count, mnk, A, B, C, cutoff, levels) != MM_OK) return 0;
  mm_plan_s tmp{std::move(P)};
  if (info) mm_plan_info(&tmp, info, ninfo);
  const size_t r = mm_plan_describe(&tmp, buf, len);
  return r ? r : 1;
}

size_t mm_batched_table(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                        int dtype, const int* cutoff, const int* levels, unsigned flags, void* buf, size_t len) {
  if (count < 0 || (count > 0 && (!mnk || !A || !B || !C))) return 0;
  if (check_enums(MM_ALGO_WINOGRAD, MM_SCHED_GROUPED, dtype) != MM_OK) return 0;
  Plan P;
  P.algo = MM_ALGO_WINOGRAD;
  P.sched = MM_SCHED_GROUPED;
  P.dtype = dtype;
  P.batched = true;
  P.flags = flags;
  P.tile_cfg = (int)((flags >> 8) & 0xff) - 1;
  if (build_batch_plan(P, count, mnk, A, B, C, cutoff, levels) != MM_OK) return 0;
  if (buf) std::memcpy(buf, P.table.data(), std::min(len, P.table.size()));
  return P.table.size();
}

int mm_batched_plan_create(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C,
                           int dtype, const int* cutoff, const int* levels, unsigned flags, mm_plan_t* plan) {
  if (!plan) return fail(MM_E_INVALID, "NULL plan pointer");
  *plan = nullptr;
  if (count < 0 || (count > 0 && (!mnk || !A || !B || !C))) return fail(MM_E_INVALID, "bad batch arrays");
  int rc = check_enums(MM_ALGO_WINOGRAD, MM_SCHED_GROUPED, dtype);
  if (rc != MM_OK) return rc;
  if (flags & MM_PLAN_ACCUMULATE) return fail(MM_E_UNSUPPORTED, "batched plans do not accumulate");
  std::unique_ptr<Plan> P(new Plan);
  P->algo = MM_ALGO_WINOGRAD;
  P->sched = MM_SCHED_GROUPED;
  P->dtype = dtype;
  P->batched = true;
  P->flags = flags;
  P->tile_cfg = (int)((flags >> 8) & 0xff) - 1;
  if (P->tile_cfg >= kNumGemmCfg) return fail(MM_E_INVALID, "unknown tile configuration");
  rc = build_batch_plan(*P, count, mnk, A, B, C, cutoff, levels);
  if (rc != MM_OK) return rc;
  rc = upload(*P);
  if (rc != MM_OK) return rc;
  *plan = new mm_plan_s{std::move(P)};
  return MM_OK;
}

int mm_batched_levels(int count, const int64_t* mnk, int dtype, const int* cutoff, const int* levels,
                      int* levels_out) {
  if (count < 0 || (count > 0 && (!mnk || !levels_out))) return fail(MM_E_INVALID, "bad batch arrays");
  int rc = check_enums(MM_ALGO_WINOGRAD, MM_SCHED_GROUPED, dtype);
  if (rc != MM_OK) return rc;
  for (int i = 0; i < count; ++i)
    if (mnk[3 * i] < 0 || mnk[3 * i + 1] < 0 || mnk[3 * i + 2] < 0)
      return fail(MM_E_INVALID, "negative dimension in batch");
  std::vector<int> cut, lev;
  resolve_batch(count, mnk, dtype, cutoff, levels, cut, lev);
  for (int i = 0; i < count; ++i) {
    const int64_t m = mnk[3 * i], n = mnk[3 * i + 1], k = mnk[3 * i + 2];
    levels_out[i] = (m == 0 || n == 0 || k == 0) ? 0 : count_levels(m, n, k, cut[i], lev[i]);
  }
  return MM_OK;
}

const char* mm_tuning_source(void) { return class_table().source.c_str(); }

int mm_plan_check(mm_plan_t plan, hipStream_t stream) {
  if (!plan || !plan->p) return fail(MM_E_INVALID, "NULL plan");
  Plan& P = *plan->p;
  if (!P.persistent || !P.dctr) return MM_OK;
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(MM_E_HIP, "hipStreamSynchronize failed");
  int flag = 0;
  if (hipMemcpy(&flag, P.dctr + PC_ERROR, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MM_E_HIP, "reading the plan's error flag failed");
  if (flag) {
    const int zero = 0;
    (void)hipMemcpy(P.dctr + PC_ERROR, &zero, sizeof zero, hipMemcpyHostToDevice);
    return fail(MM_E_HIP, "a task of the persistent launch waited past its bound; results since the last "
                          "check are not reliable");
  }
  return MM_OK;
}

int mm_batched(int count, const int64_t* mnk, void* const* A, void* const* B, void* const* C, int dtype,
               const int* cutoff, const int* levels, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (count < 0 || (count > 0 && (!mnk || !A || !B || !C))) return fail(MM_E_INVALID, "bad batch arrays");
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != MM_OK) return rc;
  std::ostringstream key;
  for (int i = 0; i < count; ++i)
    if (mnk[3 * i] < 0 || mnk[3 * i + 1] < 0 || mnk[3 * i + 2] < 0)
      return fail(MM_E_INVALID, "negative dimension in batch");
  std::vector<int> cut, lev;
  resolve_batch(count, mnk, dtype, cutoff, levels, cut, lev);
  key << "B|" << dev << "|" << dtype << "|" << count;
  for (int i = 0; i < count; ++i)
    key << "|" << mnk[3 * i] << "," << mnk[3 * i + 1] << "," << mnk[3 * i + 2] << "," << A[i] << "," << B[i]
        << "," << C[i] << "," << cut[i] << "," << lev[i];
  Plan* P = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_plans.find(key.str());
    if (it == g_plans.end()) {
      std::unique_ptr<Plan> np(new Plan);
      np->algo = MM_ALGO_WINOGRAD;
      np->sched = MM_SCHED_GROUPED;
      np->dtype = dtype;
      np->batched = true;
      rc = check_enums(MM_ALGO_WINOGRAD, MM_SCHED_GROUPED, dtype);
      if (rc != MM_OK) return rc;
      rc = build_batch_plan(*np, count, mnk, A, B, C, cut.data(), lev.data());
      if (rc != MM_OK) return rc;
      rc = upload(*np);
      if (rc != MM_OK) return rc;
      it = g_plans.emplace(key.str(), std::move(np)).first;
    }
    P = it->second.get();
  }
  return execute(*P, nullptr, nullptr, nullptr, ws, ws_bytes, stream);
}

}  // extern "C"
