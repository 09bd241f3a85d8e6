// Internal structures shared by the planner (host) and the kernels (device).
#pragma once

#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

#include "fmm_tables.h"

namespace fmm {

// Buffers a descriptor can point into.  A, B and C are the caller's operands
// (their leading dimensions arrive with each multiply); WS is the workspace.
enum Buf : int32_t { BUF_A = 0, BUF_B = 1, BUF_C = 2, BUF_WS = 3, BUF_NONE = -1 };

// Element type of a buffer region.  ELT_BF16X2 is a split FP32 operand of the
// BF16x3 path: two bfloat16 planes, hi = bf16(x) and lo = bf16(x - hi), the lo
// plane `plane` elements after the hi plane.  Leaf S operands are split
// row-major (element (i, j) of a plane at i * ld + j); leaf T operands are
// split in k-octets (element (k, n) at (k / 8) * ld + n * 8 + k % 8, ld = 8 *
// columns), so the 8 consecutive k of one column that a matrix-core fragment
// takes are one 16-byte group in both cases.
enum Elt : int32_t { ELT_F64 = 0, ELT_F32 = 1, ELT_BF16X2 = 2 };

// A strided matrix view: element (i, j) is at
//   base[buf] + off + (row + i) * LD + (col + j),  LD = ld[buf] for A/B/C, else ld.
// alpha scales every element read through the view (single-non-zero columns of
// U or V become such views instead of copies).  Split regions (ELT_BF16X2)
// are never views; their addressing is the one described above.
struct Ref {
  int32_t buf;
  int32_t elt;
  int64_t off;
  int64_t row;
  int64_t col;
  int64_t ld;
  double alpha;
  int64_t plane = 0;  // ELT_BF16X2: element offset of the lo plane
};

struct Bases {
  void* ptr[4];
  int64_t ld[4];
};

// One pass of operand formation: every group has one source view and R^lv
// outputs (workspace element offsets, -1 where the output is a view instead).
// Output element (p, q) of output o of group g is
//   sum over the lv-level Kronecker product of the side's coefficient matrix
//   applied to the (BR*BC)^lv blocks of the group's source at position (p, q).
struct FormPass {
  int alg = -1;   // base case of the pass's levels
  int side;       // 0: A side (U, blocks M x K); 1: B side (V, blocks K x N)
  int lv;         // levels fused in this pass (1 or 2)
  int depth_in;   // depth of the sources (0 = the input matrix)
  int64_t h, w;   // output block dims = position grid
  int64_t out_ld;
  int out_elt;
  int64_t out_plane = 0;  // ELT_BF16X2 outputs: offset of the lo plane
  int ngroups;
  int nout;       // R^lv
  std::vector<Ref> groups;
  std::vector<int64_t> outs;  // ngroups * nout
  size_t dev_groups = 0, dev_outs = 0;  // byte offsets in the plan's device table
};

// One pass of the W-combination: group g reads R^lv inputs laid out at
// in_off + r * in_stride (r in leaf order, ld in_ld) and writes one output
// matrix of (BR^lv h) x (BC^lv w) through `out`.  The last pass (depth 0)
// writes C and adds the k-peel product P when present.
struct CombinePass {
  int alg = -1;   // base case of the pass's levels
  int lv;
  int depth_in;
  int64_t h, w;
  int in_elt;
  int64_t in_ld, in_stride;
  int ngroups;
  std::vector<int64_t> in_off;  // per group
  std::vector<Ref> out;         // per group
  bool has_p = false;
  Ref p;                        // k-peel product (m0 x n0) when has_p
  size_t dev_in = 0, dev_out = 0;
};

// A leaf operand formed while the GEMM stages it (plans with leaf_form): the
// sum over n terms of coef * (alpha times the block at (row + drow, col +
// dcol) of the operand's view), as the formation pass would have written it.
// Unused terms have coef 0.
constexpr int kMaxLeafTerms = 2;
struct LeafTerms {
  int32_t n;
  int32_t coef[kMaxLeafTerms];
  int32_t pad_;
  int64_t drow[kMaxLeafTerms], dcol[kMaxLeafTerms];
};

struct GemmProb {
  Ref a, b, c;
  double alpha;
  double pad;
  LeafTerms fa, fb;  // read only by the forming kernels (GemmArgs::form_terms > 0)
};

// Problems of identical shape; tiles of all groups form one flat index space.
// A launch may hold the groups of several plans (a batch): each group names
// its plan's problem array and the slot of that plan's operand bases.
struct GemmGroup {
  int64_t m, n, k;
  int64_t count;
  int64_t tiles_m, tiles_n;
  int64_t tile_start;  // first flat tile index of this group
  int64_t prob_start;  // index of the group's first problem in `probs`
  const GemmProb* probs = nullptr;  // device array; NULL means GemmArgs::single
  int32_t slot = 0;                 // index into GemmArgs::bases
  int32_t split = 0;                // 1: every problem's operands are split planes (ELT_BF16X2)
};

constexpr int kMaxGemmGroups = 24;  // groups per launch (a plan has at most 4)
constexpr int kMaxGemmSlots = 8;    // plans per launch

struct GemmArgs {
  Bases bases[kMaxGemmSlots];
  GemmProb single;
  int ngroups;
  int elt;
  int tile;  // output tile edge of the FP64 / FP32 kernel: 64, 128, or 0 (chosen at launch)
  int form_terms;  // 0: plain operands; kMaxLeafTerms: every problem forms A and B from LeafTerms
  int dma;         // FP64 / FP32: every problem's operands allow the direct-load kernels (leaf_dma_ok)
  int pad_;
  int64_t total_tiles;
  GemmGroup groups[kMaxGemmGroups];
};

struct FormArgs {
  Bases bases;
  const Ref* groups;
  const int64_t* outs;
  int64_t h, w, out_ld;
  int out_elt;
  int nout;
  int64_t out_plane;
};

struct CombineArgs {
  Bases bases;
  const int64_t* in_off;
  const Ref* out;
  int64_t h, w, in_ld, in_stride;
  int in_elt;
  int has_p;
  Ref p;
  // set by the host: FP32 products and outputs, no k-peel term, and every
  // pair of adjacent positions 8-byte aligned in the products and in C
  int pairs;
};

// --- plan -----------------------------------------------------------------

struct LeafRef {
  Ref s, t, m;
};

struct Plan {
  int alg_id = -1;  // -1: classical (no recursion); else the top level's base case
  std::vector<int> lv_alg;  // base case of every level, top first
  std::string alg_name;     // "classical", a base case, or one base case per level joined by '+'
  int M = 1, K = 1, N = 1, R = 1;
  int64_t m = 0, k = 0, n = 0;
  int levels = 0;
  int dtype = 0;
  int fuse = 1;       // recursion levels fused per addition pass
  int elt = ELT_F64;  // element type of A, B, C and the leaf operands
  int64_t m0 = 0, k0 = 0, n0 = 0, ml = 0, kl = 0, nl = 0;

  std::vector<FormPass> s_passes, t_passes;
  std::vector<CombinePass> w_passes;
  std::vector<GemmGroup> gemm_groups;
  std::vector<GemmProb> gemm_probs;
  std::vector<LeafRef> leaves;
  int64_t gemm_tiles = 0;
  int64_t s_mat = 0, t_mat = 0;

  size_t ws_bytes = 0;
  size_t table_bytes = 0;
  std::vector<unsigned char> table;  // host image of the device descriptor table
  size_t dev_probs = 0;

  // device side
  bool host_only = true;
  int device = -1;
  void* ws = nullptr;
  void* dev_table = nullptr;
  int timing_slots = 0;         // 0: timing off; else ring of this many multiplies
  std::vector<void*> events;    // (stages + 1) HIP events per slot
  int64_t timed = 0;            // timed multiplies since timing was enabled
  bool external = false;        // device memory bound by the caller (not owned)
  bool use_graph = false;       // replay the stages as a captured HIP graph
  bool pair_form = false;       // S and T formed by one launch (small one-level plans)
  int leaf_form = 0;            // > 0: the leaf GEMM forms S and T while staging them, with
                                // this many term slots (kMaxLeafTerms); multiply skips the passes
  int leaf_tile = 0;            // FP64 / FP32 leaf tile edge: 64, 128, or 0 (chosen per launch)
  void* graph_exec = nullptr;   // hipGraphExec_t of the last capture
  void* cap_stream = nullptr;   // private stream the capture is recorded on
  Bases graph_key{};            // operand bases the captured graph was made for

  double leaf_flops = 0, add_bytes = 0, gemm_min_bytes = 0;
};

// Plans on the host only; fills every field above except the device side.
// Returns an empty string on success, else the error message (and sets *code).
std::string make_plan(Plan& P, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                      int dtype, int fuse, int* code, int leaf_form = 0);

int find_algorithm(const char* name);  // -1 for "classical", -2 unknown

// Base case of every recursion level, top first.  `alg` names one base case
// (used at every level) or one per level joined by '+' (Section 5.2 composes
// different base cases across levels; their count must equal `levels`).
// Returns -1 for "classical" (ids empty), 0 with `levels` ids, or an error
// status (FMM_EALG unknown name, FMM_EINVAL malformed list) with *err set.
int parse_levels(const char* alg, int levels, std::vector<int>* ids, std::string* err);

// What make_plan would produce, without its R^L descriptors: the GEMM groups
// (tiles filled in), the addition bytes, the workspace bytes and the pass
// counts, computed per pass from view counts in O(levels).  Equal to the
// corresponding fields of make_plan for every input (a host test checks it).
struct PlanSummary {
  int levels = 0, fuse = 0;
  std::vector<GemmGroup> groups;
  double add_bytes = 0, leaf_flops = 0;
  size_t ws_bytes = 0;
  int form_passes = 0, comb_passes = 0;
  bool pair_form = false;  // S and T formed by one launch (Plan::pair_form)
  int leaf_form = 0;       // S and T formed inside the leaf GEMM (Plan::leaf_form)
};



// Plans of one level whose S and T passes together cover at most this many
// output positions form both in one launch (Plan::pair_form).
constexpr int64_t kPairFormMaxPositions = int64_t(1) << 20;
std::string summarize_plan(PlanSummary& S, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                           int dtype, int fuse, int leaf_form = 0);

// Sets the calling thread's error message (fmm_last_error); returns code.
int set_error(int code, const std::string& msg);

// One candidate of the cost model (fmm_tune.cpp).
struct Candidate {
  char alg[80];
  int levels = 0;
  int fuse = 0;
  int tile = 0;  // leaf tile edge of a recorded choice; 0: chosen per launch
  double model_ms = 0, leaf_ms = 0, add_ms = 0;
  size_t ws_bytes = 0;
  double err = 0;  // predicted error bound (error_bound)
};

// Root-mean-square growth of the rounding error per recursive step of base
// case `id`, for operands with i.i.d. zero-mean entries:
//   sqrt(sum_r |u_r|^2 |v_r|^2 |w_r|^2 / (M K N))
// (u_r, v_r: columns r of U and V; w_r: column r of W).  1 for a classical
// step, 2 for Strassen.
double growth(int id);

// Predicted bound on the relative Frobenius error of C against the exact
// product for a plan whose levels use the base cases `ids` (top first; empty
// for the classical product), inner dimension k and dtype:
//   e0 * prod growth(ids),  e0 = c + (2 + sqrt(k)) u
// with u the unit roundoff of the leaf arithmetic (2^-53 FP64, 2^-24 FP32)
// and c = 3 * 2^-16 on the BF16x3 path (two split residuals and the dropped
// lo*lo term per product term), 0 otherwise.
double error_bound(const std::vector<int>& ids, int64_t k, int dtype);

// Largest error bound the automatic choice accepts for dtype when the caller
// gives 0: 1e-12 (FP64), 1e-4 (FP32), 5e-4 (BF16x3).
double default_max_error(int dtype);

// Argument checks of one product C = A*B (m x k by k x n, element size es):
// leading dimensions, NULL pointers with non-zero sizes, C overlapping A or
// B.  0 when valid, else an fmm_status with *why set.
int check_operands(int64_t m, int64_t k, int64_t n, size_t es, const void* A, int64_t lda, const void* B,
                   int64_t ldb, const void* C, int64_t ldc, std::string* why);

// Workspace budget: FMM_HBM_BUDGET (bytes) if set, else 3/4 of the current
// device's free memory, else 3/4 of 288 GB.
size_t default_budget();

// Candidates for (m, k, n, dtype), best predicted first; alg NULL or "auto"
// for every base case, else only that one ("classical" gives the plain GEMM).
// Candidates whose workspace exceeds `budget` (0: default_budget) or whose
// error bound exceeds `max_error` (0: default_max_error, < 0: no limit) are
// left out.  Returns an error message or "".
std::string rank_candidates(int64_t m, int64_t k, int64_t n, int dtype, const char* alg, size_t budget,
                            int fuse, double max_error, std::vector<Candidate>& out);

// Measured choices recorded by an autotuner (fmm_tune_record), keyed by the
// exact (m, k, n, dtype).
void record_tuned(int64_t m, int64_t k, int64_t n, int dtype, const Candidate& c);
bool lookup_tuned(int64_t m, int64_t k, int64_t n, int dtype, Candidate* c);
void clear_tuned();

// The plan to make for alg ("auto"/NULL = any base case) at `levels` (-1 =
// any depth): a recorded measured choice when alg is "auto" and levels -1 and
// one exists for the shape (and fits the budget and max_error), else the
// model's best within both.  False with *why on failure.
bool choose(int64_t m, int64_t k, int64_t n, int dtype, const char* alg, int levels, size_t budget, int fuse,
            double max_error, Candidate* pick, std::string* why);

constexpr int64_t kTileM = 128, kTileN = 128;

// Which 128 x 128 kernel a launch would run, for use_small_tiles.
enum TileKernel { kTilesStaged = 0, kTilesBf16x3 = 1, kTilesF64Dma = 2, kTilesF32Dma = 3 };

// Whether a leaf launch of `tiles128` tiles of kTileM x kTileN on `cus`
// compute units runs 64 x 64 tiles instead: when the large tiles would leave
// compute units idle.  Every kernel: fewer tiles than compute units.  The
// register-staged FP64 / FP32 kernel (whose small tile keeps 74-93% of its
// rate) also at most four waves of two tiles per CU whose last wave is at most
// half full; the FP64 direct-load kernel, faster than the small tile by more,
// only when that last wave is partial and follows a full one (at exactly one
// tile per CU the large tiles measured 16% faster); the FP32 direct-load
// kernel, which holds four tiles per CU, and BF16x3 (68%) never.
inline bool use_small_tiles(int64_t tiles128, int64_t cus, int kind = kTilesStaged) {
  if (tiles128 < cus) return true;
  const int64_t rem = tiles128 % (2 * cus);
  const bool partial = tiles128 < 4 * cus && rem > 0 && rem <= cus;
  if (kind == kTilesStaged) return partial;
  if (kind == kTilesF64Dma) return partial && tiles128 > 2 * cus;
  return false;
}

}  // namespace fmm
