// Planner: static peeling, the operand tree with single-non-zero views, the
// pass schedule of the addition kernels, the workspace layout and the grouped
// GEMM problem list.  Host-only code; no HIP calls.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "fmm_internal.h"

namespace fmm {

namespace {

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

size_t elt_size(int elt) { return elt == ELT_F64 ? 8 : 4; }

// Leading dimension of a workspace matrix of width w (elements of es bytes):
// a multiple of 16 elements; FP64 rows of 2 KB or more get 16 more, so that
// the rows of one leaf tile are not a power-of-two stride apart (such rows
// crowd into a few L2 sets and memory channels).  Measured at 16384^3: the
// FP64 leaf launch gains 2%; FP32 leaves gain less than the FP32
// combination pass loses reading padded products, so FP32 rows stay unpadded.
int64_t ws_ld(int64_t w, size_t es) {
  const int64_t ld = round_up(w, 16);
  return es == 8 && ld * 8 >= 2048 ? ld + 16 : ld;
}

struct Arena {
  size_t used = 0;
  // Returns the byte offset of a fresh 256-byte aligned region.
  size_t alloc(size_t bytes) {
    size_t off = round_up((int64_t)used, 256);
    used = off + bytes;
    return off;
  }
};

// Number of non-zeros in column r of a (rows x R) coefficient table, and the
// row of the last one.
int col_nnz(const signed char* X, int rows, int R, int r, int* where, int* coef) {
  int cnt = 0;
  for (int i = 0; i < rows; ++i) {
    if (X[i * R + r] != 0) {
      ++cnt;
      *where = i;
      *coef = X[i * R + r];
    }
  }
  return cnt;
}

// Levels fused per addition pass (1 or 2).  An explicit request wins, then
// the FMM_FUSE environment variable; by default two levels are fused (fewer
// bytes: the level-one intermediates are never written), except for BF16x3
// plans of wide base cases (R > 8), whose split T operands in k-octets are
// formed by the register kernel, which measured slower fused than unfused.
// Plans whose levels use different base cases always run one level per pass.
// Whether base case `id` can fuse two levels per addition pass: narrow ones
// (R <= 8) in registers, wide ones through LDS, which holds the (BR*BC)^2
// sources of 64 positions (at most 11 blocks per side) and the products of 4
// top-level indices (R <= 32).  The kernels compile the two-level variants
// only for these (kFuse2 in fmm_add_kernels.h states the same rule).
bool fuse2_ok(int id) {
  const AlgInfo& a = alg_info(id);
  return a.R <= 8 || (a.M * a.K <= 11 && a.K * a.N <= 11 && a.R <= 32);
}

int resolve_fuse(int requested, int R, int dtype, const std::vector<int>& ids) {
  for (int id : ids)
    if (id != ids[0]) return 1;  // levels of different base cases: one level per pass
  if (!ids.empty() && !fuse2_ok(ids[0])) return 1;  // too wide for the two-level kernels
  if (requested == 1 || requested == 2) return requested;
  const char* e = std::getenv("FMM_FUSE");
  if (e && (e[0] == '1' || e[0] == '2') && e[1] == 0) return e[0] - '0';
  return (dtype == 2 && R > 8) ? 1 : 2;  // dtype 2: FP32 inputs with BF16x3 leaves
}

// Term slots a plan needs to form its leaf operands inside the leaf GEMM
// (kMaxLeafTerms), or 0 when it cannot: one level, FP64 / FP32 (the BF16x3
// leaves read split operands), every S and T column with at most
// kMaxLeafTerms non-zeros (Strassen and its direct sums), all of them +-1 (a
// multiply-add then rounds like the pass's add or subtract).
int leaf_form_terms(const std::vector<int>& ids, int levels, int dtype) {
  if (levels != 1 || dtype == 2 || ids.size() != 1) return 0;
  const AlgInfo& A = alg_info(ids[0]);
  int most = 0;
  for (int side = 0; side < 2; ++side) {
    const signed char* X = side == 0 ? A.U : A.V;
    const int rows = side == 0 ? A.M * A.K : A.K * A.N;
    for (int r = 0; r < A.R; ++r) {
      int nz = 0;
      for (int i = 0; i < rows; ++i) {
        const int c = X[i * A.R + r];
        if (c != 0 && c != 1 && c != -1) return 0;
        nz += c != 0;
      }
      most = nz > most ? nz : most;
    }
  }
  return most <= kMaxLeafTerms ? kMaxLeafTerms : 0;
}

// Splits L levels into passes of at most `fuse` levels.  Operand formation
// runs top-down and keeps the fused pass at the bottom (fewest bytes: the
// R^L outputs are written once); the combination runs bottom-up with the
// fused pass first, for the same reason.
std::vector<int> schedule(int L, int fuse, bool top_down) {
  std::vector<int> s;
  int rest = L;
  while (rest > 0) {
    int lv = rest >= fuse ? fuse : rest;
    if (top_down && rest > fuse) lv = 1;
    s.push_back(lv);
    rest -= lv;
  }
  return s;
}

// Passes of a plan whose levels use the base cases `ids`: as schedule() when
// every level uses the same one, else one level per pass (a fused pass needs
// one base case for both of its levels).
std::vector<int> schedule_ids(const std::vector<int>& ids, int fuse, bool top_down) {
  for (int id : ids)
    if (id != ids[0]) return std::vector<int>(ids.size(), 1);
  return schedule((int)ids.size(), fuse, top_down);
}

// Products of a per-level dimension over the first d levels, d = 0..L.
std::vector<int64_t> prefix(const std::vector<int>& ids, int which) {
  std::vector<int64_t> p(ids.size() + 1, 1);
  for (size_t l = 0; l < ids.size(); ++l) {
    const AlgInfo& A = alg_info(ids[l]);
    const int v = which == 0 ? A.M : which == 1 ? A.K : which == 2 ? A.N : A.R;
    p[l + 1] = p[l] * v;
  }
  return p;
}

// Layout of a split (BF16x3) leaf operand of h x w elements: S (side 0)
// row-major with rows padded to 8 elements; T (side 1) in k-octets, one group
// of 8 consecutive rows per `ld` = 8 w elements.  *plane = elements per plane
// (the lo plane follows the hi plane).
void split_layout(int side, int64_t h, int64_t w, int64_t* ld, int64_t* plane) {
  if (side == 0) {
    *ld = round_up(w, 8);
    *plane = h * *ld;
  } else {
    *ld = 8 * w;
    *plane = round_up(h, 8) / 8 * *ld;
  }
}

struct Node {
  Ref ref;
};

// Builds the operand-formation passes of one side.  Returns leaf refs.
std::vector<Ref> plan_side(Plan& P, int side, Arena& ws, std::vector<FormPass>& passes,
                           int64_t* materialized, double* bytes) {
  const std::vector<int64_t> rdiv = prefix(P.lv_alg, side == 0 ? 0 : 1);
  const std::vector<int64_t> cdiv = prefix(P.lv_alg, side == 0 ? 1 : 2);
  const int64_t rows0 = side == 0 ? P.m0 : P.k0;
  const int64_t cols0 = side == 0 ? P.k0 : P.n0;
  const int in_elt = P.elt;

  std::vector<Ref> nodes(1);
  nodes[0] = Ref{side == 0 ? BUF_A : BUF_B, in_elt, 0, 0, 0, 0, 1.0};
  int depth = 0;
  *materialized = 0;
  for (int lv : schedule_ids(P.lv_alg, P.fuse, true)) {
    const AlgInfo& A = alg_info(P.lv_alg[depth]);  // every level of a fused pass uses it
    const int BC = side == 0 ? A.K : A.N;
    const int NB = (side == 0 ? A.M : A.K) * BC;
    const int R = A.R;
    const signed char* coef = side == 0 ? A.U : A.V;
    const int d2 = depth + lv;
    const bool final_pass = d2 == P.levels;
    // the BF16x3 path writes its leaf operands split (hi / lo planes)
    const bool split = final_pass && P.dtype == 2;
    FormPass fp;
    fp.alg = P.lv_alg[depth];
    fp.side = side;
    fp.lv = lv;
    fp.depth_in = depth;
    fp.h = rows0 / rdiv[d2];
    fp.w = cols0 / cdiv[d2];
    fp.out_elt = split ? ELT_BF16X2 : final_pass ? P.elt : ELT_F64;
    fp.out_ld = ws_ld(fp.w, elt_size(fp.out_elt));
    fp.ngroups = (int)nodes.size();
    fp.nout = (int)ipow(R, lv);
    size_t region = (size_t)fp.h * fp.out_ld * elt_size(fp.out_elt);
    if (split) {
      split_layout(side, fp.h, fp.w, &fp.out_ld, &fp.out_plane);
      region = (size_t)fp.out_plane * 2 * 2;  // two planes of bf16
    }
    std::vector<Ref> next;
    next.reserve(nodes.size() * fp.nout);
    for (const Ref& g : nodes) {
      fp.groups.push_back(g);
      *bytes += (double)ipow(NB, lv) * fp.h * fp.w * elt_size(g.elt);
      for (int o = 0; o < fp.nout; ++o) {
        // digits r_1..r_lv of o, r_1 most significant
        int digits[8];
        int t = o;
        for (int j = lv - 1; j >= 0; --j) {
          digits[j] = t % R;
          t /= R;
        }
        bool single = true;
        double alpha = g.alpha;
        int64_t row = g.row, col = g.col;
        for (int j = 0; j < lv && single; ++j) {
          int where = 0, c = 0;
          if (col_nnz(coef, NB, R, digits[j], &where, &c) != 1) {
            single = false;
            break;
          }
          alpha *= c;
          const int64_t bh = rows0 / rdiv[depth + j + 1];
          const int64_t bw = cols0 / cdiv[depth + j + 1];
          row += (int64_t)(where / BC) * bh;
          col += (int64_t)(where % BC) * bw;
        }
        const bool view_ok = single && !split && (!final_pass || g.elt == P.elt);
        if (view_ok) {
          Ref v = g;
          v.alpha = alpha;
          v.row = row;
          v.col = col;
          next.push_back(v);
          fp.outs.push_back(-1);
        } else {
          const size_t off = ws.alloc(region);
          const size_t es_out = split ? 2 : elt_size(fp.out_elt);
          Ref v{BUF_WS, fp.out_elt, (int64_t)(off / es_out), 0, 0, fp.out_ld, 1.0};
          v.plane = fp.out_plane;
          next.push_back(v);
          fp.outs.push_back(v.off);
          *bytes += (double)fp.h * fp.w * (split ? 4 : elt_size(fp.out_elt));
          if (final_pass) ++*materialized;
        }
      }
    }
    passes.push_back(std::move(fp));
    nodes.swap(next);
    depth = d2;
  }
  return nodes;
}

}  // namespace

// Closed-form mirror of make_plan's accounting (see the header).  Per pass,
// outputs come in two kinds: those whose digits all name single-non-zero
// columns stay views of their group (and keep its element type), the rest are
// written to the workspace.  Counting groups by element type is enough to
// reproduce every byte and allocation make_plan makes.
namespace {

struct ArenaSim {
  size_t used = 0;
  void alloc_many(int64_t count, size_t bytes) {
    if (count <= 0) return;
    const size_t first = (size_t)round_up((int64_t)used, 256);
    used = first + (size_t)(count - 1) * (size_t)round_up((int64_t)bytes, 256) + bytes;
  }
};

int single_columns(const signed char* X, int rows, int R) {
  int cnt = 0;
  for (int r = 0; r < R; ++r) {
    int where = 0, c = 0;
    if (col_nnz(X, rows, R, r, &where, &c) == 1) ++cnt;
  }
  return cnt;
}

void summarize_side(const std::vector<int>& ids, int side, int fuse, int dtype, int elt, int64_t rows0,
                    int64_t cols0, ArenaSim& ws, double* bytes, int* passes) {
  const int levels = (int)ids.size();
  const std::vector<int64_t> rdiv = prefix(ids, side == 0 ? 0 : 1);
  const std::vector<int64_t> cdiv = prefix(ids, side == 0 ? 1 : 2);
  // groups whose element type is the path's, and FP64 groups of an FP32 path
  int64_t g_in = 1, g_f64 = 0;
  int depth = 0;
  for (int lv : schedule_ids(ids, fuse, true)) {
    const AlgInfo& A = alg_info(ids[depth]);
    const int NB = (side == 0 ? A.M : A.K) * (side == 0 ? A.K : A.N);
    const int64_t ns = single_columns(side == 0 ? A.U : A.V, NB, A.R);
    const int d2 = depth + lv;
    const bool final_pass = d2 == levels;
    const bool split = final_pass && dtype == 2;
    const int64_t h = rows0 / rdiv[d2], w = cols0 / cdiv[d2];
    const int out_elt = final_pass ? elt : ELT_F64;
    const int64_t nout = ipow(A.R, lv), nv = split ? 0 : ipow(ns, lv);
    // reads: every group reads NB^lv blocks of its element type
    *bytes += (double)ipow(NB, lv) * h * w * ((double)g_in * elt_size(elt) + (double)g_f64 * 8);
    // views kept: a group of the path's type keeps nv views; an FP64 group
    // keeps nv views unless this is the final pass of an FP32 path; split
    // outputs are never views
    const bool f64_views = !final_pass || elt == ELT_F64;
    const int64_t mat = (g_in + g_f64) * (nout - nv) + (f64_views ? 0 : g_f64 * nv);
    // allocations happen group by group, output by output, all the same size
    if (split) {
      int64_t sld = 0, plane = 0;
      split_layout(side, h, w, &sld, &plane);
      ws.alloc_many(mat, (size_t)plane * 4);
      *bytes += (double)mat * h * w * 4;
    } else {
      ws.alloc_many(mat, (size_t)h * ws_ld(w, elt_size(out_elt)) * elt_size(out_elt));
      *bytes += (double)mat * h * w * elt_size(out_elt);
    }
    const int64_t in_views = g_in * nv, f64_kept = f64_views ? g_f64 * nv : 0;
    if (out_elt == elt) {
      g_in = in_views + mat + (elt == ELT_F64 ? f64_kept : 0);
      g_f64 = elt == ELT_F64 ? 0 : f64_kept;
    } else {  // FP64 outputs on an FP32 path
      g_in = in_views;
      g_f64 = f64_kept + mat;
    }
    ++*passes;
    depth = d2;
  }
}

}  // namespace

std::string summarize_plan(PlanSummary& S, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                           int dtype, int fuse, int leaf_form) {
  S = PlanSummary();
  if (m < 0 || k < 0 || n < 0) return "sizes must be non-negative";
  if (levels < 0 || levels > 6) return "levels must be in [0, 6]";
  if (dtype < 0 || dtype > 2) return "unknown dtype";
  std::vector<int> ids;
  std::string err;
  const int pr = parse_levels(alg, levels, &ids, &err);
  if (pr > 0) return err;
  const int elt = dtype == 0 ? ELT_F64 : ELT_F32;
  const size_t es = elt_size(elt);
  int L = pr < 0 ? 0 : levels;
  if (m == 0 || n == 0 || k == 0) L = 0;
  S.levels = L;
  if (L == 0) {
    if (m > 0 && n > 0) S.groups.push_back(GemmGroup{m, n, k, 1, 0, 0, 0, 0});
  } else {
    S.fuse = resolve_fuse(fuse, alg_info(ids[0]).R, dtype, ids);
    const std::vector<int64_t> pm = prefix(ids, 0), pk = prefix(ids, 1), pn = prefix(ids, 2), prr = prefix(ids, 3);
    const int64_t fm = pm[L], fk = pk[L], fn = pn[L];
    const int64_t m0 = m / fm * fm, k0 = k / fk * fk, n0 = n / fn * fn;
    const int64_t ml = m0 / fm, kl = k0 / fk, nl = n0 / fn;
    if (ml < 1 || kl < 1 || nl < 1) return "recursion depth leaves a leaf dimension < 1";
    ArenaSim ws;
    summarize_side(ids, 0, S.fuse, dtype, elt, m0, k0, ws, &S.add_bytes, &S.form_passes);
    summarize_side(ids, 1, S.fuse, dtype, elt, k0, n0, ws, &S.add_bytes, &S.form_passes);
    const int64_t nleaves = prr[L];
    const int64_t m_ld = ws_ld(nl, es);
    const int64_t m_stride = round_up(ml * m_ld * (int64_t)es, 256) / (int64_t)es;
    ws.alloc_many(1, (size_t)m_stride * es * nleaves);
    S.groups.push_back(GemmGroup{ml, nl, kl, nleaves, 0, 0, 0, 0});
    S.groups.back().split = dtype == 2 ? 1 : 0;
    const bool has_p = k0 < k;
    if (has_p) {
      ws.alloc_many(1, (size_t)m0 * round_up(n0, 16) * es);
      S.groups.push_back(GemmGroup{m0, n0, k - k0, 1, 0, 0, 0, 0});
    }
    if (n0 < n) S.groups.push_back(GemmGroup{m0, n - n0, k, 1, 0, 0, 0, 0});
    if (m0 < m) S.groups.push_back(GemmGroup{m - m0, n, k, 1, 0, 0, 0, 0});
    int depth = L;
    size_t node_es = es;
    for (int lv : schedule_ids(ids, S.fuse, false)) {
      const int d2 = depth - lv;
      const int64_t h = m0 / pm[depth], w = n0 / pn[depth];
      const int64_t ngroups = prr[d2], per = prr[depth] / prr[d2];
      S.add_bytes += (double)ngroups * per * h * w * node_es;
      const int64_t oh = h * (pm[depth] / pm[d2]), ow = w * (pn[depth] / pn[d2]);
      if (d2 == 0) {
        if (has_p) S.add_bytes += (double)m0 * n0 * es;
        S.add_bytes += (double)m0 * n0 * es;
      } else {
        const int64_t o_stride = round_up(oh * round_up(ow, 16) * 8, 256) / 8;
        ws.alloc_many(1, (size_t)o_stride * 8 * ngroups);
        S.add_bytes += (double)ngroups * oh * ow * 8;
        node_es = 8;
      }
      ++S.comb_passes;
      depth = d2;
    }
    S.ws_bytes = ws.used;
    // the condition make_plan applies: one unsplit pass per side of one level
    S.pair_form = L == 1 && dtype != 2 && S.form_passes == 2 &&
                  (m0 / fm) * (k0 / fk) + (k0 / fk) * (n0 / fn) <= kPairFormMaxPositions;
    const int nt = leaf_form_terms(ids, L, dtype);
    S.leaf_form = leaf_form == 2 ? nt : 0;
    if (leaf_form == 2 && nt == 0) return "leaf_form 2 needs a one-level FP64 / FP32 plan";
  }
  for (GemmGroup& g : S.groups) {
    g.tiles_m = (g.m + kTileM - 1) / kTileM;
    g.tiles_n = (g.n + kTileN - 1) / kTileN;
    S.leaf_flops += 2.0 * g.m * g.n * g.k * g.count;
  }
  return std::string();
}

int find_algorithm(const char* name) {
  if (!name) return -2;
  if (std::strcmp(name, "classical") == 0) return -1;
  for (int i = 0; i < kNumAlgorithms; ++i)
    if (std::strcmp(alg_info(i).name, name) == 0) return i;
  return -2;
}

int parse_levels(const char* alg, int levels, std::vector<int>* ids, std::string* err) {
  ids->clear();
  if (!alg) {
    *err = "unknown algorithm '(null)'";
    return 5;  // FMM_EALG
  }
  if (std::strlen(alg) >= 80) {
    *err = "algorithm name longer than 79 characters";
    return 1;  // FMM_EINVAL
  }
  if (!std::strchr(alg, '+')) {
    const int id = find_algorithm(alg);
    if (id == -2) {
      *err = std::string("unknown algorithm '") + alg + "'";
      return 5;
    }
    if (id == -1) return -1;
    ids->assign(levels > 0 ? levels : 0, id);
    return 0;
  }
  std::string part;
  for (const char* c = alg;; ++c) {
    if (*c == '+' || *c == 0) {
      const int id = find_algorithm(part.c_str());
      if (id < 0) {
        *err = "'" + part + "' in '" + alg + "' is not a base case";
        return 5;
      }
      ids->push_back(id);
      part.clear();
      if (*c == 0) break;
    } else {
      part += *c;
    }
  }
  if ((int)ids->size() != levels) {
    *err = std::string("'") + alg + "' names " + std::to_string(ids->size()) +
           " levels; levels must equal that count";
    ids->clear();
    return 1;  // FMM_EINVAL
  }
  return 0;
}

std::string make_plan(Plan& P, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                      int dtype, int fuse, int* code, int leaf_form) {
  *code = 1;  // FMM_EINVAL
  if (m < 0 || k < 0 || n < 0) return "sizes must be non-negative";
  if (levels < 0 || levels > 6) return "levels must be in [0, 6]";
  if (dtype < 0 || dtype > 2) return "unknown dtype";
  if (fuse < 0 || fuse > 2) return "fuse must be 0 (default), 1 or 2";
  if (leaf_form < 0 || leaf_form > 2) return "leaf_form must be 0 (default), 1 or 2";
  std::vector<int> ids;
  std::string perr;
  const int pr = parse_levels(alg, levels, &ids, &perr);
  if (pr > 0) {
    *code = pr;
    return perr;
  }
  const int id = pr < 0 ? -1 : ids.empty() ? find_algorithm(alg) : ids[0];
  P = Plan();
  P.alg_name = alg;
  P.m = m;
  P.k = k;
  P.n = n;
  P.dtype = dtype;
  P.elt = dtype == 0 ? ELT_F64 : ELT_F32;
  const size_t es = elt_size(P.elt);
  P.alg_id = id;
  P.levels = id < 0 ? 0 : levels;
  if (m == 0 || n == 0 || k == 0) P.levels = 0;  // nothing to recurse on
  if (P.levels > 0) {
    const AlgInfo& A = alg_info(id);
    P.lv_alg = ids;
    P.M = A.M;
    P.K = A.K;
    P.N = A.N;
    P.R = A.R;
    P.fuse = resolve_fuse(fuse, A.R, dtype, ids);
    const int64_t fm = prefix(ids, 0)[P.levels], fk = prefix(ids, 1)[P.levels], fn = prefix(ids, 2)[P.levels];
    P.m0 = m / fm * fm;
    P.k0 = k / fk * fk;
    P.n0 = n / fn * fn;
    P.ml = P.m0 / fm;
    P.kl = P.k0 / fk;
    P.nl = P.n0 / fn;
    if (P.ml < 1 || P.kl < 1 || P.nl < 1)
      return "recursion depth leaves a leaf dimension < 1 (m, k or n smaller than M^L, K^L or N^L)";
  } else {
    P.m0 = m;
    P.k0 = k;
    P.n0 = n;
    P.ml = m;
    P.kl = k;
    P.nl = n;
  }

  Arena ws;
  double add_bytes = 0;
  const Ref refA{BUF_A, P.elt, 0, 0, 0, 0, 1.0};
  const Ref refB{BUF_B, P.elt, 0, 0, 0, 0, 1.0};
  const Ref refC{BUF_C, P.elt, 0, 0, 0, 0, 1.0};

  if (P.levels > 0) {
    const int L = P.levels;
    const std::vector<int64_t> pm = prefix(P.lv_alg, 0), pn = prefix(P.lv_alg, 2), prr = prefix(P.lv_alg, 3);
    std::vector<Ref> S = plan_side(P, 0, ws, P.s_passes, &P.s_mat, &add_bytes);
    std::vector<Ref> T = plan_side(P, 1, ws, P.t_passes, &P.t_mat, &add_bytes);
    const int64_t nleaves = prr[L];
    // Leaf products M_rho, contiguous with a uniform stride.
    const int64_t m_ld = ws_ld(P.nl, es);
    const int64_t m_stride = round_up(P.ml * m_ld * (int64_t)es, 256) / (int64_t)es;
    const size_t m_base = ws.alloc((size_t)m_stride * es * nleaves);
    GemmGroup g0{P.ml, P.nl, P.kl, nleaves, 0, 0, 0, 0};
    g0.split = S[0].elt == ELT_BF16X2 ? 1 : 0;  // BF16x3 leaves read split operands, never views
    P.gemm_groups.push_back(g0);
    for (int64_t r = 0; r < nleaves; ++r) {
      GemmProb pr{};
      pr.a = S[r];
      pr.b = T[r];
      pr.alpha = S[r].alpha * T[r].alpha;
      pr.a.alpha = 1.0;
      pr.b.alpha = 1.0;
      pr.c = Ref{BUF_WS, P.elt, (int64_t)(m_base / es) + r * m_stride, 0, 0, m_ld, 1.0};
      P.gemm_probs.push_back(pr);
      P.leaves.push_back(LeafRef{S[r], T[r], pr.c});
    }
    // Peel problems (classical, Section 3.5).
    Ref pref{};
    bool has_p = false;
    if (P.k0 < k) {
      const int64_t p_ld = round_up(P.n0, 16);
      const size_t off = ws.alloc((size_t)P.m0 * p_ld * es);
      pref = Ref{BUF_WS, P.elt, (int64_t)(off / es), 0, 0, p_ld, 1.0};
      has_p = true;
      GemmProb pr{};
      pr.a = refA;
      pr.a.col = P.k0;
      pr.b = refB;
      pr.b.row = P.k0;
      pr.c = pref;
      pr.alpha = 1.0;
      P.gemm_groups.push_back(GemmGroup{P.m0, P.n0, k - P.k0, 1, 0, 0, 0, 0});
      P.gemm_probs.push_back(pr);
    }
    if (P.n0 < n) {
      GemmProb pr{};
      pr.a = refA;
      pr.b = refB;
      pr.b.col = P.n0;
      pr.c = refC;
      pr.c.col = P.n0;
      pr.alpha = 1.0;
      P.gemm_groups.push_back(GemmGroup{P.m0, n - P.n0, k, 1, 0, 0, 0, 0});
      P.gemm_probs.push_back(pr);
    }
    if (P.m0 < m) {
      GemmProb pr{};
      pr.a = refA;
      pr.a.row = P.m0;
      pr.b = refB;
      pr.c = refC;
      pr.c.row = P.m0;
      pr.alpha = 1.0;
      P.gemm_groups.push_back(GemmGroup{m - P.m0, n, k, 1, 0, 0, 0, 0});
      P.gemm_probs.push_back(pr);
    }
    // Combination passes, deepest level first.
    std::vector<int64_t> node_off(nleaves);
    for (int64_t r = 0; r < nleaves; ++r) node_off[r] = (int64_t)(m_base / es) + r * m_stride;
    int64_t node_stride = m_stride, node_ld = m_ld;
    int node_elt = P.elt;
    int depth = L;
    std::vector<int> sched = schedule_ids(P.lv_alg, P.fuse, false);
    for (size_t pi = 0; pi < sched.size(); ++pi) {
      const int lv = sched[pi];
      const int d2 = depth - lv;
      CombinePass cp;
      cp.alg = P.lv_alg[d2];  // every level of a fused pass uses it
      cp.lv = lv;
      cp.depth_in = depth;
      cp.h = P.m0 / pm[depth];
      cp.w = P.n0 / pn[depth];
      cp.in_elt = node_elt;
      cp.in_ld = node_ld;
      cp.in_stride = node_stride;
      const int64_t ngroups = prr[d2];
      const int64_t per = prr[depth] / prr[d2];
      cp.ngroups = (int)ngroups;
      add_bytes += (double)ngroups * per * cp.h * cp.w * elt_size(node_elt);
      const int64_t oh = cp.h * (pm[depth] / pm[d2]), ow = cp.w * (pn[depth] / pn[d2]);
      std::vector<int64_t> next_off;
      if (d2 == 0) {
        cp.in_off.push_back(node_off[0]);
        cp.out.push_back(refC);
        if (has_p) {
          cp.has_p = true;
          cp.p = pref;
          add_bytes += (double)P.m0 * P.n0 * es;
        }
        add_bytes += (double)P.m0 * P.n0 * es;
      } else {
        const int64_t o_ld = round_up(ow, 16);
        const int64_t o_stride = round_up(oh * o_ld * 8, 256) / 8;
        const size_t base = ws.alloc((size_t)o_stride * 8 * ngroups);
        for (int64_t g = 0; g < ngroups; ++g) {
          cp.in_off.push_back(node_off[g * per]);
          const int64_t off = (int64_t)(base / 8) + g * o_stride;
          cp.out.push_back(Ref{BUF_WS, ELT_F64, off, 0, 0, o_ld, 1.0});
          next_off.push_back(off);
          add_bytes += (double)oh * ow * 8;
        }
        node_stride = o_stride;
        node_ld = o_ld;
        node_elt = ELT_F64;
      }
      P.w_passes.push_back(std::move(cp));
      node_off.swap(next_off);
      depth = d2;
    }
  } else if (m > 0 && n > 0) {
    GemmProb pr{};
    pr.a = refA;
    pr.b = refB;
    pr.c = refC;
    pr.alpha = 1.0;
    P.gemm_groups.push_back(GemmGroup{m, n, k, 1, 0, 0, 0, 0});
    P.gemm_probs.push_back(pr);
  }
  if (P.gemm_groups.size() > (size_t)kMaxGemmGroups) return "too many GEMM groups";

  // Tiles and flop/byte accounting.
  int64_t tiles = 0, prob = 0;
  for (GemmGroup& g : P.gemm_groups) {
    g.tiles_m = (g.m + kTileM - 1) / kTileM;
    g.tiles_n = (g.n + kTileN - 1) / kTileN;
    g.tile_start = tiles;
    g.prob_start = prob;
    tiles += g.tiles_m * g.tiles_n * g.count;
    prob += g.count;
    P.leaf_flops += 2.0 * g.m * g.n * g.k * g.count;
    P.gemm_min_bytes += (double)es * (g.m * g.k + g.k * g.n + g.m * g.n) * g.count;
  }
  P.gemm_tiles = tiles;
  P.add_bytes = add_bytes;
  P.ws_bytes = ws.used;
  // Leaf operands formed inside the leaf GEMM: every problem's A and B become
  // term lists (leaf r: the non-zeros of column r of U and V over the blocks
  // of A and B, in ascending block order, the pass's chain order; views and
  // peel strips: one term).  The S and T passes stay in the plan (the
  // FMM_STAGE_FORM_* stages still write them) but fmm_multiply skips them.
  {
    const int nt = P.levels > 0 ? leaf_form_terms(P.lv_alg, P.levels, dtype) : 0;
    if (leaf_form == 2 && nt == 0)
      return "leaf_form 2 needs a one-level FP64 / FP32 plan whose S and T columns have at most " +
             std::to_string(kMaxLeafTerms) + " non-zeros, each +-1";
    P.leaf_form = leaf_form == 2 ? nt : 0;
  }
  if (P.leaf_form) {
    const AlgInfo& A = alg_info(P.lv_alg[0]);
    auto one = [](LeafTerms& t) {
      std::memset(&t, 0, sizeof(t));
      t.n = 1;
      t.coef[0] = 1;
    };
    for (GemmProb& pr : P.gemm_probs) {
      one(pr.fa);
      one(pr.fb);
    }
    for (int r = 0; r < A.R; ++r) {
      GemmProb& pr = P.gemm_probs[r];
      for (int side = 0; side < 2; ++side) {
        Ref& op = side == 0 ? pr.a : pr.b;
        if (op.buf != BUF_WS) continue;  // a view: one term
        LeafTerms& t = side == 0 ? pr.fa : pr.fb;
        const signed char* X = side == 0 ? A.U : A.V;
        const int BC = side == 0 ? A.K : A.N, rows = side == 0 ? A.M * A.K : A.K * A.N;
        const int64_t bh = side == 0 ? P.ml : P.kl, bw = side == 0 ? P.kl : P.nl;
        std::memset(&t, 0, sizeof(t));
        for (int i = 0; i < rows; ++i) {
          const int c = X[i * A.R + r];
          if (c == 0) continue;
          t.coef[t.n] = c;
          t.drow[t.n] = (int64_t)(i / BC) * bh;
          t.dcol[t.n] = (int64_t)(i % BC) * bw;
          ++t.n;
        }
        op = Ref{side == 0 ? BUF_A : BUF_B, P.elt, 0, 0, 0, 0, 1.0};
      }
    }
  }
  // Small one-level plans form S and T in one launch: between two dependent
  // launches the queue idles about as long as one such pass takes.
  if (P.s_passes.size() == 1 && P.t_passes.size() == 1) {
    const FormPass& fs = P.s_passes[0];
    const FormPass& ft = P.t_passes[0];
    P.pair_form = fs.lv == 1 && ft.lv == 1 && fs.alg == ft.alg && fs.out_elt != ELT_BF16X2 &&
                  ft.out_elt != ELT_BF16X2 && fs.h > 0 && fs.w > 0 && ft.h > 0 && ft.w > 0 &&
                  fs.ngroups > 0 && ft.ngroups > 0 &&
                  fs.h * fs.w * fs.ngroups + ft.h * ft.w * ft.ngroups <= kPairFormMaxPositions;
  }

  // Host image of the device descriptor table.
  Arena tab;
  P.dev_probs = tab.alloc(sizeof(GemmProb) * P.gemm_probs.size());
  for (FormPass& fp : P.s_passes) {
    fp.dev_groups = tab.alloc(sizeof(Ref) * fp.groups.size());
    fp.dev_outs = tab.alloc(sizeof(int64_t) * fp.outs.size());
  }
  for (FormPass& fp : P.t_passes) {
    fp.dev_groups = tab.alloc(sizeof(Ref) * fp.groups.size());
    fp.dev_outs = tab.alloc(sizeof(int64_t) * fp.outs.size());
  }
  for (CombinePass& cp : P.w_passes) {
    cp.dev_in = tab.alloc(sizeof(int64_t) * cp.in_off.size());
    cp.dev_out = tab.alloc(sizeof(Ref) * cp.out.size());
  }
  P.table_bytes = tab.used ? tab.used : 256;
  P.table.assign(P.table_bytes, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(P.table.data() + off, src, bytes);
  };
  put(P.dev_probs, P.gemm_probs.data(), sizeof(GemmProb) * P.gemm_probs.size());
  for (FormPass& fp : P.s_passes) {
    put(fp.dev_groups, fp.groups.data(), sizeof(Ref) * fp.groups.size());
    put(fp.dev_outs, fp.outs.data(), sizeof(int64_t) * fp.outs.size());
  }
  for (FormPass& fp : P.t_passes) {
    put(fp.dev_groups, fp.groups.data(), sizeof(Ref) * fp.groups.size());
    put(fp.dev_outs, fp.outs.data(), sizeof(int64_t) * fp.outs.size());
  }
  for (CombinePass& cp : P.w_passes) {
    put(cp.dev_in, cp.in_off.data(), sizeof(int64_t) * cp.in_off.size());
    put(cp.dev_out, cp.out.data(), sizeof(Ref) * cp.out.size());
  }
  *code = 0;
  return std::string();
}

}  // namespace fmm
