// Cost model for choosing the base case and recursion depth.
//
// The paper chooses per shape by measurement and observes that recursion pays
// only while the leaf multiplication stays on the flat part of its
// performance curve (Section 5); the model below is the library's prior for
// that choice.  For each candidate (base case, depth) it takes the plan's
// closed-form summary (no descriptors are built) and predicts
//   t = t_leaf + t_add + launches * t_launch
// where t_leaf walks the grouped launch as the persistent kernel does: every
// 128 x 128 output tile of a problem with inner dimension k costs (k + kFix)
// units, the units are spread over `slots` resident workgroups, and the last
// partial wave costs a whole tile; t_add moves the plan's algorithmic bytes of
// the formation and combination passes at the measured streaming rate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

namespace {

// Sustained rates of this library's kernels on MI355X at large sizes
// (16384^3 leaf launches; streaming addition kernels).
constexpr double kRateF64 = 65e12;          // flop/s, FP64 MFMA
constexpr double kRateF32 = 110e12;         // flop/s, FP32 MFMA
constexpr double kRateBf16x3Split = 300e12; // FP32-equivalent flop/s, BF16x3 on split leaf operands
constexpr double kRateBf16x3 = 245e12;      // FP32-equivalent flop/s, BF16x3 splitting FP32 tiles
constexpr double kRateBf16x3Big = 430e12;   // FP32-equivalent flop/s, BF16x3 256 x 256 tiles (split operands)
constexpr double kAddBw = 4.8e12;           // byte/s, formation / combination passes
constexpr double kLaunch = 6e-6;       // s per kernel launch on a busy stream
constexpr double kFix = 32;            // per-tile fixed cost, in units of k
constexpr int kSlots = 512;            // resident leaf workgroups (2 per compute unit)
constexpr int kCUs = kSlots / 2;
constexpr int kSlotsSmall = 4 * kCUs;  // resident 64 x 64 leaf workgroups (4 per compute unit)
// full-occupancy rate of the 64 x 64 tile relative to the 128 x 128 one
constexpr double kSmallF64 = 0.93, kSmallF32 = 0.74, kSmallBf16x3 = 0.68;
// rate of a 32 x 32 tile alone on its compute unit relative to the 128 x 128
// rate (512^3 FP64: 256 such tiles in 15.6 us; taken for FP32 as well)
constexpr double kTiny = 0.28;
constexpr int64_t kMaxLeaves = 60000;  // candidates with more leaves are not offered

// Rate of group g of a plan: on the BF16x3 path the leaf group (the first
// group of a recursive plan) reads split operands, the others FP32 ones.
double rate(int dtype, bool split_leaf) {
  if (dtype == 0) return kRateF64;
  if (dtype == 1) return kRateF32;
  return split_leaf ? kRateBf16x3Split : kRateBf16x3;
}

void predict(const PlanSummary& P, int dtype, Candidate& c) {
  // leaf: tile-work units of every group (scaled to the group's rate),
  // quantised to whole waves of the largest tile cost
  const double ref = rate(dtype, false);
  double units = 0, wmax = 0, tiles = 0;
  for (size_t i = 0; i < P.groups.size(); ++i) {
    const GemmGroup& g = P.groups[i];
    const double t = (double)g.tiles_m * g.tiles_n * g.count;
    const double w = ((double)g.k + kFix) * ref / rate(dtype, i == 0 && P.levels > 0);
    units += t * w;
    tiles += t;
    wmax = std::max(wmax, w);
  }
  // Tiles of one launch share the compute units: with fewer tiles than
  // resident slots each compute unit holds ceil(tiles / CUs) of them and
  // splits its rate among those.
  auto waves_time = [](double u, double w, double ntiles, int per_cu, double tile_edge, double r) {
    const double resident = std::min<double>(per_cu, std::max(1.0, std::ceil(ntiles / kCUs)));
    const double slots = kCUs * resident;
    return std::ceil(u / (slots * w)) * w * 2.0 * tile_edge * tile_edge / (r / slots);
  };
  double leaf_s = 0;
  // BF16x3: split-operand groups with whole k-octets run 256 x 256 tiles,
  // one workgroup per compute unit, when they have two such tiles per CU;
  // the other groups then take a launch of 128 x 128 tiles of their own
  double big_tiles = 0, big_units = 0, big_w = 0;
  if (dtype == 2)
    for (const GemmGroup& g : P.groups)
      if (g.split && g.k % 8 == 0) {
        const double t = (double)((g.m + 255) / 256) * ((g.n + 255) / 256) * g.count;
        big_tiles += t;
        big_units += t * ((double)g.k + kFix);
        big_w = std::max(big_w, (double)g.k + kFix);
      }
  if (big_tiles >= 2.0 * kCUs) {
    leaf_s = waves_time(big_units, big_w, big_tiles, 1, 256, kRateBf16x3Big);
    double units_r = 0, w_r = 0, tiles_r = 0;
    for (const GemmGroup& g : P.groups)
      if (!(g.split && g.k % 8 == 0)) {
        const double t = (double)g.tiles_m * g.tiles_n * g.count;
        units_r += t * ((double)g.k + kFix);
        tiles_r += t;
        w_r = std::max(w_r, (double)g.k + kFix);
      }
    if (tiles_r > 0) leaf_s += waves_time(units_r, w_r, tiles_r, kSlots / kCUs, (double)kTileM, kRateBf16x3) + kLaunch;
  } else if (tiles > 0 && dtype != 2 && [&] {
               double t64 = 0;
               for (const GemmGroup& g : P.groups) t64 += (double)((g.m + 63) / 64) * ((g.n + 63) / 64) * g.count;
               return 2.0 * t64 <= kCUs;
             }()) {
    // the launch runs 32 x 32 tiles (launch_gemm: at most half as many 64 x 64
    // tiles as compute units)
    double units32 = 0, tiles32 = 0;
    for (size_t i = 0; i < P.groups.size(); ++i) {
      const GemmGroup& g = P.groups[i];
      const double t = (double)((g.m + 31) / 32) * ((g.n + 31) / 32) * g.count;
      units32 += t * ((double)g.k + kFix) * ref / rate(dtype, i == 0 && P.levels > 0);
      tiles32 += t;
    }
    leaf_s = waves_time(units32, wmax, tiles32, kSlotsSmall / kCUs, 32, ref * kTiny);
  } else if (tiles > 0 && use_small_tiles((int64_t)tiles, kCUs, dtype == 2 ? kTilesBf16x3 : dtype == 0 ? kTilesF64Dma : kTilesF32Dma)) {
    // the launch runs 64 x 64 tiles (units weighted by each group's rate,
    // as for the large tiles)
    double units64 = 0, tiles64 = 0;
    for (size_t i = 0; i < P.groups.size(); ++i) {
      const GemmGroup& g = P.groups[i];
      const double t = (double)((g.m + 63) / 64) * ((g.n + 63) / 64) * g.count;
      units64 += t * ((double)g.k + kFix) * ref / rate(dtype, i == 0 && P.levels > 0);
      tiles64 += t;
    }
    const double f = dtype == 0 ? kSmallF64 : dtype == 1 ? kSmallF32 : kSmallBf16x3;
    leaf_s = waves_time(units64, wmax, tiles64, kSlotsSmall / kCUs, 64, ref * f);
  } else if (tiles > 0) {
    leaf_s = waves_time(units, wmax, tiles, kSlots / kCUs, (double)kTileM, ref);
  }
  const double add_s = P.add_bytes / kAddBw;
  // a pair-formed plan forms S and T in one launch, a leaf-formed one in none
  const double launches = 1.0 + P.comb_passes + (P.leaf_form ? 0 : P.form_passes - (P.pair_form ? 1 : 0));
  c.leaf_ms = leaf_s * 1e3;
  c.add_ms = add_s * 1e3;
  c.model_ms = (leaf_s + add_s + launches * kLaunch) * 1e3;
  c.ws_bytes = P.ws_bytes;
}

}  // namespace

double growth(int id) {
  const AlgInfo& a = alg_info(id);
  const int MK = a.M * a.K, KN = a.K * a.N, MN = a.M * a.N;
  double s = 0;
  for (int r = 0; r < a.R; ++r) {
    double u = 0, v = 0, w = 0;
    for (int i = 0; i < MK; ++i) u += (double)a.U[i * a.R + r] * a.U[i * a.R + r];
    for (int j = 0; j < KN; ++j) v += (double)a.V[j * a.R + r] * a.V[j * a.R + r];
    for (int k = 0; k < MN; ++k) w += (double)a.W[k * a.R + r] * a.W[k * a.R + r];
    s += u * v * w;
  }
  return std::sqrt(s / ((double)a.M * a.K * a.N));
}

double error_bound(const std::vector<int>& ids, int64_t k, int dtype) {
  const double sk = 2.0 + std::sqrt((double)std::max<int64_t>(k, 1));
  double e = dtype == 0 ? sk * std::ldexp(1.0, -53)
             : dtype == 1 ? sk * std::ldexp(1.0, -24)
                          : 3.0 * std::ldexp(1.0, -16) + sk * std::ldexp(1.0, -24);
  for (int id : ids) e *= growth(id);
  return e;
}

double default_max_error(int dtype) { return dtype == 0 ? 1e-12 : dtype == 1 ? 1e-4 : 5e-4; }

size_t default_budget() {
  if (const char* b = std::getenv("FMM_HBM_BUDGET")) {
    const double v = std::atof(b);
    if (v > 0) return (size_t)v;
  }
  size_t free_b = 0, total_b = 0;
  int n = 0;
  if (hipGetDeviceCount(&n) == hipSuccess && n > 0 && hipMemGetInfo(&free_b, &total_b) == hipSuccess)
    return free_b / 4 * 3;
  (void)hipGetLastError();
  return (size_t)288e9 / 4 * 3;
}

std::string rank_candidates(int64_t m, int64_t k, int64_t n, int dtype, const char* alg, size_t budget,
                            int fuse, double max_error, std::vector<Candidate>& out) {
  out.clear();
  if (m < 0 || k < 0 || n < 0) return "sizes must be non-negative";
  if (dtype < 0 || dtype > 2) return "unknown dtype";
  if (!budget) budget = default_budget();
  if (max_error == 0) max_error = default_max_error(dtype);
  const bool any = !alg || !std::strcmp(alg, "auto");
  const bool listed = !any && std::strchr(alg, '+');  // one base case per level
  std::vector<int> ids;
  if (any) {
    for (int i = 0; i < kNumAlgorithms; ++i)
      if (std::strcmp(alg_info(i).name, "classical_222_8")) ids.push_back(i);
  } else if (!listed) {
    const int id = find_algorithm(alg);
    if (id == -2) return std::string("unknown algorithm '") + alg + "'";
    if (id >= 0) ids.push_back(id);
  }
  auto add = [&](const char* name, int levels) {
    PlanSummary P;
    if (!summarize_plan(P, name, m, k, n, levels, dtype, fuse).empty()) return;
    if (P.ws_bytes > budget) return;
    std::vector<int> lv;
    std::string perr;
    if (parse_levels(name, levels, &lv, &perr) > 0) return;
    const double err = error_bound(P.levels > 0 ? lv : std::vector<int>(), k, dtype);
    if (max_error > 0 && err > max_error) return;
    Candidate c;
    c.err = err;
    std::snprintf(c.alg, sizeof(c.alg), "%s", name);
    c.levels = levels;
    c.fuse = P.levels > 0 ? P.fuse : 0;
    predict(P, dtype, c);
    out.push_back(c);
  };
  if (listed) {
    std::vector<int> lv;
    std::string err;
    const int count = (int)std::count(alg, alg + std::strlen(alg), '+') + 1;
    if (parse_levels(alg, count, &lv, &err) > 0) return err;
    add(alg, count);
  }
  if (any || (!listed && find_algorithm(alg) == -1)) add("classical", 0);
  if (any) {
    // two levels of different base cases (Section 5.2's composition), when
    // every leaf dimension keeps 64 or more
    for (int a : ids)
      for (int b : ids) {
        if (a == b) continue;
        const AlgInfo &A = alg_info(a), &B = alg_info(b);
        if (m / (A.M * B.M) < 64 || k / (A.K * B.K) < 64 || n / (A.N * B.N) < 64) continue;
        const std::string name = std::string(A.name) + "+" + B.name;
        add(name.c_str(), 2);
      }
  }
  for (int id : ids) {
    const AlgInfo& a = alg_info(id);
    if (!any) add(a.name, 0);  // depth 0 of a named base case: the classical product
    // recurse while every leaf dimension keeps at least 64 rows, columns and
    // depth (deeper leaves only lose) and the leaf count stays below
    // kMaxLeaves (descriptor tables of that size cost planning time)
    int64_t fm = 1, fk = 1, fn = 1, leaves = 1;
    for (int L = 1; L <= 5; ++L) {
      fm *= a.M;
      fk *= a.K;
      fn *= a.N;
      leaves *= a.R;
      if (m / fm < 64 || n / fn < 64 || k / fk < 64 || leaves > kMaxLeaves) break;
      add(a.name, L);
    }
  }
  std::stable_sort(out.begin(), out.end(),
                   [](const Candidate& x, const Candidate& y) { return x.model_ms < y.model_ms; });
  return "";
}

namespace {
using TuneKey = std::tuple<int64_t, int64_t, int64_t, int>;
std::mutex g_tuned_mu;
std::map<TuneKey, Candidate>& tuned_table() {
  static std::map<TuneKey, Candidate> t;
  return t;
}
}  // namespace

void record_tuned(int64_t m, int64_t k, int64_t n, int dtype, const Candidate& c) {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  tuned_table()[TuneKey{m, k, n, dtype}] = c;
}

bool lookup_tuned(int64_t m, int64_t k, int64_t n, int dtype, Candidate* c) {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  auto it = tuned_table().find(TuneKey{m, k, n, dtype});
  if (it == tuned_table().end()) return false;
  *c = it->second;
  return true;
}

void clear_tuned() {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  tuned_table().clear();
}

bool choose(int64_t m, int64_t k, int64_t n, int dtype, const char* alg, int levels, size_t budget, int fuse,
            double max_error, Candidate* pick, std::string* why) {
  const bool any = !alg || !std::strcmp(alg, "auto");
  const double limit = max_error == 0 ? default_max_error(dtype) : max_error;
  if (any && levels < 0) {
    Candidate c;
    if (lookup_tuned(m, k, n, dtype, &c)) {
      PlanSummary P;
      std::vector<int> lv;
      std::string perr;
      if (summarize_plan(P, c.alg, m, k, n, c.levels, dtype, c.fuse).empty() &&
          P.ws_bytes <= (budget ? budget : default_budget()) && parse_levels(c.alg, c.levels, &lv, &perr) <= 0 &&
          (limit < 0 || error_bound(P.levels > 0 ? lv : std::vector<int>(), k, dtype) <= limit)) {
        *pick = c;
        return true;
      }
    }
  }
  std::vector<Candidate> cands;
  *why = rank_candidates(m, k, n, dtype, alg, budget, fuse, max_error, cands);
  if (!why->empty()) return false;
  for (const Candidate& c : cands)
    if (levels < 0 || c.levels == levels) {
      *pick = c;
      return true;
    }
  *why = "no candidate fits the workspace budget and the error budget";
  return false;
}

}  // namespace fmm
