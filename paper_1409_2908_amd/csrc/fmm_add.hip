// Dispatch of the addition kernels by base case: every base case's
// launchers are instantiated in a generated source file of their own
// (csrc/gen/fmm_add_NN.hip, one per table), so they compile in parallel; this
// file maps the run-time algorithm id to them.
#include <hip/hip_runtime.h>

#include <array>
#include <utility>

#include "fmm_launch.h"

namespace fmm {

template <int ID>
hipError_t launch_form_id(const FormArgs& a, int side, int lv, int ngroups, hipStream_t s);
template <int ID>
hipError_t launch_form_pair_id(const FormArgs& sa, int ngs, const FormArgs& ta, int ngt, hipStream_t st);
template <int ID>
hipError_t launch_combine_id(const CombineArgs& a, int lv, int ngroups, hipStream_t s);

namespace {

using FormFn = hipError_t (*)(const FormArgs&, int, int, int, hipStream_t);
using PairFn = hipError_t (*)(const FormArgs&, int, const FormArgs&, int, hipStream_t);
using CombFn = hipError_t (*)(const CombineArgs&, int, int, hipStream_t);

template <int... I>
constexpr auto form_table(std::integer_sequence<int, I...>) {
  return std::array<FormFn, sizeof...(I)>{&launch_form_id<I>...};
}
template <int... I>
constexpr auto pair_table(std::integer_sequence<int, I...>) {
  return std::array<PairFn, sizeof...(I)>{&launch_form_pair_id<I>...};
}
template <int... I>
constexpr auto comb_table(std::integer_sequence<int, I...>) {
  return std::array<CombFn, sizeof...(I)>{&launch_combine_id<I>...};
}

const auto kFormFns = form_table(std::make_integer_sequence<int, kNumAlgorithms>{});
const auto kPairFns = pair_table(std::make_integer_sequence<int, kNumAlgorithms>{});
const auto kCombFns = comb_table(std::make_integer_sequence<int, kNumAlgorithms>{});

}  // namespace

hipError_t launch_form_pair(int alg, const FormArgs& sa, int ngs, const FormArgs& ta, int ngt, hipStream_t st) {
  // one-level passes with unsplit outputs and non-empty grids on both sides
  if (sa.out_elt == ELT_BF16X2 || ta.out_elt == ELT_BF16X2 || sa.h <= 0 || sa.w <= 0 || ta.h <= 0 || ta.w <= 0 ||
      ngs <= 0 || ngt <= 0)
    return hipErrorInvalidValue;
  if (alg < 0 || alg >= kNumAlgorithms) return hipErrorInvalidValue;
  return kPairFns[alg](sa, ngs, ta, ngt, st);
}

hipError_t launch_form(int alg, const FormArgs& a, int side, int lv, int ngroups, hipStream_t s) {
  if (a.h == 0 || a.w == 0 || ngroups == 0) return hipSuccess;
  if (alg < 0 || alg >= kNumAlgorithms) return hipErrorInvalidValue;
  return kFormFns[alg](a, side, lv, ngroups, s);
}

hipError_t launch_combine(int alg, const CombineArgs& a, int lv, int ngroups, hipStream_t s) {
  if (a.h == 0 || a.w == 0 || ngroups == 0) return hipSuccess;
  if (alg < 0 || alg >= kNumAlgorithms) return hipErrorInvalidValue;
  return kCombFns[alg](a, lv, ngroups, s);
}

}  // namespace fmm
