// Device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fmm_internal.h"

namespace fmm {

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Coefficients of one side of a base case as compile-time constants.
//   side 0: U (A blocks, BR x BC = M x K), side 1: V (B blocks, K x N),
//   side 2: W transposed view (rows = products r, columns = C blocks k).
template <int ID, int SIDE>
struct Side {
  using A = Alg<ID>;
  static constexpr int R = A::R;
  static constexpr int BR = SIDE == 0 ? A::M : A::K;
  static constexpr int BC = SIDE == 0 ? A::K : A::N;
  static constexpr int NB = BR * BC;
  // coefficient of block i in output r
  static constexpr int coef(int i, int r) { return SIDE == 0 ? A::U[i][r] : A::V[i][r]; }
  static constexpr int first_nz(int r) {
    for (int i = 0; i < NB; ++i)
      if (coef(i, r) != 0) return i;
    return -1;
  }
};

template <int ID>
struct Comb {
  using A = Alg<ID>;
  static constexpr int R = A::R;
  static constexpr int MN = A::M * A::N;
  static constexpr int coef(int k, int r) { return A::W[k][r]; }
  static constexpr int first_nz(int k) {
    for (int r = 0; r < R; ++r)
      if (coef(k, r) != 0) return r;
    return -1;
  }
};

// One term of an addition chain: the first term initialises (copy, negation or
// exact power-of-two scaling), later terms add; each operation rounds once.
template <int C, bool FIRST>
__device__ __forceinline__ void chain_term(double& acc, double x) {
  // c * x and the add round separately, also for |c| = 3 (where a contracted
  // multiply-add would round once and differ in the last bit); for c = +-2^e
  // the product is exact and both forms agree
#pragma clang fp contract(off)
  if constexpr (FIRST) {
    if constexpr (C == 1) acc = x;
    else if constexpr (C == -1) acc = -x;
    else acc = __dmul_rn((double)C, x);
  } else {
    if constexpr (C == 1) acc = __dadd_rn(acc, x);
    else if constexpr (C == -1) acc = __dsub_rn(acc, x);
    else acc = __dadd_rn(acc, __dmul_rn((double)C, x));
  }
}

// sum_i coef(i, r) * x[i * STRIDE] over i = 0..NB-1 in ascending order.
template <class S, int R_IDX, int STRIDE, int NB>
__device__ __forceinline__ double chain_col(const double* x) {
  double acc = 0.0;
  constexpr int first = S::first_nz(R_IDX);
  static_for<0, NB>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int c = S::coef(i, R_IDX);
    if constexpr (c != 0) chain_term<c, i == first>(acc, x[i * STRIDE]);
  });
  return acc;
}

// sum_r W[k][r] * m[r] over r ascending.
template <int ID, int K_IDX>
__device__ __forceinline__ double chain_row(const double* mv) {
  using CB = Comb<ID>;
  double acc = 0.0;
  constexpr int first = CB::first_nz(K_IDX);
  static_for<0, CB::R>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    constexpr int c = CB::coef(K_IDX, r);
    if constexpr (c != 0) chain_term<c, r == first>(acc, mv[r]);
  });
  return acc;
}

// bfloat16 bits of a finite FP32 value, rounded to nearest with ties to even
// on the bit pattern (add 0x7FFF plus the lowest kept bit, drop 16 bits).
// The hardware conversion does not break ties to even, and the BF16x3 split
// is defined with round to nearest even.
__device__ __forceinline__ unsigned short bf16_bits_rne(float x) {
  const unsigned u = __builtin_bit_cast(unsigned, x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// The BF16x3 split of x: hi = bf16(x), lo = bf16(x - hi), both to nearest
// even; x - hi is exact in FP32.
__device__ __forceinline__ void split_bits(float x, unsigned short* hi, unsigned short* lo) {
  *hi = bf16_bits_rne(x);
  *lo = bf16_bits_rne(x - __builtin_bit_cast(float, (unsigned)*hi << 16));
}

__device__ __forceinline__ char* buf_ptr(const Bases& b, const Ref& r, int64_t* ld) {
  *ld = r.buf == BUF_WS ? r.ld : b.ld[r.buf];
  return (char*)b.ptr[r.buf];
}

__device__ __forceinline__ double load_elt(const char* base, int elt, int64_t idx) {
  return elt == ELT_F64 ? ((const double*)base)[idx] : (double)((const float*)base)[idx];
}

}  // namespace fmm
