// Streaming addition kernels (templates; each base case is instantiated in a
// source file of its own): operand formation (S_r from A with U, T_r from B
// with V) and the W-combination of the leaf products into C.
//
// Section 3.2 of the paper compares pairwise, write-once and streaming
// addition chains.  Here one thread owns one element position (p, q) of the
// output blocks: it reads the (BR*BC)^lv source elements at that position
// exactly once, keeps every partial sum in registers, and writes each
// materialised output exactly once -- the streaming variant's read count with
// the write-once variant's single output stream per store instruction.  A
// wavefront covers 64 consecutive q, so every load and store instruction moves
// 512 contiguous bytes (FP64).  Up to two recursion levels are fused per pass
// (their Kronecker-product coefficients are applied level by level, top level
// first, which is the recursion's own order): in registers for narrow base
// cases (R <= 8), and through LDS for wide ones, where a workgroup stages the
// (BR*BC)^2 sources (formation) or the R^2 products (combination) of 64
// positions once and its wavefronts share the level-one sums; the two-level
// combination always takes the LDS path.  Every variant performs the same
// roundings in the same order, so fused and one-level passes agree bit for
// bit.
#pragma once

#include <hip/hip_runtime.h>

#include "fmm_device.h"
#include "fmm_launch.h"

namespace fmm {

// Whether a base case fuses two recursion levels per addition pass: narrow
// ones (R <= 8) in registers; wide ones through LDS, which holds the
// (BR*BC)^2 sources of 64 positions (at most 11 blocks per side: 61 KB) and
// the products of 4 top-level indices (R <= 32: 64 KB).  Wider base cases
// run one level per pass (the planner's fuse2_ok states the same rule).
template <int ID>
constexpr bool kFuse2 = Alg<ID>::R <= 8 ||
                        (Alg<ID>::M * Alg<ID>::K <= 11 && Alg<ID>::K * Alg<ID>::N <= 11 && Alg<ID>::R <= 32);

constexpr int kAddTX = 64, kAddTY = 4;

__device__ __forceinline__ void store_out(char* ws, int elt, int64_t idx, int64_t plane, double v) {
  if (elt == ELT_F64) {
    ((double*)ws)[idx] = v;
  } else if (elt == ELT_F32) {
    ((float*)ws)[idx] = (float)v;  // one round-to-nearest-even from the FP64 sum
  } else {
    // BF16x3 leaf operand: the FP32 value x of the sum, then its split
    unsigned short hi, lo;
    split_bits((float)v, &hi, &lo);
    ((unsigned short*)ws)[idx] = hi;
    ((unsigned short*)ws)[idx + plane] = lo;
  }
}

// OCT: the output is a split T operand stored in k-octets; each wavefront
// then covers 8 consecutive rows p of 8 consecutive columns q, so every
// 2-byte store instruction of the wavefront fills 128 contiguous bytes (8
// whole octets) instead of scattering over 1 KB.
template <int ID, int SIDE, int LV, bool OCT>
__device__ __forceinline__ void form_body(const FormArgs& a, unsigned bx, unsigned by, unsigned bz) {
  using S = Side<ID, SIDE>;
  constexpr int NB = S::NB, R = S::R, BR = S::BR, BC = S::BC;
  constexpr int NIN = LV == 1 ? NB : NB * NB;
  const int t = threadIdx.y * kAddTX + threadIdx.x;
  const int64_t q = OCT ? (int64_t)bx * 32 + (t >> 3) : (int64_t)bx * kAddTX + threadIdx.x;
  const int64_t p = OCT ? (int64_t)by * 8 + (t & 7) : (int64_t)by * kAddTY + threadIdx.y;
  if (q >= a.w || p >= a.h) return;
  const int g = (int)bz;
  const Ref src = a.groups[g];
  int64_t ld;
  const char* base = buf_ptr(a.bases, src, &ld);
  const int64_t h = a.h, w = a.w;
  double x[NIN];
  static_for<0, NIN>([&](auto ic) {
    constexpr int idx = decltype(ic)::value;
    constexpr int i1 = LV == 1 ? idx : idx / NB;
    constexpr int i2 = LV == 1 ? 0 : idx % NB;
    constexpr int a1 = i1 / BC, b1 = i1 % BC, a2 = i2 / BC, b2 = i2 % BC;
    const int64_t row = src.row + (LV == 1 ? a1 * h : (a1 * BR + a2) * h) + p;
    const int64_t col = src.col + (LV == 1 ? b1 * w : (b1 * BC + b2) * w) + q;
    x[idx] = load_elt(base, src.elt, src.off + row * ld + col) * src.alpha;
  });
  char* ws = (char*)a.bases.ptr[BUF_WS];
  const int64_t* outs = a.outs + (int64_t)g * a.nout;
  // split T operands are stored in k-octets (see Elt): row p, column q
  const int64_t pos = (SIDE == 1 && a.out_elt == ELT_BF16X2) ? (p >> 3) * a.out_ld + q * 8 + (p & 7)
                                                            : p * a.out_ld + q;
  if constexpr (LV == 1) {
    static_for<0, R>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int64_t off = outs[r];
      if (off >= 0) store_out(ws, a.out_elt, off + pos, a.out_plane, chain_col<S, r, 1, NB>(x));
    });
  } else {
    static_for<0, R>([&](auto r1c) {
      constexpr int r1 = decltype(r1c)::value;
      double y[NB];
      // top level: y[i2] = sum_i1 U[i1][r1] x[i1][i2]
      static_for<0, NB>([&](auto i2c) {
        constexpr int i2 = decltype(i2c)::value;
        y[i2] = chain_col<S, r1, NB, NB>(x + i2);
      });
      static_for<0, R>([&](auto r2c) {
        constexpr int r2 = decltype(r2c)::value;
        const int64_t off = outs[r1 * R + r2];
        if (off >= 0) store_out(ws, a.out_elt, off + pos, a.out_plane, chain_col<S, r2, 1, NB>(y));
      });
    });
  }
}

template <int ID, int SIDE, int LV, bool OCT = false>
__global__ void __launch_bounds__(kAddTX * kAddTY) form_kernel(FormArgs a) {
  form_body<ID, SIDE, LV, OCT>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// form_kernel with two adjacent positions (p, q), (p, q + 1) per thread for
// unsplit outputs: one 8-byte (FP32) or 16-byte (FP64) store per output where
// the pair is aligned.  Same chains, same order.  The launcher runs it for
// FP32 outputs, where it measured 4-5% faster per pass (Strassen L=2 at
// 16384^3: 1.31 -> 1.25 ms); for FP64 outputs it measured 3% slower.
// PAIRS: FP32 source and FP32 outputs with every pair 8-byte aligned (even
// offsets, columns, widths and leading dimensions, an 8-byte aligned source
// pointer): each pair is one 8-byte load and one 8-byte store, with no
// run-time element-type or alignment test per access.
template <int ID, int SIDE, int LV, bool PAIRS>
__device__ __forceinline__ void form2p_body(const FormArgs& a, const Ref& src, const char* base, int64_t ld,
                                            int64_t p, int64_t q) {
  using S = Side<ID, SIDE>;
  constexpr int NB = S::NB, R = S::R, BR = S::BR, BC = S::BC;
  constexpr int NIN = LV == 1 ? NB : NB * NB;
  const bool two = PAIRS || q + 1 < a.w;
  const int g = (int)blockIdx.z;
  const int64_t h = a.h, w = a.w;
  double x0[NIN], x1[NIN];
  static_for<0, NIN>([&](auto ic) {
    constexpr int idx = decltype(ic)::value;
    constexpr int i1 = LV == 1 ? idx : idx / NB;
    constexpr int i2 = LV == 1 ? 0 : idx % NB;
    constexpr int a1 = i1 / BC, b1 = i1 % BC, a2 = i2 / BC, b2 = i2 % BC;
    const int64_t row = src.row + (LV == 1 ? a1 * h : (a1 * BR + a2) * h) + p;
    const int64_t col = src.col + (LV == 1 ? b1 * w : (b1 * BC + b2) * w) + q;
    const int64_t e = src.off + row * ld + col;
    if constexpr (PAIRS) {
      const float2 v = *(const float2*)((const float*)base + e);
      x0[idx] = (double)v.x * src.alpha;
      x1[idx] = (double)v.y * src.alpha;
    } else {
      x0[idx] = load_elt(base, src.elt, e) * src.alpha;
      x1[idx] = load_elt(base, src.elt, two ? e + 1 : e) * src.alpha;
    }
  });
  char* ws = (char*)a.bases.ptr[BUF_WS];
  const int64_t* outs = a.outs + (int64_t)g * a.nout;
  const int64_t pos = p * a.out_ld + q;
  const bool f64 = a.out_elt == ELT_F64;
  auto put = [&](int64_t off, double v0, double v1) {
    const int64_t i = off + pos;
    if constexpr (PAIRS) {
      if ((off & 1) == 0) {  // uniform: the pair's parity is the offset's
        *(float2*)((float*)ws + i) = make_float2((float)v0, (float)v1);
      } else {
        ((float*)ws)[i] = (float)v0;
        ((float*)ws)[i + 1] = (float)v1;
      }
    } else if (two && (i & 1) == 0) {
      if (f64) *(double2*)((double*)ws + i) = make_double2(v0, v1);
      else *(float2*)((float*)ws + i) = make_float2((float)v0, (float)v1);
    } else {
      store_out(ws, a.out_elt, i, a.out_plane, v0);
      if (two) store_out(ws, a.out_elt, i + 1, a.out_plane, v1);
    }
  };
  if constexpr (LV == 1) {
    static_for<0, R>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int64_t off = outs[r];
      if (off >= 0) put(off, chain_col<S, r, 1, NB>(x0), chain_col<S, r, 1, NB>(x1));
    });
  } else {
    static_for<0, R>([&](auto r1c) {
      constexpr int r1 = decltype(r1c)::value;
      double y0[NB], y1[NB];
      static_for<0, NB>([&](auto i2c) {
        constexpr int i2 = decltype(i2c)::value;
        y0[i2] = chain_col<S, r1, NB, NB>(x0 + i2);
        y1[i2] = chain_col<S, r1, NB, NB>(x1 + i2);
      });
      static_for<0, R>([&](auto r2c) {
        constexpr int r2 = decltype(r2c)::value;
        const int64_t off = outs[r1 * R + r2];
        if (off >= 0) put(off, chain_col<S, r2, 1, NB>(y0), chain_col<S, r2, 1, NB>(y1));
      });
    });
  }
}

template <int ID, int SIDE, int LV>
__global__ void __launch_bounds__(kAddTX * kAddTY) form2p_kernel(FormArgs a) {
  const int64_t q = ((int64_t)blockIdx.x * kAddTX + threadIdx.x) * 2;
  const int64_t p = (int64_t)blockIdx.y * kAddTY + threadIdx.y;
  if (q >= a.w || p >= a.h) return;
  const Ref src = a.groups[blockIdx.z];
  int64_t ld;
  const char* base = buf_ptr(a.bases, src, &ld);
  // every value below is uniform over the launch's group
  const bool pairs = a.out_elt == ELT_F32 && src.elt == ELT_F32 &&
                     ((src.off | src.col | ld | a.w | a.out_ld) & 1) == 0 &&
                     ((uintptr_t)base & 7) == 0;
  if (pairs) form2p_body<ID, SIDE, LV, true>(a, src, base, ld, p, q);
  else form2p_body<ID, SIDE, LV, false>(a, src, base, ld, p, q);
}

// One level of S and of T in a single launch, for small problems where the
// idle time between dependent launches is comparable to a pass: blocks
// [0, xs) of the x dimension form S on an xs x ys x zs grid, the rest form T
// on its own yt x zt extent; blocks outside a side's grid do nothing.  The
// body (and so every stored value) is the one form_kernel runs.
template <int ID>
__global__ void __launch_bounds__(kAddTX * kAddTY) form_pair_kernel(FormArgs s, FormArgs t, unsigned xs,
                                                                    unsigned ys, unsigned zs, unsigned yt,
                                                                    unsigned zt) {
  if (blockIdx.x < xs) {
    if (blockIdx.y < ys && blockIdx.z < zs) form_body<ID, 0, 1, false>(s, blockIdx.x, blockIdx.y, blockIdx.z);
  } else if (blockIdx.y < yt && blockIdx.z < zt) {
    form_body<ID, 1, 1, false>(t, blockIdx.x - xs, blockIdx.y, blockIdx.z);
  }
}


// Coefficients of one side as a device table with one row of NB integers per
// output r, so a wave-uniform r reads its row with scalar loads.
template <int ID, int SIDE>
struct ColTable {
  int c[Side<ID, SIDE>::R][Side<ID, SIDE>::NB];
};

template <int ID, int SIDE>
constexpr ColTable<ID, SIDE> make_col_table() {
  ColTable<ID, SIDE> t{};
  for (int r = 0; r < Side<ID, SIDE>::R; ++r)
    for (int i = 0; i < Side<ID, SIDE>::NB; ++i) t.c[r][i] = Side<ID, SIDE>::coef(i, r);
  return t;
}

template <int ID, int SIDE>
__constant__ ColTable<ID, SIDE> kColTable = make_col_table<ID, SIDE>();

// Two levels of operand formation in one pass for wide base cases, staged
// through LDS.  A workgroup owns 64 * NP consecutive columns q of one row p
// of the leaf-sized grid, NP adjacent ones per lane: it first loads the NB^2
// source elements of those positions into LDS (a thread has NP * NB^2 / 4
// loads in flight), then each wavefront takes every fourth top-level output
// r1, forms the NB level-two sums y[i2] = sum_i1 U[i1][r1] x[i1][i2] from
// LDS, and writes S_{r1,r2} = sum_i2 U[i2][r2] y[i2] for every r2 (with NP =
// 2 and FP64 outputs one 16-byte store per lane, 1 KB per wavefront).  Sums
// run in ascending index order from -0.0 with fused multiply-adds: with
// coefficients +-2^e the first step returns c*x exactly and every later one
// rounds like the corresponding add or subtract of the chain, so the results
// equal the register kernel's bit for bit, for either NP.
template <int ID, int SIDE, int NP>
__global__ void __launch_bounds__(256) form2_kernel(FormArgs a) {
  using S = Side<ID, SIDE>;
  constexpr int NB = S::NB, R = S::R, BR = S::BR, BC = S::BC, NIN = NB * NB;
  __shared__ double xs[NIN][64 * NP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * (64 * NP) + NP * lane;
  const int64_t p = blockIdx.y;
  const int g = blockIdx.z;
  const Ref src = a.groups[g];
  int64_t ld;
  const char* base = buf_ptr(a.bases, src, &ld);
  const int64_t h = a.h, w = a.w;
  // Branch-free loads, all in flight before the first LDS store: positions
  // past the last column read column w - 1 and store 0.
  bool ok[NP];
  int64_t qc[NP];
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    ok[e] = q + e < w;
    qc[e] = ok[e] ? q + e : w - 1;
  }
  constexpr int NJ = (NIN + 3) / 4;
  double v[NJ][NP];
  auto load_all = [&](auto tag) {
    using T = decltype(tag);
    const T* bp = (const T*)base + src.off;
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
      const int idx = wave + 4 * k < NIN ? wave + 4 * k : NIN - 1;
      const int i1 = idx / NB, i2 = idx % NB;
      const int a1 = i1 / BC, b1 = i1 % BC, a2 = i2 / BC, b2 = i2 % BC;
      const int64_t row = src.row + (a1 * BR + a2) * h + p;
      const int64_t col = src.col + (b1 * BC + b2) * w;
#pragma unroll
      for (int e = 0; e < NP; ++e) v[k][e] = (double)bp[row * ld + col + qc[e]];
    }
  };
  if (src.elt == ELT_F64) load_all(double{});
  else load_all(float{});
#pragma unroll
  for (int k = 0; k < NJ; ++k)
    if (wave + 4 * k < NIN) {
#pragma unroll
      for (int e = 0; e < NP; ++e) xs[wave + 4 * k][NP * lane + e] = ok[e] ? v[k][e] * src.alpha : 0.0;
    }
  __syncthreads();
  if (!ok[0]) return;
  char* ws = (char*)a.bases.ptr[BUF_WS];
  const int64_t* outs = a.outs + (int64_t)g * a.nout;
  const int64_t pos = p * a.out_ld + q;
  const ColTable<ID, SIDE>& tab = kColTable<ID, SIDE>;
  // both positions of a lane in one 16-byte store: FP64 outputs, the pair
  // inside the row and 16-byte aligned (workspace outputs start 256-byte
  // aligned, so an even row length and an even q make it so)
  const bool pair = NP == 2 && ok[NP - 1] && a.out_elt == ELT_F64 && (a.out_ld & 1) == 0;
  for (int r1 = wave; r1 < R; r1 += 4) {
    double y[NP][NB];
#pragma unroll
    for (int i2 = 0; i2 < NB; ++i2) {
      double acc[NP];
#pragma unroll
      for (int e = 0; e < NP; ++e) acc[e] = -0.0;
#pragma unroll
      for (int i1 = 0; i1 < NB; ++i1) {
        const int c = tab.c[r1][i1];
        if (c != 0) {
#pragma unroll
          for (int e = 0; e < NP; ++e) acc[e] = __fma_rn((double)c, xs[i1 * NB + i2][NP * lane + e], acc[e]);
        }
      }
#pragma unroll
      for (int e = 0; e < NP; ++e) y[e][i2] = acc[e];
    }
    const int64_t* o = outs + r1 * R;
    static_for<0, R>([&](auto r2c) {
      constexpr int r2 = decltype(r2c)::value;
      const int64_t off = o[r2];
      if (off < 0) return;
      if constexpr (NP == 2) {
        const double s0 = chain_col<S, r2, 1, NB>(y[0]), s1 = chain_col<S, r2, 1, NB>(y[1]);
        if (pair && ((off + pos) & 1) == 0) {
          *(double2*)((double*)ws + off + pos) = make_double2(s0, s1);
        } else {
          store_out(ws, a.out_elt, off + pos, a.out_plane, s0);
          if (ok[1]) store_out(ws, a.out_elt, off + pos + 1, a.out_plane, s1);
        }
      } else {
        store_out(ws, a.out_elt, off + pos, a.out_plane, chain_col<S, r2, 1, NB>(y[0]));
      }
    });
  }
}

// Split (BF16x3) leaf operands (one level, or two levels of a narrow base
// case) with two positions per thread, so each store instruction writes two
// bf16 of a plane (4 bytes per lane) instead of one.  S operands (row-major
// planes): positions (p, q) and (p, q + 1), a workgroup covering 512
// consecutive columns of one row (1 KB of each plane, as for T; four rows of
// 128 columns measured the same).  T operands (k-octets): positions (p, q) and
// (p + 1, q) of one octet, a wavefront covering 16 columns of one octet (256
// contiguous bytes per plane, 1 KB per workgroup).  Same chains, in the same
// order, as form_kernel.
// F32IN: an FP32 source, read without a run-time element-type test; for S
// operands (pairs along a row) with every pair 8-byte aligned, as one 8-byte
// load per pair.
template <int ID, int SIDE, int LV, bool F32IN>
__device__ __forceinline__ void form_split2_body(const FormArgs& a, const Ref& src, const char* base, int64_t ld,
                                                 int64_t p, int64_t q) {
  using S = Side<ID, SIDE>;
  constexpr int NB = S::NB, R = S::R, BR = S::BR, BC = S::BC;
  constexpr int NIN = LV == 1 ? NB : NB * NB;
  constexpr int dp = SIDE == 0 ? 0 : 1, dq = SIDE == 0 ? 1 : 0;
  constexpr bool kPairLoad = F32IN && SIDE == 0;
  const bool two = kPairLoad || (q + dq < a.w && p + dp < a.h);
  const int g = blockIdx.z;
  const int64_t h = a.h, w = a.w;
  double x0[NIN], x1[NIN];
  static_for<0, NIN>([&](auto ic) {
    constexpr int idx = decltype(ic)::value;
    constexpr int i1 = LV == 1 ? idx : idx / NB;
    constexpr int i2 = LV == 1 ? 0 : idx % NB;
    constexpr int a1 = i1 / BC, b1 = i1 % BC, a2 = i2 / BC, b2 = i2 % BC;
    const int64_t row = src.row + (LV == 1 ? a1 * h : (a1 * BR + a2) * h) + p;
    const int64_t col = src.col + (LV == 1 ? b1 * w : (b1 * BC + b2) * w) + q;
    const int64_t e = src.off + row * ld + col;
    if constexpr (kPairLoad) {
      const float2 v = *(const float2*)((const float*)base + e);
      x0[idx] = (double)v.x * src.alpha;
      x1[idx] = (double)v.y * src.alpha;
    } else if constexpr (F32IN) {
      const float* bf = (const float*)base;
      x0[idx] = (double)bf[e] * src.alpha;
      x1[idx] = (double)bf[two ? e + dp * ld + dq : e] * src.alpha;
    } else {
      x0[idx] = load_elt(base, src.elt, e) * src.alpha;
      x1[idx] = load_elt(base, src.elt, two ? e + dp * ld + dq : e) * src.alpha;
    }
  });
  unsigned short* ws = (unsigned short*)a.bases.ptr[BUF_WS];
  const int64_t* outs = a.outs + (int64_t)g * a.nout;
  const int64_t pos = SIDE == 0 ? p * a.out_ld + q : (p >> 3) * a.out_ld + q * 8 + (p & 7);
  auto put = [&](int64_t off, double v0, double v1) {
    unsigned short h0, l0, h1, l1;
    split_bits((float)v0, &h0, &l0);
    split_bits((float)v1, &h1, &l1);
    const int64_t i = off + pos;  // even: planes, rows and octets have even lengths
    if (two) {
      *(unsigned*)(ws + i) = (unsigned)h0 | ((unsigned)h1 << 16);
      *(unsigned*)(ws + i + a.out_plane) = (unsigned)l0 | ((unsigned)l1 << 16);
    } else {
      ws[i] = h0;
      ws[i + a.out_plane] = l0;
    }
  };
  if constexpr (LV == 1) {
    static_for<0, R>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int64_t off = outs[r];
      if (off >= 0) put(off, chain_col<S, r, 1, NB>(x0), chain_col<S, r, 1, NB>(x1));
    });
  } else {
    static_for<0, R>([&](auto r1c) {
      constexpr int r1 = decltype(r1c)::value;
      double y0[NB], y1[NB];
      static_for<0, NB>([&](auto i2c) {
        constexpr int i2 = decltype(i2c)::value;
        y0[i2] = chain_col<S, r1, NB, NB>(x0 + i2);
        y1[i2] = chain_col<S, r1, NB, NB>(x1 + i2);
      });
      static_for<0, R>([&](auto r2c) {
        constexpr int r2 = decltype(r2c)::value;
        const int64_t off = outs[r1 * R + r2];
        if (off >= 0) put(off, chain_col<S, r2, 1, NB>(y0), chain_col<S, r2, 1, NB>(y1));
      });
    });
  }
}

template <int ID, int SIDE, int LV>
__global__ void __launch_bounds__(256) form_split2_kernel(FormArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t p, q;
  if constexpr (SIDE == 0) {
    // blockIdx.x enumerates (row, 512-column block) pairs, rows outer
    const int64_t ncb = (a.w + 511) / 512;
    p = (int64_t)blockIdx.x / ncb;
    q = ((int64_t)blockIdx.x % ncb * 256 + threadIdx.x) * 2;
  } else {
    q = (int64_t)blockIdx.x * 64 + wave * 16 + (lane >> 2);
    p = (int64_t)blockIdx.y * 8 + 2 * (lane & 3);
  }
  if (q >= a.w || p >= a.h) return;
  const Ref src = a.groups[blockIdx.z];
  int64_t ld;
  const char* base = buf_ptr(a.bases, src, &ld);
  // uniform over the launch's group
  const bool f32 = src.elt == ELT_F32;
  const bool pairs = SIDE == 0 ? f32 && ((src.off | src.col | ld | a.w) & 1) == 0 && ((uintptr_t)base & 7) == 0
                               : f32;
  if (pairs) form_split2_body<ID, SIDE, LV, true>(a, src, base, ld, p, q);
  else form_split2_body<ID, SIDE, LV, false>(a, src, base, ld, p, q);
}

// W-combination, one level: C_k = sum_r W[k][r] M_r at each position.
template <int ID>
__global__ void __launch_bounds__(kAddTX * kAddTY) combine1_kernel(CombineArgs a) {
  using CB = Comb<ID>;
  constexpr int R = CB::R, MN = CB::MN, N = Alg<ID>::N;
  const int64_t q = (int64_t)blockIdx.x * kAddTX + threadIdx.x;
  const int64_t p = (int64_t)blockIdx.y * kAddTY + threadIdx.y;
  if (q >= a.w || p >= a.h) return;
  const int g = blockIdx.z;
  const char* ws = (const char*)a.bases.ptr[BUF_WS];
  const int64_t in0 = a.in_off[g] + p * a.in_ld + q;
  double mv[R];
  static_for<0, R>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    mv[r] = load_elt(ws, a.in_elt, in0 + r * a.in_stride);
  });
  const Ref out = a.out[g];
  int64_t ld;
  char* ob = buf_ptr(a.bases, out, &ld);
  int64_t pld = 0;
  const char* pb = a.has_p ? buf_ptr(a.bases, a.p, &pld) : nullptr;
  static_for<0, MN>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int ba = k / N, bc = k % N;
    double v = chain_row<ID, k>(mv);
    const int64_t row = ba * a.h + p, col = bc * a.w + q;
    if (a.has_p) v = __dadd_rn(v, load_elt(pb, a.p.elt, a.p.off + row * pld + col));
    const int64_t idx = out.off + (out.row + row) * ld + out.col + col;
    if (out.elt == ELT_F64) ((double*)ob)[idx] = v;
    else ((float*)ob)[idx] = (float)v;
  });
}

template <int ID>
struct WTable {
  int c[Comb<ID>::MN][Comb<ID>::R];
};

template <int ID>
constexpr WTable<ID> make_w_table() {
  WTable<ID> t{};
  for (int k = 0; k < Comb<ID>::MN; ++k)
    for (int r = 0; r < Comb<ID>::R; ++r) t.c[k][r] = Comb<ID>::coef(k, r);
  return t;
}

template <int ID>
__constant__ WTable<ID> kWTable = make_w_table<ID>();

// Whether every W coefficient of a base case is 0 or +-2^e: then c * y is
// exact and a fused multiply-add rounds like the scaled add of the one-level
// chains, so the fused combination kernels below keep their bits.
template <int ID>
constexpr bool w_pow2() {
  for (int k = 0; k < Comb<ID>::MN; ++k)
    for (int r = 0; r < Comb<ID>::R; ++r) {
      const int c = Comb<ID>::coef(k, r) < 0 ? -Comb<ID>::coef(k, r) : Comb<ID>::coef(k, r);
      if (c != 0 && (c & (c - 1)) != 0) return false;
    }
  return true;
}

// W-combination, two levels fused, for narrow base cases (R <= 8) with FP32
// products and FP32 outputs whose pairs of adjacent positions are all 8-byte
// aligned (the host sets CombineArgs::pairs), in registers: each thread owns
// positions (p, q) and (p, q + 1) of one row, reads its R^2 products there
// with one 8-byte load each, and accumulates every C_{c1,c2} with the same
// FMAs in the same order as combine2_kernel (Y_{r1,c2} from -0.0 over
// ascending r2, then C_{c1,c2} over ascending r1), so the two agree bit for
// bit; each output pair is one 8-byte store.  A scheduling fence between
// consecutive r1 keeps each r1's seven loads together (130 registers, three
// wavefronts per SIMD).
template <int ID>
__global__ void __launch_bounds__(kAddTX * kAddTY) combine2p_kernel(CombineArgs a) {
  static_assert(w_pow2<ID>(), "fused combination needs W coefficients 0 or +-2^e");
  using CB = Comb<ID>;
  constexpr int R = CB::R, MN = CB::MN, N = Alg<ID>::N, M = Alg<ID>::M;
  const int64_t q = ((int64_t)blockIdx.x * kAddTX + threadIdx.x) * 2;
  const int64_t p = (int64_t)blockIdx.y * kAddTY + threadIdx.y;
  if (q >= a.w || p >= a.h) return;
  const int g = blockIdx.z;
  const float* ws = (const float*)a.bases.ptr[BUF_WS];
  const int64_t gbase = a.in_off[g] + p * a.in_ld + q;
  double acc0[MN][MN], acc1[MN][MN];
  static_for<0, MN>([&](auto c1c) {
    static_for<0, MN>([&](auto c2c) {
      acc0[decltype(c1c)::value][decltype(c2c)::value] = -0.0;
      acc1[decltype(c1c)::value][decltype(c2c)::value] = -0.0;
    });
  });
  static_for<0, R>([&](auto r1c) {
    constexpr int r1 = decltype(r1c)::value;
    double m0[R], m1[R];
    static_for<0, R>([&](auto r2c) {
      constexpr int r2 = decltype(r2c)::value;
      const float2 v = *(const float2*)(ws + gbase + (int64_t)(r1 * R + r2) * a.in_stride);
      m0[r2] = v.x;
      m1[r2] = v.y;
    });
    double y0[MN], y1[MN];
    static_for<0, MN>([&](auto c2c) {
      constexpr int c2 = decltype(c2c)::value;
      double t0 = -0.0, t1 = -0.0;
      static_for<0, R>([&](auto r2c) {
        constexpr int r2 = decltype(r2c)::value;
        constexpr int c = CB::coef(c2, r2);
        if constexpr (c != 0) {
          t0 = __fma_rn((double)c, m0[r2], t0);
          t1 = __fma_rn((double)c, m1[r2], t1);
        }
      });
      y0[c2] = t0;
      y1[c2] = t1;
    });
    static_for<0, MN>([&](auto c1c) {
      constexpr int c1 = decltype(c1c)::value;
      constexpr int c = CB::coef(c1, r1);
      if constexpr (c != 0) {
        static_for<0, MN>([&](auto c2c) {
          constexpr int c2 = decltype(c2c)::value;
          acc0[c1][c2] = __fma_rn((double)c, y0[c2], acc0[c1][c2]);
          acc1[c1][c2] = __fma_rn((double)c, y1[c2], acc1[c1][c2]);
        });
      }
    });
    __builtin_amdgcn_sched_barrier(0);
  });
  const Ref out = a.out[g];
  int64_t ld;
  float* ob = (float*)buf_ptr(a.bases, out, &ld);
  static_for<0, MN>([&](auto c1c) {
    constexpr int c1 = decltype(c1c)::value;
    constexpr int a1 = c1 / N, cc1 = c1 % N;
    static_for<0, MN>([&](auto c2c) {
      constexpr int c2 = decltype(c2c)::value;
      constexpr int a2 = c2 / N, cc2 = c2 % N;
      const int64_t row = (int64_t)(a1 * M + a2) * a.h + p;
      const int64_t col = (int64_t)(cc1 * N + cc2) * a.w + q;
      const int64_t idx = out.off + (out.row + row) * ld + out.col + col;
      *(float2*)(ob + idx) = make_float2((float)acc0[c1][c2], (float)acc1[c1][c2]);
    });
  });
}

// W-combination, two levels fused, for wide base cases.  A workgroup of four
// wavefronts owns 64 consecutive positions of one row; wavefront w owns the
// top-level output blocks c1 = w, w+4, ... and accumulates C_{c1,c2} for
// every deeper block c2 in registers.  The products are staged through LDS
// RC top-level indices r1 at a time (R*RC*64 elements, every element read
// from HBM once, RC*R/4 loads in flight per thread); from LDS each wavefront
// forms Y_{r1,c2} = sum_r2 W[c2][r2] M_{r1,r2} for all c2 (compile-time
// chains) and adds W[c1][r1] Y_{r1,c2}.  Same summation order as the
// one-level passes, so the results are bitwise theirs.
template <int ID>
__global__ void __launch_bounds__(256) combine2_kernel(CombineArgs a) {
  static_assert(w_pow2<ID>(), "fused combination needs W coefficients 0 or +-2^e");
  using CB = Comb<ID>;
  constexpr int R = CB::R, MN = CB::MN, N = Alg<ID>::N, M = Alg<ID>::M;
  constexpr int RC = 4, CPW = (MN + 3) / 4;
  constexpr int NLD = RC * R * 64 / 256;  // loads per thread and stage
  __shared__ double sm[RC * R][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const int64_t p = blockIdx.y;
  const int g = blockIdx.z;
  const char* ws = (const char*)a.bases.ptr[BUF_WS];
  const int64_t gbase = a.in_off[g] + p * a.in_ld;
  const WTable<ID>& tab = kWTable<ID>;
  double acc[CPW][MN];
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
    for (int c2 = 0; c2 < MN; ++c2) acc[cc][c2] = -0.0;
  for (int r0 = 0; r0 < R; r0 += RC) {
    double v[NLD];
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int e = (int)threadIdx.x + 256 * j;
      const int rr = e >> 6, l = e & 63;
      const int64_t qq = (int64_t)blockIdx.x * 64 + l;
      v[j] = (r0 * R + rr < R * R && qq < a.w)
                 ? load_elt(ws, a.in_elt, gbase + (int64_t)(r0 * R + rr) * a.in_stride + qq)
                 : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int e = (int)threadIdx.x + 256 * j;
      sm[e >> 6][e & 63] = v[j];
    }
    __syncthreads();
    for (int j = 0; j < RC && r0 + j < R; ++j) {
      const int r1 = r0 + j;
      double y[MN];
      static_for<0, MN>([&](auto c2c) {
        constexpr int c2 = decltype(c2c)::value;
        double t = -0.0;
        static_for<0, R>([&](auto r2c) {
          constexpr int r2 = decltype(r2c)::value;
          constexpr int c = CB::coef(c2, r2);
          if constexpr (c != 0) t = __fma_rn((double)c, sm[j * R + r2][lane], t);
        });
        y[c2] = t;
      });
#pragma unroll
      for (int cc = 0; cc < CPW; ++cc) {
        const int c1 = wave + 4 * cc;
        if (c1 < MN) {
          const int c = tab.c[c1][r1];
          if (c != 0) {
#pragma unroll
            for (int c2 = 0; c2 < MN; ++c2) acc[cc][c2] = __fma_rn((double)c, y[c2], acc[cc][c2]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (q >= a.w) return;
  const Ref out = a.out[g];
  int64_t ld;
  char* ob = buf_ptr(a.bases, out, &ld);
  int64_t pld = 0;
  const char* pb = a.has_p ? buf_ptr(a.bases, a.p, &pld) : nullptr;
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc) {
    const int c1 = wave + 4 * cc;
    if (c1 >= MN) continue;
    const int a1 = c1 / N, cc1 = c1 % N;
#pragma unroll
    for (int c2 = 0; c2 < MN; ++c2) {
      const int a2 = c2 / N, cc2 = c2 % N;
      const int64_t row = (int64_t)(a1 * M + a2) * a.h + p;
      const int64_t col = (int64_t)(cc1 * N + cc2) * a.w + q;
      double v = acc[cc][c2];
      if (a.has_p) v = __dadd_rn(v, load_elt(pb, a.p.elt, a.p.off + row * pld + col));
      const int64_t idx = out.off + (out.row + row) * ld + out.col + col;
      if (out.elt == ELT_F64) ((double*)ob)[idx] = v;
      else ((float*)ob)[idx] = (float)v;
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers of one base case (instantiated once per base case, in the
// generated files csrc/gen/fmm_add_NN.hip)


template <int ID>
hipError_t launch_form_id(const FormArgs& a, int side, int lv, int ngroups, hipStream_t s) {
  dim3 block(kAddTX, kAddTY);
  if (a.out_elt == ELT_BF16X2 && (lv == 1 || (lv == 2 && Alg<ID>::R <= 8))) {
    const dim3 g2 = side == 0 ? dim3((unsigned)((a.w + 511) / 512 * a.h), 1, (unsigned)ngroups)
                              : dim3((unsigned)((a.w + 63) / 64), (unsigned)((a.h + 7) / 8), (unsigned)ngroups);
    if (side == 0 && lv == 1) hipLaunchKernelGGL((form_split2_kernel<ID, 0, 1>), g2, dim3(256), 0, s, a);
    else if (side == 1 && lv == 1) hipLaunchKernelGGL((form_split2_kernel<ID, 1, 1>), g2, dim3(256), 0, s, a);
    else if constexpr (Alg<ID>::R <= 8) {
      if (side == 0) hipLaunchKernelGGL((form_split2_kernel<ID, 0, 2>), g2, dim3(256), 0, s, a);
      else hipLaunchKernelGGL((form_split2_kernel<ID, 1, 2>), g2, dim3(256), 0, s, a);
    }
    return hipGetLastError();
  }
  if (lv == 2 && !kFuse2<ID>) return hipErrorInvalidValue;  // planned one level per pass
  if constexpr (Alg<ID>::R > 8 && kFuse2<ID>) {
    // split T operands of two fused levels of a wide base case: the register
    // kernel with the 8 x 8 wavefront mapping of the k-octet layout
    if (side == 1 && a.out_elt == ELT_BF16X2 && lv == 2) {
      dim3 grid((unsigned)((a.w + 31) / 32), (unsigned)((a.h + 7) / 8), (unsigned)ngroups);
      hipLaunchKernelGGL((form_kernel<ID, 1, 2, true>), grid, block, 0, s, a);
      return hipGetLastError();
    }
  }
  // Two fused levels of a wide base case go through LDS, except split T
  // operands (k-octet layout), which keep the register kernel's 8 x 8 mapping.
  if constexpr (kFuse2<ID>) {
    if (lv == 2 && Alg<ID>::R > 8 && !(side == 1 && a.out_elt == ELT_BF16X2)) {
      // two positions per lane while the staged sources of 128 positions fit
      // two workgroups in a compute unit's LDS (at most 8 blocks per side:
      // 64 KB); measured 2-3% faster per pass on <4,2,4> at 16384^3
      constexpr bool two = Alg<ID>::M * Alg<ID>::K <= 8 && Alg<ID>::K * Alg<ID>::N <= 8;
      constexpr int NP = two ? 2 : 1;
      dim3 g2((unsigned)((a.w + 64 * NP - 1) / (64 * NP)), (unsigned)a.h, (unsigned)ngroups);
      if (side == 0) hipLaunchKernelGGL((form2_kernel<ID, 0, NP>), g2, dim3(256), 0, s, a);
      else hipLaunchKernelGGL((form2_kernel<ID, 1, NP>), g2, dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
  if (a.out_elt == ELT_F32 && (lv == 1 || Alg<ID>::R <= 8)) {
    dim3 gp((unsigned)((a.w + 2 * kAddTX - 1) / (2 * kAddTX)), (unsigned)((a.h + kAddTY - 1) / kAddTY),
            (unsigned)ngroups);
    if (side == 0 && lv == 1) hipLaunchKernelGGL((form2p_kernel<ID, 0, 1>), gp, block, 0, s, a);
    else if (side == 1 && lv == 1) hipLaunchKernelGGL((form2p_kernel<ID, 1, 1>), gp, block, 0, s, a);
    else if constexpr (Alg<ID>::R <= 8) {
      if (side == 0) hipLaunchKernelGGL((form2p_kernel<ID, 0, 2>), gp, block, 0, s, a);
      else hipLaunchKernelGGL((form2p_kernel<ID, 1, 2>), gp, block, 0, s, a);
    }
    return hipGetLastError();
  }
  dim3 grid((unsigned)((a.w + kAddTX - 1) / kAddTX), (unsigned)((a.h + kAddTY - 1) / kAddTY),
            (unsigned)ngroups);
  if (side == 0 && lv == 1) hipLaunchKernelGGL((form_kernel<ID, 0, 1>), grid, block, 0, s, a);
  else if (side == 1 && lv == 1) hipLaunchKernelGGL((form_kernel<ID, 1, 1>), grid, block, 0, s, a);
  else if constexpr (Alg<ID>::R <= 8) {
    if (side == 0 && lv == 2) hipLaunchKernelGGL((form_kernel<ID, 0, 2>), grid, block, 0, s, a);
    else if (side == 1 && lv == 2) hipLaunchKernelGGL((form_kernel<ID, 1, 2>), grid, block, 0, s, a);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ID>
hipError_t launch_form_pair_id(const FormArgs& sa, int ngs, const FormArgs& ta, int ngt, hipStream_t st) {
  const unsigned xs = (unsigned)((sa.w + kAddTX - 1) / kAddTX), ys = (unsigned)((sa.h + kAddTY - 1) / kAddTY);
  const unsigned xt = (unsigned)((ta.w + kAddTX - 1) / kAddTX), yt = (unsigned)((ta.h + kAddTY - 1) / kAddTY);
  const dim3 grid(xs + xt, ys > yt ? ys : yt, (unsigned)(ngs > ngt ? ngs : ngt));
  hipLaunchKernelGGL((form_pair_kernel<ID>), grid, dim3(kAddTX, kAddTY), 0, st, sa, ta, xs, ys, (unsigned)ngs, yt,
                     (unsigned)ngt);
  return hipGetLastError();
}

template <int ID>
hipError_t launch_combine_id(const CombineArgs& a, int lv, int ngroups, hipStream_t s) {
  if (lv == 1) {
    dim3 block(kAddTX, kAddTY);
    dim3 grid((unsigned)((a.w + kAddTX - 1) / kAddTX), (unsigned)((a.h + kAddTY - 1) / kAddTY),
              (unsigned)ngroups);
    hipLaunchKernelGGL((combine1_kernel<ID>), grid, block, 0, s, a);
  } else if (lv == 2) {
    if constexpr (Alg<ID>::R <= 8) {
      if (a.pairs) {  // FP32 products and outputs, aligned pairs: the register kernel
        dim3 grid((unsigned)((a.w + 2 * kAddTX - 1) / (2 * kAddTX)), (unsigned)((a.h + kAddTY - 1) / kAddTY),
                  (unsigned)ngroups);
        hipLaunchKernelGGL((combine2p_kernel<ID>), grid, dim3(kAddTX, kAddTY), 0, s, a);
        return hipGetLastError();
      }
    }
    if constexpr (kFuse2<ID>) {
      dim3 grid((unsigned)((a.w + 63) / 64), (unsigned)a.h, (unsigned)ngroups);
      hipLaunchKernelGGL((combine2_kernel<ID>), grid, dim3(256), 0, s, a);
    } else {
      return hipErrorInvalidValue;  // planned one level per pass
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fmm
