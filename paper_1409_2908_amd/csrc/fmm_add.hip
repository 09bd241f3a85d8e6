// Streaming addition kernels: operand formation (S_r from A with U, T_r from B
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
// (their Kronecker-product coefficients are applied level by level in
// registers, top level first, which is the recursion's own order).
#include <hip/hip_runtime.h>

#include "fmm_device.h"
#include "fmm_launch.h"

namespace fmm {

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
template <int ID, int SIDE, int LV, bool OCT = false>
__global__ void __launch_bounds__(kAddTX * kAddTY) form_kernel(FormArgs a) {
  using S = Side<ID, SIDE>;
  constexpr int NB = S::NB, R = S::R, BR = S::BR, BC = S::BC;
  constexpr int NIN = LV == 1 ? NB : NB * NB;
  const int t = threadIdx.y * kAddTX + threadIdx.x;
  const int64_t q = OCT ? (int64_t)blockIdx.x * 32 + (t >> 3) : (int64_t)blockIdx.x * kAddTX + threadIdx.x;
  const int64_t p = OCT ? (int64_t)blockIdx.y * 8 + (t & 7) : (int64_t)blockIdx.y * kAddTY + threadIdx.y;
  if (q >= a.w || p >= a.h) return;
  const int g = blockIdx.z;
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

// W-combination, two levels fused.  A workgroup of MN wavefronts covers 64
// consecutive positions; wavefront c2 owns the deeper-level output block c2
// and accumulates the top-level outputs C_{c1,c2} for every c1 in registers.
// For each top-level product r1 the workgroup stages the R products
// M_{r1,r2} of its 64 positions in LDS (each element read from HBM once),
// every wavefront forms Y_{r1,c2} = sum_r2 W[c2][r2] M_{r1,r2} from LDS, and
// adds W[c1][r1] Y_{r1,c2} into its accumulators.  Sums run in ascending
// index order starting from zero; with coefficients 0 or +-2^e each fused
// multiply-add rounds exactly like the corresponding chain step.
template <int ID>
__global__ void __launch_bounds__(1024) combine2_kernel(CombineArgs a) {
  using CB = Comb<ID>;
  constexpr int R = CB::R, MN = CB::MN, N = Alg<ID>::N, M = Alg<ID>::M;
  __shared__ double sm[2][R][64];
  const int lane = threadIdx.x & 63;
  const int c2 = threadIdx.x >> 6;  // wave-uniform
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const int64_t p = blockIdx.y;
  const int g = blockIdx.z;
  const char* ws = (const char*)a.bases.ptr[BUF_WS];
  const int64_t gbase = a.in_off[g] + p * a.in_ld;
  // Accumulators start at -0.0 so that the first fused multiply-add returns
  // exactly c*x, signed zeros included, like the first term of a chain.
  double acc[MN];
#pragma unroll
  for (int c1 = 0; c1 < MN; ++c1) acc[c1] = -0.0;
  auto stage = [&](int buf, int r1) {
    for (int e = threadIdx.x; e < R * 64; e += MN * 64) {
      const int r2 = e >> 6, l = e & 63;
      const int64_t qq = (int64_t)blockIdx.x * 64 + l;
      double v = 0.0;
      if (qq < a.w) v = load_elt(ws, a.in_elt, gbase + ((int64_t)r1 * R + r2) * a.in_stride + qq);
      sm[buf][r2][l] = v;
    }
  };
  stage(0, 0);
  __syncthreads();
  for (int r1 = 0; r1 < R; ++r1) {
    const int cur = r1 & 1;
    if (r1 + 1 < R) stage(cur ^ 1, r1 + 1);
    double y = -0.0;
    for (int r2 = 0; r2 < R; ++r2) {
      const int c = a.wc[c2][r2];
      if (c != 0) y = __fma_rn((double)c, sm[cur][r2][lane], y);
    }
#pragma unroll
    for (int c1 = 0; c1 < MN; ++c1) {
      const int c = a.wc[c1][r1];
      if (c != 0) acc[c1] = __fma_rn((double)c, y, acc[c1]);
    }
    __syncthreads();
  }
  if (q >= a.w) return;
  const Ref out = a.out[g];
  int64_t ld;
  char* ob = buf_ptr(a.bases, out, &ld);
  int64_t pld = 0;
  const char* pb = a.has_p ? buf_ptr(a.bases, a.p, &pld) : nullptr;
  const int a2 = c2 / N, cc2 = c2 % N;
#pragma unroll
  for (int c1 = 0; c1 < MN; ++c1) {
    const int a1 = c1 / N, cc1 = c1 % N;
    const int64_t row = (int64_t)(a1 * M + a2) * a.h + p;
    const int64_t col = (int64_t)(cc1 * N + cc2) * a.w + q;
    double v = acc[c1];
    if (a.has_p) v = __dadd_rn(v, load_elt(pb, a.p.elt, a.p.off + row * pld + col));
    const int64_t idx = out.off + (out.row + row) * ld + out.col + col;
    if (out.elt == ELT_F64) ((double*)ob)[idx] = v;
    else ((float*)ob)[idx] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// host launchers

template <int ID>
static hipError_t launch_form_id(const FormArgs& a, int side, int lv, int ngroups, hipStream_t s) {
  dim3 block(kAddTX, kAddTY);
  if (side == 1 && a.out_elt == ELT_BF16X2) {
    dim3 grid((unsigned)((a.w + 31) / 32), (unsigned)((a.h + 7) / 8), (unsigned)ngroups);
    if (lv == 1) hipLaunchKernelGGL((form_kernel<ID, 1, 1, true>), grid, block, 0, s, a);
    else if (lv == 2) hipLaunchKernelGGL((form_kernel<ID, 1, 2, true>), grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  dim3 grid((unsigned)((a.w + kAddTX - 1) / kAddTX), (unsigned)((a.h + kAddTY - 1) / kAddTY),
            (unsigned)ngroups);
  if (side == 0 && lv == 1) hipLaunchKernelGGL((form_kernel<ID, 0, 1>), grid, block, 0, s, a);
  else if (side == 0 && lv == 2) hipLaunchKernelGGL((form_kernel<ID, 0, 2>), grid, block, 0, s, a);
  else if (side == 1 && lv == 1) hipLaunchKernelGGL((form_kernel<ID, 1, 1>), grid, block, 0, s, a);
  else if (side == 1 && lv == 2) hipLaunchKernelGGL((form_kernel<ID, 1, 2>), grid, block, 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_form(int alg, const FormArgs& a, int side, int lv, int ngroups, hipStream_t s) {
  if (a.h == 0 || a.w == 0 || ngroups == 0) return hipSuccess;
  switch (alg) {
    case 0: return launch_form_id<0>(a, side, lv, ngroups, s);
    case 1: return launch_form_id<1>(a, side, lv, ngroups, s);
    case 2: return launch_form_id<2>(a, side, lv, ngroups, s);
    case 3: return launch_form_id<3>(a, side, lv, ngroups, s);
    case 4: return launch_form_id<4>(a, side, lv, ngroups, s);
    case 5: return launch_form_id<5>(a, side, lv, ngroups, s);
  }
  return hipErrorInvalidValue;
}

template <int ID>
static hipError_t launch_combine_id(const CombineArgs& a, int lv, int ngroups, hipStream_t s) {
  if (lv == 1) {
    dim3 block(kAddTX, kAddTY);
    dim3 grid((unsigned)((a.w + kAddTX - 1) / kAddTX), (unsigned)((a.h + kAddTY - 1) / kAddTY),
              (unsigned)ngroups);
    hipLaunchKernelGGL((combine1_kernel<ID>), grid, block, 0, s, a);
  } else if (lv == 2) {
    constexpr int MN = Comb<ID>::MN;
    dim3 block(64 * MN);
    dim3 grid((unsigned)((a.w + 63) / 64), (unsigned)a.h, (unsigned)ngroups);
    hipLaunchKernelGGL((combine2_kernel<ID>), grid, block, 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine(int alg, const CombineArgs& a, int lv, int ngroups, hipStream_t s) {
  if (a.h == 0 || a.w == 0 || ngroups == 0) return hipSuccess;
  switch (alg) {
    case 0: return launch_combine_id<0>(a, lv, ngroups, s);
    case 1: return launch_combine_id<1>(a, lv, ngroups, s);
    case 2: return launch_combine_id<2>(a, lv, ngroups, s);
    case 3: return launch_combine_id<3>(a, lv, ngroups, s);
    case 4: return launch_combine_id<4>(a, lv, ngroups, s);
    case 5: return launch_combine_id<5>(a, lv, ngroups, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace fmm
