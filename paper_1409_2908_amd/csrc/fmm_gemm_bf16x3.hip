// Grouped, persistent leaf GEMM for FP32 operands with BF16x3 products.
//
// Each FP32 operand element x is carried as
//   hi = bf16(x)   and   lo = bf16(x - hi)     (round to nearest even),
// and every leaf product is accumulated in FP32 by the BF16 matrix cores as
//   A_hi B_hi + A_hi B_lo + A_lo B_hi
// (the lo*lo term, below FP32 resolution of the result, is dropped).  The
// split keeps about 16 significant bits of each operand; the W-combination and
// the operand sums stay in FP64/FP32 outside this kernel.  Leaf operands
// arrive already split (the formation kernels write hi / lo planes), so their
// tiles go from HBM to LDS as 16-byte groups with no arithmetic; FP32
// operands (peel strips, the classical product) are split on their way into
// LDS.
//
// Work decomposition and scheduling follow the FP64/FP32 kernel: one flat tile
// space over all problems, ~2 workgroups of 4 wavefronts per CU, 128 x 128
// tiles, 64 x 64 per wavefront = 4 x 4 blocks of v_mfma_f32_16x16x32_bf16, XCD
// aware tile order.  K advances 32 per step through double-buffered LDS that
// holds the hi and lo planes of A (row-major, k contiguous) and of B
// transposed (n-major, k contiguous), so each lane's MFMA fragment (8
// consecutive k of one row / column) is one 16-byte LDS read.  Operands are
// read with raw buffer loads (out-of-range lanes read 0, stores past the
// edge are dropped).
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "fmm_gemm_common.h"
#include "fmm_launch.h"

namespace fmm {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));

constexpr int XBM = 128, XBN = 128, XBK = 32, XNT = 256;
constexpr int XKP = XBK + 8;  // LDS row length in bf16 (keeps 16-byte rows, shifts banks)

struct Bf16x3Smem {
  __bf16 a_hi[2][XBM][XKP];
  __bf16 a_lo[2][XBM][XKP];
  __bf16 b_hi[2][XBN][XKP];
  __bf16 b_lo[2][XBN][XKP];
};

__device__ __forceinline__ void split(float x, __bf16& hi, __bf16& lo) {
  unsigned short h, l;
  split_bits(x, &h, &l);
  hi = __builtin_bit_cast(__bf16, h);
  lo = __builtin_bit_cast(__bf16, l);
}

__device__ __forceinline__ float load_f32(__amdgpu_buffer_rsrc_t r, int off, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}

typedef unsigned u4_t __attribute__((ext_vector_type(4)));

// Keeps the first `nvalid` (0..8) bf16 elements of an 8-element group held in
// four dwords (element e in dword e / 2, low half for even e) and zeroes the
// rest: the part of a 16-byte group past the end of K.
__device__ __forceinline__ u4_t keep_first(u4_t v, int nvalid) {
  u4_t r;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const unsigned m = 2 * d + 1 < nvalid ? 0xffffffffu : 2 * d < nvalid ? 0x0000ffffu : 0u;
    r[d] = v[d] & m;
  }
  return r;
}

// One 128 x 128 output tile of a leaf whose operands were split by the
// formation kernels: S planes row-major (row stride lda), T planes in
// k-octets (group stride ldb).  Every 16-byte global load is one MFMA
// fragment's worth of k and goes to LDS unchanged; no arithmetic precedes the
// matrix cores except zeroing the part of the last K group past K.
__device__ __forceinline__ void bf16x3_tile_split(Bf16x3Smem& sm, const __bf16* Ah, const __bf16* Al,
                                                  const __bf16* Bh, const __bf16* Bl, float* C, int lda,
                                                  int ldb, int ldc, int mrem, int nrem, int64_t K,
                                                  float alpha) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;

  // A: rows ar and ar + 64, k group ak; B: k groups bg and bg + 2, column bn
  const int ar = tid >> 2, ak = tid & 3;
  const int bg = tid >> 7, bn = tid & 127;
  const int a_base = (ar * lda + 8 * ak) * 2;
  const int a_step = uniform_int(64 * lda * 2);
  const int b_base = bn < nrem ? (bg * ldb + 8 * bn) * 2 : kInvalidOff;
  const int b_step = uniform_int(2 * ldb * 2);

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  u4_t rah[2], ral[2], rbh[2], rbl[2];
  auto ld16 = [](__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
  };
  auto gload = [&](int64_t k0) {
    const __amdgpu_buffer_rsrc_t sah = make_rsrc(Ah + k0), sal = make_rsrc(Al + k0);
    const __amdgpu_buffer_rsrc_t sbh = make_rsrc(Bh + (k0 >> 3) * ldb), sbl = make_rsrc(Bl + (k0 >> 3) * ldb);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int ao = (ar + 64 * j < mrem && k0 + 8 * ak < K) ? a_base : kInvalidOff;
      rah[j] = ld16(sah, ao, j * a_step);
      ral[j] = ld16(sal, ao, j * a_step);
      const int bo = k0 + 8 * (bg + 2 * j) < K ? b_base : kInvalidOff;
      rbh[j] = ld16(sbh, bo, j * b_step);
      rbl[j] = ld16(sbl, bo, j * b_step);
    }
  };
  auto lstore = [&](int buf, int64_t k0) {
    if (k0 + XBK > K) {  // last, partial K step (uniform)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int na = (int)(K - k0) - 8 * ak, nb = (int)(K - k0) - 8 * (bg + 2 * j);
        rah[j] = keep_first(rah[j], na);
        ral[j] = keep_first(ral[j], na);
        rbh[j] = keep_first(rbh[j], nb);
        rbl[j] = keep_first(rbl[j], nb);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      *(u4_t*)&sm.a_hi[buf][ar + 64 * j][8 * ak] = rah[j];
      *(u4_t*)&sm.a_lo[buf][ar + 64 * j][8 * ak] = ral[j];
      *(u4_t*)&sm.b_hi[buf][bn][8 * (bg + 2 * j)] = rbh[j];
      *(u4_t*)&sm.b_lo[buf][bn][8 * (bg + 2 * j)] = rbl[j];
    }
  };

  const int64_t nk = (K + XBK - 1) / XBK;
  // Fragments: A (hi, lo) of the step, B (hi, lo) of the column block in use
  // and of the next one.  The barrier sits after the third column block:
  // every read of the current buffer is issued before it, the next buffer is
  // written before it, and after it the next step's A fragments and first B
  // fragments are read while the last column block's MFMAs run.
  bf8_t ah[4], al[4], bh[2], bl[2];
  auto rd_a = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = *(const bf8_t*)&sm.a_hi[buf][wm * 64 + i * 16 + li][8 * lg];
      al[i] = *(const bf8_t*)&sm.a_lo[buf][wm * 64 + i * 16 + li][8 * lg];
    }
  };
  auto rd_b = [&](int buf, int j) {
    bh[j & 1] = *(const bf8_t*)&sm.b_hi[buf][wn * 64 + j * 16 + li][8 * lg];
    bl[j & 1] = *(const bf8_t*)&sm.b_lo[buf][wn * 64 + j * 16 + li][8 * lg];
  };
  auto mma = [&](int j) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j & 1], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j & 1], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j & 1], acc[i][j], 0, 0, 0);
    }
  };
  if (nk > 0) {
    gload(0);
    lstore(0, 0);
  }
  __syncthreads();
  if (nk > 0) {
    rd_a(0);
    rd_b(0, 0);
  }
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) gload((kt + 1) * XBK);
    rd_b(cur, 1);
    mma(0);
    rd_b(cur, 2);
    mma(1);
    if (more) lstore(cur ^ 1, (kt + 1) * XBK);
    rd_b(cur, 3);
    mma(2);
    __syncthreads();
    if (more) rd_b(cur ^ 1, 0);
    // last column block: once a row block's three MFMAs are issued, its A
    // fragments are replaced by the next step's
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[1], acc[i][3], 0, 0, 0);
      acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[1], acc[i][3], 0, 0, 0);
      acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[1], acc[i][3], 0, 0, 0);
      if (more) {
        ah[i] = *(const bf8_t*)&sm.a_hi[cur ^ 1][wm * 64 + i * 16 + li][8 * lg];
        al[i] = *(const bf8_t*)&sm.a_lo[cur ^ 1][wm * 64 + i * 16 + li][8 * lg];
      }
    }
  }

  const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wm * 64 + i * 16 + 4 * lg + v;
        const int c = wn * 64 + j * 16 + li;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, alpha * acc[i][j][v]), sc,
                                              (r < mrem && c < nrem) ? (r * ldc + c) * 4 : kInvalidOff, 0, 0);
      }
}

// One 128 x 128 output tile with FP32 operands (peel strips and the
// classical product), split on the way into LDS.  PAIR: K is even, so A is
// read as aligned element pairs (8-byte loads); otherwise element by element.
template <bool PAIR>
__device__ __forceinline__ void bf16x3_tile(Bf16x3Smem& sm, const float* A, const float* B, float* C, int lda,
                                            int ldb, int ldc, int mrem, int nrem, int64_t K, float alpha) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;

  // A staging: PAIR: 8 pairs per thread (rows ar + 16 j, k = 2 kp, 2 kp + 1);
  // otherwise 16 singles (rows ar1 + 8 j, k = ak1).
  const int ar = tid >> 4, kp = tid & 15;
  const int ar1 = tid >> 5, ak1 = tid & 31;
  // B staging: column bn, 16 consecutive k from bk0 (two chunks of 8).
  const int bn = tid & 127, bk0 = (tid >> 7) * 16;
  const int a_step = uniform_int(PAIR ? 16 * lda * 4 : 8 * lda * 4);
  const int b_step = uniform_int(ldb * 4);
  const int a_base = PAIR ? (ar * lda + 2 * kp) * 4 : (ar1 * lda + ak1) * 4;
  const int a_rows = PAIR ? (mrem - ar + 15) / 16 : (mrem - ar1 + 7) / 8;
  const int b_base = bn < nrem ? (bk0 * ldb + bn) * 4 : kInvalidOff;

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  float ra[16], rb[16];
  auto gload = [&](int64_t k0) {
    const __amdgpu_buffer_rsrc_t sa = make_rsrc(A + k0);
    const __amdgpu_buffer_rsrc_t sb = make_rsrc(B + k0 * (int64_t)ldb);
    const int kr = K - k0 < XBK ? (int)(K - k0) : XBK;
    if constexpr (PAIR) {
      const int av = 2 * kp < kr ? a_base : kInvalidOff;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // the builtin returns a vector_size(8) value: reinterpret its 8 bytes
        // as two floats (element-wise conversion to another vector kind is
        // not a reinterpretation)
        const f2_t v = __builtin_bit_cast(
            f2_t, __builtin_amdgcn_raw_buffer_load_b64(sa, j < a_rows ? av : kInvalidOff, j * a_step, 0));
        ra[2 * j] = v.x;
        ra[2 * j + 1] = v.y;
      }
    } else {
      const int av = ak1 < kr ? a_base : kInvalidOff;
#pragma unroll
      for (int j = 0; j < 16; ++j) ra[j] = load_f32(sa, j < a_rows ? av : kInvalidOff, j * a_step);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) rb[e] = load_f32(sb, bk0 + e < kr ? b_base : kInvalidOff, e * b_step);
  };
  auto lstore = [&](int buf) {
    if constexpr (PAIR) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 h0, l0, h1, l1;
        split(ra[2 * j], h0, l0);
        split(ra[2 * j + 1], h1, l1);
        *(bf2_t*)&sm.a_hi[buf][ar + 16 * j][2 * kp] = bf2_t{h0, h1};
        *(bf2_t*)&sm.a_lo[buf][ar + 16 * j][2 * kp] = bf2_t{l0, l1};
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) split(ra[j], sm.a_hi[buf][ar1 + 8 * j][ak1], sm.a_lo[buf][ar1 + 8 * j][ak1]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      bf8_t h, l;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 x, y;
        split(rb[8 * c + e], x, y);
        h[e] = x;
        l[e] = y;
      }
      *(bf8_t*)&sm.b_hi[buf][bn][bk0 + 8 * c] = h;
      *(bf8_t*)&sm.b_lo[buf][bn][bk0 + 8 * c] = l;
    }
  };

  const int64_t nk = (K + XBK - 1) / XBK;
  // Same schedule as bf16x3_tile_split: barrier after the third column block,
  // the next step's fragments read under the last block's MFMAs.
  bf8_t ah[4], al[4], bh[2], bl[2];
  auto rd_a = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = *(const bf8_t*)&sm.a_hi[buf][wm * 64 + i * 16 + li][8 * lg];
      al[i] = *(const bf8_t*)&sm.a_lo[buf][wm * 64 + i * 16 + li][8 * lg];
    }
  };
  auto rd_b = [&](int buf, int j) {
    bh[j & 1] = *(const bf8_t*)&sm.b_hi[buf][wn * 64 + j * 16 + li][8 * lg];
    bl[j & 1] = *(const bf8_t*)&sm.b_lo[buf][wn * 64 + j * 16 + li][8 * lg];
  };
  auto mma = [&](int j) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j & 1], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j & 1], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j & 1], acc[i][j], 0, 0, 0);
    }
  };
  if (nk > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  if (nk > 0) {
    rd_a(0);
    rd_b(0, 0);
  }
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) gload((kt + 1) * XBK);
    rd_b(cur, 1);
    mma(0);
    rd_b(cur, 2);
    mma(1);
    if (more) lstore(cur ^ 1);
    rd_b(cur, 3);
    mma(2);
    __syncthreads();
    if (more) rd_b(cur ^ 1, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[1], acc[i][3], 0, 0, 0);
      acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[1], acc[i][3], 0, 0, 0);
      acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[1], acc[i][3], 0, 0, 0);
      if (more) {
        ah[i] = *(const bf8_t*)&sm.a_hi[cur ^ 1][wm * 64 + i * 16 + li][8 * lg];
        al[i] = *(const bf8_t*)&sm.a_lo[cur ^ 1][wm * 64 + i * 16 + li][8 * lg];
      }
    }
  }

  const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // 16x16 f32 MFMA output: register v of lane l is row 4 (l / 16) + v, column l % 16
        const int r = wm * 64 + i * 16 + 4 * lg + v;
        const int c = wn * 64 + j * 16 + li;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, alpha * acc[i][j][v]), sc,
                                              (r < mrem && c < nrem) ? (r * ldc + c) * 4 : kInvalidOff, 0, 0);
      }
}

// 64 x 64 tiles (launches whose 128 x 128 tiles would leave compute units
// idle): 4 wavefronts of 32 x 32 outputs (2 x 2 MFMA blocks), the same LDS
// layout, loads and split as the 128 x 128 tiles, and the plain schedule of
// one barrier per K step after the step's MFMAs.
struct Bf16x3Smem64 {
  __bf16 a_hi[2][64][XKP];
  __bf16 a_lo[2][64][XKP];
  __bf16 b_hi[2][64][XKP];
  __bf16 b_lo[2][64][XKP];
};

// MFMAs and the C store of one 64 x 64 tile from the LDS buffers; `stage`
// (k0, buf) writes the next step's operands into LDS buffer buf.
template <class Stage, class Load>
__device__ __forceinline__ void bf16x3_mma64(Bf16x3Smem64& sm, Load&& gload, Stage&& lstore, float* C, int ldc,
                                             int mrem, int nrem, int64_t K, float alpha) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;
  f4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0, 0, 0, 0};
  const int64_t nk = (K + XBK - 1) / XBK;
  if (nk > 0) {
    gload(0);
    lstore(0, 0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) gload((kt + 1) * XBK);
    bf8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *(const bf8_t*)&sm.a_hi[cur][wm * 32 + i * 16 + li][8 * lg];
      al[i] = *(const bf8_t*)&sm.a_lo[cur][wm * 32 + i * 16 + li][8 * lg];
      bh[i] = *(const bf8_t*)&sm.b_hi[cur][wn * 32 + i * 16 + li][8 * lg];
      bl[i] = *(const bf8_t*)&sm.b_lo[cur][wn * 32 + i * 16 + li][8 * lg];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    // the other buffer's readers all passed the previous barrier
    if (more) lstore(cur ^ 1, (kt + 1) * XBK);
    __syncthreads();
  }
  const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wm * 32 + i * 16 + 4 * lg + v;
        const int c = wn * 32 + j * 16 + li;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, alpha * acc[i][j][v]), sc,
                                              (r < mrem && c < nrem) ? (r * ldc + c) * 4 : kInvalidOff, 0, 0);
      }
}

// 64 x 64 tile of a leaf with split operands (layouts as bf16x3_tile_split).
__device__ __forceinline__ void bf16x3_tile_split64(Bf16x3Smem64& sm, const __bf16* Ah, const __bf16* Al,
                                                    const __bf16* Bh, const __bf16* Bl, float* C, int lda,
                                                    int ldb, int ldc, int mrem, int nrem, int64_t K,
                                                    float alpha) {
  const int tid = threadIdx.x;
  // A: row ar, k group ak; B: k group bg, column bn (one 16-byte group each)
  const int ar = tid >> 2, ak = tid & 3;
  const int bg = tid >> 6, bn = tid & 63;
  const int a_base = (ar * lda + 8 * ak) * 2;
  const int b_base = bn < nrem ? (bg * ldb + 8 * bn) * 2 : kInvalidOff;
  u4_t rah, ral, rbh, rbl;
  auto ld16 = [](__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  };
  auto gload = [&](int64_t k0) {
    const __amdgpu_buffer_rsrc_t sah = make_rsrc(Ah + k0), sal = make_rsrc(Al + k0);
    const __amdgpu_buffer_rsrc_t sbh = make_rsrc(Bh + (k0 >> 3) * ldb), sbl = make_rsrc(Bl + (k0 >> 3) * ldb);
    const int ao = (ar < mrem && k0 + 8 * ak < K) ? a_base : kInvalidOff;
    const int bo = k0 + 8 * bg < K ? b_base : kInvalidOff;
    rah = ld16(sah, ao);
    ral = ld16(sal, ao);
    rbh = ld16(sbh, bo);
    rbl = ld16(sbl, bo);
  };
  auto lstore = [&](int buf, int64_t k0) {
    if (k0 + XBK > K) {  // last, partial K step (uniform)
      const int na = (int)(K - k0) - 8 * ak, nb = (int)(K - k0) - 8 * bg;
      rah = keep_first(rah, na);
      ral = keep_first(ral, na);
      rbh = keep_first(rbh, nb);
      rbl = keep_first(rbl, nb);
    }
    *(u4_t*)&sm.a_hi[buf][ar][8 * ak] = rah;
    *(u4_t*)&sm.a_lo[buf][ar][8 * ak] = ral;
    *(u4_t*)&sm.b_hi[buf][bn][8 * bg] = rbh;
    *(u4_t*)&sm.b_lo[buf][bn][8 * bg] = rbl;
  };
  bf16x3_mma64(sm, gload, lstore, C, ldc, mrem, nrem, K, alpha);
}

// 64 x 64 tile with FP32 operands, split on the way into LDS (as bf16x3_tile).
template <bool PAIR>
__device__ __forceinline__ void bf16x3_tile64(Bf16x3Smem64& sm, const float* A, const float* B, float* C, int lda,
                                              int ldb, int ldc, int mrem, int nrem, int64_t K, float alpha) {
  const int tid = threadIdx.x;
  // A staging: PAIR: 4 pairs per thread (rows ar + 16 j, k = 2 kp, 2 kp + 1);
  // otherwise 8 singles (rows ar1 + 8 j, k = ak1).  B: column bn, 8
  // consecutive k from bk0.
  const int ar = tid >> 4, kp = tid & 15;
  const int ar1 = tid >> 5, ak1 = tid & 31;
  const int bn = tid & 63, bk0 = (tid >> 6) * 8;
  const int a_step = PAIR ? 16 * lda * 4 : 8 * lda * 4;
  const int a_base = PAIR ? (ar * lda + 2 * kp) * 4 : (ar1 * lda + ak1) * 4;
  const int a_rows = PAIR ? (mrem - ar + 15) / 16 : (mrem - ar1 + 7) / 8;
  const int b_base = bn < nrem ? (bk0 * ldb + bn) * 4 : kInvalidOff;
  const int b_step = ldb * 4;
  float ra[8], rb[8];
  auto gload = [&](int64_t k0) {
    const __amdgpu_buffer_rsrc_t sa = make_rsrc(A + k0);
    const __amdgpu_buffer_rsrc_t sb = make_rsrc(B + k0 * (int64_t)ldb);
    const int kr = K - k0 < XBK ? (int)(K - k0) : XBK;
    if constexpr (PAIR) {
      const int av = 2 * kp < kr ? a_base : kInvalidOff;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f2_t v = __builtin_bit_cast(
            f2_t, __builtin_amdgcn_raw_buffer_load_b64(sa, j < a_rows ? av : kInvalidOff, j * a_step, 0));
        ra[2 * j] = v.x;
        ra[2 * j + 1] = v.y;
      }
    } else {
      const int av = ak1 < kr ? a_base : kInvalidOff;
#pragma unroll
      for (int j = 0; j < 8; ++j) ra[j] = load_f32(sa, j < a_rows ? av : kInvalidOff, j * a_step);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) rb[e] = load_f32(sb, bk0 + e < kr ? b_base : kInvalidOff, e * b_step);
  };
  auto lstore = [&](int buf, int64_t) {
    if constexpr (PAIR) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        __bf16 h0, l0, h1, l1;
        split(ra[2 * j], h0, l0);
        split(ra[2 * j + 1], h1, l1);
        *(bf2_t*)&sm.a_hi[buf][ar + 16 * j][2 * kp] = bf2_t{h0, h1};
        *(bf2_t*)&sm.a_lo[buf][ar + 16 * j][2 * kp] = bf2_t{l0, l1};
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) split(ra[j], sm.a_hi[buf][ar1 + 8 * j][ak1], sm.a_lo[buf][ar1 + 8 * j][ak1]);
    }
    bf8_t h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 x, y;
      split(rb[e], x, y);
      h[e] = x;
      l[e] = y;
    }
    *(bf8_t*)&sm.b_hi[buf][bn][bk0] = h;
    *(bf8_t*)&sm.b_lo[buf][bn][bk0] = l;
  };
  bf16x3_mma64(sm, gload, lstore, C, ldc, mrem, nrem, K, alpha);
}

// 256 x 256 tiles (launches with many tiles): one workgroup of 4 wavefronts
// per compute unit, each wavefront 128 x 128 outputs (8 x 8 blocks of
// v_mfma_f32_16x16x32_bf16).  Per K step of 32 a wavefront reads 32 KB of
// fragments from LDS for 192 MFMAs, half the LDS bytes per MFMA of the
// 64 x 64 wavefront tile, and the workgroup writes 64 KB of staged operands for
// 4x the MFMAs of a 128 x 128 workgroup tile: the LDS traffic drops from about
// the whole LDS bandwidth at full matrix-core rate to about half of it.  Every
// output accumulates the same three MFMAs per K step of 32 in the same order
// as the 64 x 64 and 128 x 128 tiles, so all tile shapes agree bit for bit.
// LDS holds 16-byte k groups (8 bf16: one fragment's worth), 4 per row and
// K step, at slot g ^ ((r >> 1) & 3) of their row so that the 8 rows 8
// consecutive lanes read together land in 8 distinct 16-byte slots of a
// 128-byte line; two buffers of 64 KB (A and B, hi and lo planes).
constexpr int ZBM = 256;

struct Bf16x3SmemBig {
  u4_t a[2][2][ZBM * 4];  // [buffer][plane][row * 4 + slot]
  u4_t b[2][2][ZBM * 4];  // [buffer][plane][column * 4 + slot]
};
static_assert(sizeof(Bf16x3SmemBig) == 128 * 1024, "LDS layout of the 256 x 256 tile");

__device__ __forceinline__ int zslot(int r, int g) { return r * 4 + (g ^ ((r >> 1) & 3)); }

// One 256 x 256 output tile of a leaf with split operands (layouts as
// bf16x3_tile_split: S planes row-major, T planes in k-octets) and K a
// multiple of 8.  Operands go from memory to LDS by direct loads
// (buffer_load_dwordx4 ... lds): each instruction moves 64 16-byte groups and
// lane i lands at byte 16 i of its wave's 1 KB LDS chunk, so a chunk is 16
// rows (or columns) x 4 slots and lane i fetches the k group that the swizzle
// puts in its slot; lanes past the tile edge or past K read through an
// out-of-range offset and write zeros.  No registers hold staged data and no
// LDS store instructions are issued.
__device__ __forceinline__ void bf16x3_tile_split256(Bf16x3SmemBig& sm, const __bf16* Ah, const __bf16* Al,
                                                     const __bf16* Bh, const __bf16* Bl, float* C, int lda,
                                                     int ldb, int ldc, int mrem, int nrem, int K, float alpha) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;

  // direct-load lanes: wave w fills chunks 4 w .. 4 w + 3 of each plane;
  // lane i covers row / column 64 w + 16 q + i / 4 of chunk q and the k
  // group g = (i & 3) ^ ((i >> 3) & 3) (the swizzle of that row)
  const int dr = wave * 64 + (lane >> 2);
  const int dg = (lane & 3) ^ ((lane >> 3) & 3);
  const int a_lane = (dr * lda + 8 * dg) * 2;
  const int a_q = uniform_int(16 * lda * 2);
  const int b_lane = (dg * ldb + 8 * dr) * 2;
  bool a_ok[4], b_ok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a_ok[q] = dr + 16 * q < mrem;
    b_ok[q] = dr + 16 * q < nrem;
  }
  typedef __attribute__((address_space(3))) void* lds_ptr;
  // plane p of A (side 0) or B (side 1), chunks of wave `wave`, step k0
  auto dma = [&](int side, int p, int buf, int k0) {
    const bool kv = k0 + 8 * dg < K;
    if (side == 0) {
      const __amdgpu_buffer_rsrc_t r = make_rsrc((p ? Al : Ah) + k0);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)&sm.a[buf][p][(wave * 4 + q) * 64], 16,
                                                 (a_ok[q] && kv) ? a_lane : kInvalidOff, q * a_q, 0, 0);
    } else {
      const __amdgpu_buffer_rsrc_t r = make_rsrc((p ? Bl : Bh) + (int64_t)(k0 >> 3) * ldb);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)&sm.b[buf][p][(wave * 4 + q) * 64], 16,
                                                 (b_ok[q] && kv) ? b_lane : kInvalidOff, q * 256, 0, 0);
    }
  };

  f4_t acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  const int nk = (K + XBK - 1) / XBK;
  // Fragments: A (hi, lo) of all 8 row blocks of the step, B (hi, lo) of the
  // column block in use and of the next one.  One barrier per K step, after
  // the seventh column block: every read of the current buffer is issued
  // before it, and the direct loads of the next step (issued over the first
  // four column blocks) have landed in the other buffer; after it the next
  // step's fragments are read while the last column block's MFMAs run, each A
  // fragment replaced right after its last use.  The loop body has no
  // branches: the last step also loads and reads a step past K (out-of-range
  // loads write zeros; nothing uses those values).
  bf8_t ah[8], al[8], bh[2], bl[2];
  auto frag = [&](const u4_t* plane, int r) { return __builtin_bit_cast(bf8_t, plane[zslot(r, lg)]); };
  auto rd_b = [&](int buf, int j) {
    bh[j & 1] = frag(sm.b[buf][0], wn * 128 + j * 16 + li);
    bl[j & 1] = frag(sm.b[buf][1], wn * 128 + j * 16 + li);
  };
  auto mma = [&](int j) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j & 1], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j & 1], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j & 1], acc[i][j], 0, 0, 0);
    }
  };
  // vmcnt(0) only (expcnt and lgkmcnt at their maxima): the direct loads
  // count as vector-memory loads until their data is in LDS
  constexpr int kWaitVm0 = 0x0F70;
  dma(0, 0, 0, 0);
  dma(0, 1, 0, 0);
  dma(1, 0, 0, 0);
  dma(1, 1, 0, 0);
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ah[i] = frag(sm.a[0][0], wm * 128 + i * 16 + li);
    al[i] = frag(sm.a[0][1], wm * 128 + i * 16 + li);
  }
  rd_b(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1, nxt = cur ^ 1;
    const int k1 = (kt + 1) * XBK;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      if (j < 4) dma(j >> 1, j & 1, nxt, k1);
      rd_b(cur, j + 1);
      mma(j);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    // last column block: once a row block's three MFMAs are issued, its A
    // fragments are replaced by the next step's
    const bf8_t bh7 = bh[1], bl7 = bl[1];
    rd_b(nxt, 0);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      acc[i][7] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh7, acc[i][7], 0, 0, 0);
      acc[i][7] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl7, acc[i][7], 0, 0, 0);
      acc[i][7] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh7, acc[i][7], 0, 0, 0);
      ah[i] = frag(sm.a[nxt][0], wm * 128 + i * 16 + li);
      al[i] = frag(sm.a[nxt][1], wm * 128 + i * 16 + li);
    }
    __builtin_amdgcn_sched_barrier(0);
  }

  const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wm * 128 + i * 16 + 4 * lg + v;
        const int c = wn * 128 + j * 16 + li;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, alpha * acc[i][j][v]), sc,
                                              (r < mrem && c < nrem) ? (r * ldc + c) * 4 : kInvalidOff, 0, 0);
      }
  // the next tile's first loads write buffer 0, which other wavefronts may
  // still be reading (the reads after the last step)
  __syncthreads();
}

// Grouped launch on 256 x 256 tiles of problems with split operands and K a
// multiple of 8 (the launcher gives it only such groups).
__global__ void __launch_bounds__(XNT) __attribute__((amdgpu_waves_per_eu(1, 1)))
gemm_bf16x3_big_kernel(GemmArgs args) {
  const GemmArgs* ap = kernarg_args();
  __shared__ Bf16x3SmemBig sm;
  const int64_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
  for (int64_t t = slot; t < ap->total_tiles; t += G) {
    const TileJob job = decode_tile(ap, t);
    const GemmProb pr = job.probs ? job.probs[job.prob] : ap->single;
    int64_t lda, ldb, ldc;
    const char* abase = slot_ptr(ap, job.slot, pr.a, &lda);
    const char* bbase = slot_ptr(ap, job.slot, pr.b, &ldb);
    float* C = (float*)slot_ptr(ap, job.slot, pr.c, &ldc) + pr.c.off;
    C = uniform_ptr(C + (pr.c.row + job.tm * ZBM) * ldc + pr.c.col + job.tn * ZBM);
    const int64_t mr = job.m - job.tm * ZBM, nr = job.n - job.tn * ZBM;
    const int mrem = uniform_int(mr < ZBM ? (int)mr : ZBM);
    const int nrem = uniform_int(nr < ZBM ? (int)nr : ZBM);
    const __bf16* Ah = uniform_ptr((const __bf16*)abase + pr.a.off + job.tm * ZBM * lda);
    const __bf16* Bh = uniform_ptr((const __bf16*)bbase + pr.b.off + job.tn * ZBM * 8);
    bf16x3_tile_split256(sm, Ah, uniform_ptr(Ah + pr.a.plane), Bh, uniform_ptr(Bh + pr.b.plane), C,
                         uniform_int((int)lda), uniform_int((int)ldb), uniform_int((int)ldc), mrem, nrem,
                         uniform_int((int)job.k), (float)uniform_double(pr.alpha));
  }
}

template <int TM>
__global__ void __launch_bounds__(XNT) __attribute__((amdgpu_waves_per_eu(2, TM == 128 ? 2 : 4)))
gemm_bf16x3_kernel(GemmArgs args) {
  const GemmArgs* ap = kernarg_args();
  using Smem = std::conditional_t<TM == 128, Bf16x3Smem, Bf16x3Smem64>;
  __shared__ Smem sm;
  const int64_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
  for (int64_t t = slot; t < ap->total_tiles; t += G) {
    const TileJob job = decode_tile(ap, t);
    const GemmProb pr = job.probs ? job.probs[job.prob] : ap->single;
    int64_t lda, ldb, ldc;
    const char* abase = slot_ptr(ap, job.slot, pr.a, &lda);
    const char* bbase = slot_ptr(ap, job.slot, pr.b, &ldb);
    float* C = (float*)slot_ptr(ap, job.slot, pr.c, &ldc) + pr.c.off;
    C = uniform_ptr(C + (pr.c.row + job.tm * TM) * ldc + pr.c.col + job.tn * TM);
    const int64_t mr = job.m - job.tm * TM, nr = job.n - job.tn * TM;
    const int mrem = uniform_int(mr < TM ? (int)mr : TM);
    const int nrem = uniform_int(nr < TM ? (int)nr : TM);
    const int ilda = uniform_int((int)lda), ildb = uniform_int((int)ldb), ildc = uniform_int((int)ldc);
    const float alpha = (float)uniform_double(pr.alpha);
    if (uniform_int(pr.a.elt) == ELT_BF16X2) {
      // leaf operands split by the formation kernels (workspace regions, never
      // views): S rows of lda, T k-octets of ldb; offsets in bf16 elements
      const __bf16* Ah = uniform_ptr((const __bf16*)abase + pr.a.off + job.tm * TM * lda);
      const __bf16* Bh = uniform_ptr((const __bf16*)bbase + pr.b.off + job.tn * TM * 8);
      if constexpr (TM == 128)
        bf16x3_tile_split(sm, Ah, uniform_ptr(Ah + pr.a.plane), Bh, uniform_ptr(Bh + pr.b.plane), C, ilda, ildb,
                          ildc, mrem, nrem, job.k, alpha);
      else
        bf16x3_tile_split64(sm, Ah, uniform_ptr(Ah + pr.a.plane), Bh, uniform_ptr(Bh + pr.b.plane), C, ilda,
                            ildb, ildc, mrem, nrem, job.k, alpha);
      continue;
    }
    const float* A = uniform_ptr((const float*)abase + pr.a.off + (pr.a.row + job.tm * TM) * lda + pr.a.col);
    const float* B = uniform_ptr((const float*)bbase + pr.b.off + pr.b.row * ldb + pr.b.col + job.tn * TM);
    // even K and 8-byte aligned rows allow pair loads of A
    const bool pair = ((job.k | ilda) & 1) == 0 && (((uintptr_t)A) & 7) == 0;
    if constexpr (TM == 128) {
      if (pair)
        bf16x3_tile<true>(sm, A, B, C, ilda, ildb, ildc, mrem, nrem, job.k, alpha);
      else
        bf16x3_tile<false>(sm, A, B, C, ilda, ildb, ildc, mrem, nrem, job.k, alpha);
    } else {
      if (pair)
        bf16x3_tile64<true>(sm, A, B, C, ilda, ildb, ildc, mrem, nrem, job.k, alpha);
      else
        bf16x3_tile64<false>(sm, A, B, C, ilda, ildb, ildc, mrem, nrem, job.k, alpha);
    }
  }
}

template <int TM>
static hipError_t launch_bf16x3_tiles(const GemmArgs& a, int num_cus, hipStream_t s) {
  const GemmArgs* pa = &a;
  GemmArgs re;
  if (TM != kTileM) {
    re = a;
    int64_t tiles = 0;
    for (int i = 0; i < re.ngroups; ++i) {
      GemmGroup& g = re.groups[i];
      g.tiles_m = (g.m + TM - 1) / TM;
      g.tiles_n = (g.n + TM - 1) / TM;
      g.tile_start = tiles;
      tiles += g.tiles_m * g.tiles_n * g.count;
    }
    re.total_tiles = tiles;
    pa = &re;
  }
  static std::atomic<int> cached{0};
  int per_cu = cached.load(std::memory_order_relaxed);
  if (!per_cu) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_bf16x3_kernel<TM>, XNT, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cached.store(per_cu, std::memory_order_relaxed);
  }
  const int64_t G = leaf_grid((int64_t)per_cu * num_cus, pa->total_tiles);
  hipLaunchKernelGGL(gemm_bf16x3_kernel<TM>, dim3((unsigned)G), dim3(XNT), 0, s, *pa);
  return hipGetLastError();
}

// Re-counts the flat tile space of `a` for TM x TM tiles.
static GemmArgs retile(const GemmArgs& a, int tm) {
  GemmArgs re = a;
  int64_t tiles = 0;
  for (int i = 0; i < re.ngroups; ++i) {
    GemmGroup& g = re.groups[i];
    g.tiles_m = (g.m + tm - 1) / tm;
    g.tiles_n = (g.n + tm - 1) / tm;
    g.tile_start = tiles;
    tiles += g.tiles_m * g.tiles_n * g.count;
  }
  re.total_tiles = tiles;
  return re;
}

static hipError_t launch_bf16x3_big(const GemmArgs& a, int num_cus, hipStream_t s) {
  const GemmArgs re = retile(a, ZBM);
  static std::atomic<int> cached{0};
  int per_cu = cached.load(std::memory_order_relaxed);
  if (!per_cu) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_bf16x3_big_kernel, XNT, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cached.store(per_cu, std::memory_order_relaxed);
  }
  const int64_t G = leaf_grid((int64_t)per_cu * num_cus, re.total_tiles);
  hipLaunchKernelGGL(gemm_bf16x3_big_kernel, dim3((unsigned)G), dim3(XNT), 0, s, re);
  return hipGetLastError();
}

// Groups the 256 x 256 kernel takes: split operands and K a multiple of 8
// (whole k-octets, which its direct loads need: a partial octet's padding
// would have to be zeroed in registers).
static bool big_group(const GemmGroup& g) { return g.split && g.k % 8 == 0; }

// Number of 256 x 256 tiles of the groups the big kernel takes.
static int64_t split_tiles256(const GemmArgs& a) {
  int64_t t = 0;
  for (int i = 0; i < a.ngroups; ++i) {
    const GemmGroup& g = a.groups[i];
    if (big_group(g)) t += ((g.m + ZBM - 1) / ZBM) * ((g.n + ZBM - 1) / ZBM) * g.count;
  }
  return t;
}

// The groups of `a` the big kernel takes (big) or not, tile counts for 128 x 128.
static GemmArgs select_groups(const GemmArgs& a, bool big) {
  GemmArgs re = a;
  re.ngroups = 0;
  for (int i = 0; i < a.ngroups; ++i)
    if (big_group(a.groups[i]) == big) re.groups[re.ngroups++] = a.groups[i];
  return retile(re, XBM);
}

// Tile edge: an explicit 64, 128 or 256 wins (256 for split-operand groups
// only); otherwise the split-operand groups run 256 x 256 tiles when they
// have at least two per compute unit, and the rest (or everything) 64 x 64
// tiles when the launch has fewer 128 x 128 tiles than compute units
// (use_small_tiles), else 128 x 128.  The big tiles take a launch of their
// own, so a plan with peel strips then makes two launches.
hipError_t launch_gemm_bf16x3(const GemmArgs& a, int num_cus, hipStream_t s) {
  if (a.total_tiles <= 0) return hipSuccess;
  const int64_t big = split_tiles256(a);
  if (big > 0 && (a.tile == 256 || (a.tile == 0 && big >= 2 * (int64_t)num_cus))) {
    hipError_t e = launch_bf16x3_big(select_groups(a, true), num_cus, s);
    if (e != hipSuccess) return e;
    const GemmArgs rest = select_groups(a, false);
    if (rest.total_tiles <= 0) return hipSuccess;
    const bool small = use_small_tiles(rest.total_tiles, num_cus, kTilesBf16x3);
    return small ? launch_bf16x3_tiles<64>(rest, num_cus, s) : launch_bf16x3_tiles<128>(rest, num_cus, s);
  }
  const bool small = a.tile == 64 || (a.tile != 128 && use_small_tiles(a.total_tiles, num_cus, kTilesBf16x3));
  return small ? launch_bf16x3_tiles<64>(a, num_cus, s) : launch_bf16x3_tiles<128>(a, num_cus, s);
}

}  // namespace fmm
