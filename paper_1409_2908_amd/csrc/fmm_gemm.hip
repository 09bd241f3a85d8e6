// Grouped, persistent leaf GEMM on the CDNA4 matrix cores.
//
// One launch multiplies every leaf product M_rho = alpha_rho S_rho T_rho of a
// plan (Section 3.1, second bullet; all R^L leaves at once, the breadth-first
// layout of Section 4.2) together with the classical peel problems
// (Section 3.5).  All problems' 128 x 128 output tiles form one flat index
// space; a grid of about two workgroups per compute unit walks it with a
// static stride, so there is no per-problem launch and no load imbalance
// beyond one tile.
//
// Tile: 128 x 128 per workgroup of 4 wavefronts (2 x 2), 64 x 64 per
// wavefront = 4 x 4 MFMA 16x16x4 blocks.  Two workgroups share each compute
// unit (so each SIMD runs two wavefronts of different workgroups, whose
// barriers do not line up and keep the matrix pipe fed).  K advances 16 at a
// time through a double-buffered LDS stage: global loads for step k+1 are
// issued before the MFMAs of step k and stored to the other LDS buffer before
// its last quarter of MFMAs, one barrier per step.  Within a K step lane group g of a wavefront
// supplies k = 4g + kk (FP32) or k = 4kk + g (FP64) for MFMA kk (any bijection
// of k works when A and B use the same one), so each lane reads its A
// fragment from one LDS row.  Every FP64 kernel (all tile edges, and the
// direct-load kernel in fmm_gemm_f64dma.hip) takes the FP64 bijection, so
// they accumulate the same products in the same order.
//
// Operands are read and C is written with raw buffer instructions: a
// per-step 128-bit resource in scalar registers plus one 32-bit byte offset
// per element, so a lane needs no 64-bit address.  Out-of-range elements
// (tile edges, the K tail) get an offset past the resource's size: the
// hardware returns 0 for such loads and drops such stores, so edges need no
// branches.  This bounds each operand row offset: ld * 128 * 8 bytes must
// stay below 2^31 (the host rejects larger leading dimensions).
//
// Order: consecutive workgroup ids are dispatched round-robin over the 8 XCDs,
// each with its own L2; workgroup b is given flat slot (b mod 8) * (G/8) + b/8
// so the tiles running at once on one XCD are neighbours in a grouped raster
// (8 tile rows per group) and share A and B panels in that XCD's L2.
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "fmm_device.h"
#include "fmm_gemm_common.h"
#include "fmm_launch.h"

namespace fmm {

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  using acc_t = d4_t;
  // B rows of BN + 16 doubles: the four k rows one fragment read touches
  // (adjacent k, see the K loop) start 128 bytes apart in the LDS banks
  static constexpr int APAD = 1, BPAD = 16;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row of register v in lane l (16x16 block; column is l % 16)
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
  }
  static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, int off, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, x), r, off, 0, 0);
  }
};

template <>
struct Mfma<float> {
  using acc_t = f4_t;
  static constexpr int APAD = 1, BPAD = 4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
  }
  static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, int off, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
  }
};


// BM x BN output tile per workgroup of 4 wavefronts (2 x 2): 128 x 128 (the
// large-problem shape, two workgroups per CU), 64 x 64 (for launches with
// fewer large tiles than compute units, where four times as many tiles keep
// more of the chip busy) or 32 x 32 (launches with at most half as many 64 x
// 64 tiles as units).
//
// NT > 0 (plans with leaf-side formation): every problem's A and B tiles are
// formed while they are staged, as sum_t coef_t * X_t over up to NT blocks
// X_t of the operand (LeafTerms; views and peel strips have one term of
// coefficient 1).  The loads of all terms are issued with the step's other
// loads; the sums are taken in lstore, once they have landed, in the order
// and precision of the formation pass (FP64, ascending block index, the first
// term initialising, one rounding per add or subtract; then one rounding to
// T), so the staged values, and the products, equal those of a plan that
// writes S and T first, bit for bit.
template <typename T, int BM, int BN, int NT>
__global__ void __launch_bounds__(GNT) __attribute__((amdgpu_waves_per_eu(2, BM == 128 ? 2 : 8)))
gemm_kernel(GemmArgs args) {
  const GemmArgs* ap = kernarg_args();
  using MF = Mfma<T>;
  using acc_t = typename MF::acc_t;
  constexpr int ES = (int)sizeof(T);
  constexpr int WTM = BM / 2, WTN = BN / 2, TI = WTM / 16, TJ = WTN / 16;
  constexpr int EA = BM * GBK / GNT, EB = GBK * BN / GNT;  // elements per thread: 8 and 8 (128 x 128)
  constexpr int RA = GNT / GBK, RB = GNT / BN;               // rows per load step: 16 and 2 (128 x 128)
  constexpr int KPL = GBK / 4;                               // k per lane group per step
  __shared__ T As[2][BM][GBK + MF::APAD];
  __shared__ T Bs[2][GBK][BN + MF::BPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;
  const int ar = tid / GBK, ac = tid % GBK, br = tid / BN, bc = tid % BN;
  const int64_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;

  for (int64_t t = slot; t < ap->total_tiles; t += G) {
    const TileJob job = decode_tile(ap, t);
    const GemmProb pr = job.probs ? job.probs[job.prob] : ap->single;
    int64_t lda, ldb, ldc;
    const T* A = (const T*)slot_ptr(ap, job.slot, pr.a, &lda) + pr.a.off;
    const T* B = (const T*)slot_ptr(ap, job.slot, pr.b, &ldb) + pr.b.off;
    T* C = (T*)slot_ptr(ap, job.slot, pr.c, &ldc) + pr.c.off;
    // Everything below is the same for the whole workgroup; saying so keeps
    // the buffer resources in scalar registers.
    const T* A0 = A;
    const T* B0 = B;
    A = uniform_ptr(A + (pr.a.row + job.tm * BM) * lda + pr.a.col);
    B = uniform_ptr(B + pr.b.row * ldb + pr.b.col + job.tn * BN);
    C = uniform_ptr(C + (pr.c.row + job.tm * BM) * ldc + pr.c.col + job.tn * BN);
    // formed operands: the tile's origin in each term's block, and its coefficient
    const T* At[NT > 0 ? NT : 1];
    const T* Bt[NT > 0 ? NT : 1];
    int ca[NT > 0 ? NT : 1], cb[NT > 0 ? NT : 1];
    if constexpr (NT > 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        ca[t] = uniform_int(pr.fa.coef[t]);
        cb[t] = uniform_int(pr.fb.coef[t]);
        At[t] = uniform_ptr(A0 + (pr.a.row + pr.fa.drow[t] + job.tm * BM) * lda + pr.a.col + pr.fa.dcol[t]);
        Bt[t] = uniform_ptr(B0 + (pr.b.row + pr.fb.drow[t]) * ldb + pr.b.col + pr.fb.dcol[t] + job.tn * BN);
      }
    }
    const int64_t mr = job.m - job.tm * BM, nr = job.n - job.tn * BN;
    const int mrem = uniform_int(mr < BM ? (int)mr : BM);
    const int nrem = uniform_int(nr < BN ? (int)nr : BN);
    const int64_t K = job.k;
    const int ilda = uniform_int((int)lda), ildb = uniform_int((int)ldb), ildc = uniform_int((int)ldc);
    const T alpha = (T)uniform_double(pr.alpha);

    // One byte offset per operand and lane; the EA (EB) rows a lane loads are
    // RA (RB) rows apart, a stride passed as the scalar offset.  Lanes past the
    // tile's last row or column (or past K) load through kInvalidOff and read 0.
    const int a_base = (ar * ilda + ac) * ES;
    const int a_rows = (mrem - ar + RA - 1) / RA;  // valid rows of this lane
    const int b_base = bc < nrem ? (br * ildb + bc) * ES : kInvalidOff;
    const int a_step = uniform_int(RA * ilda * ES), b_step = uniform_int(RB * ildb * ES);

    acc_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    constexpr int NTL = NT > 0 ? NT : 1;  // loads per staged element
    T ra[NTL][EA], rb[NTL][EB];
    auto gload = [&](int64_t k0) {
      // One branch-free path for full and partial K steps: a branch here would
      // merge the loaded registers and force a wait for the loads to land.
      const int kr = K - k0 < GBK ? (int)(K - k0) : GBK;
      const int av = ac < kr ? a_base : kInvalidOff;
      const int b_rows = (kr - br + RB - 1) / RB;
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        // unused term slots (coefficient 0) read through the invalid offset
        const T* a_src = NT > 0 ? At[t] : A;
        const T* b_src = NT > 0 ? Bt[t] : B;
        const bool a_on = NT == 0 || ca[t] != 0, b_on = NT == 0 || cb[t] != 0;
        const __amdgpu_buffer_rsrc_t sa = make_rsrc(a_src + k0);
        const __amdgpu_buffer_rsrc_t sb = make_rsrc(b_src + k0 * (int64_t)ildb);
#pragma unroll
        for (int j = 0; j < EA; ++j) ra[t][j] = MF::load(sa, a_on && j < a_rows ? av : kInvalidOff, j * a_step);
#pragma unroll
        for (int j = 0; j < EB; ++j)
          rb[t][j] = MF::load(sb, b_on && j < b_rows ? b_base : kInvalidOff, j * b_step);
      }
    };
    // sum_t c[t] * x[t] in FP64, ascending t, the first non-zero term
    // initialising (c * x is exact for c = +-1, and a fused multiply-add then
    // rounds exactly like the add or subtract of the formation pass)
    auto chain = [&](const double* v, const int* c) -> T {
      double acc = 0.0;
      bool first = true;
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        if (c[t] == 0) continue;
        acc = first ? (double)c[t] * v[t] : __fma_rn((double)c[t], v[t], acc);
        first = false;
      }
      return (T)acc;
    };
    auto form_a = [&](int j) -> T {
      double v[NTL];
#pragma unroll
      for (int t = 0; t < NTL; ++t) v[t] = (double)ra[t][j];
      return chain(v, ca);
    };
    auto form_b = [&](int j) -> T {
      double v[NTL];
#pragma unroll
      for (int t = 0; t < NTL; ++t) v[t] = (double)rb[t][j];
      return chain(v, cb);
    };
    auto lstore = [&](int buf) {
      if constexpr (NT == 0) {
#pragma unroll
        for (int j = 0; j < EA; ++j) As[buf][ar + RA * j][ac] = ra[0][j];
#pragma unroll
        for (int j = 0; j < EB; ++j) Bs[buf][br + RB * j][bc] = rb[0][j];
      } else {
#pragma unroll
        for (int j = 0; j < EA; ++j) As[buf][ar + RA * j][ac] = form_a(j);
#pragma unroll
        for (int j = 0; j < EB; ++j) Bs[buf][br + RB * j][bc] = form_b(j);
      }
    };

    const int64_t nk = (K + GBK - 1) / GBK;
    if constexpr (std::is_same_v<T, float>) {
      // FP32: fragment registers for the four sub-steps of a K step, and the
      // barrier between the MFMAs of sub-steps 2 and 3.  Every read of the
      // current buffer is issued before it and the next buffer has been
      // written before it; after it the next step's first fragments are read
      // while sub-step 3's MFMAs run.  (Measured +5% over the schedule below
      // for FP32, -2% for FP64, whose longer MFMAs already hide the reads.)
      T af[KPL][TI], bf[KPL][TJ];
      auto rd = [&](int buf, int kk) {
#pragma unroll
        for (int i = 0; i < TI; ++i) af[kk][i] = As[buf][wm * WTM + i * 16 + li][lg * KPL + kk];
#pragma unroll
        for (int j = 0; j < TJ; ++j) bf[kk][j] = Bs[buf][lg * KPL + kk][wn * WTN + j * 16 + li];
      };
      auto mma = [&](int kk) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) acc[i][j] = MF::op(af[kk][i], bf[kk][j], acc[i][j]);
      };
      if (nk > 0) {
        gload(0);
        lstore(0);
      }
      __syncthreads();
      if (nk > 0) rd(0, 0);
      for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) gload((kt + 1) * GBK);
        rd(cur, 1);
        mma(0);
        rd(cur, 2);
        rd(cur, 3);
        mma(1);
        if (more) lstore(cur ^ 1);
        mma(2);
        __syncthreads();
        if (more) rd(cur ^ 1, 0);
        mma(3);
      }
    } else {
      if (nk > 0) {
        gload(0);
        lstore(0);
      }
      __syncthreads();
      for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload((kt + 1) * GBK);
#pragma unroll
        for (int kk = 0; kk < KPL; ++kk) {
          T af[TI], bf[TJ];
#pragma unroll
          for (int i = 0; i < TI; ++i) af[i] = As[cur][wm * WTM + i * 16 + li][kk * 4 + lg];
#pragma unroll
          for (int j = 0; j < TJ; ++j) bf[j] = Bs[cur][kk * 4 + lg][wn * WTN + j * 16 + li];
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = MF::op(af[i], bf[j], acc[i][j]);
          // The other buffer's readers all passed the previous barrier, so the
          // next step's tile can be written now; doing it before the last
          // sub-step hides the LDS writes behind its MFMAs (the loads issued at
          // the top of the step have had three sub-steps to land).
          if (kk == KPL - 2 && kt + 1 < nk) lstore(cur ^ 1);
        }
        __syncthreads();
      }
    }

    const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = wm * WTM + i * 16 + MF::row(lane, v);
          const int c = wn * WTN + j * 16 + li;
          MF::store(sc, (r < mrem && c < nrem) ? (r * ildc + c) * ES : kInvalidOff, alpha * acc[i][j][v]);
        }
  }
}

// Persistent grids: as many workgroups as fit at once (each walks tiles with
// a stride), or one per tile when there are fewer tiles.  (One workgroup per
// tile throughout measured the same for the FP64 leaves and 7% slower for the
// 256 x 256 BF16x3 leaves.)
int64_t leaf_grid(int64_t resident, int64_t tiles) {
  const int64_t want = (tiles + 7) / 8 * 8;
  int64_t G = want < resident ? want : resident;
  if (G < 8) G = 8;
  return G / 8 * 8;
}

template <typename T, int BM, int NT>
static int blocks_per_cu() {
  static std::atomic<int> cached{0};
  int b = cached.load(std::memory_order_relaxed);
  if (!b) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, gemm_kernel<T, BM, BM, NT>, GNT, 0) != hipSuccess ||
        b < 1)
      b = 1;
    cached.store(b, std::memory_order_relaxed);
  }
  return b;
}

// Tile shape of a launch: an explicit 64 or 128 wins; otherwise (0) 64 x 64
// when the 128 x 128 tiles would leave compute units idle (use_small_tiles,
// per the kernel the large tiles would run) and 128 x 128 else.  The planner counts tiles of kTileM x kTileN;
// a launch with another shape re-counts every group's tiles.
static int pick_tile(const GemmArgs& a, int num_cus, int kind) {
  if (a.tile == 64 || a.tile == 128) return a.tile;
  return use_small_tiles(a.total_tiles, num_cus, kind) ? 64 : 128;
}

template <typename T, int BM, int NT>
static hipError_t launch_tiles(const GemmArgs& a, int num_cus, hipStream_t s) {
  const GemmArgs* pa = &a;
  GemmArgs re;
  if (BM != kTileM) {
    re = a;
    int64_t tiles = 0;
    for (int i = 0; i < re.ngroups; ++i) {
      GemmGroup& g = re.groups[i];
      g.tiles_m = (g.m + BM - 1) / BM;
      g.tiles_n = (g.n + BM - 1) / BM;
      g.tile_start = tiles;
      tiles += g.tiles_m * g.tiles_n * g.count;
    }
    re.total_tiles = tiles;
    pa = &re;
  }
  const int64_t G = leaf_grid((int64_t)blocks_per_cu<T, BM, NT>() * num_cus, pa->total_tiles);
  hipLaunchKernelGGL((gemm_kernel<T, BM, BM, NT>), dim3((unsigned)G), dim3(GNT), 0, s, *pa);
  return hipGetLastError();
}

// Launches that form their operands run 64 x 64 tiles (the plans that use
// them have small leaf launches, and the 128 x 128 tile's registers could not
// hold the terms' loads in flight).
// 64 x 64 tiles of a launch.
static int64_t tiles64(const GemmArgs& a) {
  int64_t t = 0;
  for (int i = 0; i < a.ngroups; ++i) t += ((a.groups[i].m + 63) / 64) * ((a.groups[i].n + 63) / 64) * a.groups[i].count;
  return t;
}

// Launches with so few 64 x 64 tiles that most compute units would idle
// (at most half as many as units) run 32 x 32 tiles: a tile's time is then
// bound by its one compute unit's matrix and load rate, and four times as many
// tiles spread the product over four times as many units.  Every tile edge
// accumulates each output element over the same K steps in the same order.
template <typename T, int NT>
static hipError_t launch_typed(const GemmArgs& a, int num_cus, hipStream_t s, int kind) {
  if (a.tile == 0 && 2 * tiles64(a) <= num_cus) return launch_tiles<T, 32, NT>(a, num_cus, s);
  if constexpr (NT > 0) return launch_tiles<T, 64, NT>(a, num_cus, s);
  else
    return pick_tile(a, num_cus, kind) == 64 ? launch_tiles<T, 64, 0>(a, num_cus, s)
                                             : launch_tiles<T, 128, 0>(a, num_cus, s);
}

template <typename T>
static hipError_t launch_forms(const GemmArgs& a, int num_cus, hipStream_t s) {
  // launches on 128 x 128 tiles whose operands allow it stage them by direct
  // loads (fmm_gemm_f64dma.hip, fmm_gemm_f32dma.hip); same products, same
  // order.  The tile rule follows the kernel the large tiles would run.
  const bool dma = a.form_terms == 0 && a.dma;
  const int kind = !dma ? kTilesStaged : std::is_same_v<T, double> ? kTilesF64Dma : kTilesF32Dma;
  if (dma && !(a.tile == 0 && 2 * tiles64(a) <= num_cus) && pick_tile(a, num_cus, kind) == 128)
    return std::is_same_v<T, double> ? launch_gemm_f64_dma(a, num_cus, s) : launch_gemm_f32_dma(a, num_cus, s);
  if (a.form_terms == 0) return launch_typed<T, 0>(a, num_cus, s, kind);
  if (a.form_terms == kMaxLeafTerms) return launch_typed<T, kMaxLeafTerms>(a, num_cus, s, kind);
  return hipErrorInvalidValue;
}

hipError_t launch_gemm(const GemmArgs& a, int dtype, int num_cus, hipStream_t s) {
  if (a.total_tiles <= 0) return hipSuccess;
  if (dtype == 2) return a.form_terms ? hipErrorInvalidValue : launch_gemm_bf16x3(a, num_cus, s);
  if (dtype == 0) return launch_forms<double>(a, num_cus, s);
  if (dtype == 1) return launch_forms<float>(a, num_cus, s);
  return hipErrorInvalidValue;
}

}  // namespace fmm
