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
// Tile: 128 x 128 per workgroup of 8 wavefronts (4 x 2), 32 x 64 per
// wavefront = 2 x 4 MFMA 16x16x4 blocks (64 FP64 accumulator values per lane,
// so two wavefronts fit each SIMD without spilling).  K advances 16 at a time through a
// double-buffered LDS stage: global loads for step k+1 are issued before the
// MFMAs of step k, stored to the other LDS buffer after them, one barrier per
// step.  Within a K step lane group g of a wavefront supplies k = 4g + kk for
// MFMA kk (any bijection of k works when A and B use the same one), so each
// lane reads its A fragment from one LDS row.
//
// Order: consecutive workgroup ids are dispatched round-robin over the 8 XCDs,
// each with its own L2; workgroup b is given flat slot (b mod 8) * (G/8) + b/8
// so the tiles running at once on one XCD are neighbours in a grouped raster
// (8 tile rows per group) and share A and B panels in that XCD's L2.
#include <hip/hip_runtime.h>

#include "fmm_device.h"
#include "fmm_launch.h"

namespace fmm {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int GBM = 128, GBN = 128, GBK = 16, GNT = 512;

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  using acc_t = d4_t;
  static constexpr int APAD = 1, BPAD = 4;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row of register v in lane l (16x16 block; column is l % 16)
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
  using acc_t = f4_t;
  static constexpr int APAD = 1, BPAD = 4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

struct TileJob {
  int64_t m, n, k, tm, tn, prob;
};

__device__ __forceinline__ TileJob decode_tile(const GemmArgs& args, int64_t t) {
  int64_t gm = 0, gn = 0, gk = 0, tiles_m = 1, tiles_n = 1, tstart = 0, pstart = 0;
#pragma unroll
  for (int i = 0; i < kMaxGemmGroups; ++i) {
    if (i < args.ngroups && t >= args.groups[i].tile_start) {
      gm = args.groups[i].m;
      gn = args.groups[i].n;
      gk = args.groups[i].k;
      tiles_m = args.groups[i].tiles_m;
      tiles_n = args.groups[i].tiles_n;
      tstart = args.groups[i].tile_start;
      pstart = args.groups[i].prob_start;
    }
  }
  const int64_t lt = t - tstart;
  const int64_t tpp = tiles_m * tiles_n;
  const int64_t pi = lt / tpp;
  const int64_t tt = lt - pi * tpp;
  const int64_t gsz = 8 * tiles_n;
  const int64_t grp = tt / gsz;
  const int64_t first = grp * 8;
  const int64_t rows = tiles_m - first < 8 ? tiles_m - first : 8;
  const int64_t rin = tt - grp * gsz;
  TileJob j;
  j.m = gm;
  j.n = gn;
  j.k = gk;
  j.tm = first + rin % rows;
  j.tn = rin / rows;
  j.prob = pstart + pi;
  return j;
}

template <typename T>
__global__ void __launch_bounds__(GNT) gemm_kernel(GemmArgs args) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc_t;
  __shared__ T As[2][GBM][GBK + MF::APAD];
  __shared__ T Bs[2][GBK][GBN + MF::BPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // 4 x 2 wavefronts
  const int li = lane & 15, lg = lane >> 4;
  const int64_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;

  for (int64_t t = slot; t < args.total_tiles; t += G) {
    const TileJob job = decode_tile(args, t);
    const GemmProb pr = args.probs ? args.probs[job.prob] : args.single;
    int64_t lda, ldb, ldc;
    const T* A = (const T*)buf_ptr(args.bases, pr.a, &lda) + pr.a.off;
    const T* B = (const T*)buf_ptr(args.bases, pr.b, &ldb) + pr.b.off;
    T* C = (T*)buf_ptr(args.bases, pr.c, &ldc) + pr.c.off;
    A += (pr.a.row + job.tm * GBM) * lda + pr.a.col;
    B += pr.b.row * ldb + pr.b.col + job.tn * GBN;
    C += (pr.c.row + job.tm * GBM) * ldc + pr.c.col + job.tn * GBN;
    const int64_t mrem = job.m - job.tm * GBM;
    const int64_t nrem = job.n - job.tn * GBN;
    const int64_t K = job.k;

    acc_t acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // Each thread moves 4 elements of the A tile and 4 of the B tile per K
    // step; 16 (A) or 128 (B) consecutive threads cover one contiguous row.
    T ra[4], rb[4];
    const int ar = tid >> 4, ac = tid & 15, br = tid >> 7, bc = tid & 127;
    auto gload = [&](int64_t k0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = ar + 32 * j;
        ra[j] = (r < mrem && k0 + ac < K) ? A[r * lda + k0 + ac] : T(0);
        const int kr = br + 4 * j;
        rb[j] = (k0 + kr < K && bc < nrem) ? B[(k0 + kr) * ldb + bc] : T(0);
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        As[buf][ar + 32 * j][ac] = ra[j];
        Bs[buf][br + 4 * j][bc] = rb[j];
      }
    };

    const int64_t nk = (K + GBK - 1) / GBK;
    if (nk > 0) {
      gload(0);
      lstore(0);
    }
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int cur = (int)(kt & 1);
      if (kt + 1 < nk) gload((kt + 1) * GBK);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        T af[2], bf[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = As[cur][wm * 32 + i * 16 + li][lg * 4 + kk];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][lg * 4 + kk][wn * 64 + j * 16 + li];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = MF::op(af[i], bf[j], acc[i][j]);
      }
      if (kt + 1 < nk) lstore(cur ^ 1);
      __syncthreads();
    }

    const T alpha = (T)pr.alpha;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = wm * 32 + i * 16 + MF::row(lane, v);
          const int c = wn * 64 + j * 16 + li;
          if (r < mrem && c < nrem) C[r * ldc + c] = alpha * acc[i][j][v];
        }
  }
}

template <typename T>
static int blocks_per_cu() {
  static int cached = 0;
  if (!cached) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, gemm_kernel<T>, GNT, 0) != hipSuccess || b < 1) b = 1;
    cached = b;
  }
  return cached;
}

hipError_t launch_gemm(const GemmArgs& a, int dtype, int num_cus, hipStream_t s) {
  if (a.total_tiles <= 0) return hipSuccess;
  const int per_cu = dtype == 0 ? blocks_per_cu<double>() : blocks_per_cu<float>();
  int64_t G = (int64_t)per_cu * num_cus;
  const int64_t want = (a.total_tiles + 7) / 8 * 8;
  if (want < G) G = want;
  if (G < 8) G = 8;
  G = G / 8 * 8;
  if (dtype == 0) {
    hipLaunchKernelGGL((gemm_kernel<double>), dim3((unsigned)G), dim3(GNT), 0, s, a);
  } else if (dtype == 1) {
    hipLaunchKernelGGL((gemm_kernel<float>), dim3((unsigned)G), dim3(GNT), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fmm
