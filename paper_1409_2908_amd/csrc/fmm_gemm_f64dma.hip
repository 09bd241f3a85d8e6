// FP64 leaf GEMM on 128 x 128 tiles with operands staged by direct
// global-to-LDS loads.
//
// Same grouped, persistent launch as gemm_kernel (fmm_gemm.hip): every
// problem's 128 x 128 output tiles form one flat index space walked with a
// static stride, XCD-aware.  The difference is the staging: each K step of 16
// moves the A tile (128 rows x 16 k) and the B tile (16 k x 128 columns)
// from memory to LDS with buffer_load_dwordx4 ... lds, which writes the 16
// bytes of lane i of a wavefront at byte 16 i of the instruction's 1 KB LDS
// chunk.  No registers hold staged data and no LDS store instructions are
// issued: between barriers the wavefronts issue only the direct loads,
// fragment reads and MFMAs.
//
// Layouts.  A: row r of the tile holds its 16 k as 8 slots of one k pair
// (16 bytes); k pair p sits in slot p ^ ((r >> 1) & 7), so a chunk is 8 rows
// x 8 slots and lane i fetches the k pair that the swizzle puts in its slot.
// B: k row kk holds its 128 columns contiguously (1 KB, one chunk, lane i =
// columns 2i and 2i + 1) at kk * 144 doubles.  Fragment reads: lane (li, g)
// of a wavefront supplies k = 4 kk + g to MFMA kk (the bijection every FP64
// kernel of this library uses); its A read (row li, k pair 2 kk + g / 2,
// half g % 2) and its B read (k row 4 kk + g, column li) then touch 64
// distinct 4-byte banks across each half-wavefront.
//
// Requirements (checked on the host, leaf_dma_ok): every problem's A and B
// rows start 16-byte aligned with even leading dimensions, and every group
// has even K and N, so a k pair or column pair never straddles the end of a
// row.  Rows past M, column pairs past N and k pairs past K read through an
// out-of-range offset and land as zeros.
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "fmm_device.h"
#include "fmm_gemm_common.h"
#include "fmm_launch.h"

namespace fmm {

namespace {

constexpr int QBM = 128, QBK = 16, QBS = 144;  // tile edge, k per step, B row stride (doubles)

struct F64DmaSmem {
  double a[2][QBM * QBK];  // [buffer][row * 16 + 2 * slot + half]
  double b[2][QBK * QBS];  // [buffer][k * 144 + column]
};
static_assert(sizeof(F64DmaSmem) == 69632, "LDS layout of the direct-load FP64 tile");

__device__ __forceinline__ int aslot(int r, int p) { return r * QBK + 2 * (p ^ ((r >> 1) & 7)); }

// One 128 x 128 output tile: C = alpha * A B over K, A / B / C at the tile's
// origin.
__device__ __forceinline__ void f64_tile_dma(F64DmaSmem& sm, const double* A, const double* B, double* C,
                                             int lda, int ldb, int ldc, int mrem, int nrem, int K,
                                             double alpha) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;
  typedef __attribute__((address_space(3))) void* lds_ptr;

  // A: wavefront w fills rows 32 w .. 32 w + 31, chunk q = rows 32 w + 8 q ..
  // + 7; lane i covers row 32 w + 8 q + i / 8 and the k pair of slot i % 8
  int a_off[4], a_p[4];
  bool a_ok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 32 * wave + 8 * q + (lane >> 3);
    a_p[q] = (lane & 7) ^ ((r >> 1) & 7);
    a_off[q] = (r * lda + 2 * a_p[q]) * 8;
    a_ok[q] = r < mrem;
  }
  // B: wavefront w fills k rows 4 w .. 4 w + 3; lane i covers columns 2i, 2i + 1
  const int b_off = 16 * lane;
  const bool b_ok = 2 * lane < nrem;
  // a step wholly inside K needs only the row / column checks, folded into
  // the offsets once (`checked` false); the tail step and the steps past K
  // that the pipeline loads check every k pair and k row
  int a_offv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) a_offv[q] = a_ok[q] ? a_off[q] : kInvalidOff;
  const int b_offv = b_ok ? b_off : kInvalidOff;
  auto dma = [&](int buf, int k0, auto checked) {
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + k0);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(B + (int64_t)k0 * ldb);
    if constexpr (!decltype(checked)::value) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)&sm.a[buf][(32 * wave + 8 * q) * QBK], 16, a_offv[q], 0,
                                                 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 4 * wave + q;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)&sm.b[buf][kk * QBS], 16, b_offv, kk * ldb * 8, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)&sm.a[buf][(32 * wave + 8 * q) * QBK], 16,
                                                 (a_ok[q] && k0 + 2 * a_p[q] < K) ? a_off[q] : kInvalidOff, 0, 0,
                                                 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 4 * wave + q;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)&sm.b[buf][kk * QBS], 16,
                                                 (b_ok && k0 + kk < K) ? b_off : kInvalidOff, kk * ldb * 8, 0, 0);
      }
    }
  };

  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0, 0, 0, 0};

  // vmcnt(0) only (expcnt and lgkmcnt at their maxima): the direct loads
  // count as vector-memory loads until their data is in LDS
  constexpr int kWaitVm0 = 0x0F70;
  const int nk = (K + QBK - 1) / QBK;
  // Fragments are read one sub-step ahead of their MFMAs (two register
  // sets), and the barrier sits between the third and the fourth sub-step:
  // every read of the current buffer is issued before it, and the direct
  // loads of the step after next go out right after it into the buffer just
  // released, so they have a whole step of MFMAs to land in.  The next
  // step's first fragments are read while the fourth sub-step's MFMAs run.
  // Scheduling fences keep the compiler from sinking a fragment read down to
  // its MFMAs (which would expose the LDS latency) or the loads below them.
  // The last two steps load steps past K, which write zeros nothing reads.
  double af[2][4], bf[2][4];
  auto rd = [&](int buf, int kk) {
    const int p = 2 * kk + (lg >> 1), h = lg & 1, s = kk & 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) af[s][i] = sm.a[buf][aslot(wm * 64 + i * 16 + li, p) + h];
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[s][j] = sm.b[buf][(kk * 4 + lg) * QBS + wn * 64 + j * 16 + li];
  };
  // The first three sub-steps issue their MFMAs at raised wavefront
  // priority, so of the two wavefronts sharing a SIMD the one in its MFMA
  // burst keeps the pipe while the other issues its reads (0.4% on the
  // 16384^3 leaves); the fourth, whose MFMAs carry the interleaved direct
  // loads, stays at the base priority.
  auto mma = [&](int kk) {
    const int s = kk & 1;
    if (kk < 3) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s][i], bf[s][j], acc[i][j], 0, 0, 0);
    if (kk < 3) __builtin_amdgcn_s_setprio(0);
  };
  auto fence = [] { __builtin_amdgcn_sched_barrier(0); };
  constexpr std::true_type kChecked{};
  constexpr std::false_type kPlain{};
  dma(0, 0, kChecked);
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  dma(1, QBK, kChecked);
  rd(0, 0);
  auto step = [&](int kt, auto checked) {
    const int cur = kt & 1;
    rd(cur, 1);
    fence();
    mma(0);
    fence();
    rd(cur, 2);
    fence();
    mma(1);
    fence();
    rd(cur, 3);
    fence();
    mma(2);
    fence();
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    rd(cur ^ 1, 0);
    fence();
    dma(cur, (kt + 2) * QBK, checked);
    mma(3);
    if constexpr (!decltype(checked)::value) {
      // one direct load between every two MFMAs of the last sub-step, so
      // the loads leave in a steady stream instead of one burst per step
#pragma unroll
      for (int g = 0; g < 8; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // a VMEM read
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // two MFMAs
      }
    }
    fence();
  };
  // the steps whose loads (two steps ahead) lie wholly inside K run a loop
  // body without branches, which the interleaving needs
  const int nplain = K / QBK - 2 > 0 ? K / QBK - 2 : 0;
  int kt = 0;
  for (; kt < nplain; ++kt) step(kt, kPlain);
  for (; kt < nk; ++kt) step(kt, kChecked);
  // the loads past K have landed before the next tile's first loads reuse
  // the buffers
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();

  const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // 16x16 f64 block: register v of lane l holds row l / 16 + 4 v, column l % 16
        const int r = wm * 64 + i * 16 + lg + 4 * v;
        const int c = wn * 64 + j * 16 + li;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, alpha * acc[i][j][v]), sc,
                                              (r < mrem && c < nrem) ? (r * ldc + c) * 8 : kInvalidOff, 0, 0);
      }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm_f64_dma_kernel(GemmArgs args) {
  const GemmArgs* ap = kernarg_args();
  __shared__ F64DmaSmem sm;
  const int64_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
  for (int64_t t = slot; t < ap->total_tiles; t += G) {
    const TileJob job = decode_tile(ap, t);
    const GemmProb pr = job.probs ? job.probs[job.prob] : ap->single;
    int64_t lda, ldb, ldc;
    const double* A = (const double*)slot_ptr(ap, job.slot, pr.a, &lda) + pr.a.off;
    const double* B = (const double*)slot_ptr(ap, job.slot, pr.b, &ldb) + pr.b.off;
    double* C = (double*)slot_ptr(ap, job.slot, pr.c, &ldc) + pr.c.off;
    A = uniform_ptr(A + (pr.a.row + job.tm * QBM) * lda + pr.a.col);
    B = uniform_ptr(B + pr.b.row * ldb + pr.b.col + job.tn * QBM);
    C = uniform_ptr(C + (pr.c.row + job.tm * QBM) * ldc + pr.c.col + job.tn * QBM);
    const int64_t mr = job.m - job.tm * QBM, nr = job.n - job.tn * QBM;
    f64_tile_dma(sm, A, B, C, uniform_int((int)lda), uniform_int((int)ldb), uniform_int((int)ldc),
                 uniform_int(mr < QBM ? (int)mr : QBM), uniform_int(nr < QBM ? (int)nr : QBM),
                 uniform_int((int)job.k), uniform_double(pr.alpha));
  }
}

}  // namespace

hipError_t launch_gemm_f64_dma(const GemmArgs& a, int num_cus, hipStream_t s) {
  static std::atomic<int> cached{0};
  int per_cu = cached.load(std::memory_order_relaxed);
  if (!per_cu) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_f64_dma_kernel, 256, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cached.store(per_cu, std::memory_order_relaxed);
  }
  // the planner counts 128 x 128 tiles (kTileM), this kernel's tile
  const int64_t G = leaf_grid((int64_t)per_cu * num_cus, a.total_tiles);
  hipLaunchKernelGGL(gemm_f64_dma_kernel, dim3((unsigned)G), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fmm
