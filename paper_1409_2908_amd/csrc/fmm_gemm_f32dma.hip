// FP32 leaf GEMM on 128 x 128 tiles with operands staged by direct
// global-to-LDS loads (the FP32 counterpart of fmm_gemm_f64dma.hip).
//
// Each K step of 16 moves the A tile (128 rows x 16 k) and the B tile (16 k
// x 128 columns) to LDS with buffer_load_dwordx4 ... lds: lane i of a
// wavefront lands its 16 bytes at byte 16 i of the instruction's 1 KB chunk.
//
// Layouts.  A: row r holds its 16 k as 4 slots of one k quad (16 bytes); k
// quad p sits in slot p ^ ((r >> 2) & 3), so a chunk is 16 rows x 4 slots.
// B: a chunk holds k rows 2c and 2c + 1 (128 columns each, 512 bytes), and
// chunk c starts at 1056 c bytes.  Fragment reads follow the FP32 bijection
// every FP32 kernel of this library uses (lane group g supplies k = 4 g + kk
// to MFMA kk, fmm_gemm.hip), so the products and their order, and the bits,
// are those of the other FP32 tile shapes: lane (li, g) reads its four A
// values of a step (row li, k quad g) with one 16-byte read, 16 rows of one
// quad falling on distinct banks, and its B value of MFMA kk from k row
// 4 g + kk, the four rows of one read starting 64 bytes apart in the banks.
//
// Requirements (checked on the host, leaf_dma_ok): every problem's A and B
// rows start 16-byte aligned with leading dimensions a multiple of 4, and
// every group has K and N a multiple of 4, so a k quad or a column quad never
// straddles the end of a row.  Rows past M, column quads past N and k quads
// or k rows past K read through an out-of-range offset and land as zeros.
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "fmm_device.h"
#include "fmm_gemm_common.h"
#include "fmm_launch.h"

namespace fmm {

namespace {

constexpr int SBM = 128, SBK = 16, SBC = 264;  // tile edge, k per step, B chunk stride (floats)

struct F32DmaSmem {
  f4_t a[2][SBM * 4];        // [buffer][row * 4 + slot]: k quads
  float b[2][(SBK / 2) * SBC];  // [buffer][chunk * 264 + (k % 2) * 128 + column]
};
static_assert(sizeof(F32DmaSmem) == 2 * 8192 + 2 * 8 * 264 * 4, "LDS layout of the direct-load FP32 tile");

__device__ __forceinline__ int aquad(int r, int p) { return r * 4 + (p ^ ((r >> 2) & 3)); }
__device__ __forceinline__ int brow(int k) { return (k >> 1) * SBC + (k & 1) * SBM; }

__device__ __forceinline__ void f32_tile_dma(F32DmaSmem& sm, const float* A, const float* B, float* C, int lda,
                                             int ldb, int ldc, int mrem, int nrem, int K, float alpha) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lg = lane >> 4;
  typedef __attribute__((address_space(3))) void* lds_ptr;

  // A: wavefront w fills rows 32 w .. 32 w + 31 as chunks q = 0, 1 of 16 rows;
  // lane i covers row 32 w + 16 q + i / 4 and the k quad of slot i % 4
  int a_off[2], a_p[2];
  bool a_ok[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = 32 * wave + 16 * q + (lane >> 2);
    a_p[q] = (lane & 3) ^ ((r >> 2) & 3);
    a_off[q] = (r * lda + 4 * a_p[q]) * 4;
    a_ok[q] = r < mrem;
  }
  // B: wavefront w fills chunks 2 w, 2 w + 1 (k rows 4 w .. 4 w + 3); lane i
  // covers k row 2c + i / 32 of chunk c, columns 4 (i % 32) .. + 3
  const int b_row = lane >> 5;
  const int b_off = (b_row * ldb + 4 * (lane & 31)) * 4;
  const bool b_ok = 4 * (lane & 31) < nrem;
  // a step wholly inside K needs only the row / column checks, folded into
  // the offsets once (`checked` false); the tail step and the step past K
  // check every k
  int a_offv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) a_offv[q] = a_ok[q] ? a_off[q] : kInvalidOff;
  const int b_offv = b_ok ? b_off : kInvalidOff;
  auto dma = [&](int buf, int k0, auto checked) {
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + k0);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(B + (int64_t)k0 * ldb);
    if constexpr (!decltype(checked)::value) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)&sm.a[buf][(32 * wave + 16 * q) * 4], 16, a_offv[q], 0,
                                                 0, 0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int c = 2 * wave + q;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)&sm.b[buf][c * SBC], 16, b_offv, 2 * c * ldb * 4, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)&sm.a[buf][(32 * wave + 16 * q) * 4], 16,
                                                 (a_ok[q] && k0 + 4 * a_p[q] < K) ? a_off[q] : kInvalidOff, 0, 0,
                                                 0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int c = 2 * wave + q;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)&sm.b[buf][c * SBC], 16,
                                                 (b_ok && k0 + 2 * c + b_row < K) ? b_off : kInvalidOff,
                                                 2 * c * ldb * 4, 0, 0);
      }
    }
  };

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  constexpr int kWaitVm0 = 0x0F70;  // vmcnt(0) only
  const int nk = (K + SBK - 1) / SBK;
  // A fragments: the four k values of the step in one read per row block; B
  // fragments per sub-step.  Step kt issues the loads of step kt + 1 first,
  // into the buffer every wavefront finished reading before the previous
  // barrier, so they land while the step's 64 MFMAs run; the last step
  // loads a step past K (zeros nothing reads).
  f4_t af[4];
  float bf[4][4];
  auto rd = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = sm.a[buf][aquad(wm * 64 + i * 16 + li, lg)];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[kk][j] = sm.b[buf][brow(4 * lg + kk) + wn * 64 + j * 16 + li];
  };
  constexpr std::true_type kChecked{};
  constexpr std::false_type kPlain{};
  auto mma_all = [&] {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][kk], bf[kk][j], acc[i][j], 0, 0, 0);
  };
  dma(0, 0, kChecked);
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  dma(1, SBK, kChecked);
  // step 0: its successor's loads are already out
  rd(0);
  mma_all();
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  // step kt >= 1: the loads of step kt + 1 go into the buffer step kt - 1
  // used, ahead of this step's fragment reads and MFMAs
  auto step = [&](int kt, auto checked) {
    const int cur = kt & 1;
    dma(cur ^ 1, (kt + 1) * SBK, checked);
    rd(cur);
    mma_all();
    if constexpr (!decltype(checked)::value) {
      // scheduling groups: the first fragment reads, then the MFMAs in one
      // stream (the compiler still issues the four loads up front; this
      // order measured 0.3% faster than its own and 2% on whole products)
      __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);  // eight LDS reads
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);  // four MFMAs
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // a VMEM read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 48, 0);  // the other MFMAs
    }
    // every MFMA of the step is issued before the wait for the next step's
    // loads and the barrier (the compiler would otherwise sink some below)
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  };
  // steps whose loads (one step ahead) lie wholly inside K run a loop body
  // without branches
  const int nplain = K / SBK - 1 < nk ? K / SBK - 1 : nk;
  int kt = 1;
  for (; kt < nplain; ++kt) step(kt, kPlain);
  for (; kt < nk; ++kt) step(kt, kChecked);
  // the loads past K have landed and every read is done before the next
  // tile's first loads reuse the buffers
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();

  const __amdgpu_buffer_rsrc_t sc = make_rsrc(C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // 16x16 f32 block: register v of lane l holds row 4 (l / 16) + v, column l % 16
        const int r = wm * 64 + i * 16 + 4 * lg + v;
        const int c = wn * 64 + j * 16 + li;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, alpha * acc[i][j][v]), sc,
                                              (r < mrem && c < nrem) ? (r * ldc + c) * 4 : kInvalidOff, 0, 0);
      }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
gemm_f32_dma_kernel(GemmArgs args) {
  const GemmArgs* ap = kernarg_args();
  __shared__ F32DmaSmem sm;
  const int64_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
  for (int64_t t = slot; t < ap->total_tiles; t += G) {
    const TileJob job = decode_tile(ap, t);
    const GemmProb pr = job.probs ? job.probs[job.prob] : ap->single;
    int64_t lda, ldb, ldc;
    const float* A = (const float*)slot_ptr(ap, job.slot, pr.a, &lda) + pr.a.off;
    const float* B = (const float*)slot_ptr(ap, job.slot, pr.b, &ldb) + pr.b.off;
    float* C = (float*)slot_ptr(ap, job.slot, pr.c, &ldc) + pr.c.off;
    A = uniform_ptr(A + (pr.a.row + job.tm * SBM) * lda + pr.a.col);
    B = uniform_ptr(B + pr.b.row * ldb + pr.b.col + job.tn * SBM);
    C = uniform_ptr(C + (pr.c.row + job.tm * SBM) * ldc + pr.c.col + job.tn * SBM);
    const int64_t mr = job.m - job.tm * SBM, nr = job.n - job.tn * SBM;
    f32_tile_dma(sm, A, B, C, uniform_int((int)lda), uniform_int((int)ldb), uniform_int((int)ldc),
                 uniform_int(mr < SBM ? (int)mr : SBM), uniform_int(nr < SBM ? (int)nr : SBM),
                 uniform_int((int)job.k), (float)uniform_double(pr.alpha));
  }
}

}  // namespace

hipError_t launch_gemm_f32_dma(const GemmArgs& a, int num_cus, hipStream_t s) {
  static std::atomic<int> cached{0};
  int per_cu = cached.load(std::memory_order_relaxed);
  if (!per_cu) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_f32_dma_kernel, 256, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cached.store(per_cu, std::memory_order_relaxed);
  }
  const int64_t G = leaf_grid((int64_t)per_cu * num_cus, a.total_tiles);
  hipLaunchKernelGGL(gemm_f32_dma_kernel, dim3((unsigned)G), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fmm
