// Host-side launchers of the HIP kernels (defined in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include "fmm_internal.h"

namespace fmm {

// BF16x3 leaf kernels are compiled in.
constexpr bool kHaveBf16x3 = true;

hipError_t launch_form(int alg, const FormArgs& a, int side, int lv, int ngroups, hipStream_t s);
// One-level S and T passes (unsplit outputs) in one launch; the same values as two launch_form calls.
hipError_t launch_form_pair(int alg, const FormArgs& sa, int ngs, const FormArgs& ta, int ngt, hipStream_t st);
hipError_t launch_combine(int alg, const CombineArgs& a, int lv, int ngroups, hipStream_t s);
// Grouped GEMM over every problem in `a`; the element type (a.elt) and the
// dtype (0: FP64 MFMA, 1: FP32 MFMA, 2: BF16x3 MFMA) select the kernel.
hipError_t launch_gemm(const GemmArgs& a, int dtype, int num_cus, hipStream_t s);
hipError_t launch_gemm_bf16x3(const GemmArgs& a, int num_cus, hipStream_t s);
// FP64, 128 x 128 tiles, operands staged by direct global-to-LDS loads (a.dma
// must be set: 16-byte aligned rows, even leading dimensions, even K and N).
hipError_t launch_gemm_f64_dma(const GemmArgs& a, int num_cus, hipStream_t s);
// FP32 (FP32 MFMA path) likewise: 16-byte aligned rows, leading dimensions,
// K and N multiples of 4.
hipError_t launch_gemm_f32_dma(const GemmArgs& a, int num_cus, hipStream_t s);
// Workgroups of a grouped leaf launch over `tiles` tiles, `resident` of
// which fit on the device at once (a multiple of 8, at least 8).
int64_t leaf_grid(int64_t resident, int64_t tiles);

}  // namespace fmm
