// Shared pieces of the grouped leaf-GEMM kernels: buffer resources, uniform
// values, and the flat-tile decoder.
#pragma once

#include <hip/hip_runtime.h>

#include "fmm_device.h"

namespace fmm {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned u2_t __attribute__((ext_vector_type(2)));

constexpr int GBM = 128, GBN = 128, GBK = 16, GNT = 256;
constexpr int kInvalidOff = (int)0x80000000;  // beyond kNumRecords: loads read 0, stores drop
constexpr int kNumRecords = 0x7ffffff0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p) {
  // 0x00020000: 32-bit data format word of a raw (unformatted) gfx9 buffer
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, kNumRecords, 0x00020000);
}

__device__ __forceinline__ int uniform_int(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ double uniform_double(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const unsigned long long u = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}


// The launch's argument block, read through the kernel-argument segment
// pointer (the block is the kernels' only explicit argument, so it starts the
// segment).  Indexing it at run time then compiles to scalar loads at a
// computed address; indexing the by-value parameter would copy the whole
// block to scratch first.
__device__ __forceinline__ const GemmArgs* kernarg_args() {
  return (const GemmArgs*)__builtin_amdgcn_kernarg_segment_ptr();
}

// Base pointer and leading dimension of view r of the plan in `slot`.
__device__ __forceinline__ char* slot_ptr(const GemmArgs* a, int slot, const Ref& r, int64_t* ld) {
  const int buf = uniform_int(r.buf);
  *ld = buf == BUF_WS ? r.ld : a->bases[slot].ld[buf];
  return (char*)a->bases[slot].ptr[buf];
}

struct TileJob {
  int64_t m, n, k, tm, tn, prob;
  const GemmProb* probs;
  int slot;
};

__device__ __forceinline__ TileJob decode_tile(const GemmArgs* args, int64_t t) {
  int gi = 0;
  for (int i = 1; i < args->ngroups; ++i)
    if (t >= args->groups[i].tile_start) gi = i;
  const GemmGroup& g = args->groups[gi];
  const int64_t gm = g.m, gn = g.n, gk = g.k, tiles_m = g.tiles_m, tiles_n = g.tiles_n;
  const int64_t tstart = g.tile_start, pstart = g.prob_start;
  const GemmProb* probs = g.probs;
  const int slot = g.slot;
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
  j.probs = probs;
  j.slot = slot;
  return j;
}

}  // namespace fmm
