// C ABI and executor: validates arguments, owns the device resources of a
// plan, and enqueues the stages (operand formation, grouped leaf GEMM,
// W-combination) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_internal.h"
#include "fmm_launch.h"

struct fmm_plan_s {
  fmm::Plan P;
};

namespace {

thread_local std::string g_err;

fmm_status fail(fmm_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

fmm_status hip_fail(hipError_t e, const char* what) {
  return fail(FMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int num_cus(int device) {
  static std::atomic<int> cached[64];  // 0 = not queried yet
  if (device < 0 || device >= 64) return 256;
  int v = cached[device].load(std::memory_order_relaxed);
  if (!v) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0)
      v = 256;
    cached[device].store(v, std::memory_order_relaxed);
  }
  return v;
}

// Exact Brent check of one table (Equation (2) against the tensor of
// Section 2.2): sum_r U[i][r] V[j][r] W[k][r] == [A_i B_j contributes to C_k].
bool brent_ok(const fmm::AlgInfo& a, std::string* why) {
  const int MK = a.M * a.K, KN = a.K * a.N, MN = a.M * a.N, R = a.R;
  for (int i = 0; i < MK; ++i)
    for (int j = 0; j < KN; ++j)
      for (int k = 0; k < MN; ++k) {
        long long s = 0;
        for (int r = 0; r < R; ++r) s += (long long)a.U[i * R + r] * a.V[j * R + r] * a.W[k * R + r];
        const int ia = i / a.K, ib = i % a.K, jb = j / a.N, jc = j % a.N, ka = k / a.N, kc = k % a.N;
        const long long t = (ib == jb && jc == kc && ia == ka) ? 1 : 0;
        if (s != t) {
          *why = std::string("table ") + a.name + " fails the Brent equation at (i,j,k)=(" +
                 std::to_string(i) + "," + std::to_string(j) + "," + std::to_string(k) + ")";
          return false;
        }
      }
  return true;
}

fmm_status check_tables_once() {
  static std::once_flag once;
  static bool ok = true;
  static std::string why;
  std::call_once(once, [] {
    for (int i = 0; i < fmm::kNumAlgorithms; ++i)
      if (!brent_ok(fmm::alg_info(i), &why)) {
        ok = false;
        break;
      }
  });
  return ok ? FMM_OK : fail(FMM_EALG, why);
}

size_t elt_size(int elt) { return elt == fmm::ELT_F64 ? 8 : 4; }

constexpr int64_t kMaxLd = (int64_t)1 << 21;

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return abytes && bbytes && x < y + bbytes && y < x + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t es) {
  if (rows <= 0 || cols <= 0) return 0;
  return ((size_t)(rows - 1) * ld + cols) * es;
}

fmm_status validate(const fmm::Plan& P, const void* A, int64_t lda, const void* B, int64_t ldb,
                    const void* C, int64_t ldc) {
  std::string why;
  const int st = fmm::check_operands(P.m, P.k, P.n, elt_size(P.elt), A, lda, B, ldb, C, ldc, &why);
  return st ? fail((fmm_status)st, why) : FMM_OK;
}

fmm::Bases make_bases(const fmm::Plan& P, const void* A, int64_t lda, const void* B, int64_t ldb,
                      void* C, int64_t ldc) {
  fmm::Bases b;
  b.ptr[0] = const_cast<void*>(A);
  b.ptr[1] = const_cast<void*>(B);
  b.ptr[2] = C;
  b.ptr[3] = P.ws;
  b.ld[0] = lda;
  b.ld[1] = ldb;
  b.ld[2] = ldc;
  b.ld[3] = 0;
  return b;
}

template <typename T>
const T* table_ptr(const fmm::Plan& P, size_t off) {
  return (const T*)((const char*)P.dev_table + off);
}

hipError_t run_form(const fmm::Plan& P, const std::vector<fmm::FormPass>& passes, const fmm::Bases& b,
                    hipStream_t s) {
  for (const fmm::FormPass& fp : passes) {
    fmm::FormArgs a;
    a.bases = b;
    a.groups = table_ptr<fmm::Ref>(P, fp.dev_groups);
    a.outs = table_ptr<int64_t>(P, fp.dev_outs);
    a.h = fp.h;
    a.w = fp.w;
    a.out_ld = fp.out_ld;
    a.out_plane = fp.out_plane;
    a.out_elt = fp.out_elt;
    a.nout = fp.nout;
    hipError_t e = fmm::launch_form(fp.alg, a, fp.side, fp.lv, fp.ngroups, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Both one-level passes of a pair_form plan in one launch (T is formed by
// the S stage; the T stage then has nothing to do).
hipError_t run_form_pair(const fmm::Plan& P, const fmm::Bases& b, hipStream_t s) {
  fmm::FormArgs a[2];
  const fmm::FormPass* fp[2] = {&P.s_passes[0], &P.t_passes[0]};
  for (int i = 0; i < 2; ++i) {
    a[i].bases = b;
    a[i].groups = table_ptr<fmm::Ref>(P, fp[i]->dev_groups);
    a[i].outs = table_ptr<int64_t>(P, fp[i]->dev_outs);
    a[i].h = fp[i]->h;
    a[i].w = fp[i]->w;
    a[i].out_ld = fp[i]->out_ld;
    a[i].out_plane = fp[i]->out_plane;
    a[i].out_elt = fp[i]->out_elt;
    a[i].nout = fp[i]->nout;
  }
  return fmm::launch_form_pair(fp[0]->alg, a[0], fp[0]->ngroups, a[1], fp[1]->ngroups, s);
}

// Whether every problem of plan P (or the single problem of a plain GEMM)
// suits the direct-load leaf kernels (FP64 and FP32 MFMA paths): rows of A
// and B 16-byte aligned with leading dimensions a multiple of e = 16 bytes /
// element size (the kernels add row offsets and column offsets that keep
// that alignment), and K and N multiples of e in every group.
bool ref_dma_ok(const fmm::Ref& r, const fmm::Bases& b, void* ws, int e) {
  const int64_t ld = r.buf == fmm::BUF_WS ? r.ld : b.ld[r.buf];
  const void* base = r.buf == fmm::BUF_WS ? ws : b.ptr[r.buf];
  return ld % e == 0 && (r.off + r.row * ld + r.col) % e == 0 && (uintptr_t)base % 16 == 0;
}

bool leaf_dma_ok(const fmm::Plan& P, const fmm::Bases& b) {
  if (P.dtype == 2 || P.leaf_form) return false;
  const int e = P.dtype == 0 ? 2 : 4;
  for (const fmm::GemmGroup& g : P.gemm_groups)
    if (g.n % e || g.k % e) return false;
  for (const fmm::GemmProb& pr : P.gemm_probs)
    if (!ref_dma_ok(pr.a, b, P.ws, e) || !ref_dma_ok(pr.b, b, P.ws, e)) return false;
  return true;
}

// Appends plan P's GEMM groups to a (possibly shared) grouped launch, with
// P's operand bases in slot `slot`.
void append_leaf(fmm::GemmArgs& a, const fmm::Plan& P, const fmm::Bases& b, int slot) {
  a.bases[slot] = b;
  a.elt = P.elt;
  for (const fmm::GemmGroup& g0 : P.gemm_groups) {
    fmm::GemmGroup g = g0;
    g.tile_start += a.total_tiles;
    g.probs = table_ptr<fmm::GemmProb>(P, P.dev_probs);
    g.slot = slot;
    a.groups[a.ngroups++] = g;
  }
  a.total_tiles += P.gemm_tiles;
}

hipError_t run_leaf(const fmm::Plan& P, const fmm::Bases& b, hipStream_t s) {
  if (P.gemm_groups.empty()) return hipSuccess;
  fmm::GemmArgs a;
  std::memset(&a, 0, sizeof(a));
  append_leaf(a, P, b, 0);
  a.tile = P.leaf_tile;
  a.form_terms = P.leaf_form;
  a.dma = leaf_dma_ok(P, b) ? 1 : 0;
  return fmm::launch_gemm(a, P.dtype, num_cus(P.device), s);
}

// Whether every pair of adjacent positions (p, q), (p, q + 1), q even, of a
// combination pass is 8-byte aligned in the FP32 products and in the FP32
// output blocks (the register combination kernel's 8-byte accesses).
bool combine_pairs_ok(const fmm::CombinePass& cp, const fmm::Bases& b) {
  if (cp.in_elt != fmm::ELT_F32 || cp.has_p || (cp.w & 1) || ((cp.in_ld | cp.in_stride) & 1)) return false;
  if (((uintptr_t)b.ptr[fmm::BUF_WS] & 7) != 0) return false;
  for (int64_t off : cp.in_off)
    if (off & 1) return false;
  for (const fmm::Ref& o : cp.out) {
    const int64_t ld = o.buf == fmm::BUF_WS ? o.ld : b.ld[o.buf];
    if (o.elt != fmm::ELT_F32 || ((o.off | o.col | ld) & 1) || ((uintptr_t)b.ptr[o.buf] & 7) != 0) return false;
  }
  return true;
}

hipError_t run_combine(const fmm::Plan& P, const fmm::Bases& b, hipStream_t s) {
  for (const fmm::CombinePass& cp : P.w_passes) {
    fmm::CombineArgs a;
    std::memset(&a, 0, sizeof(a));
    a.bases = b;
    a.in_off = table_ptr<int64_t>(P, cp.dev_in);
    a.out = table_ptr<fmm::Ref>(P, cp.dev_out);
    a.h = cp.h;
    a.w = cp.w;
    a.in_ld = cp.in_ld;
    a.in_stride = cp.in_stride;
    a.in_elt = cp.in_elt;
    a.has_p = cp.has_p ? 1 : 0;
    a.p = cp.p;
    a.pairs = combine_pairs_ok(cp, b) ? 1 : 0;
    hipError_t e = fmm::launch_combine(cp.alg, a, cp.lv, cp.ngroups, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_stage(const fmm::Plan& P, int stage, const fmm::Bases& b, hipStream_t s) {
  switch (stage) {
    case FMM_STAGE_FORM_S: return P.pair_form ? run_form_pair(P, b, s) : run_form(P, P.s_passes, b, s);
    case FMM_STAGE_FORM_T: return P.pair_form ? hipSuccess : run_form(P, P.t_passes, b, s);
    case FMM_STAGE_LEAF: return run_leaf(P, b, s);
    case FMM_STAGE_COMBINE: return run_combine(P, b, s);
  }
  return hipErrorInvalidValue;
}

// A stage as a multiply runs it: plans that form their leaf operands inside
// the leaf GEMM skip the formation stages (fmm_run_stage still runs them, so
// the formed operands can be inspected).
hipError_t run_multiply_stage(const fmm::Plan& P, int stage, const fmm::Bases& b, hipStream_t s) {
  if (P.leaf_form && (stage == FMM_STAGE_FORM_S || stage == FMM_STAGE_FORM_T)) return hipSuccess;
  return run_stage(P, stage, b, s);
}

constexpr size_t kTableAlign = 256;

size_t table_offset(const fmm::Plan& P) { return (P.ws_bytes + kTableAlign - 1) / kTableAlign * kTableAlign; }

fmm_status check_runnable(const fmm::Plan& P) {
  if (P.host_only) return fail(FMM_EINVAL, "host-only plan cannot run");
  if (P.external && !P.dev_table) return fail(FMM_EINVAL, "no device memory bound to the plan (fmm_plan_bind)");
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != P.device) return fail(FMM_EINVAL, "plan belongs to another device");
  return FMM_OK;
}

void drop_graph(fmm::Plan& P) {
  if (P.graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)P.graph_exec);
  P.graph_exec = nullptr;
  std::memset(&P.graph_key, 0, sizeof(P.graph_key));
}

// Records the four stages on the plan's private stream into a graph and
// (re)instantiates the plan's executable graph from it.
fmm_status capture_graph(fmm::Plan& P, const fmm::Bases& b) {
  hipError_t e;
  if (!P.cap_stream) {
    hipStream_t cs;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    P.cap_stream = cs;
  }
  hipStream_t cs = (hipStream_t)P.cap_stream;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t le = hipSuccess;
  for (int stage = 0; stage < FMM_NUM_STAGES && le == hipSuccess; ++stage) le = run_multiply_stage(P, stage, b, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  if (le != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    drop_graph(P);
    return hip_fail(le != hipSuccess ? le : e, "graph capture");
  }
  if (P.graph_exec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult r;
    if (hipGraphExecUpdate((hipGraphExec_t)P.graph_exec, g, &bad, &r) != hipSuccess ||
        r != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      drop_graph(P);
    }
  }
  if (!P.graph_exec) {
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "hipGraphInstantiate");
    }
    P.graph_exec = ex;
  }
  (void)hipGraphDestroy(g);
  P.graph_key = b;
  return FMM_OK;
}

// Device memory of fmm_multiply_noalloc: a fixed array that every GPU the
// library runs on holds from module load until the process ends.  In host
// code the name `scratch` only stands in for the device symbol; the array's
// device address on each GPU comes from hipGetSymbolAddress (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[FMM_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, NULL until looked up

// Address of `scratch` on device `dev`, which must be the current device:
// looked up once per device (each GPU holds its own copy at its own address).
fmm_status scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FMM_EUNSUPPORTED, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the no-allocation scratch array");
    if (!p) return fail(FMM_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FMM_OK;
}

fmm_status plan_common(fmm_plan_t* out, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                       int dtype, int fuse, bool device, bool defer = false, bool graph = false,
                       int leaf_tile = 0, double max_error = 0, int leaf_form = 0) {
  if (!out) return fail(FMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (leaf_tile != 0 && leaf_tile != 64 && leaf_tile != 128 && !(leaf_tile == 256 && dtype == FMM_F32_BF16X3))
    return fail(FMM_EINVAL, "leaf_tile must be 0, 64 or 128 (or 256 on the BF16x3 path)");
  fmm_status st = check_tables_once();
  if (st != FMM_OK) return st;
  if (dtype == FMM_F32_BF16X3 && !fmm::kHaveBf16x3)
    return fail(FMM_EUNSUPPORTED, "BF16x3 leaves are not compiled into this library");
  // "auto" (any base case) or levels -1 (best depth of `alg`): the cost model's choice
  std::string chosen;
  if ((alg && !std::strcmp(alg, "auto")) || levels < 0) {
    if (levels < -1) return fail(FMM_EINVAL, "levels must be >= -1");
    fmm::Candidate pick;
    std::string why;
    if (!fmm::choose(m, k, n, dtype, alg, levels, 0, fuse, max_error, &pick, &why))
      return fail(why.rfind("unknown algorithm", 0) == 0 ? FMM_EALG
                  : why.rfind("no candidate", 0) == 0    ? FMM_ENOMEM
                                                         : FMM_EINVAL,
                  why);
    chosen = pick.alg;
    alg = chosen.c_str();
    levels = pick.levels;
    if (!fuse) fuse = pick.fuse;
    if (!leaf_tile) leaf_tile = pick.tile;
  }
  fmm_plan_s* h = new (std::nothrow) fmm_plan_s();
  if (!h) return fail(FMM_ENOMEM, "host allocation failed");
  int code = 0;
  std::string err = fmm::make_plan(h->P, alg, m, k, n, levels, dtype, fuse, &code, leaf_form);
  if (!err.empty()) {
    delete h;
    return fail((fmm_status)code, err);
  }
  fmm::Plan& P = h->P;
  P.leaf_tile = leaf_tile;
  if (device) {
    if (const char* bud = std::getenv("FMM_HBM_BUDGET")) {
      const double budget = std::atof(bud);
      if (budget > 0 && (double)P.ws_bytes > budget) {
        delete h;
        return fail(FMM_ENOMEM, "workspace of " + std::to_string(P.ws_bytes) +
                                    " bytes exceeds FMM_HBM_BUDGET");
      }
    }
    hipError_t e = hipGetDevice(&P.device);
    if (e != hipSuccess) {
      delete h;
      return hip_fail(e, "hipGetDevice");
    }
    P.use_graph = graph;
    if (defer) {
      // The caller binds device memory (fmm_plan_bind) before the first run.
      P.external = true;
      P.host_only = false;
      *out = h;
      return FMM_OK;
    }
    if (P.ws_bytes) {
      e = hipMalloc(&P.ws, P.ws_bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        P.ws = nullptr;
        delete h;
        return fail(FMM_ENOMEM, "hipMalloc of " + std::to_string(P.ws_bytes) + " workspace bytes failed");
      }
    }
    e = hipMalloc(&P.dev_table, P.table_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (P.ws) (void)hipFree(P.ws);
      delete h;
      return fail(FMM_ENOMEM, "hipMalloc of the descriptor table failed");
    }
    e = hipMemcpy(P.dev_table, P.table.data(), P.table_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (P.ws) (void)hipFree(P.ws);
      (void)hipFree(P.dev_table);
      delete h;
      return hip_fail(e, "hipMemcpy of the descriptor table");
    }
    P.host_only = false;
  }
  *out = h;
  return FMM_OK;
}

}  // namespace

namespace fmm {
int set_error(int code, const std::string& msg) { return (int)fail((fmm_status)code, msg); }

int check_operands(int64_t m, int64_t k, int64_t n, size_t es, const void* A, int64_t lda, const void* B,
                   int64_t ldb, const void* C, int64_t ldc, std::string* why) {
  if (m == 0 || n == 0) return FMM_OK;
  if (!C) return *why = "C is NULL", FMM_EINVAL;
  if (ldc < n) return *why = "ldc < n", FMM_EINVAL;
  // The leaf kernels address a 128-row tile with 32-bit byte offsets.
  if (lda >= kMaxLd || ldb >= kMaxLd || ldc >= kMaxLd)
    return *why = "leading dimensions must be below 2^21 elements", FMM_EUNSUPPORTED;
  if (k > 0) {
    if (!A || !B) return *why = "A or B is NULL", FMM_EINVAL;
    if (lda < k) return *why = "lda < k", FMM_EINVAL;
    if (ldb < n) return *why = "ldb < n", FMM_EINVAL;
    const size_t cb = span_bytes(m, n, ldc, es);
    if (overlaps(C, cb, A, span_bytes(m, k, lda, es)) || overlaps(C, cb, B, span_bytes(k, n, ldb, es)))
      return *why = "C overlaps A or B", FMM_EINVAL;
  }
  return FMM_OK;
}
}  // namespace fmm

extern "C" {

fmm_status fmm_plan(fmm_plan_t* out, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                    int dtype) {
  return plan_common(out, alg, m, k, n, levels, dtype, 0, true);
}

fmm_status fmm_plan_host(fmm_plan_t* out, const char* alg, int64_t m, int64_t k, int64_t n,
                         int levels, int dtype) {
  return plan_common(out, alg, m, k, n, levels, dtype, 0, false);
}

fmm_status fmm_plan_ex(fmm_plan_t* out, const char* alg, int64_t m, int64_t k, int64_t n, int levels,
                       int dtype, const fmm_plan_options_t* opts) {
  const int fuse = opts ? opts->fuse_levels : 0;
  const bool host_only = opts && opts->host_only;
  const bool defer = opts && opts->defer_device_memory;
  const bool graph = opts && opts->use_graph;
  const int tile = opts ? opts->leaf_tile : 0;
  const double max_error = opts ? opts->max_error : 0;
  const int leaf_form = opts ? opts->leaf_form : 0;
  return plan_common(out, alg, m, k, n, levels, dtype, fuse, !host_only, defer, graph, tile, max_error,
                     leaf_form);
}

size_t fmm_plan_device_bytes(fmm_plan_t p) {
  if (!p) return 0;
  return table_offset(p->P) + p->P.table_bytes;
}

fmm_status fmm_plan_bind(fmm_plan_t p, void* mem, size_t bytes, void* stream) {
  if (!p) return fail(FMM_EINVAL, "plan is NULL");
  fmm::Plan& P = p->P;
  if (!P.external) return fail(FMM_EINVAL, "plan owns its device memory (not made with defer_device_memory)");
  if (!mem) return fail(FMM_EINVAL, "mem is NULL");
  if ((uintptr_t)mem % kTableAlign) return fail(FMM_EINVAL, "mem must be 256-byte aligned");
  if (bytes < fmm_plan_device_bytes(p)) return fail(FMM_EINVAL, "bytes < fmm_plan_device_bytes(p)");
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != P.device) return fail(FMM_EINVAL, "plan belongs to another device");
  drop_graph(P);
  P.ws = P.ws_bytes ? mem : nullptr;
  P.dev_table = (char*)mem + table_offset(P);
  hipError_t e = hipMemcpyAsync(P.dev_table, P.table.data(), P.table_bytes, hipMemcpyHostToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) {
    P.ws = nullptr;
    P.dev_table = nullptr;
    return hip_fail(e, "hipMemcpyAsync of the descriptor table");
  }
  return FMM_OK;
}

fmm_status fmm_run_stage(fmm_plan_t p, int stage, const void* A, int64_t lda, const void* B,
                         int64_t ldb, void* C, int64_t ldc, void* stream) {
  if (!p) return fail(FMM_EINVAL, "plan is NULL");
  const fmm::Plan& P = p->P;
  if (P.host_only) return fail(FMM_EINVAL, "host-only plan cannot run");
  if (stage < 0 || stage >= FMM_NUM_STAGES) return fail(FMM_EINVAL, "bad stage");
  fmm_status st = validate(P, A, lda, B, ldb, C, ldc);
  if (st != FMM_OK) return st;
  if (P.m == 0 || P.n == 0) return FMM_OK;
  st = check_runnable(P);
  if (st != FMM_OK) return st;
  const fmm::Bases b = make_bases(P, A, lda, B, ldb, C, ldc);
  hipError_t e = run_stage(P, stage, b, (hipStream_t)stream);
  return e == hipSuccess ? FMM_OK : hip_fail(e, "kernel launch");
}

fmm_status fmm_multiply(fmm_plan_t p, const void* A, int64_t lda, const void* B, int64_t ldb,
                        void* C, int64_t ldc, void* stream) {
  if (!p) return fail(FMM_EINVAL, "plan is NULL");
  fmm::Plan& P = p->P;
  if (P.host_only) return fail(FMM_EINVAL, "host-only plan cannot run");
  fmm_status st = validate(P, A, lda, B, ldb, C, ldc);
  if (st != FMM_OK) return st;
  if (P.m == 0 || P.n == 0) return FMM_OK;
  st = check_runnable(P);
  if (st != FMM_OK) return st;
  const fmm::Bases b = make_bases(P, A, lda, B, ldb, C, ldc);
  hipStream_t s = (hipStream_t)stream;
  if (P.use_graph && !P.timing_slots) {
    if (!P.graph_exec || std::memcmp(&P.graph_key, &b, sizeof(b)) != 0) {
      st = capture_graph(P, b);
      if (st != FMM_OK) return st;
    }
    hipError_t e = hipGraphLaunch((hipGraphExec_t)P.graph_exec, s);
    return e == hipSuccess ? FMM_OK : hip_fail(e, "hipGraphLaunch");
  }
  const size_t slot = P.timing_slots ? (size_t)(P.timed % P.timing_slots) * (FMM_NUM_STAGES + 1) : 0;
  for (int stage = 0; stage < FMM_NUM_STAGES; ++stage) {
    if (P.timing_slots) {
      hipError_t e = hipEventRecord((hipEvent_t)P.events[slot + stage], s);
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    hipError_t e = run_multiply_stage(P, stage, b, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  if (P.timing_slots) {
    hipError_t e = hipEventRecord((hipEvent_t)P.events[slot + FMM_NUM_STAGES], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ++P.timed;
  }
  return FMM_OK;
}

fmm_status fmm_multiply_noalloc(fmm_plan_t p, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                                int64_t ldc, void* stream) {
  if (!p) return fail(FMM_EINVAL, "plan is NULL");
  fmm::Plan& P = p->P;
  if (P.host_only) return fail(FMM_EINVAL, "host-only plan cannot run");
  fmm_status st = validate(P, A, lda, B, ldb, C, ldc);
  if (st != FMM_OK) return st;
  if (P.m == 0 || P.n == 0) return FMM_OK;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != P.device) return fail(FMM_EINVAL, "plan belongs to another device");
  const size_t need = table_offset(P) + P.table_bytes;
  if (need > (size_t)FMM_NOALLOC_MAX_BYTES)
    return fail(FMM_ENOMEM, "plan needs " + std::to_string(need) + " device bytes (workspace + tables); " +
                                "fmm_multiply_noalloc has " + std::to_string((size_t)FMM_NOALLOC_MAX_BYTES));
  void* mem = nullptr;
  st = scratch_ptr(cur, &mem);
  if (st != FMM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // The plan's device pointers name the array for this call only; every
  // launch below takes them as kernel arguments, so the plan's own memory (or
  // its binding) is left as it was.
  void* const ws0 = P.ws;
  void* const tab0 = P.dev_table;
  P.ws = P.ws_bytes ? mem : nullptr;
  P.dev_table = (char*)mem + table_offset(P);
  e = hipMemcpyAsync(P.dev_table, P.table.data(), P.table_bytes, hipMemcpyHostToDevice, s);
  const fmm::Bases b = make_bases(P, A, lda, B, ldb, C, ldc);
  for (int stage = 0; stage < FMM_NUM_STAGES && e == hipSuccess; ++stage) e = run_multiply_stage(P, stage, b, s);
  P.ws = ws0;
  P.dev_table = tab0;
  return e == hipSuccess ? FMM_OK : hip_fail(e, "no-allocation multiply");
}

fmm_status fmm_multiply_batched(const fmm_plan_t* plans, const void* const* A, const int64_t* lda,
                                const void* const* B, const int64_t* ldb, void* const* C,
                                const int64_t* ldc, int count, void* stream) {
  if (count < 0) return fail(FMM_EINVAL, "count < 0");
  if (count == 0) return FMM_OK;
  if (!plans || !A || !lda || !B || !ldb || !C || !ldc) return fail(FMM_EINVAL, "NULL array");
  std::vector<int> live;
  std::vector<fmm::Bases> bases((size_t)count);
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return fail(FMM_EINVAL, "plan " + std::to_string(i) + " is NULL");
    const fmm::Plan& P = plans[i]->P;
    fmm_status st = validate(P, A[i], lda[i], B[i], ldb[i], C[i], ldc[i]);
    if (st != FMM_OK) return fail(st, "request " + std::to_string(i) + ": " + g_err);
    if (P.m == 0 || P.n == 0) continue;
    st = check_runnable(P);
    if (st != FMM_OK) return fail(st, "request " + std::to_string(i) + ": " + g_err);
    for (int j : live)
      if (plans[j] == plans[i]) return fail(FMM_EINVAL, "a plan appears twice in one batch (shared workspace)");
    bases[i] = make_bases(P, A[i], lda[i], B[i], ldb[i], C[i], ldc[i]);
    live.push_back(i);
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int stage : {FMM_STAGE_FORM_S, FMM_STAGE_FORM_T})
    for (int i : live)
      if ((e = run_multiply_stage(plans[i]->P, stage, bases[i], s)) != hipSuccess)
        return hip_fail(e, "kernel launch");
  // Leaves of all requests of one dtype (and one way of staging operands)
  // share grouped launches, as many plans per launch as the argument block
  // holds.
  for (int key = 0; key < 3 * 2; ++key) {
    const int dtype = key / 2, form = (key % 2) * fmm::kMaxLeafTerms;  // plain, or forming, operands
    fmm::GemmArgs a;
    std::memset(&a, 0, sizeof(a));
    int slots = 0;
    bool dma = true;
    auto flush = [&]() -> hipError_t {
      hipError_t fe = hipSuccess;
      a.form_terms = form;
      a.dma = dma ? 1 : 0;
      if (slots) fe = fmm::launch_gemm(a, dtype, num_cus(plans[live[0]]->P.device), s);
      std::memset(&a, 0, sizeof(a));
      slots = 0;
      dma = true;
      return fe;
    };
    for (int i : live) {
      const fmm::Plan& P = plans[i]->P;
      if (P.dtype != dtype || P.leaf_form != form || P.gemm_groups.empty()) continue;
      if (slots == fmm::kMaxGemmSlots || a.ngroups + (int)P.gemm_groups.size() > fmm::kMaxGemmGroups)
        if ((e = flush()) != hipSuccess) return hip_fail(e, "kernel launch");
      append_leaf(a, P, bases[i], slots++);
      dma = dma && leaf_dma_ok(P, bases[i]);
    }
    if ((e = flush()) != hipSuccess) return hip_fail(e, "kernel launch");
  }
  for (int i : live)
    if ((e = run_stage(plans[i]->P, FMM_STAGE_COMBINE, bases[i], s)) != hipSuccess)
      return hip_fail(e, "kernel launch");
  return FMM_OK;
}

fmm_status fmm_plan_enable_timing(fmm_plan_t p, int slots) {
  if (!p) return fail(FMM_EINVAL, "plan is NULL");
  fmm::Plan& P = p->P;
  if (P.host_only) return fail(FMM_EINVAL, "host-only plan");
  if (slots < 0) return fail(FMM_EINVAL, "slots must be >= 0");
  const size_t need = (size_t)slots * (FMM_NUM_STAGES + 1);
  while (P.events.size() < need) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    P.events.push_back(ev);
  }
  P.timing_slots = slots;
  P.timed = 0;
  return FMM_OK;
}

fmm_status fmm_plan_stage_ms(fmm_plan_t p, double ms[FMM_NUM_STAGES]) {
  if (!p || !ms) return fail(FMM_EINVAL, "NULL argument");
  fmm::Plan& P = p->P;
  if (!P.timing_slots || P.timed == 0) return fail(FMM_EINVAL, "no timed multiply yet");
  const int64_t n = P.timed < P.timing_slots ? P.timed : P.timing_slots;
  for (int i = 0; i < FMM_NUM_STAGES; ++i) ms[i] = 0;
  for (int64_t t = P.timed - n; t < P.timed; ++t) {
    const size_t slot = (size_t)(t % P.timing_slots) * (FMM_NUM_STAGES + 1);
    hipError_t e = hipEventSynchronize((hipEvent_t)P.events[slot + FMM_NUM_STAGES]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    for (int i = 0; i < FMM_NUM_STAGES; ++i) {
      float f = 0;
      e = hipEventElapsedTime(&f, (hipEvent_t)P.events[slot + i], (hipEvent_t)P.events[slot + i + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      ms[i] += f;
    }
  }
  for (int i = 0; i < FMM_NUM_STAGES; ++i) ms[i] /= (double)n;
  return FMM_OK;
}

fmm_status fmm_plan_operand(fmm_plan_t p, int side, int64_t leaf, int* loc, int64_t* offset,
                            int64_t* row, int64_t* col, int64_t* ld, double* alpha) {
  if (!p) return fail(FMM_EINVAL, "plan is NULL");
  const fmm::Plan& P = p->P;
  if (leaf < 0 || leaf >= (int64_t)P.leaves.size()) return fail(FMM_EINVAL, "leaf out of range");
  if (side < 0 || side > 2) return fail(FMM_EINVAL, "side must be 0, 1 or 2");
  const fmm::LeafRef& L = P.leaves[leaf];
  const fmm::Ref& r = side == 0 ? L.s : side == 1 ? L.t : L.m;
  const bool ws = r.buf == fmm::BUF_WS;
  if (loc) *loc = r.buf;
  if (offset) *offset = ws ? r.off + r.row * r.ld + r.col : 0;
  if (row) *row = ws ? 0 : r.row;
  if (col) *col = ws ? 0 : r.col;
  if (ld) *ld = ws ? r.ld : 0;
  if (alpha) *alpha = r.alpha;
  return FMM_OK;
}

void* fmm_plan_workspace(fmm_plan_t p) { return p ? p->P.ws : nullptr; }

size_t fmm_plan_workspace_bytes(fmm_plan_t p) { return p ? p->P.ws_bytes : 0; }

fmm_status fmm_plan_info(fmm_plan_t p, fmm_plan_info_t* info) {
  if (!p || !info) return fail(FMM_EINVAL, "NULL argument");
  const fmm::Plan& P = p->P;
  std::memset(info, 0, sizeof(*info));
  info->m = P.m;
  info->k = P.k;
  info->n = P.n;
  info->levels = P.levels;
  info->dtype = P.dtype;
  info->M = P.M;
  info->K = P.K;
  info->N = P.N;
  info->R = P.R;
  info->m0 = P.m0;
  info->k0 = P.k0;
  info->n0 = P.n0;
  info->leaf_m = P.ml;
  info->leaf_k = P.kl;
  info->leaf_n = P.nl;
  info->num_leaves = (int64_t)P.leaves.size();
  info->num_s_materialized = P.s_mat;
  info->num_t_materialized = P.t_mat;
  info->num_gemm_problems = (int64_t)P.gemm_probs.size();
  info->gemm_tiles = P.gemm_tiles;
  info->workspace_bytes = P.ws_bytes;
  info->leaf_flops = P.leaf_flops;
  info->classical_flops = 2.0 * (double)P.m * (double)P.k * (double)P.n;
  info->add_bytes = P.add_bytes;
  info->fuse_levels = P.levels > 0 ? P.fuse : 0;
  info->gemm_min_bytes = P.gemm_min_bytes;
  // one base case per level joined by '+' when the levels differ
  const bool mixed = P.alg_name.find('+') != std::string::npos;
  std::snprintf(info->alg, sizeof(info->alg), "%s",
                P.alg_id < 0 ? "classical" : mixed ? P.alg_name.c_str() : fmm::alg_info(P.alg_id).name);
  info->leaf_tile = P.leaf_tile;
  info->pair_form = P.pair_form ? 1 : 0;
  info->leaf_form = P.leaf_form;
  info->error_bound = fmm::error_bound(P.levels > 0 ? P.lv_alg : std::vector<int>(), P.k, P.dtype);
  return FMM_OK;
}

fmm_status fmm_plan_destroy(fmm_plan_t p) {
  if (!p) return FMM_OK;
  fmm::Plan& P = p->P;
  fmm_status st = FMM_OK;
  if (!P.host_only) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != P.device) (void)hipSetDevice(P.device);
    drop_graph(P);
    if (P.cap_stream) (void)hipStreamDestroy((hipStream_t)P.cap_stream);
    if (!P.external) {
      if (P.ws && hipFree(P.ws) != hipSuccess) st = fail(FMM_EHIP, "hipFree of the workspace failed");
      if (P.dev_table && hipFree(P.dev_table) != hipSuccess) st = fail(FMM_EHIP, "hipFree of the table failed");
    }
    for (void* ev : P.events) (void)hipEventDestroy((hipEvent_t)ev);
    if (prev != P.device && prev >= 0) (void)hipSetDevice(prev);
  }
  delete p;
  return st;
}

fmm_status fmm_gemm(int dtype, int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                    const void* B, int64_t ldb, void* C, int64_t ldc, void* stream) {
  if (m < 0 || k < 0 || n < 0) return fail(FMM_EINVAL, "sizes must be non-negative");
  if (dtype < 0 || dtype > 2) return fail(FMM_EINVAL, "unknown dtype");
  if (dtype == FMM_F32_BF16X3 && !fmm::kHaveBf16x3)
    return fail(FMM_EUNSUPPORTED, "BF16x3 leaves are not compiled into this library");
  fmm::Plan P;
  P.m = m;
  P.k = k;
  P.n = n;
  P.dtype = dtype;
  P.elt = dtype == 0 ? fmm::ELT_F64 : fmm::ELT_F32;
  fmm_status st = validate(P, A, lda, B, ldb, C, ldc);
  if (st != FMM_OK) return st;
  if (m == 0 || n == 0) return FMM_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  fmm::GemmArgs a;
  std::memset(&a, 0, sizeof(a));
  a.bases[0] = make_bases(P, A, lda, B, ldb, C, ldc);
  a.single.a = fmm::Ref{fmm::BUF_A, P.elt, 0, 0, 0, 0, 1.0};
  a.single.b = fmm::Ref{fmm::BUF_B, P.elt, 0, 0, 0, 0, 1.0};
  a.single.c = fmm::Ref{fmm::BUF_C, P.elt, 0, 0, 0, 0, 1.0};
  a.single.alpha = 1.0;
  a.ngroups = 1;
  a.elt = P.elt;
  fmm::GemmGroup& g = a.groups[0];
  g.m = m;
  g.n = n;
  g.k = k;
  g.count = 1;
  g.tiles_m = (m + fmm::kTileM - 1) / fmm::kTileM;
  g.tiles_n = (n + fmm::kTileN - 1) / fmm::kTileN;
  g.tile_start = 0;
  g.prob_start = 0;
  g.probs = nullptr;
  g.slot = 0;
  a.total_tiles = g.tiles_m * g.tiles_n;
  {
    const int e = dtype == 0 ? 2 : 4;
    a.dma = dtype != 2 && n % e == 0 && k % e == 0 && ref_dma_ok(a.single.a, a.bases[0], nullptr, e) &&
            ref_dma_ok(a.single.b, a.bases[0], nullptr, e);
  }
  hipError_t e = fmm::launch_gemm(a, dtype, num_cus(dev), (hipStream_t)stream);
  return e == hipSuccess ? FMM_OK : hip_fail(e, "kernel launch");
}

int fmm_num_algorithms(void) { return fmm::kNumAlgorithms; }

const char* fmm_algorithm_name(int index) {
  if (index < 0 || index >= fmm::kNumAlgorithms) return nullptr;
  return fmm::alg_info(index).name;
}

fmm_status fmm_algorithm_coeffs(const char* alg, int* M, int* K, int* N, int* R, int8_t* U, int8_t* V,
                                int8_t* W) {
  const int id = fmm::find_algorithm(alg);
  if (id < 0) return fail(FMM_EALG, std::string("unknown algorithm '") + (alg ? alg : "(null)") + "'");
  const fmm::AlgInfo& a = fmm::alg_info(id);
  if (M) *M = a.M;
  if (K) *K = a.K;
  if (N) *N = a.N;
  if (R) *R = a.R;
  if (U) std::memcpy(U, a.U, (size_t)a.M * a.K * a.R);
  if (V) std::memcpy(V, a.V, (size_t)a.K * a.N * a.R);
  if (W) std::memcpy(W, a.W, (size_t)a.M * a.N * a.R);
  return FMM_OK;
}

fmm_status fmm_check_algorithms(void) {
  std::string why;
  for (int i = 0; i < fmm::kNumAlgorithms; ++i)
    if (!brent_ok(fmm::alg_info(i), &why)) return fail(FMM_EALG, why);
  return FMM_OK;
}

fmm_status fmm_rank_candidates(int64_t m, int64_t k, int64_t n, int dtype, const char* alg,
                               size_t budget_bytes, double max_error, fmm_candidate_t* out, int max,
                               int* count) {
  if (count) *count = 0;
  if (max < 0 || (max > 0 && !out)) return fail(FMM_EINVAL, "bad output array");
  fmm_status st = check_tables_once();
  if (st != FMM_OK) return st;
  std::vector<fmm::Candidate> cands;
  std::string why = fmm::rank_candidates(m, k, n, dtype, alg, budget_bytes, 0, max_error, cands);
  if (!why.empty()) return fail(why.rfind("unknown algorithm", 0) == 0 ? FMM_EALG : FMM_EINVAL, why);
  const int nout = std::min<int>(max, (int)cands.size());
  for (int i = 0; i < nout; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::snprintf(out[i].alg, sizeof(out[i].alg), "%s", cands[i].alg);
    out[i].levels = cands[i].levels;
    out[i].fuse_levels = cands[i].fuse;
    out[i].leaf_tile = cands[i].tile;
    out[i].model_ms = cands[i].model_ms;
    out[i].leaf_ms = cands[i].leaf_ms;
    out[i].add_ms = cands[i].add_ms;
    out[i].workspace_bytes = cands[i].ws_bytes;
    out[i].error_bound = cands[i].err;
  }
  if (count) *count = nout;
  return FMM_OK;
}

fmm_status fmm_tune_record(int64_t m, int64_t k, int64_t n, int dtype, const char* alg, int levels,
                           int fuse_levels, int leaf_tile) {
  if (m < 0 || k < 0 || n < 0) return fail(FMM_EINVAL, "sizes must be non-negative");
  if (dtype < 0 || dtype > 2) return fail(FMM_EINVAL, "unknown dtype");
  if (!alg) return fail(FMM_EINVAL, "alg is NULL");
  if (std::strlen(alg) >= sizeof(fmm::Candidate::alg)) return fail(FMM_EINVAL, "algorithm name too long");
  {
    std::vector<int> ids;
    std::string err;
    const int pr = fmm::parse_levels(alg, levels, &ids, &err);
    if (pr > 0) return fail((fmm_status)pr, err);
  }
  if (levels < 0 || fuse_levels < 0 || fuse_levels > 2) return fail(FMM_EINVAL, "bad levels or fuse_levels");
  if (leaf_tile != 0 && leaf_tile != 64 && leaf_tile != 128 && !(leaf_tile == 256 && dtype == FMM_F32_BF16X3))
    return fail(FMM_EINVAL, "leaf_tile must be 0, 64 or 128 (or 256 on the BF16x3 path)");
  fmm::Plan P;
  int code = 0;
  std::string err = fmm::make_plan(P, alg, m, k, n, levels, dtype, fuse_levels, &code);
  if (!err.empty()) return fail((fmm_status)code, err);
  fmm::Candidate c;
  std::snprintf(c.alg, sizeof(c.alg), "%s", alg);
  c.levels = levels;
  c.fuse = fuse_levels;
  c.tile = leaf_tile;
  fmm::record_tuned(m, k, n, dtype, c);
  return FMM_OK;
}

fmm_status fmm_tune_clear(void) {
  fmm::clear_tuned();
  return FMM_OK;
}

const char* fmm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
