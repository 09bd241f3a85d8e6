// Serving runtime: a request queue with continuous batching in front of
// fmm_multiply_batched.
//
// Admission is first come, first served.  A request is admitted when its
// plan's device bytes (workspace + descriptor tables) fit the arena; the
// batch being built closes when it reaches max_batch requests or the head of
// the queue does not fit.  At most max_inflight batches are enqueued at once,
// so the host plans batch b+1 while the device runs batch b.  Each batch ends
// with one HIP event; when it has completed, the batch's arena ranges are
// freed and its requests are reported.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_internal.h"

namespace {

// First-fit allocator over [0, size) in 256-byte units, coalescing on free.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
    if (!bytes) bytes = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    if (!bytes) bytes = 256;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Queued {
  int64_t id;
  fmm_request_t r;
  std::string alg;  // chosen base case (after the model, if asked)
  int levels;
  double submit_ms;
  fmm_plan_t plan = nullptr;  // made once, kept while the request waits for room
  hipEvent_t ready = nullptr; // recorded on the request's stream at submit (NULL: none)
};

struct Admitted {
  int64_t id;
  fmm_request_t r;
  std::string alg;
  int levels;
  double submit_ms;
  fmm_plan_t plan;
  size_t off, bytes;
};

struct Batch {
  hipEvent_t ev;
  double launch_ms;
  std::vector<Admitted> reqs;
  hipGraphExec_t exec = nullptr;  // the batch's graph (use_graph), freed when it completes
};

}  // namespace

struct fmm_server_s {
  fmm_server_options_t opt;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap_stream = nullptr;  // records batch graphs (use_graph); never runs work
  char* arena_mem = nullptr;
  Arena arena;
  std::deque<Queued> queue;
  std::deque<Batch> inflight;
  std::vector<hipEvent_t> spare_events;
  std::deque<fmm_completion_t> ready;
  int64_t next_id = 0;
  int64_t pending = 0;
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

fmm_status fail(fmm_status code, const std::string& msg) { return (fmm_status)fmm::set_error(code, msg); }

void complete(fmm_server_s& S, int64_t id, void* user, fmm_status st, double submit_ms, double launch_ms,
              int batch, const std::string& alg, int levels) {
  fmm_completion_t c;
  std::memset(&c, 0, sizeof(c));
  c.id = id;
  c.user = user;
  c.status = st;
  c.submit_ms = submit_ms;
  c.launch_ms = launch_ms;
  c.done_ms = S.now_ms();
  c.batch_size = batch;
  std::snprintf(c.alg, sizeof(c.alg), "%s", alg.c_str());
  c.levels = levels;
  S.ready.push_back(c);
  --S.pending;
}

void finish_batch(fmm_server_s& S, Batch& b, fmm_status st) {
  if (b.exec) {
    (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
  }
  for (Admitted& a : b.reqs) {
    S.arena.release(a.off, a.bytes);
    (void)fmm_plan_destroy(a.plan);
    complete(S, a.id, a.r.user, st, a.submit_ms, b.launch_ms, (int)b.reqs.size(), a.alg, a.levels);
  }
  S.spare_events.push_back(b.ev);
}

// Retires completed batches in order; with block, waits for the oldest.
fmm_status retire(fmm_server_s& S, bool block) {
  while (!S.inflight.empty()) {
    Batch& b = S.inflight.front();
    hipError_t e = block ? hipEventSynchronize(b.ev) : hipEventQuery(b.ev);
    if (e == hipErrorNotReady) break;
    block = false;
    if (e != hipSuccess) {
      finish_batch(S, b, FMM_EHIP);
      S.inflight.pop_front();
      return fail(FMM_EHIP, std::string("batch completion: ") + hipGetErrorString(e));
    }
    finish_batch(S, b, FMM_OK);
    S.inflight.pop_front();
  }
  return FMM_OK;
}

// use_graph: records the batch's launches (kernels only: the descriptor
// tables were uploaded when the plans were bound) on the capture stream,
// instantiates the graph and launches it on the server's stream.  Every
// batch holds other requests, so each is instantiated once; the executable
// graph lives until the batch's completion event has been seen.
fmm_status launch_graph(fmm_server_s& S, Batch& b, std::vector<fmm_plan_t>& plans, std::vector<const void*>& A,
                        std::vector<int64_t>& lda, std::vector<const void*>& B, std::vector<int64_t>& ldb,
                        std::vector<void*>& C, std::vector<int64_t>& ldc) {
  hipError_t e;
  if (!S.cap_stream) {
    e = hipStreamCreateWithFlags(&S.cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(FMM_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  }
  e = hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail(FMM_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  const fmm_status st = fmm_multiply_batched(plans.data(), A.data(), lda.data(), B.data(), ldb.data(), C.data(),
                                             ldc.data(), (int)plans.size(), S.cap_stream);
  const std::string err = st != FMM_OK ? std::string(fmm_last_error()) : std::string();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(S.cap_stream, &g);
  if (st != FMM_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != FMM_OK ? fail(st, err) : fail(FMM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b.exec = nullptr;
    return fail(FMM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  e = hipGraphLaunch(b.exec, S.stream);
  if (e != hipSuccess) return fail(FMM_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return FMM_OK;
}

// An event of the server's pool (created when the pool is empty).
fmm_status take_event(fmm_server_s& S, hipEvent_t* ev) {
  if (S.spare_events.empty()) {
    hipEvent_t e0;
    hipError_t e = hipEventCreateWithFlags(&e0, hipEventDisableTiming);
    if (e != hipSuccess) return fail(FMM_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    S.spare_events.push_back(e0);
  }
  *ev = S.spare_events.back();
  S.spare_events.pop_back();
  return FMM_OK;
}

// Returns a queued request's stream event to the pool (a wait on it that was
// already enqueued keeps the state the event had then).
void drop_ready(fmm_server_s& S, Queued& q) {
  if (q.ready) S.spare_events.push_back(q.ready);
  q.ready = nullptr;
}

// Admits and launches batches while there is room.
fmm_status admit(fmm_server_s& S) {
  const size_t arena_bytes = S.opt.arena_bytes;
  while ((int)S.inflight.size() < S.opt.max_inflight && !S.queue.empty()) {
    Batch b;
    bool blocked = false;
    while (!S.queue.empty() && (int)b.reqs.size() < S.opt.max_batch && !blocked) {
      Queued& q = S.queue.front();
      if (!q.plan) {
        fmm_plan_options_t o;
        std::memset(&o, 0, sizeof(o));
        o.fuse_levels = S.opt.fuse_levels;
        o.defer_device_memory = 1;
        fmm_status st = fmm_plan_ex(&q.plan, q.alg.c_str(), q.r.m, q.r.k, q.r.n, q.levels, q.r.dtype, &o);
        if (st != FMM_OK) {
          drop_ready(S, q);
          complete(S, q.id, q.r.user, st, q.submit_ms, S.now_ms(), 0, q.alg, q.levels);
          S.queue.pop_front();
          continue;
        }
      }
      const size_t bytes = fmm_plan_device_bytes(q.plan);
      if (bytes > arena_bytes) {
        (void)fmm_plan_destroy(q.plan);
        drop_ready(S, q);
        complete(S, q.id, q.r.user, FMM_ENOMEM, q.submit_ms, S.now_ms(), 0, q.alg, q.levels);
        S.queue.pop_front();
        continue;
      }
      size_t off = 0;
      if (!S.arena.alloc(bytes, &off)) {
        blocked = true;  // first come, first served: wait for arena space
        break;
      }
      // the batch runs after the work the request's stream had enqueued at submit
      if (q.ready) {
        hipError_t we = hipStreamWaitEvent(S.stream, q.ready, 0);
        drop_ready(S, q);
        if (we != hipSuccess) {
          (void)fmm_plan_destroy(q.plan);
          complete(S, q.id, q.r.user, FMM_EHIP, q.submit_ms, S.now_ms(), 0, q.alg, q.levels);
          S.queue.pop_front();
          continue;
        }
      }
      fmm_status st = fmm_plan_bind(q.plan, S.arena_mem + off, bytes, S.stream);
      if (st != FMM_OK) {
        S.arena.release(off, bytes);
        (void)fmm_plan_destroy(q.plan);
        complete(S, q.id, q.r.user, st, q.submit_ms, S.now_ms(), 0, q.alg, q.levels);
        S.queue.pop_front();
        continue;
      }
      b.reqs.push_back(Admitted{q.id, q.r, q.alg, q.levels, q.submit_ms, q.plan, off, bytes});
      S.queue.pop_front();
    }
    if (b.reqs.empty()) break;
    const size_t nb = b.reqs.size();
    std::vector<fmm_plan_t> plans(nb);
    std::vector<const void*> A(nb), B(nb);
    std::vector<void*> C(nb);
    std::vector<int64_t> lda(nb), ldb(nb), ldc(nb);
    for (size_t i = 0; i < nb; ++i) {
      const fmm_request_t& r = b.reqs[i].r;
      plans[i] = b.reqs[i].plan;
      A[i] = r.A;
      B[i] = r.B;
      C[i] = r.C;
      lda[i] = r.lda;
      ldb[i] = r.ldb;
      ldc[i] = r.ldc;
    }
    {
      const fmm_status est = take_event(S, &b.ev);
      if (est != FMM_OK) return est;
    }
    b.launch_ms = S.now_ms();
    fmm_status st = S.opt.use_graph
                        ? launch_graph(S, b, plans, A, lda, B, ldb, C, ldc)
                        : fmm_multiply_batched(plans.data(), A.data(), lda.data(), B.data(), ldb.data(), C.data(),
                                               ldc.data(), (int)nb, S.stream);
    hipError_t e = hipEventRecord(b.ev, S.stream);
    if (st != FMM_OK || e != hipSuccess) {
      // nothing of the batch may still read the arena when its ranges are reused
      (void)hipStreamSynchronize(S.stream);
      finish_batch(S, b, st != FMM_OK ? st : FMM_EHIP);
      continue;
    }
    S.inflight.push_back(std::move(b));
  }
  return FMM_OK;
}

}  // namespace

extern "C" {

fmm_status fmm_server_create(fmm_server_t* out, const fmm_server_options_t* opts, void* stream) {
  if (!out) return fail(FMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!opts) return fail(FMM_EINVAL, "opts is NULL");
  if (opts->max_batch < 1 || opts->max_batch > 64) return fail(FMM_EINVAL, "max_batch must be in [1, 64]");
  if (opts->max_inflight < 1) return fail(FMM_EINVAL, "max_inflight must be >= 1");
  if (opts->arena_bytes == 0) return fail(FMM_EINVAL, "arena_bytes must be > 0");
  fmm_server_s* S = new fmm_server_s();
  S->opt = *opts;
  S->t0 = std::chrono::steady_clock::now();
  hipError_t e = hipGetDevice(&S->device);
  if (e == hipSuccess && !stream) {
    e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    S->own_stream = e == hipSuccess;
  } else {
    S->stream = (hipStream_t)stream;
  }
  if (e != hipSuccess) {
    delete S;
    return fail(FMM_EHIP, std::string("server stream: ") + hipGetErrorString(e));
  }
  e = hipMalloc((void**)&S->arena_mem, opts->arena_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(FMM_ENOMEM, "hipMalloc of the serving arena failed");
  }
  S->arena.reset(opts->arena_bytes);
  *out = S;
  return FMM_OK;
}

fmm_status fmm_server_submit(fmm_server_t s, const fmm_request_t* req, int64_t* id) {
  if (!s || !req) return fail(FMM_EINVAL, "NULL argument");
  const fmm_request_t& r = *req;
  if (r.m < 0 || r.k < 0 || r.n < 0) return fail(FMM_EINVAL, "sizes must be non-negative");
  if (r.dtype < 0 || r.dtype > 2) return fail(FMM_EINVAL, "unknown dtype");
  {
    // the checks fmm_multiply_batched makes, per request: a request that
    // would fail them is refused here and never makes its batch fail
    std::string why;
    const int st = fmm::check_operands(r.m, r.k, r.n, r.dtype == FMM_F64 ? 8 : 4, r.A, r.lda, r.B, r.ldb, r.C,
                                       r.ldc, &why);
    if (st) return fail((fmm_status)st, why);
  }
  Queued q;
  q.r = r;
  q.submit_ms = s->now_ms();
  const bool auto_alg = !r.alg || !std::strcmp(r.alg, "auto");
  if (auto_alg || r.levels < 0) {
    // a measured choice for the exact shape if one was recorded, else the model
    fmm::Candidate pick;
    std::string why;
    if (!fmm::choose(r.m, r.k, r.n, r.dtype, auto_alg ? nullptr : r.alg, r.levels, s->opt.arena_bytes,
                     s->opt.fuse_levels, s->opt.max_error[r.dtype], &pick, &why))
      return fail(why.rfind("no candidate", 0) == 0 ? FMM_ENOMEM : FMM_EINVAL, why);
    q.alg = pick.alg;
    q.levels = pick.levels;
  } else {
    q.alg = r.alg;
    q.levels = r.levels;
  }
  if (r.wait_stream && (hipStream_t)r.stream != s->stream) {
    fmm_status est = take_event(*s, &q.ready);
    if (est != FMM_OK) return est;
    hipError_t e = hipEventRecord(q.ready, (hipStream_t)r.stream);
    if (e != hipSuccess) {
      drop_ready(*s, q);
      return fail(FMM_EHIP, std::string("hipEventRecord on the request's stream: ") + hipGetErrorString(e));
    }
  }
  q.id = s->next_id++;
  s->queue.push_back(q);
  ++s->pending;
  if (id) *id = q.id;
  return FMM_OK;
}

fmm_status fmm_server_progress(fmm_server_t s, int wait, fmm_completion_t* done, int max_done,
                               int* num_done) {
  if (num_done) *num_done = 0;
  if (!s) return fail(FMM_EINVAL, "server is NULL");
  if (max_done < 0 || (max_done > 0 && !done)) return fail(FMM_EINVAL, "bad completion array");
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != s->device) (void)hipSetDevice(s->device);
  fmm_status st = retire(*s, false);
  if (st == FMM_OK) st = admit(*s);
  if (st == FMM_OK && wait && s->ready.empty() && !s->inflight.empty()) {
    st = retire(*s, true);
    if (st == FMM_OK) st = admit(*s);
  }
  if (prev != s->device && prev >= 0) (void)hipSetDevice(prev);
  int n = 0;
  while (n < max_done && !s->ready.empty()) {
    done[n++] = s->ready.front();
    s->ready.pop_front();
  }
  if (num_done) *num_done = n;
  return st;
}

int64_t fmm_server_pending(fmm_server_t s) { return s ? s->pending + (int64_t)s->ready.size() : 0; }

fmm_status fmm_server_destroy(fmm_server_t s) {
  if (!s) return FMM_OK;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != s->device) (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  for (Batch& b : s->inflight) {
    for (Admitted& a : b.reqs) (void)fmm_plan_destroy(a.plan);
    (void)hipEventDestroy(b.ev);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
  }
  for (Queued& q : s->queue) {
    if (q.plan) (void)fmm_plan_destroy(q.plan);
    if (q.ready) (void)hipEventDestroy(q.ready);
  }
  for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (prev != s->device && prev >= 0) (void)hipSetDevice(prev);
  delete s;
  return FMM_OK;
}

}  // extern "C"
