// Serving runtime: a request queue with continuous batching in front of
// fmm_multiply_batched.
//
// Batches run on one to four HIP streams ("lanes", all of the default
// priority).  With one lane every request shares it.  With more, lane 0 runs
// the large requests (2mkn >= large_flops), one per batch: such a request
// fills the device by itself, and batching it would hold every request of the
// batch until the largest is done; the other lanes run the small requests,
// each batch on the small lane with the fewest batches in flight, so a small
// arrival never queues behind a large product and its kernels are dispatched
// alongside the large one's workgroups as those retire.
//
// Small requests are admitted first come, first served; large ones shortest
// first (fewest flops), except that one waiting over 100 ms goes first.  A
// request is admitted when its plan's device bytes (workspace + descriptor
// tables) fit the arena; the batch being built closes when it reaches its
// size limit or the next request of its class does not fit.  At most
// max_inflight batches are enqueued per lane, so the host plans the next
// batches while the device runs the current ones.  Each batch ends with one
// HIP event on its lane; when it has completed, the batch's arena ranges are
// freed and its requests are reported.  Plans own their workspaces and take
// their kernel arguments by value, so batches on different lanes share no
// device memory.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <string>
#include <thread>
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

struct Lane {
  hipStream_t stream = nullptr;
  bool own = false;
  std::deque<Batch> inflight;  // in launch order
};

}  // namespace

struct fmm_server_s {
  fmm_server_options_t opt;
  int device = 0;
  std::vector<Lane> lanes;
  hipStream_t cap_stream = nullptr;  // records batch graphs (use_graph); never runs work
  char* arena_mem = nullptr;
  Arena arena;
  std::deque<Queued> queue;
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
              int batch, const std::string& alg, int levels, int lane = -1) {
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
  c.lane = lane;
  S.ready.push_back(c);
  --S.pending;
}

void finish_batch(fmm_server_s& S, Batch& b, fmm_status st, int lane) {
  if (b.exec) {
    (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
  }
  for (Admitted& a : b.reqs) {
    S.arena.release(a.off, a.bytes);
    (void)fmm_plan_destroy(a.plan);
    complete(S, a.id, a.r.user, st, a.submit_ms, b.launch_ms, (int)b.reqs.size(), a.alg, a.levels, lane);
  }
  S.spare_events.push_back(b.ev);
}

// Retires the completed batches at the front of one lane, in launch order.
fmm_status retire_lane(fmm_server_s& S, int li) {
  Lane& L = S.lanes[li];
  while (!L.inflight.empty()) {
    Batch& b = L.inflight.front();
    const hipError_t e = hipEventQuery(b.ev);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) {
      finish_batch(S, b, FMM_EHIP, li);
      L.inflight.pop_front();
      return fail(FMM_EHIP, std::string("batch completion: ") + hipGetErrorString(e));
    }
    finish_batch(S, b, FMM_OK, li);
    L.inflight.pop_front();
  }
  return FMM_OK;
}

// Retires completed batches of every lane; with block, first waits until
// some batch has completed (if any is in flight).  Waiting on one lane's
// event would miss an earlier completion on another, so with several busy
// lanes the wait polls their oldest batches.
fmm_status retire(fmm_server_s& S, bool block) {
  if (block) {
    int busy = -1, nbusy = 0;
    for (int li = 0; li < (int)S.lanes.size(); ++li)
      if (!S.lanes[li].inflight.empty()) busy = li, ++nbusy;
    if (nbusy == 1) {
      const hipError_t e = hipEventSynchronize(S.lanes[busy].inflight.front().ev);
      if (e != hipSuccess) {
        Lane& L = S.lanes[busy];
        finish_batch(S, L.inflight.front(), FMM_EHIP, busy);
        L.inflight.pop_front();
        return fail(FMM_EHIP, std::string("batch completion: ") + hipGetErrorString(e));
      }
    } else if (nbusy > 1) {
      for (bool done = false; !done;) {
        for (const Lane& L : S.lanes)
          if (!L.inflight.empty() && hipEventQuery(L.inflight.front().ev) != hipErrorNotReady) done = true;
        if (!done) std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  }
  for (int li = 0; li < (int)S.lanes.size(); ++li) {
    const fmm_status st = retire_lane(S, li);
    if (st != FMM_OK) return st;
  }
  return FMM_OK;
}

// use_graph: records the batch's launches (kernels only: the descriptor
// tables were uploaded when the plans were bound) on the capture stream,
// instantiates the graph and launches it on the server's stream.  Every
// batch holds other requests, so each is instantiated once; the executable
// graph lives until the batch's completion event has been seen.
fmm_status launch_graph(fmm_server_s& S, hipStream_t stream, Batch& b, std::vector<fmm_plan_t>& plans,
                        std::vector<const void*>& A,
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
  e = hipGraphLaunch(b.exec, stream);
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

bool is_large(const fmm_server_s& S, const fmm_request_t& r) {
  return S.lanes.size() > 1 && 2.0 * (double)r.m * (double)r.k * (double)r.n >= S.opt.large_flops;
}

// The lane a batch of the class goes to (-1: every lane of the class is full).
int pick_lane(const fmm_server_s& S, bool large) {
  const int nl = (int)S.lanes.size();
  if (nl == 1 || large) return (int)S.lanes[0].inflight.size() < S.opt.max_inflight ? 0 : -1;
  int best = -1;
  for (int li = 1; li < nl; ++li) {
    const int f = (int)S.lanes[li].inflight.size();
    if (f < S.opt.max_inflight && (best < 0 || f < (int)S.lanes[best].inflight.size())) best = li;
  }
  return best;
}

enum class Take { kAdmitted, kDropped, kBlocked };

// Plans the queued request at `it` (once), reserves its arena range, orders
// lane L after the request's stream and binds the plan; the request then
// leaves the queue for batch b.  A request that can never run completes
// with its error and leaves the queue (kDropped); one that does not fit the
// arena now stays (kBlocked).
Take take_one(fmm_server_s& S, Lane& L, std::deque<Queued>::iterator it, Batch& b) {
  Queued& q = *it;
  auto drop = [&](fmm_status code, bool had_plan) {
    if (had_plan) (void)fmm_plan_destroy(q.plan);
    drop_ready(S, q);
    complete(S, q.id, q.r.user, code, q.submit_ms, S.now_ms(), 0, q.alg, q.levels);
    S.queue.erase(it);
    return Take::kDropped;
  };
  if (!q.plan) {
    fmm_plan_options_t o;
    std::memset(&o, 0, sizeof(o));
    o.fuse_levels = S.opt.fuse_levels;
    o.defer_device_memory = 1;
    const fmm_status pst = fmm_plan_ex(&q.plan, q.alg.c_str(), q.r.m, q.r.k, q.r.n, q.levels, q.r.dtype, &o);
    if (pst != FMM_OK) {
      q.plan = nullptr;
      return drop(pst, false);
    }
  }
  const size_t bytes = fmm_plan_device_bytes(q.plan);
  if (bytes > S.opt.arena_bytes) return drop(FMM_ENOMEM, true);
  size_t off = 0;
  if (!S.arena.alloc(bytes, &off)) return Take::kBlocked;
  // the batch runs after the work the request's stream had enqueued at submit
  if (q.ready) {
    const hipError_t we = hipStreamWaitEvent(L.stream, q.ready, 0);
    if (we != hipSuccess) {
      S.arena.release(off, bytes);
      return drop(FMM_EHIP, true);
    }
    drop_ready(S, q);
  }
  const fmm_status bst = fmm_plan_bind(q.plan, S.arena_mem + off, bytes, L.stream);
  if (bst != FMM_OK) {
    S.arena.release(off, bytes);
    return drop(bst, true);
  }
  b.reqs.push_back(Admitted{q.id, q.r, q.alg, q.levels, q.submit_ms, q.plan, off, bytes});
  S.queue.erase(it);
  return Take::kAdmitted;
}

// The large request to run next: the one with the fewest flops (shortest
// first keeps the many medium-large requests from waiting behind the
// largest), except that requests waiting longer than kLargeMaxWaitMs go
// first, oldest first, so none waits without bound.
constexpr double kLargeMaxWaitMs = 100.0;
std::deque<Queued>::iterator pick_large(fmm_server_s& S) {
  const double now = S.now_ms();
  auto best = S.queue.end();
  bool best_aged = false;
  double best_flops = 0;
  for (auto it = S.queue.begin(); it != S.queue.end(); ++it) {
    if (!is_large(S, it->r)) continue;
    const bool aged = now - it->submit_ms > kLargeMaxWaitMs;
    const double fl = (double)it->r.m * (double)it->r.k * (double)it->r.n;
    if (best == S.queue.end() || (aged && !best_aged) || (!best_aged && !aged && fl < best_flops)) {
      best = it;
      best_aged = aged;
      best_flops = fl;
    }
    // among aged requests the first met (the oldest) stays
  }
  return best;
}

// Builds one batch of the class on lane li and launches it: small requests
// in arrival order, up to max_batch of them; large requests one per batch,
// by pick_large.  Returns the number of requests taken off the queue
// (admitted or completed with an error); *st is set on a failure of the
// server itself.
int admit_batch(fmm_server_s& S, bool large, int li, fmm_status* st) {
  *st = FMM_OK;
  Lane& L = S.lanes[li];
  Batch b;
  int taken = 0;
  if (large) {
    for (;;) {
      auto it = pick_large(S);
      if (it == S.queue.end()) break;
      const Take t = take_one(S, L, it, b);
      if (t == Take::kBlocked) break;  // waits for arena space
      ++taken;
      if (t == Take::kAdmitted) break;
    }
  } else {
    for (auto it = S.queue.begin(); it != S.queue.end() && (int)b.reqs.size() < S.opt.max_batch;) {
      if (S.lanes.size() > 1 && is_large(S, it->r)) {
        ++it;
        continue;
      }
      const auto next = std::next(it);
      const bool last = next == S.queue.end();
      const int64_t next_id = last ? -1 : next->id;
      const Take t = take_one(S, L, it, b);
      if (t == Take::kBlocked) break;  // first come, first served: wait for arena space
      ++taken;
      // take_one erased `it`; continue from the request that followed it
      if (last) break;
      it = S.queue.begin();
      while (it != S.queue.end() && it->id != next_id) ++it;
    }
  }
  if (b.reqs.empty()) return taken;
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
  if ((*st = take_event(S, &b.ev)) != FMM_OK) {
    // nothing was launched: give the ranges back and report the requests
    b.ev = nullptr;
    for (Admitted& a : b.reqs) {
      S.arena.release(a.off, a.bytes);
      (void)fmm_plan_destroy(a.plan);
      complete(S, a.id, a.r.user, *st, a.submit_ms, S.now_ms(), 0, a.alg, a.levels);
    }
    return taken;
  }
  b.launch_ms = S.now_ms();
  const fmm_status lst = S.opt.use_graph
                             ? launch_graph(S, L.stream, b, plans, A, lda, B, ldb, C, ldc)
                             : fmm_multiply_batched(plans.data(), A.data(), lda.data(), B.data(), ldb.data(),
                                                    C.data(), ldc.data(), (int)nb, L.stream);
  const hipError_t e = hipEventRecord(b.ev, L.stream);
  if (lst != FMM_OK || e != hipSuccess) {
    // nothing of the batch may still read the arena when its ranges are reused
    (void)hipStreamSynchronize(L.stream);
    finish_batch(S, b, lst != FMM_OK ? lst : FMM_EHIP, li);
    return taken;
  }
  L.inflight.push_back(std::move(b));
  return taken;
}

// Admits and launches batches while a lane has room and its class has
// requests waiting that fit.
fmm_status admit(fmm_server_s& S) {
  for (bool progressed = true; progressed && !S.queue.empty();) {
    progressed = false;
    for (const bool large : {true, false}) {
      if (S.lanes.size() == 1 && large) continue;  // one lane: a single class
      const int li = pick_lane(S, large);
      if (li < 0) continue;
      fmm_status st;
      if (admit_batch(S, large, li, &st) > 0) progressed = true;
      if (st != FMM_OK) return st;
    }
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
  if (opts->num_streams < 0 || opts->num_streams > 4) return fail(FMM_EINVAL, "num_streams must be in [0, 4]");
  if (!(opts->large_flops >= 0)) return fail(FMM_EINVAL, "large_flops must be >= 0");
  fmm_server_s* S = new fmm_server_s();
  S->opt = *opts;
  if (S->opt.num_streams == 0) S->opt.num_streams = 1;
  if (S->opt.large_flops == 0) S->opt.large_flops = FMM_SERVER_LARGE_FLOPS;
  S->t0 = std::chrono::steady_clock::now();
  auto undo = [&](fmm_status code, const std::string& msg) {
    for (Lane& L : S->lanes)
      if (L.own) (void)hipStreamDestroy(L.stream);
    delete S;
    return fail(code, msg);
  };
  hipError_t e = hipGetDevice(&S->device);
  if (e != hipSuccess) return undo(FMM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (S->opt.arena_bytes == 0) {
    // the device's free memory, less a reserve for the callers' operands
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return undo(FMM_EHIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
    const size_t reserve = (size_t)FMM_SERVER_RESERVE_BYTES;
    if (free_b <= reserve) return undo(FMM_ENOMEM, "less free device memory than the arena's reserve");
    S->opt.arena_bytes = free_b - reserve;
  }
  S->lanes.resize((size_t)S->opt.num_streams);
  for (int li = 0; li < S->opt.num_streams; ++li) {
    Lane& L = S->lanes[li];
    if (li == 0 && stream) {
      L.stream = (hipStream_t)stream;
      continue;
    }
    // default priority, as every stream of this library
    e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e != hipSuccess) return undo(FMM_EHIP, std::string("server stream: ") + hipGetErrorString(e));
    L.own = true;
  }
  e = hipMalloc((void**)&S->arena_mem, S->opt.arena_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return undo(FMM_ENOMEM, "hipMalloc of the serving arena failed");
  }
  S->arena.reset(S->opt.arena_bytes);
  *out = S;
  return FMM_OK;
}

size_t fmm_server_arena_bytes(fmm_server_t s) { return s ? s->opt.arena_bytes : 0; }

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
  const bool small = 2.0 * (double)r.m * (double)r.k * (double)r.n < s->opt.large_flops;
  if (auto_alg && r.levels < 0 && small && !s->opt.small_model) {
    // A small request joins a batch whose leaves share grouped launches; a
    // fast plan would add its own formation and combination launches to the
    // batch's stream, which costs more than the leaf flops it saves there.
    q.alg = "classical";
    q.levels = 0;
  } else if (auto_alg || r.levels < 0) {
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
  // (with one lane a request on the server's own stream is ordered already)
  if (r.wait_stream && !(s->lanes.size() == 1 && (hipStream_t)r.stream == s->lanes[0].stream)) {
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
  bool busy = false;
  for (const Lane& L : s->lanes) busy = busy || !L.inflight.empty();
  if (st == FMM_OK && wait && s->ready.empty() && busy) {
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
  for (Lane& L : s->lanes) {
    (void)hipStreamSynchronize(L.stream);
    for (Batch& b : L.inflight) {
      for (Admitted& a : b.reqs) (void)fmm_plan_destroy(a.plan);
      (void)hipEventDestroy(b.ev);
      if (b.exec) (void)hipGraphExecDestroy(b.exec);
    }
  }
  for (Queued& q : s->queue) {
    if (q.plan) (void)fmm_plan_destroy(q.plan);
    if (q.ready) (void)hipEventDestroy(q.ready);
  }
  for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  for (Lane& L : s->lanes)
    if (L.own) (void)hipStreamDestroy(L.stream);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (prev != s->device && prev >= 0) (void)hipSetDevice(prev);
  delete s;
  return FMM_OK;
}

}  // extern "C"
