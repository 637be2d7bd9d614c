// Serving loop of the MAPA allocation library: continuous batching of
// allocation requests over device-resident server state.
//
// One host thread owned by the context.  Per server, requests are answered
// first in, first out, one at a time; across servers they are batched.  Each
// device batch runs the same kernels as mapa_query_batch (kernels.hip) on its
// own stream and workspace; up to two batches are in flight, so requests that
// arrive while one batch is on the GPU join the next (continuous batching).
// The loop keeps a host mirror of every server's busy mask, updated from the
// results of its own batches and the releases it issues, which lets it answer
// requests that cannot fit (k > free accelerators) without a device batch
// and estimate each request's prefix work-list for admission.  Requests the
// batch path does not take (servers of more than 16 accelerators, or k > 8)
// join the same dispatch as a second, wide batch on the same stream
// (wide.hip's kernels on the slot's own buffers), admitted by embeddings.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <queue>
#include <thread>

#include "ctx.h"
#include "wide.h"

namespace mapa {

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  mapa_request r;
  double due_us;  // wall-clock time (since the loop started) at which it is due
  Req *next;      // next request of the same server's queue
};

struct Held {
  double t_us;
  int64_t handle;
};
struct HeldLater {
  bool operator()(const Held &a, const Held &b) const { return a.t_us > b.t_us; }
};

struct Slot {
  Workspace ws;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t g0 = nullptr, g1 = nullptr;  // timing: around the batch's kernels
  bool timed = false;         // this batch records g0 / g1 (one batch in kGpuSample)
  bool stream_busy = false;   // work not yet seen complete may still read the pinned buffers
  uint64_t rel_seen = 0;      // release generation this stream is already ordered after
  mapa_query *h_q = nullptr;     // pinned
  mapa_result *h_res = nullptr;  // pinned
  int64_t *h_rel = nullptr;      // pinned, read by the release kernel in place
  size_t cap_rel = 0;
  bool active = false;
  int32_t batch_id = -1;
  double t_dispatch = 0;
  std::vector<const Req *> reqs;
  std::vector<uint32_t> busy_before;
  // the dispatch's wide batch
  std::vector<const Req *> wreqs;
  std::vector<uint32_t> wbusy_before;
  mapa_query *h_wq = nullptr;          // pinned [kServeWideMax]
  mapa_result_wide *h_wres = nullptr;  // pinned [kServeWideMax]
  void *d_wide = nullptr;              // device: queries | results | wide scratch
};

// wide requests per dispatch, and the embeddings a wide batch is admitted up
// to (a single request beyond it still runs alone; one beyond the wide
// kernels' limit is answered MAPA_RES_REFUSED on the host)
constexpr int32_t kServeWideMax = 256;
constexpr unsigned long long kServeWideLeaves = 1ull << 34;
constexpr size_t kServeWideResOff = ((size_t)kServeWideMax * sizeof(mapa_query) + 255) / 256 * 256;
constexpr size_t kServeWideScratchOff =
    kServeWideResOff + ((size_t)kServeWideMax * sizeof(mapa_result_wide) + 255) / 256 * 256;

bool is_wide(int nvert, int k) { return nvert > kMaxN || k > kMaxK; }

// one device batch in kGpuSample records timing events (mean_gpu_us)
constexpr int64_t kGpuSample = 8;

// prefix items a request would need with items of at most `leaves` embeddings
unsigned long long estimate_items(int F, int k, int leaves) {
  int d = 0;
  while (d < k - 1 && perm_leaves(F - d, k - d) > (unsigned long long)leaves) ++d;
  return perm_leaves(F, d);
}

// Per (free accelerators, k): prefix items admission counts and embeddings
// (the fused-launch test), tabulated once per loop.
struct WorkTables {
  unsigned long long items[kMaxN + 1][kMaxK + 1];
  unsigned long long leaves[kMaxN + 1][kMaxK + 1];
  void build(int item_leaves) {
    for (int F = 0; F <= kMaxN; ++F)
      for (int k = 0; k <= kMaxK; ++k) {
        items[F][k] = k >= 1 && k <= F ? estimate_items(F, k, item_leaves) : 0;
        leaves[F][k] = perm_leaves(F, k);
      }
  }
};

}  // namespace

struct ServeState {
  mapa_ctx *c = nullptr;
  mapa_serve_opts opts{};
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::vector<std::vector<Req>> incoming;  // one vector per submission, guarded by mu
  std::deque<mapa_completion> done_q;  // guarded by mu
  bool stopping = false;               // guarded by mu
  double last_arrival = -1e300;        // caller side, guarded by mu
  int64_t submitted = 0;               // guarded by mu
  double origin_us = -1;               // trace time 0 (first submission), guarded by mu
  int32_t error = MAPA_OK;
  std::string error_msg;
  Clock::time_point t0;

  // loop thread only
  std::vector<Slot> slots;
  std::vector<uint32_t> busy;  // host mirror of the device busy masks
  std::vector<int32_t> nvert;
  std::vector<uint8_t> in_flight, in_ready;
  // per server, the requests due and not yet answered, oldest first: a
  // singly linked list through Req::next (requests never move: they stay in
  // their submission's vector until the loop ends)
  std::vector<Req *> fhead, ftail;
  WorkTables work;
  std::deque<int32_t> ready;
  // every submission in arrival order (kept until the loop ends, so queued
  // requests can be referred to by address); (pend_sub, pend_pos) is the
  // first request not yet due
  std::deque<std::vector<Req>> subs;
  size_t pend_sub = 0, pend_pos = 0;

  bool pending_empty() {
    while (pend_sub < subs.size() && pend_pos >= subs[pend_sub].size()) {
      ++pend_sub;
      pend_pos = 0;
    }
    return pend_sub >= subs.size();
  }
  Req &pending_front() { return subs[pend_sub][pend_pos]; }

  bool fifo_empty(int32_t s) const { return fhead[s] == nullptr; }
  void fifo_push(int32_t s, Req *r) {
    r->next = nullptr;
    if (ftail[s])
      ftail[s]->next = r;
    else
      fhead[s] = r;
    ftail[s] = r;
  }
  void fifo_pop(int32_t s) {
    fhead[s] = fhead[s]->next;
    if (!fhead[s]) ftail[s] = nullptr;
  }
  std::priority_queue<Held, std::vector<Held>, HeldLater> held;
  std::vector<Held> deferred;  // due releases whose server has a request in flight
  std::vector<int64_t> held_forever;
  std::vector<double> lat, waits, turns;
  std::vector<mapa_completion> out_buf;  // completions of one harvest, handed over under one lock
  mapa_serve_stats st{};
  int64_t completed = 0;
  int64_t batched_queries = 0;
  int64_t fused_batches = 0;
  double batch_us_sum = 0;
  double dispatch_us_sum = 0, gpu_us_sum = 0, harvest_us_sum = 0;
  double last_done_us = 0;
  hipEvent_t rel_event = nullptr;
  uint64_t rel_gen = 0;        // releases enqueued so far (generation of rel_event)
  int rel_slot = -1;           // slot whose stream recorded rel_event
  int64_t gpu_samples = 0;
  int32_t next_batch = 0;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  }
};

namespace {

int32_t loop_fail(ServeState *S, int32_t code, const char *what, hipError_t e) {
  S->error = code;
  S->error_msg = std::string(what) + ": " + hipGetErrorString(e);
  return code;
}

#define SERVE_CHK(expr)                                                     \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) return loop_fail(S, MAPA_ERR_DEVICE, #expr, e_);  \
  } while (0)

// Record a completion; it reaches mapa_serve_poll at the next flush.
void push_completion(ServeState *S, const mapa_completion &cpl, double now) {
  S->lat.push_back(cpl.latency_us);
  S->waits.push_back(cpl.wait_us);
  S->turns.push_back(cpl.latency_us - cpl.wait_us);
  S->last_done_us = now;
  ++S->completed;
  S->out_buf.push_back(cpl);
}

void flush_completions(ServeState *S) {
  if (S->out_buf.empty()) return;
  std::lock_guard<std::mutex> lk(S->mu);
  S->done_q.insert(S->done_q.end(), S->out_buf.begin(), S->out_buf.end());
  S->out_buf.clear();
}

void make_ready(ServeState *S, int32_t s) {
  if (!S->in_flight[s] && !S->in_ready[s] && !S->fifo_empty(s)) {
    S->in_ready[s] = 1;
    S->ready.push_back(s);
  }
}

// Completed device batches -> completions, mirror updates, scheduled releases.
int32_t harvest(ServeState *S, bool *did) {
  for (auto &sl : S->slots) {
    if (!sl.active) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return loop_fail(S, MAPA_ERR_DEVICE, "batch", q);
    const double now = S->now_us();
    float gms = 0;
    if (sl.timed && hipEventElapsedTime(&gms, sl.g0, sl.g1) == hipSuccess) {
      S->gpu_us_sum += 1e3 * gms;
      ++S->gpu_samples;
    }
    sl.stream_busy = false;
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
      const mapa_result &r = sl.h_res[i];
      const Req &rq = *sl.reqs[i];
      const int32_t s = rq.r.server;
      mapa_completion cpl;
      std::memset(&cpl, 0, sizeof cpl);
      cpl.id = rq.r.id;
      cpl.count = r.count;
      cpl.alloc_handle = r.alloc_handle;
      cpl.latency_us = now - rq.due_us;
      cpl.wait_us = sl.t_dispatch - rq.due_us;
      cpl.status = r.status;
      cpl.key = r.key;
      cpl.agg = r.agg;
      cpl.pres = r.pres;
      cpl.vertex_mask = r.vertex_mask;
      cpl.busy_before = sl.busy_before[i];
      cpl.batch = sl.batch_id;
      cpl.server = s;
      std::memcpy(cpl.mapping, r.mapping, 8);
      std::memset(cpl.mapping + 8, 0xFF, 8);
      S->st.embeddings += r.count;
      if (r.status == MAPA_RES_OK && r.alloc_handle >= 0) {
        ++S->st.granted;
        S->busy[s] |= r.vertex_mask;
        if (rq.r.hold >= 0) {
          const double unit = S->opts.time_unit_us > 0 ? S->opts.time_unit_us : 1.0;
          S->held.push({now + rq.r.hold * unit, r.alloc_handle});
        } else {
          S->held_forever.push_back(r.alloc_handle);
        }
      } else {
        ++S->st.nofit;
      }
      S->in_flight[s] = 0;
      push_completion(S, cpl, now);
      make_ready(S, s);
    }
    for (size_t i = 0; i < sl.wreqs.size(); ++i) {
      const mapa_result_wide &r = sl.h_wres[i];
      const Req &rq = *sl.wreqs[i];
      const int32_t s = rq.r.server;
      mapa_completion cpl;
      std::memset(&cpl, 0, sizeof cpl);
      cpl.id = rq.r.id;
      cpl.count = r.count;
      cpl.alloc_handle = r.alloc_handle;
      cpl.latency_us = now - rq.due_us;
      cpl.wait_us = sl.t_dispatch - rq.due_us;
      cpl.status = r.status;
      cpl.key = r.key;
      cpl.agg = r.agg;
      cpl.pres = r.pres;
      cpl.vertex_mask = r.vertex_mask;
      cpl.busy_before = sl.wbusy_before[i];
      cpl.batch = sl.batch_id;
      cpl.server = s;
      std::memcpy(cpl.mapping, r.mapping, 16);
      S->st.embeddings += r.count;
      if (r.status == MAPA_RES_OK && r.alloc_handle >= 0) {
        ++S->st.granted;
        S->busy[s] |= r.vertex_mask;
        if (rq.r.hold >= 0) {
          const double unit = S->opts.time_unit_us > 0 ? S->opts.time_unit_us : 1.0;
          S->held.push({now + rq.r.hold * unit, r.alloc_handle});
        } else {
          S->held_forever.push_back(r.alloc_handle);
        }
      } else {
        ++S->st.nofit;
      }
      S->in_flight[s] = 0;
      push_completion(S, cpl, now);
      make_ready(S, s);
    }
    S->batch_us_sum += now - sl.t_dispatch;
    S->harvest_us_sum += S->now_us() - now;
    sl.active = false;
    sl.reqs.clear();
    sl.wreqs.clear();
    *did = true;
  }
  flush_completions(S);
  return MAPA_OK;
}

// Dispatch releases that are due and one batch of ready requests on slot sl.
int32_t dispatch(ServeState *S, Slot &sl, bool final_release, bool *did) {
  mapa_ctx *c = S->c;
  const double now = S->now_us();
  // 1. releases due now whose server has nothing in flight
  std::vector<int64_t> rel;
  std::vector<Held> again;
  for (auto &h : S->deferred) again.push_back(h);
  S->deferred.clear();
  while (!S->held.empty() && (final_release || S->held.top().t_us <= now)) {
    again.push_back(S->held.top());
    S->held.pop();
  }
  if (final_release)
    for (int64_t h : S->held_forever) again.push_back({now, h});
  if (final_release) S->held_forever.clear();
  for (auto &h : again) {
    const int32_t s = (int32_t)(h.handle >> 32);
    if (S->in_flight[s]) {
      S->deferred.push_back(h);
      continue;
    }
    rel.push_back(h.handle);
    S->busy[s] &= ~(uint32_t)h.handle;
    make_ready(S, s);  // a release may let a waiting request fit
  }
  // 2. a batch of ready requests, one per server, within the admission budget
  const unsigned long long budget =
      S->opts.admission_items > 0 ? (unsigned long long)S->opts.admission_items
                                  : sl.ws.cap_items - (unsigned long long)kPadReserve - S->opts.max_batch;
  unsigned long long items = 0, wleaves = 0;
  sl.reqs.clear();
  sl.busy_before.clear();
  sl.wreqs.clear();
  sl.wbusy_before.clear();
  std::vector<int32_t> keep;
  const size_t nready = S->ready.size();
  for (size_t it = 0; it < nready; ++it) {
    const int32_t s = S->ready.front();
    S->ready.pop_front();
    S->in_ready[s] = 0;
    if (S->in_flight[s]) continue;
    // requests that cannot fit, or that would exceed the wide kernels'
    // embedding limit, are answered here, in order
    while (!S->fifo_empty(s)) {
      const Req &rq = *S->fhead[s];
      const int F = S->nvert[s] - __builtin_popcount(S->busy[s]);
      const bool refuse = (int)rq.r.k <= F && is_wide(S->nvert[s], rq.r.k) &&
                          wide_embeddings(F, rq.r.k) > kWideMaxLeaves;
      if ((int)rq.r.k <= F && !refuse) break;
      mapa_completion cpl;
      std::memset(&cpl, 0, sizeof cpl);
      cpl.id = rq.r.id;
      cpl.alloc_handle = -1;
      cpl.latency_us = now - rq.due_us;
      cpl.wait_us = cpl.latency_us;
      cpl.status = refuse ? MAPA_RES_REFUSED : MAPA_RES_NOFIT;
      cpl.key = INT32_MIN;
      cpl.busy_before = S->busy[s];
      cpl.batch = -1;
      cpl.server = s;
      std::memset(cpl.mapping, 0xFF, sizeof cpl.mapping);
      ++S->st.nofit;
      ++S->st.host_nofit;
      push_completion(S, cpl, now);
      S->fifo_pop(s);
      *did = true;
    }
    if (S->fifo_empty(s)) continue;
    const Req *rq = S->fhead[s];
    const int F = S->nvert[s] - __builtin_popcount(S->busy[s]);
    if (is_wide(S->nvert[s], rq->r.k)) {  // the dispatch's wide batch, admitted by embeddings
      const unsigned long long e = wide_embeddings(F, rq->r.k);
      if ((int32_t)sl.wreqs.size() >= kServeWideMax) {
        keep.push_back(s);
        continue;
      }
      if (!sl.wreqs.empty() && wleaves + e > kServeWideLeaves) {
        ++S->st.admission_waits;
        keep.push_back(s);
        continue;
      }
      wleaves += e;
      sl.wreqs.push_back(rq);
      sl.wbusy_before.push_back(S->busy[s]);
      S->in_flight[s] = 1;
      S->fifo_pop(s);
      continue;
    }
    const unsigned long long est = S->work.items[F][rq->r.k];
    if ((int32_t)sl.reqs.size() >= S->opts.max_batch) {
      keep.push_back(s);
      continue;
    }
    if (!sl.reqs.empty() && items + est > budget) {
      ++S->st.admission_waits;
      keep.push_back(s);
      continue;
    }
    items += est;
    sl.reqs.push_back(rq);
    sl.busy_before.push_back(S->busy[s]);
    S->in_flight[s] = 1;
    S->fifo_pop(s);
  }
  for (auto it = keep.rbegin(); it != keep.rend(); ++it) {
    S->in_ready[*it] = 1;
    S->ready.push_front(*it);
  }
  flush_completions(S);  // host answers
  if (rel.empty() && sl.reqs.empty() && sl.wreqs.empty()) return MAPA_OK;
  *did = true;

  // 3. enqueue: releases first (ordered before this batch and, through
  //    rel_event, before every later batch on the other stream).  The slot's
  //    pinned buffers may still feed copies of a release-only dispatch.
  // Only what is needed is waited for (each HIP call costs the loop time):
  // the slot's own earlier release-only work, and releases enqueued on the
  // other stream since this stream last ordered itself after them.
  if (sl.stream_busy) SERVE_CHK(hipEventSynchronize(sl.done));
  const int self = (int)(&sl - S->slots.data());
  if (sl.rel_seen < S->rel_gen) {
    if (S->rel_slot != self) SERVE_CHK(hipStreamWaitEvent(sl.stream, S->rel_event, 0));
    sl.rel_seen = S->rel_gen;
  }
  if (!rel.empty()) {
    if (rel.size() > sl.cap_rel) {
      SERVE_CHK(hipStreamSynchronize(sl.stream));
      if (sl.h_rel) (void)hipHostFree(sl.h_rel);
      sl.h_rel = nullptr;
      sl.cap_rel = 0;
      size_t cap = std::max<size_t>(4096, rel.size() * 2);
      SERVE_CHK(hipHostMalloc((void **)&sl.h_rel, cap * sizeof(int64_t), hipHostMallocDefault));
      sl.cap_rel = cap;
    }
    std::memcpy(sl.h_rel, rel.data(), rel.size() * sizeof(int64_t));
    SERVE_CHK(launch_release_apply(sl.h_rel, 8, (int32_t)rel.size(), (int32_t)c->server_topo.size(),
                                   c->d_busy, sl.stream));
    SERVE_CHK(hipEventRecord(S->rel_event, sl.stream));
    ++S->rel_gen;
    S->rel_slot = self;
    sl.rel_seen = S->rel_gen;
    S->st.releases += (int64_t)rel.size();
  }
  if (!sl.reqs.empty()) {
    const int32_t nq = (int32_t)sl.reqs.size();
    for (int32_t i = 0; i < nq; ++i) {
      const mapa_request &r = sl.reqs[i]->r;
      mapa_query &q = sl.h_q[i];
      q.server = r.server;
      q.kind = r.kind;
      q.k = r.k;
      q.mode = r.mode;
      q.commit = 1;
      q.a = r.a;
      q.b = r.b;
      q.metric = r.metric;
    }
    // one request per server: small batches take the fused launch, which
    // reads the requests from and writes the results to the pinned buffers
    unsigned long long total = 0;
    bool small = nq <= kFusedMaxQueries;
    for (int32_t i = 0; i < nq && small; ++i) {
      const int32_t s = sl.reqs[i]->r.server;
      const unsigned long long e =
          S->work.leaves[S->nvert[s] - __builtin_popcount(sl.busy_before[i])][sl.reqs[i]->r.k];
      small = e <= kFusedMaxQueryLeaves;
      total += e;
    }
    int32_t rc;
    sl.timed = S->st.batches % kGpuSample == 0;
    if (sl.timed) SERVE_CHK(hipEventRecord(sl.g0, sl.stream));
    if (small && total <= kFusedMaxLeaves) {
      rc = enqueue_fused(c, sl.ws, sl.h_q, sl.h_res, nq, sl.stream);
      ++S->fused_batches;
    } else {
      SERVE_CHK(hipMemcpyAsync(sl.ws.d_q, sl.h_q, nq * sizeof(mapa_query), hipMemcpyHostToDevice,
                               sl.stream));
      rc = enqueue_batch(c, sl.ws, sl.ws.d_q, sl.ws.d_res, nq, sl.stream);
      if (!rc)
        SERVE_CHK(hipMemcpyAsync(sl.h_res, sl.ws.d_res, nq * sizeof(mapa_result),
                                 hipMemcpyDeviceToHost, sl.stream));
    }
    if (rc) {
      S->error = rc;
      S->error_msg = "batch enqueue failed";
      return rc;
    }
    if (sl.timed && sl.wreqs.empty()) SERVE_CHK(hipEventRecord(sl.g1, sl.stream));
  }
  if (!sl.wreqs.empty()) {
    const int32_t nw = (int32_t)sl.wreqs.size();
    for (int32_t i = 0; i < nw; ++i) {
      const mapa_request &r = sl.wreqs[i]->r;
      mapa_query &q = sl.h_wq[i];
      q.server = r.server;
      q.kind = r.kind;
      q.k = r.k;
      q.mode = r.mode;
      q.commit = 1;
      q.a = r.a;
      q.b = r.b;
      q.metric = r.metric;
    }
    if (sl.reqs.empty()) {
      sl.timed = S->st.batches % kGpuSample == 0;
      if (sl.timed) SERVE_CHK(hipEventRecord(sl.g0, sl.stream));
    }
    char *dw = static_cast<char *>(sl.d_wide);
    WideArgs w;
    wide_ctx_args(c, w);
    wide_scratch_args(dw + kServeWideScratchOff, nw, w);
    w.q = reinterpret_cast<const mapa_query *>(dw);
    w.nq = nw;
    w.res = reinterpret_cast<mapa_result_wide *>(dw + kServeWideResOff);
    w.self_check_failures = &sl.ws.d_ctr->self_check_failures;
    SERVE_CHK(hipMemcpyAsync(dw, sl.h_wq, nw * sizeof(mapa_query), hipMemcpyHostToDevice, sl.stream));
    SERVE_CHK(launch_wide_plan(w, sl.stream));
    SERVE_CHK(launch_wide_search(w, sl.stream));
    SERVE_CHK(launch_wide_finalize(w, sl.stream));
    SERVE_CHK(hipMemcpyAsync(sl.h_wres, w.res, nw * sizeof(mapa_result_wide), hipMemcpyDeviceToHost,
                             sl.stream));
    if (sl.timed) SERVE_CHK(hipEventRecord(sl.g1, sl.stream));
  }
  if (!sl.reqs.empty() || !sl.wreqs.empty()) {
    sl.batch_id = S->next_batch++;
    sl.t_dispatch = now;
    S->dispatch_us_sum += S->now_us() - now;
    ++S->st.batches;
    S->batched_queries += (int64_t)sl.reqs.size() + (int64_t)sl.wreqs.size();
  }
  SERVE_CHK(hipEventRecord(sl.done, sl.stream));
  sl.active = !sl.reqs.empty() || !sl.wreqs.empty();
  sl.stream_busy = true;
  return MAPA_OK;
}

void loop_main(ServeState *S) {
  mapa_ctx *c = S->c;
  if (hipSetDevice(c->device) != hipSuccess) {
    S->error = MAPA_ERR_DEVICE;
    S->error_msg = "hipSetDevice";
    return;
  }
  for (;;) {
    bool did = false;
    bool stopping;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto &v : S->incoming) S->subs.push_back(std::move(v));
      S->incoming.clear();
      stopping = S->stopping;
    }
    if (harvest(S, &did)) break;
    // due arrivals join their server's queue
    const double now = S->now_us();
    while (!S->pending_empty() && S->pending_front().due_us <= now) {
      Req *r = &S->pending_front();
      ++S->pend_pos;
      S->fifo_push(r->r.server, r);
      make_ready(S, r->r.server);
      did = true;
    }
    bool outstanding;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      outstanding = S->completed < S->submitted || !S->incoming.empty();
    }
    bool any_active = false;
    for (auto &sl : S->slots) any_active |= sl.active;
    const bool final_release = stopping && !outstanding && !any_active;
    for (auto &sl : S->slots) {
      if (sl.active) continue;
      if (dispatch(S, sl, final_release, &did)) return;
      if (final_release) break;
    }
    if (final_release) {
      // everything answered and every allocation handed back
      for (auto &sl : S->slots) (void)hipStreamSynchronize(sl.stream);
      if (S->deferred.empty() && S->held.empty() && S->held_forever.empty()) return;
      continue;
    }
    if (did) continue;
    any_active = false;
    for (auto &sl : S->slots) any_active |= sl.active;
    if (any_active) {
      std::this_thread::yield();
      continue;
    }
    // idle: sleep until the next arrival, release or submission
    double next = 1e300;
    if (!S->pending_empty()) next = S->pending_front().due_us;
    if (!S->held.empty()) next = std::min(next, S->held.top().t_us);
    if (!S->deferred.empty()) next = std::min(next, S->now_us());
    const double wait_us = std::max(0.0, std::min(next - S->now_us(), 2000.0));
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->incoming.empty() && !S->stopping)
      S->cv.wait_for(lk, std::chrono::microseconds((int64_t)wait_us));
  }
}

void free_state(ServeState *S) {
  for (auto &sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    ws_destroy(sl.ws);
    if (sl.h_q) (void)hipHostFree(sl.h_q);
    if (sl.h_res) (void)hipHostFree(sl.h_res);
    if (sl.h_rel) (void)hipHostFree(sl.h_rel);
    if (sl.h_wq) (void)hipHostFree(sl.h_wq);
    if (sl.h_wres) (void)hipHostFree(sl.h_wres);
    if (sl.d_wide) (void)hipFree(sl.d_wide);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.g0) (void)hipEventDestroy(sl.g0);
    if (sl.g1) (void)hipEventDestroy(sl.g1);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (S->rel_event) (void)hipEventDestroy(S->rel_event);
  delete S;
}

double percentile(std::vector<double> &v, double p) {
  if (v.empty()) return 0;
  const size_t i = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
  std::nth_element(v.begin(), v.begin() + i, v.end());
  return v[i];
}

}  // namespace

void serve_teardown(mapa_ctx *c) {
  if (!c || !c->serve) return;
  ServeState *S = c->serve;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  c->serve = nullptr;
  free_state(S);
}

}  // namespace mapa

using namespace mapa;

extern "C" {

int32_t mapa_serve_start(mapa_ctx *c, const mapa_serve_opts *opts) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (c->serve) return fail(MAPA_ERR_STATE, "a serving loop is already running");
  mapa_serve_opts o{};
  if (opts) o = *opts;
  if (o.max_batch == 0) o.max_batch = 4096;
  if (o.inflight == 0) o.inflight = 2;
  if (o.item_leaves == 0) o.item_leaves = 4096;
  if (o.max_batch < 1 || o.max_batch > 65536)
    return fail(MAPA_ERR_INVALID_ARG, "max_batch %d outside 1..65536", o.max_batch);
  if (o.inflight < 1 || o.inflight > 2) return fail(MAPA_ERR_INVALID_ARG, "inflight must be 1 or 2");
  if (o.time_unit_us < 0 || o.admission_items < 0 || o.item_leaves < 1 || o.reserved != 0)
    return fail(MAPA_ERR_INVALID_ARG, "malformed serving options");
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  if (c->server_topo.empty()) return fail(MAPA_ERR_UNKNOWN_SERVER, "no servers created");
  int32_t rc = sync_ctx(c);
  if (rc) return rc;
  rc = wide_upload(c);  // the wide batches read every topology's rows
  if (rc) return rc;
  ServeState *S = new ServeState();
  S->c = c;
  S->opts = o;
  const size_t ns = c->server_topo.size();
  S->busy.assign(ns, 0);
  S->nvert.resize(ns);
  for (size_t s = 0; s < ns; ++s) S->nvert[s] = c->topo_n[c->server_topo[s]];
  S->in_flight.assign(ns, 0);
  S->in_ready.assign(ns, 0);
  S->fhead.assign(ns, nullptr);
  S->ftail.assign(ns, nullptr);
  S->work.build(o.item_leaves);
  auto bail = [&](int32_t code, const char *what) {
    free_state(S);
    return fail(code, "mapa_serve_start: %s", what);
  };
  if (hipMemcpy(S->busy.data(), c->d_busy, ns * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return bail(MAPA_ERR_DEVICE, "reading busy masks");
  if (hipEventCreateWithFlags(&S->rel_event, hipEventDisableTiming) != hipSuccess)
    return bail(MAPA_ERR_DEVICE, "event");
  S->slots.resize(o.inflight);
  for (auto &sl : S->slots) {
    if (ws_create(sl.ws, c->enum_bytes) != MAPA_OK || ws_ensure_q(sl.ws, o.max_batch) != MAPA_OK)
      return bail(MAPA_ERR_OOM, "workspace");
    if (sl.ws.cap_items < (unsigned long long)o.max_batch + kPadReserve)
      return bail(MAPA_ERR_ADMISSION, "max_batch exceeds the enumeration buffer");
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&sl.g0) != hipSuccess || hipEventCreate(&sl.g1) != hipSuccess ||
        hipHostMalloc((void **)&sl.h_q, o.max_batch * sizeof(mapa_query), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&sl.h_res, o.max_batch * sizeof(mapa_result), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&sl.h_wq, kServeWideMax * sizeof(mapa_query), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&sl.h_wres, kServeWideMax * sizeof(mapa_result_wide), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&sl.d_wide, kServeWideScratchOff + wide_scratch_bytes(kServeWideMax)) != hipSuccess)
      return bail(MAPA_ERR_DEVICE, "stream, event or pinned buffers");
  }
  if (hipDeviceSynchronize() != hipSuccess) return bail(MAPA_ERR_DEVICE, "device sync");
  S->t0 = Clock::now();
  c->serve = S;
  S->th = std::thread(loop_main, S);
  return MAPA_OK;
}

int32_t mapa_serve_submit(mapa_ctx *c, const mapa_request *reqs, int32_t n) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  ServeState *S = c->serve;
  if (!S) return fail(MAPA_ERR_STATE, "no serving loop is running");
  if (n < 0) return fail(MAPA_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return MAPA_OK;
  if (!reqs) return fail(MAPA_ERR_INVALID_ARG, "reqs is NULL");
  // validate and copy outside the lock; due times are relative until then
  std::vector<Req> batch((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    const mapa_request &r = reqs[i];
    if (r.server < 0 || (size_t)r.server >= c->server_topo.size())
      return fail(MAPA_ERR_UNKNOWN_SERVER, "request %d: unknown server %d", i, r.server);
    if (r.k > kWideK) return fail(MAPA_ERR_UNSUPPORTED, "request %d: k=%d > %d", i, r.k, kWideK);
    if (r.kind > MAPA_TREE) {
      const int id = r.kind - MAPA_PATTERN_BASE;
      if (id < 0 || id >= c->npat || c->pat_k[id] != r.k)
        return fail(MAPA_ERR_INVALID_ARG, "request %d: kind=%d with k=%d is neither a pattern "
                    "kind nor a registered pattern of that size", i, r.kind, r.k);
    }
    if (r.k < 1 || r.mode > 1 || r.a < 0 || r.a > MAPA_MAX_AB || r.b < 0 ||
        r.b > MAPA_MAX_AB || r.metric > MAPA_METRIC_EFFBW || r.reserved1 != 0)
      return fail(MAPA_ERR_INVALID_ARG, "request %d: malformed field", i);
    if (r.metric == MAPA_METRIC_EFFBW && c->topo_maxw[c->server_topo[r.server]] > 2)
      return fail(MAPA_ERR_UNSUPPORTED, "request %d: effective bandwidth needs link weights 0..2", i);
    if (i > 0 && !(r.t_arrival >= reqs[i - 1].t_arrival))
      return fail(MAPA_ERR_INVALID_ARG, "request %d: arrival goes back in time", i);
    batch[i] = {r, S->opts.time_unit_us > 0 ? r.t_arrival * S->opts.time_unit_us : 0.0, nullptr};
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) return fail(MAPA_ERR_STATE, "the serving loop is stopping");
  if (!(reqs[0].t_arrival >= S->last_arrival))
    return fail(MAPA_ERR_INVALID_ARG, "request 0: arrival goes back in time");
  S->last_arrival = reqs[n - 1].t_arrival;
  // the loop sees nothing of this call before the lock is released, so trace
  // time 0 is taken at the end of the first submission
  const double now = S->now_us();
  if (S->origin_us < 0) S->origin_us = now;
  const double base = S->opts.time_unit_us > 0 ? S->origin_us : now;
  for (auto &r : batch) r.due_us += base;
  S->incoming.push_back(std::move(batch));
  S->submitted += n;
  S->cv.notify_all();
  return MAPA_OK;
}

int32_t mapa_serve_poll(mapa_ctx *c, mapa_completion *out, int32_t cap, int32_t *n_out) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  ServeState *S = c->serve;
  if (!S) return fail(MAPA_ERR_STATE, "no serving loop is running");
  if (cap < 0 || (cap > 0 && !out) || !n_out) return fail(MAPA_ERR_INVALID_ARG, "bad output array");
  std::lock_guard<std::mutex> lk(S->mu);
  int32_t k = 0;
  while (k < cap && !S->done_q.empty()) {
    out[k++] = S->done_q.front();
    S->done_q.pop_front();
  }
  *n_out = k;
  if (S->error) return fail(S->error, "serving loop: %s", S->error_msg.c_str());
  return MAPA_OK;
}

int32_t mapa_serve_stop(mapa_ctx *c, mapa_serve_stats *out) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  ServeState *S = c->serve;
  if (!S) return fail(MAPA_ERR_STATE, "no serving loop is running");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  mapa_serve_stats st = S->st;
  st.requests = S->submitted;
  st.completed = S->completed;
  st.wall_s = S->origin_us >= 0 ? std::max(0.0, S->last_done_us - S->origin_us) * 1e-6 : 0.0;
  st.requests_per_s = st.wall_s > 0 ? (double)st.completed / st.wall_s : 0;
  st.embeddings_per_s = st.wall_s > 0 ? (double)st.embeddings / st.wall_s : 0;
  st.p50_us = percentile(S->lat, 0.50);
  st.p99_us = percentile(S->lat, 0.99);
  st.p999_us = percentile(S->lat, 0.999);
  st.max_us = S->lat.empty() ? 0 : *std::max_element(S->lat.begin(), S->lat.end());
  st.mean_batch = st.batches ? (double)S->batched_queries / (double)st.batches : 0;
  st.mean_batch_us = st.batches ? S->batch_us_sum / (double)st.batches : 0;
  st.fused_batches = S->fused_batches;
  st.wait_p50_us = percentile(S->waits, 0.50);
  st.wait_p99_us = percentile(S->waits, 0.99);
  st.turnaround_p50_us = percentile(S->turns, 0.50);
  st.turnaround_p99_us = percentile(S->turns, 0.99);
  st.mean_dispatch_us = st.batches ? S->dispatch_us_sum / (double)st.batches : 0;
  st.mean_gpu_us = S->gpu_samples ? S->gpu_us_sum / (double)S->gpu_samples : 0;
  st.mean_harvest_us = st.batches ? S->harvest_us_sum / (double)st.batches : 0;
  const int32_t err = S->error;
  const std::string msg = S->error_msg;
  c->serve = nullptr;
  free_state(S);
  (void)hipEventRecord(c->last, c->internal);
  if (out) *out = st;
  if (err) return fail(err, "serving loop: %s", msg.c_str());
  return MAPA_OK;
}

}  // extern "C"
