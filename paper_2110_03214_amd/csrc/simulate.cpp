// Job-trace simulation (mapa_simulate): the simulation framework of the
// paper's Sec. 5.2 on the library's allocation path.
//
// Many independent simulations run together, each on its own server with
// its own job file and policy.  Per simulation: a dispatcher moves jobs
// whose arrival cycle has come into a first-in first-out queue; whenever the
// head of the queue fits in the free accelerators it is placed; a placed job
// holds its accelerators for its duration, then the Job Finished Signal
// releases them.  The engine is cycle based and jumps from one cycle with an
// event (an arrival or a finish) to the next; within a cycle, finished jobs
// free their accelerators first, then arrivals are queued, then heads are
// placed until every simulation's head blocks or its queue is empty.
//
// The simulations are independent, so each keeps its own cycle: one round
// moves every simulation to the first cycle at which its queue head fits,
// then places all those heads together, as one device batch (the Preserve
// and Greedy policies are allocation queries with commit, on distinct
// servers) followed by one scoring kernel that also places the lowest-id
// jobs.  The number of rounds is the largest number of jobs one simulation
// places, whatever the number of simulations.
#include <algorithm>
#include <cstring>
#include <deque>
#include <queue>
#include <vector>

#include "ctx.h"
#include "simulate.h"

namespace mapa {
namespace {

struct Running {
  int32_t finish;
  int32_t job;
  uint32_t mask;
  bool operator>(const Running &o) const { return finish > o.finish; }
};

struct SimState {
  int32_t server, policy, n, capacity;
  int32_t begin, end, next;  // job range and the next job to arrive
  uint32_t busy;             // host mirror of the server's busy mask
  std::deque<int32_t> queue;
  std::priority_queue<Running, std::vector<Running>, std::greater<Running>> running;
};

int pop32(uint32_t x) { return __builtin_popcount(x); }

}  // namespace
}  // namespace mapa

using namespace mapa;

extern "C" int32_t mapa_simulate(mapa_ctx *c, int32_t nsim, const int32_t *servers,
                                 const int32_t *policies, const int32_t *job_offsets,
                                 const mapa_job *jobs, mapa_job_log *logs, mapa_sim_stats *stats) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (c->serve) return fail(MAPA_ERR_STATE, "mapa_simulate: the serving loop owns the context");
  if (nsim < 0) return fail(MAPA_ERR_INVALID_ARG, "nsim < 0");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (nsim == 0) return MAPA_OK;
  if (!servers || !policies || !job_offsets) return fail(MAPA_ERR_INVALID_ARG, "NULL array");
  if (job_offsets[0] != 0) return fail(MAPA_ERR_INVALID_ARG, "job_offsets[0] must be 0");
  const int32_t njobs = job_offsets[nsim];
  if (njobs > 0 && (!jobs || !logs)) return fail(MAPA_ERR_INVALID_ARG, "NULL job or log array");
  std::vector<uint8_t> seen(c->server_topo.size(), 0);
  for (int32_t i = 0; i < nsim; ++i) {
    const int32_t s = servers[i];
    if (s < 0 || (size_t)s >= c->server_topo.size())
      return fail(MAPA_ERR_UNKNOWN_SERVER, "simulation %d: unknown server %d", i, s);
    if (seen[s]) return fail(MAPA_ERR_INVALID_ARG, "simulation %d: server %d is used twice", i, s);
    seen[s] = 1;
    const int t = c->server_topo[s];
    if (c->topo_n[t] > kMaxN)
      return fail(MAPA_ERR_UNSUPPORTED, "simulation %d: server %d has more than %d accelerators", i, s, kMaxN);
    if (c->topo_maxw[t] > 2)
      return fail(MAPA_ERR_UNSUPPORTED, "simulation %d: the log's effective bandwidth (Eq. 2) needs "
                  "link weights 0, 1, 2; server %d has %d", i, s, c->topo_maxw[t]);
    if (policies[i] < MAPA_POLICY_PRESERVE || policies[i] > MAPA_POLICY_BASELINE)
      return fail(MAPA_ERR_INVALID_ARG, "simulation %d: policy %d", i, policies[i]);
    if (job_offsets[i + 1] < job_offsets[i])
      return fail(MAPA_ERR_INVALID_ARG, "job_offsets must not decrease");
    for (int32_t j = job_offsets[i]; j < job_offsets[i + 1]; ++j) {
      const mapa_job &jb = jobs[j];
      if (jb.k < 1 || jb.k > kMaxK)
        return fail(MAPA_ERR_INVALID_ARG, "job %d: k=%d outside 1..%d", j, jb.k, kMaxK);
      if (jb.kind > MAPA_TREE) {
        const int id = jb.kind - MAPA_PATTERN_BASE;
        if (id < 0 || id >= c->npat || c->pat_k[id] != jb.k)
          return fail(MAPA_ERR_INVALID_ARG, "job %d: kind=%d with k=%d is neither a pattern kind "
                      "nor a registered pattern of that size", j, jb.kind, jb.k);
      }
      if (jb.arrival < 0 || jb.duration < 1 || jb.sensitive > 1 || jb.reserved != 0)
        return fail(MAPA_ERR_INVALID_ARG, "job %d: malformed field", j);
      if (j > job_offsets[i] && jb.arrival < jobs[j - 1].arrival)
        return fail(MAPA_ERR_INVALID_ARG, "job %d: arrival goes back in time", j);
      if ((int64_t)jb.arrival + jb.duration > INT32_MAX / 2)
        return fail(MAPA_ERR_INVALID_ARG, "job %d: cycle count too large", j);
    }
  }
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  MAPA_HIPCHK(hipSetDevice(c->device));
  int32_t rc = sync_ctx(c);
  if (rc) return rc;

  // start state: every server's busy mask as it is now (those accelerators
  // stay reserved for the whole simulation)
  std::vector<int32_t> ids(servers, servers + nsim);
  std::vector<uint32_t> busy0((size_t)nsim);
  rc = mapa_get_busy(c, nsim, ids.data(), busy0.data());
  if (rc) return rc;
  std::vector<SimState> sims((size_t)nsim);
  for (int32_t i = 0; i < nsim; ++i) {
    SimState &S = sims[i];
    S.server = servers[i];
    S.policy = policies[i];
    S.n = c->topo_n[c->server_topo[S.server]];
    S.busy = busy0[i];
    S.capacity = S.n - pop32(S.busy);
    S.begin = S.next = job_offsets[i];
    S.end = job_offsets[i + 1];
  }
  for (int32_t j = 0; j < njobs; ++j) {
    std::memset(&logs[j], 0, sizeof logs[j]);
    logs[j].id = jobs[j].id;
    logs[j].status = MAPA_RES_NOFIT;
    logs[j].start = logs[j].finish = -1;
    std::memset(logs[j].mapping, 0xFF, 8);
  }

  // pinned round buffers, read and written by the kernels in place
  rc = ensure_batch_capacity(c, (size_t)nsim);
  if (rc) return rc;
  mapa_query *h_q = nullptr;
  mapa_result *h_res = nullptr;
  SimEntry *h_e = nullptr;
  SimOut *h_o = nullptr;
  int64_t *h_rel = nullptr;
  auto release_buffers = [&]() {
    if (h_q) (void)hipHostFree(h_q);
    if (h_res) (void)hipHostFree(h_res);
    if (h_e) (void)hipHostFree(h_e);
    if (h_o) (void)hipHostFree(h_o);
    if (h_rel) (void)hipHostFree(h_rel);
  };
  if (hipHostMalloc((void **)&h_q, nsim * sizeof(mapa_query), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_res, nsim * sizeof(mapa_result), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_e, nsim * sizeof(SimEntry), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_o, nsim * sizeof(SimOut), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_rel, std::max<int32_t>(1, njobs) * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    release_buffers();
    return fail(MAPA_ERR_OOM, "simulation: pinned round buffers");
  }
  hipStream_t st = c->internal;
  int32_t err = MAPA_OK;
  int64_t rounds = 0, event_cycles = 0, placed = 0, dev_batches = 0, last_cycle = 0;
  std::vector<int32_t> round_sim;
  std::vector<int32_t> clock((size_t)nsim, -1);  // each simulation's current cycle
  int32_t nrel = 0;
  // Move simulation S to its next cycle with an event: finished jobs free
  // their accelerators (queued for the release kernel), then arrivals join
  // the queue.  Returns false when nothing is left to happen.
  auto advance = [&](SimState &S, int32_t &t) -> bool {
    int64_t nxt = INT64_MAX;
    if (S.next < S.end) nxt = jobs[S.next].arrival;
    if (!S.running.empty()) nxt = std::min<int64_t>(nxt, S.running.top().finish);
    if (nxt == INT64_MAX) return false;
    t = (int32_t)std::max<int64_t>(t + 1, nxt);
    ++event_cycles;
    last_cycle = std::max<int64_t>(last_cycle, t);
    while (!S.running.empty() && S.running.top().finish <= t) {
      const Running r = S.running.top();
      S.running.pop();
      S.busy &= ~r.mask;
      h_rel[nrel++] = ((int64_t)S.server << 32) | (int64_t)r.mask;
    }
    while (S.next < S.end && jobs[S.next].arrival <= t) {
      if ((int)jobs[S.next].k <= S.capacity) S.queue.push_back(S.next);
      ++S.next;  // a job that can never fit keeps its NOFIT log
    }
    return true;
  };
  for (;;) {
    // every simulation moves to the first cycle at which its queue head
    // fits (or ends); its releases are applied before this round's placements
    nrel = 0;
    round_sim.clear();
    int32_t nq = 0;
    bool small = true;
    unsigned long long total = 0;
    for (int32_t i = 0; i < nsim; ++i) {
      SimState &S = sims[i];
      bool live = true;
      while (live && (S.queue.empty() || (int)jobs[S.queue.front()].k > S.n - pop32(S.busy)))
        live = advance(S, clock[i]);
      if (!live) continue;
      const mapa_job &jb = jobs[S.queue.front()];
      const int F = S.n - pop32(S.busy);
      SimEntry &e = h_e[round_sim.size()];
      e.server = S.server;
      e.busy_before = S.busy;
      e.k = jb.k;
      std::memset(e.pad, 0, sizeof e.pad);
      e.nbtab = pattern_nbtab(c, jb.kind, jb.k);
      e.qi = -1;
      if (S.policy != MAPA_POLICY_BASELINE) {
        mapa_query &q = h_q[nq];
        std::memset(&q, 0, sizeof q);
        q.server = S.server;
        q.kind = jb.kind;
        q.k = jb.k;
        q.mode = MAPA_ALL_INJECTIVE;
        q.commit = 1;
        if (S.policy == MAPA_POLICY_GREEDY) {
          q.a = 1;  // Greedy: AggBW (Eq. 1)
          q.b = 0;
        } else if (jb.sensitive) {
          q.metric = MAPA_METRIC_EFFBW;  // Alg. 1, bandwidth-sensitive branch (Eq. 2)
        } else {
          q.a = 0;  // Alg. 1, insensitive branch: PreservedBW (Eq. 3)
          q.b = 1;
        }
        const unsigned long long leaves = perm_leaves(F, jb.k);
        small = small && leaves <= kFusedMaxQueryLeaves;
        total += leaves;
        e.qi = nq++;
      }
      round_sim.push_back(i);
    }
    if (nrel > 0 &&
        launch_release_apply(h_rel, 8, nrel, (int32_t)c->server_topo.size(), c->d_busy, st) != hipSuccess) {
      err = fail(MAPA_ERR_DEVICE, "simulation: release launch");
      break;
    }
    if (round_sim.empty()) break;
    ++rounds;
    if (nq > 0) {
      ++dev_batches;
      if (small && total <= kFusedMaxLeaves && nq <= kFusedMaxQueries) {
        err = enqueue_fused(c, c->ws, h_q, h_res, nq, st);
      } else if (hipMemcpyAsync(c->ws.d_q, h_q, nq * sizeof(mapa_query), hipMemcpyHostToDevice, st) != hipSuccess) {
        err = fail(MAPA_ERR_DEVICE, "simulation: query copy");
      } else {
        err = enqueue_batch(c, c->ws, c->ws.d_q, c->ws.d_res, nq, st);
        if (!err && hipMemcpyAsync(h_res, c->ws.d_res, nq * sizeof(mapa_result), hipMemcpyDeviceToHost, st) != hipSuccess)
          err = fail(MAPA_ERR_DEVICE, "simulation: result copy");
      }
      if (err) break;
    }
    SimPlaceArgs a;
    a.entries = h_e;
    a.n = (int32_t)round_sim.size();
    a.qres = h_res;
    a.out = h_o;
    a.server_topo = c->d_server_topo;
    a.topo_n = c->d_topo_n;
    a.topo_W = c->d_topo_W;
    a.eff_key = c->d_eff_key;
    a.busy = c->d_busy;
    a.self_check_failures = &c->ws.d_ctr->self_check_failures;
    if (launch_sim_place(a, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      err = fail(MAPA_ERR_DEVICE, "simulation: placement kernel");
      break;
    }
    for (size_t r = 0; r < round_sim.size(); ++r) {
      SimState &S = sims[round_sim[r]];
      const int32_t t = clock[round_sim[r]];
      const int32_t j = S.queue.front();
      const SimOut &o = h_o[r];
      if (o.mask == 0 || (o.mask & S.busy) || pop32(o.mask) != (int)jobs[j].k) {
        err = fail(MAPA_ERR_DEVICE, "simulation: job %d was not placed on free accelerators", j);
        break;
      }
      S.queue.pop_front();
      S.busy |= o.mask;
      mapa_job_log &lg = logs[j];
      lg.status = MAPA_RES_OK;
      lg.start = t;
      lg.finish = t + jobs[j].duration;
      lg.vertex_mask = o.mask;
      std::memcpy(lg.mapping, o.mapping, 8);
      lg.agg = o.agg;
      lg.pres = o.pres;
      lg.effbw_milli = o.effbw_milli;
      lg.links = o.links;
      S.running.push({lg.finish, j, o.mask});
      ++placed;
    }
    if (err) break;
  }
  if (hipStreamSynchronize(st) != hipSuccess && !err) err = fail(MAPA_ERR_DEVICE, "simulation: final sync");
  (void)hipEventRecord(c->last, st);
  release_buffers();
  if (err) {
    // leave every server as it was found
    (void)mapa_set_busy(c, nsim, ids.data(), busy0.data(), 0, nullptr);
    return err;
  }
  if (stats) {
    stats->cycles = last_cycle;
    stats->event_cycles = event_cycles;
    stats->rounds = rounds;
    stats->device_batches = dev_batches;
    stats->jobs_placed = placed;
  }
  return MAPA_OK;
}
