// Context and workspace layout shared by the host core (host.cpp) and the
// serving loop (serve.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "mapa.h"
#include "mapa_internal.h"

namespace mapa {

int32_t fail(int32_t code, const char *fmt, ...);

#define MAPA_HIPCHK(expr)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::mapa::fail(MAPA_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

template <class T>
hipError_t dev_alloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc((void **)p, count * sizeof(T));
}

template <class T>
void dev_free(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Everything one in-flight batch needs on the device: per-query plans and
// accumulators, staging for host-pointer calls, the prefix work-list and the
// per-batch counters.  Two batches in flight need two workspaces.
struct Workspace {
  size_t cap_q = 0;
  Plan *d_plan = nullptr;
  unsigned long long *d_acc_count = nullptr, *d_acc_best = nullptr;  // zero between batches
  uint32_t *d_done = nullptr;  // fused launch: blocks finished per query, zero between batches
  mapa_query *d_q = nullptr;
  mapa_result *d_res = nullptr;
  uint2 *d_items = nullptr;
  unsigned long long cap_items = 0;
  Counters *d_ctr = nullptr;
};

int32_t ws_create(Workspace &w, size_t enum_bytes);
int32_t ws_ensure_q(Workspace &w, size_t nq);  // no work may be in flight on w
void ws_destroy(Workspace &w);

struct ProfEvents {
  hipEvent_t start, stop;
};

struct ServeState;  // serve.cpp

}  // namespace mapa

struct mapa_ctx {
  int device = -1;
  bool has_device = false;
  int cu_count = 0;
  hipStream_t internal = nullptr;
  hipEvent_t last = nullptr;  // completion of the last issued call
  size_t enum_bytes = 0;

  // topologies (host copy is authoritative; device copies are derived)
  std::vector<int32_t> topo_n;
  std::vector<std::array<uint8_t, 256>> topo_W;  // 16x16 padded (zero for n > 16)
  std::vector<std::array<uint8_t, 1024>> wide_W;  // 32x32 padded, every topology
  int wpr = 1;
  int32_t *d_topo_n = nullptr;
  uint8_t *d_topo_W = nullptr;
  uint32_t *d_rows = nullptr;
  std::vector<uint8_t> topo_maxw;  // largest weight per topology
  uint8_t *d_topo_maxw = nullptr;
  size_t cap_topos = 0;
  uint16_t *d_eff_rank = nullptr;  // Eq. 2 tables (eff_off layout)
  int32_t *d_eff_key = nullptr;

  // wide path (servers of up to 32 accelerators, patterns of up to 12 vertices)
  uint32_t *d_wide_rows = nullptr;  // [T][9][32]: weight bit-planes 0..7 and adjacency, one row per vertex
  size_t wide_uploaded = 0, cap_wide = 0;
  struct WideBuf {
    void *d = nullptr;
    size_t cap = 0;
  } wide_buf;  // embedding total, plans, per-block partials (and host queries, results) of one wide call

  // registered patterns (append-only; slot i = kind MAPA_PATTERN_BASE + i)
  std::vector<unsigned long long> pat_nbtab;  // host mirror, back-neighbour tables
  std::vector<uint8_t> pat_k;                 // host mirror, k per slot (0 = free)
  int32_t npat = 0;
  unsigned long long *d_pat_nbtab = nullptr;  // [MAPA_MAX_PATTERNS]
  uint8_t *d_pat_k = nullptr;                 // [MAPA_MAX_PATTERNS], zero = free
  // matching order of each registered pattern (LINKED search) and its
  // back-neighbour table in that order
  unsigned long long *d_pat_nbtab_ord = nullptr;  // [MAPA_MAX_PATTERNS]
  uint32_t *d_pat_order = nullptr;                // [MAPA_MAX_PATTERNS]

  // servers
  std::vector<int32_t> server_topo;  // host mirror, immutable per server
  int32_t *d_server_topo = nullptr;
  uint32_t *d_busy = nullptr;
  unsigned long long *d_commit_slot = nullptr;
  size_t cap_servers = 0;

  // the API calls' batch workspace
  mapa::Workspace ws;
  // small scratch for host-pointer state calls
  int32_t *d_ids = nullptr;
  uint32_t *d_masks = nullptr;
  int64_t *d_handles = nullptr;
  uint32_t *d_flag = nullptr;
  size_t cap_small = 0;
  uint8_t *d_split = nullptr;  // prefix depth per (F, k, split), from the tuning
  // pinned staging of the fused small-batch path (kFusedMaxQueries each)
  mapa_query *h_fq = nullptr;
  mapa_result *h_fres = nullptr;
  std::vector<uint32_t> srv_stamp;  // per server: last batch stamp (distinct-server test)
  uint32_t stamp = 0;

  // captured batch graphs (device-pointer batches with MAPA_USE_GRAPH)
  struct Graph {
    const void *q;
    void *res;
    int32_t nq;
    hipStream_t stream;
    uint64_t version;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  uint64_t version = 1;  // bumped whenever a value baked into a launch changes

  mapa_tuning tuning{64, 128, 0, 256, 0};
  uint64_t occ_shape = ~0ull;  // launch shape whose occupancy occ_blocks holds
  int occ_blocks = 0;
  bool profile = false;
  std::vector<mapa::ProfEvents> prof;       // recorded, not yet read
  std::vector<mapa::ProfEvents> prof_free;  // created earlier, ready for reuse
  double prof_ms = 0;
  int64_t prof_launches = 0;
  int64_t batches = 0;

  mapa::ServeState *serve = nullptr;  // non-null while the serving loop runs
};

namespace mapa {

int32_t sync_ctx(mapa_ctx *c);

// F!/(F-k)!: embeddings of a k-position pattern into F free vertices (0 if k > F).
unsigned long long perm_leaves(int F, int k);

// True when the nq queries name nq different servers (servers must be valid).
bool distinct_servers(mapa_ctx *c, const mapa_query *q, int32_t nq);
// Enqueue the fused small-batch launch for nq queries at q (device or pinned
// host memory), results to res, on stream s, counting self-check failures
// in workspace w.
int32_t enqueue_fused(mapa_ctx *c, const Workspace &w, const mapa_query *q, mapa_result *res,
                      int32_t nq, hipStream_t s);
void fill_args(mapa_ctx *c, const Workspace &w, BatchArgs &a);

// Enqueue the whole batch pipeline (prepare .. finalize) for nq queries that
// are already in device memory, writing nq results to d_res, on stream s.
int32_t enqueue_batch(mapa_ctx *c, const Workspace &w, const mapa_query *d_q,
                      mapa_result *d_res, int32_t nq, hipStream_t s);

void serve_teardown(mapa_ctx *c);  // stop and free a running serving loop

// Kernel timing (mapa_profile): record the start event of a timed launch on
// stream s (events come from a pool, so timing costs no event creation once
// warm), then its stop event, which queues the pair for mapa_get_stats.
int32_t prof_start(mapa_ctx *c, hipStream_t s, ProfEvents &ev);
int32_t prof_stop(mapa_ctx *c, hipStream_t s, const ProfEvents &ev);

// Back-neighbour table of a pattern kind (canonical or registered) with k positions.
unsigned long long pattern_nbtab(const mapa_ctx *c, int kind, int k);
// Validate nq host queries as mapa_query_batch does.
int32_t validate_queries(const mapa_ctx *c, const mapa_query *q, int32_t nq);
// Grow the API workspace to hold nq queries (no work may be in flight).
int32_t ensure_batch_capacity(mapa_ctx *c, size_t nq);

// Resolve the allocation-free batch's scratch array on `device` (current).
int32_t noalloc_setup(int device);

}  // namespace mapa
