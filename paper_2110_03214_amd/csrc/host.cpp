// Host core of the MAPA allocation library: context, topology registry,
// device-resident server state, argument validation and the batch driver.
// Every compute step runs in kernels.hip; this file only checks arguments,
// manages memory and enqueues work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>

#include "ctx.h"
#include "wide.h"

using namespace mapa;

namespace mapa {

namespace {
thread_local std::string g_err;
}

int32_t fail(int32_t code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char *last_error() { return g_err.c_str(); }

// ------------------------------------------------------------- workspace

int32_t ws_create(Workspace &w, size_t enum_bytes) {
  unsigned long long items = enum_bytes / sizeof(uint2);
  items = std::min<unsigned long long>(items, 1ull << 31);
  if (items < (unsigned long long)kPadReserve + 1024)
    return fail(MAPA_ERR_INVALID_ARG, "enumeration buffer of %zu bytes too small (need >= %llu)",
                enum_bytes, (unsigned long long)(kPadReserve + 1024) * sizeof(uint2));
  if (dev_alloc(&w.d_items, items) != hipSuccess || dev_alloc(&w.d_ctr, 1) != hipSuccess) {
    ws_destroy(w);
    return fail(MAPA_ERR_OOM, "enumeration buffer of %zu bytes: allocation failed", enum_bytes);
  }
  w.cap_items = items;
  MAPA_HIPCHK(hipMemset(w.d_ctr, 0, sizeof(Counters)));
  return MAPA_OK;
}

int32_t ws_ensure_q(Workspace &w, size_t nq) {
  if (nq <= w.cap_q) return MAPA_OK;
  size_t cap = std::max<size_t>(1024, w.cap_q);
  while (cap < nq) cap *= 2;
  dev_free(w.d_plan);
  dev_free(w.d_acc_count);
  dev_free(w.d_acc_best);
  dev_free(w.d_done);
  dev_free(w.d_q);
  dev_free(w.d_res);
  w.cap_q = 0;
  if (dev_alloc(&w.d_plan, cap) != hipSuccess || dev_alloc(&w.d_acc_count, cap) != hipSuccess ||
      dev_alloc(&w.d_acc_best, cap) != hipSuccess || dev_alloc(&w.d_done, cap) != hipSuccess ||
      dev_alloc(&w.d_q, cap) != hipSuccess || dev_alloc(&w.d_res, cap) != hipSuccess)
    return fail(MAPA_ERR_OOM, "batch workspace for %zu queries: device allocation failed", nq);
  // accumulators and block counters start at zero; every batch leaves them so
  MAPA_HIPCHK(hipMemset(w.d_acc_count, 0, cap * sizeof(unsigned long long)));
  MAPA_HIPCHK(hipMemset(w.d_acc_best, 0, cap * sizeof(unsigned long long)));
  MAPA_HIPCHK(hipMemset(w.d_done, 0, cap * sizeof(uint32_t)));
  MAPA_HIPCHK(hipDeviceSynchronize());
  w.cap_q = cap;
  return MAPA_OK;
}

void ws_destroy(Workspace &w) {
  dev_free(w.d_plan);
  dev_free(w.d_acc_count);
  dev_free(w.d_acc_best);
  dev_free(w.d_done);
  dev_free(w.d_q);
  dev_free(w.d_res);
  dev_free(w.d_items);
  dev_free(w.d_ctr);
  w.cap_q = 0;
  w.cap_items = 0;
}

// ------------------------------------------------------------- helpers

int32_t sync_ctx(mapa_ctx *c) {
  if (!c->has_device) return MAPA_OK;
  MAPA_HIPCHK(hipSetDevice(c->device));
  MAPA_HIPCHK(hipEventSynchronize(c->last));
  return MAPA_OK;
}

void fill_args(mapa_ctx *c, const Workspace &w, BatchArgs &a) {
  a.plan = w.d_plan;
  a.acc_count = w.d_acc_count;
  a.acc_best = w.d_acc_best;
  a.items = w.d_items;
  a.cap_items = w.cap_items;
  a.ctr = w.d_ctr;
  a.server_topo = c->d_server_topo;
  a.busy = c->d_busy;
  a.commit_slot = c->d_commit_slot;
  a.nservers = (int32_t)c->server_topo.size();
  a.topo_n = c->d_topo_n;
  a.topo_W = c->d_topo_W;
  a.rows = c->d_rows;
  a.topo_maxw = c->d_topo_maxw;
  a.eff_rank = c->d_eff_rank;
  a.eff_key = c->d_eff_key;
  a.ntopo = (int32_t)c->topo_n.size();
  a.wpr = c->wpr;
  a.split_d = c->d_split;
  a.pat_nbtab = c->d_pat_nbtab;
  a.pat_k = c->d_pat_k;
  a.pat_nbtab_ord = c->d_pat_nbtab_ord;
  a.pat_order = c->d_pat_order;
  const int threads = c->tuning.threads_per_block;
  const size_t lds_bytes = (size_t)a.ntopo * kTopoWords * c->wpr * sizeof(uint32_t);
  a.rows_in_lds = lds_bytes <= 48 * 1024 ? 1 : 0;
  // widest pair_level of the k_enumerate variant: the wider, the more
  // registers (fewer waves per SIMD), so up to 12 free vertices only where
  // topologies have 10 or more vertices (measured: 8 is best below that)
  const int max_n = c->topo_n.empty() ? 0 : *std::max_element(c->topo_n.begin(), c->topo_n.end());
  a.pair = c->wpr != 1 ? 0 : max_n >= 10 ? 12 : 6;
  if (c->wpr == 1 && c->tuning.pair_width != 0) a.pair = c->tuning.pair_width < 0 ? 0 : c->tuning.pair_width;
  int per_cu = c->tuning.blocks_per_cu;
  if (per_cu <= 0) {
    // the occupancy query costs microseconds: ask once per launch shape
    const uint64_t shape = ((uint64_t)lds_bytes << 24) | ((uint64_t)threads << 8) |
                           ((uint64_t)a.pair << 5) | ((uint64_t)c->wpr << 1) | (uint64_t)a.rows_in_lds;
    if (shape != c->occ_shape) {
      c->occ_blocks = enumerate_occupancy(c->wpr, a.rows_in_lds, a.pair, threads, lds_bytes);
      c->occ_shape = shape;
    }
    per_cu = c->occ_blocks;
  }
  if (per_cu <= 0) per_cu = 4;
  a.enum_blocks = std::max(1, c->cu_count) * per_cu;
  a.enum_threads = threads;
  const unsigned long long lanes = (unsigned long long)std::max(1, c->cu_count) * per_cu * threads;
  a.lanes = std::max<unsigned long long>(1, lanes);
  a.mean_leaves = (uint32_t)std::max(1, c->tuning.mean_item_leaves);
}

unsigned long long perm_leaves(int F, int k) {
  if (k > F) return 0;
  unsigned long long p = 1;
  for (int i = 0; i < k; ++i) p *= (unsigned long long)(F - i);
  return p;
}

bool distinct_servers(mapa_ctx *c, const mapa_query *q, int32_t nq) {
  if (c->srv_stamp.size() < c->server_topo.size()) c->srv_stamp.resize(c->server_topo.size(), 0);
  if (++c->stamp == 0) {  // wrapped: clear the old stamps
    std::fill(c->srv_stamp.begin(), c->srv_stamp.end(), 0u);
    c->stamp = 1;
  }
  for (int32_t i = 0; i < nq; ++i) {
    uint32_t &m = c->srv_stamp[(size_t)q[i].server];
    if (m == c->stamp) return false;
    m = c->stamp;
  }
  return true;
}

int32_t enqueue_fused(mapa_ctx *c, const Workspace &w, const mapa_query *q, mapa_result *res,
                      int32_t nq, hipStream_t s) {
  FusedArgs f;
  std::memset(&f, 0, sizeof f);
  f.q = q;
  f.res = res;
  f.nq = nq;
  f.server_topo = c->d_server_topo;
  f.busy = c->d_busy;
  f.nservers = (int32_t)c->server_topo.size();
  f.topo_n = c->d_topo_n;
  f.rows = c->d_rows;
  f.wpr = c->wpr;
  f.topo_maxw = c->d_topo_maxw;
  f.eff_rank = c->d_eff_rank;
  f.eff_key = c->d_eff_key;
  f.pat_nbtab = c->d_pat_nbtab;
  f.pat_k = c->d_pat_k;
  f.pat_nbtab_ord = c->d_pat_nbtab_ord;
  f.pat_order = c->d_pat_order;
  f.self_check_failures = &w.d_ctr->self_check_failures;
  f.acc_count = w.d_acc_count;
  f.acc_best = w.d_acc_best;
  f.done = w.d_done;
  // spread small batches over several blocks per query, up to ~4 per CU
  const int target = std::max(1, c->cu_count) * 4;
  f.bpq = std::max(1, std::min(kFusedMaxBlocksPerQuery, target / std::max(1, nq)));
  MAPA_HIPCHK(launch_fused(f, s));
  return MAPA_OK;
}

int32_t prof_start(mapa_ctx *c, hipStream_t s, ProfEvents &ev) {
  if (!c->prof_free.empty()) {
    ev = c->prof_free.back();
    c->prof_free.pop_back();
  } else {
    MAPA_HIPCHK(hipEventCreate(&ev.start));
    if (hipEventCreate(&ev.stop) != hipSuccess) {
      (void)hipEventDestroy(ev.start);
      return fail(MAPA_ERR_DEVICE, "hipEventCreate failed");
    }
  }
  const hipError_t e = hipEventRecord(ev.start, s);
  if (e != hipSuccess) {
    c->prof_free.push_back(ev);
    return fail(MAPA_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
  }
  return MAPA_OK;
}

int32_t prof_stop(mapa_ctx *c, hipStream_t s, const ProfEvents &ev) {
  const hipError_t e = hipEventRecord(ev.stop, s);
  if (e != hipSuccess) {
    c->prof_free.push_back(ev);
    return fail(MAPA_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
  }
  c->prof.push_back(ev);
  return MAPA_OK;
}

int32_t enqueue_batch(mapa_ctx *c, const Workspace &w, const mapa_query *d_q, mapa_result *d_res,
                      int32_t nq, hipStream_t s) {
  BatchArgs a;
  std::memset(&a, 0, sizeof a);
  fill_args(c, w, a);
  a.nq = nq;
  a.q = d_q;
  a.res = d_res;
  MAPA_HIPCHK(launch_batch_front(a, s));
  MAPA_HIPCHK(launch_enumerate(a, s));
  MAPA_HIPCHK(launch_finalize(a, s));
  return MAPA_OK;
}

}  // namespace mapa

namespace {

constexpr size_t kDefaultEnumBytes = 256ull << 20;

// Canonical pattern graphs (Sec. 3.1), as back-neighbour position masks:
// nb[kind][k][p] = { j < p : (j, p) is a pattern edge }.
Tables build_tables() {
  Tables t;
  std::memset(&t, 0, sizeof t);
  for (int k = 1; k <= kMaxK; ++k) {
    for (int p = 1; p < k; ++p) {
      // ring: consecutive positions, closed when k >= 3; k = 2 is one edge
      uint8_t ring = (uint8_t)(1u << (p - 1));
      if (p == k - 1 && k >= 3) ring |= 1u;
      t.nb[MAPA_RING][k][p] = ring;
      t.nb[MAPA_ALL_TO_ALL][k][p] = (uint8_t)((1u << p) - 1u);
      t.nb[MAPA_TREE][k][p] = (uint8_t)(1u << ((p - 1) / 2));
    }
  }
  for (int kind = 0; kind < 3; ++kind)
    for (int k = 1; k <= kMaxK; ++k) {
      unsigned long long tab = 0;
      for (int p = 0; p < k; ++p) tab |= (unsigned long long)t.nb[kind][k][p] << (8 * p);
      t.nbtab[kind][k] = tab;
    }
  for (int m = 2; m <= kMaxN; ++m)
    t.inv[m] = (uint32_t)(((1ull << 32) + (unsigned long long)m - 1) / (unsigned long long)m);
  for (int F = 0; F <= kMaxN; ++F)
    for (int d = 0; d <= kMaxK; ++d) {
      unsigned long long v = 1;
      for (int i = 0; i < d; ++i) v *= (unsigned long long)std::max(0, F - i);
      t.perm[F][d] = v;
    }
  // Buckets laid out costliest items first (longest-processing-time order),
  // so the last chunks the persistent waves pick up are the cheapest.  An
  // item's cost in VALU instructions, roughly: its setup, every interior
  // node of its subtree (the node's own score terms and its children's
  // bookkeeping) and every leaf.
  constexpr double kItemCost = 300, kNodeCost = 30, kLeafCost = 20;
  std::vector<std::pair<double, int>> order;
  for (int b = 0; b < kNumBuckets; ++b) {
    const int Fp = b % kFp, L = (b / kFp) % kMaxK + 1;  // see bucket_id
    double cost = 0;
    if (Fp >= L) {
      double nodes = 1;  // subtree nodes at depth i below the prefix
      cost = kItemCost;
      for (int i = 1; i <= L; ++i) {
        nodes *= (Fp - i + 1);
        cost += nodes * (i < L ? kNodeCost : kLeafCost);
      }
    }
    order.push_back({-cost, b});
  }
  std::sort(order.begin(), order.end());
  for (int r = 0; r < kNumBuckets; ++r) t.rank_bucket[r] = (uint16_t)order[r].second;
  return t;
}

// Prefix depth per (F, k, split): the smallest d <= k-1 whose items hold at
// most min_leaves * 2^j embeddings; 0 (whole query) for the last split.
std::vector<uint8_t> build_split_table(int min_leaves) {
  std::vector<uint8_t> tab(kSplitTable, 0);
  auto perm = [](int F, int k) {
    unsigned long long v = 1;
    for (int i = 0; i < k; ++i) v *= (unsigned long long)std::max(0, F - i);
    return v;
  };
  for (int F = 0; F <= kMaxN; ++F)
    for (int k = 1; k <= kMaxK; ++k)
      for (int j = 0; j < kSplitWhole; ++j) {
        const unsigned long long T = (unsigned long long)min_leaves << j;
        int d = 0;
        while (d < k - 1 && perm(F - d, k - d) > T) ++d;
        tab[((size_t)F * (kMaxK + 1) + k) * kNumSplits + j] = (uint8_t)d;
      }
  return tab;
}

int weight_class(const uint8_t *W, int n) {
  int mx = 0;
  for (int i = 0; i < n * n; ++i) mx = std::max(mx, (int)W[i]);
  return mx <= 3 ? 1 : mx <= 15 ? 2 : 4;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Order this call after every earlier call of the context.
hipError_t begin_call(mapa_ctx *c, hipStream_t s) { return hipStreamWaitEvent(s, c->last, 0); }
hipError_t end_call(mapa_ctx *c, hipStream_t s) { return hipEventRecord(c->last, s); }

int32_t not_while_serving(mapa_ctx *c, const char *fn) {
  if (c->serve) return fail(MAPA_ERR_STATE, "%s: the serving loop owns the context", fn);
  return MAPA_OK;
}

void build_rows(const uint8_t *W16, int n, int wpr, uint32_t *out /* kTopoWords * wpr */) {
  for (int v = 0; v < 16; ++v)
    for (int w = 0; w < wpr; ++w) {
      uint32_t lo = 0, hi = 0;
      if (v < n)
        for (int u = 0; u < n; ++u) {
          const uint8_t x = W16[v * 16 + u];
          lo |= ((x >> (2 * w)) & 1u) << u;
          hi |= ((x >> (2 * w + 1)) & 1u) << u;
        }
      out[v * wpr + w] = lo | (hi << 16);
    }
  // packed weights: field width 2 * wpr bits, 16 / wpr fields per word
  const int bits = 2 * wpr, per = 16 / wpr;
  uint32_t *pk = out + 16 * wpr;
  for (int v = 0; v < 16; ++v)
    for (int w = 0; w < wpr; ++w) {
      uint32_t word = 0;
      for (int f = 0; f < per; ++f) {
        const int u = w * per + f;
        if (v < n && u < n) word |= (uint32_t)W16[v * 16 + u] << (bits * f);
      }
      pk[v * wpr + w] = word;
    }
}

// Upload the device copies of the topology tables: all of them after growth
// or a change of row format, else only topology `first` onwards.  Caller has
// synchronised the context.
int32_t upload_topologies(mapa_ctx *c, size_t first, bool all) {
  const size_t T = c->topo_n.size();
  if (T > c->cap_topos) {
    all = true;
    size_t cap = std::max<size_t>(16, c->cap_topos);
    while (cap < T) cap *= 2;
    dev_free(c->d_topo_n);
    dev_free(c->d_topo_W);
    dev_free(c->d_rows);
    dev_free(c->d_topo_maxw);
    c->cap_topos = 0;
    if (dev_alloc(&c->d_topo_n, cap) != hipSuccess || dev_alloc(&c->d_topo_W, cap * 256) != hipSuccess ||
        dev_alloc(&c->d_rows, cap * kTopoWords * 4) != hipSuccess ||
        dev_alloc(&c->d_topo_maxw, cap) != hipSuccess)
      return fail(MAPA_ERR_OOM, "topology tables: device allocation failed");
    c->cap_topos = cap;
  }
  const size_t t0 = all ? 0 : first;
  if (t0 >= T) return MAPA_OK;
  const size_t nt = T - t0;
  std::vector<uint8_t> W(nt * 256);
  std::vector<uint32_t> rows(nt * kTopoWords * c->wpr);
  for (size_t t = t0; t < T; ++t) {
    std::memcpy(&W[(t - t0) * 256], c->topo_W[t].data(), 256);
    build_rows(c->topo_W[t].data(), std::min(c->topo_n[t], kMaxN), c->wpr,
               &rows[(t - t0) * kTopoWords * c->wpr]);
  }
  MAPA_HIPCHK(hipMemcpy(c->d_topo_n + t0, c->topo_n.data() + t0, nt * sizeof(int32_t),
                        hipMemcpyHostToDevice));
  MAPA_HIPCHK(hipMemcpy(c->d_topo_W + t0 * 256, W.data(), W.size(), hipMemcpyHostToDevice));
  MAPA_HIPCHK(hipMemcpy(c->d_rows + t0 * kTopoWords * c->wpr, rows.data(), rows.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
  MAPA_HIPCHK(hipMemcpy(c->d_topo_maxw + t0, c->topo_maxw.data() + t0, nt, hipMemcpyHostToDevice));
  return MAPA_OK;
}

// Eq. 2, the predicted effective bandwidth of a link mix: x double NVLinks,
// y single NVLinks, z PCIe links, coefficients of Table "Values of
// Coefficients" in the order of the equation's features.
double effbw_eq2(int x, int y, int z) {
  static const double theta[14] = {16.396, 4.536,  1.556,  -20.694, -9.467, 7.615,  -7.973,
                                   12.733, -4.195, -8.413, 62.851,  27.418, -5.114, -46.973};
  const double X = x, Y = y, Z = z;
  const double f[14] = {X,           Y,           Z,           1 / (X + 1),     1 / (Y + 1),
                        1 / (Z + 1), X * Y,       Y * Z,       Z * X,           1 / (X * Y + 1),
                        1 / (Y * Z + 1), 1 / (Z * X + 1), X * Y * Z, 1 / (X * Y * Z + 1)};
  double v = 0;
  for (int i = 0; i < 14; ++i) v += theta[i] * f[i];
  return v;
}

// The device's Eq. 2 tables: per edge count E (up to 66, the wide path's
// 12-vertex all-to-all), each mix's dense rank (equal values share a rank,
// so maximising the rank maximises EffBW and keeps its ties) and its
// reported key round(1000 * EffBW).
int32_t upload_effbw_tables(mapa_ctx *c) {
  std::vector<uint16_t> rank(kEffEntriesWide, 0);
  std::vector<int32_t> key(kEffEntriesWide, 0);
  for (int E = 0; E <= kWideMaxEdges; ++E) {
    std::vector<double> vals;
    for (int x = 0; x <= E; ++x)
      for (int y = 0; x + y <= E; ++y) vals.push_back(effbw_eq2(x, y, E - x - y));
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    for (int x = 0; x <= E; ++x)
      for (int y = 0; x + y <= E; ++y) {
        const double v = effbw_eq2(x, y, E - x - y);
        const size_t at = (size_t)eff_off(E) + (size_t)x * (E + 1) + y;
        rank[at] = (uint16_t)(std::lower_bound(vals.begin(), vals.end(), v) - vals.begin());
        key[at] = (int32_t)std::llround(1000.0 * v);
      }
  }
  if (dev_alloc(&c->d_eff_rank, kEffEntriesWide) != hipSuccess ||
      dev_alloc(&c->d_eff_key, kEffEntriesWide) != hipSuccess)
    return fail(MAPA_ERR_OOM, "effective-bandwidth tables: device allocation failed");
  MAPA_HIPCHK(hipMemcpy(c->d_eff_rank, rank.data(), rank.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  MAPA_HIPCHK(hipMemcpy(c->d_eff_key, key.data(), key.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return MAPA_OK;
}

int32_t grow_servers(mapa_ctx *c, size_t need) {
  if (need <= c->cap_servers) return MAPA_OK;
  size_t cap = std::max<size_t>(1024, c->cap_servers);
  while (cap < need) cap *= 2;
  int32_t *st = nullptr;
  uint32_t *busy = nullptr;
  unsigned long long *slot = nullptr;
  if (dev_alloc(&st, cap) != hipSuccess || dev_alloc(&busy, cap) != hipSuccess ||
      dev_alloc(&slot, cap) != hipSuccess) {
    dev_free(st);
    dev_free(busy);
    dev_free(slot);
    return fail(MAPA_ERR_OOM, "server tables: device allocation failed");
  }
  MAPA_HIPCHK(hipMemset(busy, 0, cap * sizeof(uint32_t)));
  MAPA_HIPCHK(hipMemset(st, 0, cap * sizeof(int32_t)));
  MAPA_HIPCHK(hipMemset(slot, 0xFF, cap * sizeof(unsigned long long)));
  if (c->cap_servers) {
    MAPA_HIPCHK(hipMemcpy(st, c->d_server_topo, c->cap_servers * sizeof(int32_t), hipMemcpyDeviceToDevice));
    MAPA_HIPCHK(hipMemcpy(busy, c->d_busy, c->cap_servers * sizeof(uint32_t), hipMemcpyDeviceToDevice));
    MAPA_HIPCHK(hipMemcpy(slot, c->d_commit_slot, c->cap_servers * sizeof(unsigned long long),
                          hipMemcpyDeviceToDevice));
  }
  dev_free(c->d_server_topo);
  dev_free(c->d_busy);
  dev_free(c->d_commit_slot);
  c->d_server_topo = st;
  c->d_busy = busy;
  c->d_commit_slot = slot;
  c->cap_servers = cap;
  return MAPA_OK;
}

void drop_graphs(mapa_ctx *c) {
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
  ++c->version;
}

int32_t upload_split_table(mapa_ctx *c) {
  const std::vector<uint8_t> tab = build_split_table(std::max(1, c->tuning.min_leaves_per_item));
  if (!c->d_split && dev_alloc(&c->d_split, kSplitTable) != hipSuccess)
    return fail(MAPA_ERR_OOM, "split table: device allocation failed");
  MAPA_HIPCHK(hipMemcpy(c->d_split, tab.data(), tab.size(), hipMemcpyHostToDevice));
  return MAPA_OK;
}


int32_t ensure_small(mapa_ctx *c, size_t n) {
  if (n <= c->cap_small) return MAPA_OK;
  int32_t rc = sync_ctx(c);
  if (rc) return rc;
  size_t cap = std::max<size_t>(1024, c->cap_small);
  while (cap < n) cap *= 2;
  dev_free(c->d_ids);
  dev_free(c->d_masks);
  dev_free(c->d_handles);
  c->cap_small = 0;
  if (dev_alloc(&c->d_ids, cap) != hipSuccess || dev_alloc(&c->d_masks, cap) != hipSuccess ||
      dev_alloc(&c->d_handles, cap) != hipSuccess)
    return fail(MAPA_ERR_OOM, "state scratch: device allocation failed");
  c->cap_small = cap;
  return MAPA_OK;
}

int32_t validate_query(const mapa_ctx *c, const mapa_query &q, int32_t i) {
  if (q.server < 0 || (size_t)q.server >= c->server_topo.size())
    return fail(MAPA_ERR_UNKNOWN_SERVER, "query %d: unknown server %d", i, q.server);
  if (q.k > kMaxK)
    return fail(MAPA_ERR_UNSUPPORTED, "query %d: k=%d > %d (mapa_query_batch_wide takes up to %d)", i,
                q.k, kMaxK, MAPA_MAX_K_WIDE);
  if (c->topo_n[c->server_topo[q.server]] > kMaxN)
    return fail(MAPA_ERR_UNSUPPORTED, "query %d: server %d has %d accelerators (> %d: use "
                "mapa_query_batch_wide)", i, q.server, c->topo_n[c->server_topo[q.server]], kMaxN);
  if (q.k < 1) return fail(MAPA_ERR_INVALID_ARG, "query %d: k=%d < 1", i, q.k);
  if (q.kind > MAPA_TREE) {
    const int id = q.kind - MAPA_PATTERN_BASE;
    if (id < 0 || id >= c->npat)
      return fail(MAPA_ERR_INVALID_ARG, "query %d: kind=%d is neither a pattern kind nor a "
                  "registered pattern", i, q.kind);
    if (c->pat_k[id] != q.k)
      return fail(MAPA_ERR_INVALID_ARG, "query %d: k=%d but registered pattern %d has %d "
                  "vertices", i, q.k, id, c->pat_k[id]);
  }
  if (q.mode > 1) return fail(MAPA_ERR_INVALID_ARG, "query %d: mode=%d", i, q.mode);
  if (q.commit > 1) return fail(MAPA_ERR_INVALID_ARG, "query %d: commit=%d", i, q.commit);
  if (q.a < 0 || q.a > MAPA_MAX_AB || q.b < 0 || q.b > MAPA_MAX_AB)
    return fail(MAPA_ERR_INVALID_ARG, "query %d: key weights (%d,%d) outside 0..%d", i, q.a, q.b,
                MAPA_MAX_AB);
  if (q.metric != MAPA_METRIC_WEIGHTED && q.metric != MAPA_METRIC_EFFBW)
    return fail(MAPA_ERR_INVALID_ARG, "query %d: metric=%d", i, q.metric);
  if (q.metric == MAPA_METRIC_EFFBW && c->topo_maxw[c->server_topo[q.server]] > 2)
    return fail(MAPA_ERR_UNSUPPORTED,
                "query %d: effective bandwidth needs link weights 0, 1, 2 (PCIe, single, double "
                "NVLink); server %d has weight %d", i, q.server, c->topo_maxw[c->server_topo[q.server]]);
  return MAPA_OK;
}

}  // namespace

namespace mapa {

int32_t ensure_batch_capacity(mapa_ctx *c, size_t nq) {
  if (nq <= c->ws.cap_q) return MAPA_OK;
  int32_t rc = sync_ctx(c);
  if (rc) return rc;
  drop_graphs(c);
  return ws_ensure_q(c->ws, nq);
}

int32_t validate_queries(const mapa_ctx *c, const mapa_query *q, int32_t nq) {
  for (int32_t i = 0; i < nq; ++i)
    if (int32_t rc = validate_query(c, q[i], i)) return rc;
  return MAPA_OK;
}

unsigned long long pattern_nbtab(const mapa_ctx *c, int kind, int k) {
  if (kind > MAPA_TREE) return c->pat_nbtab[(size_t)(kind - MAPA_PATTERN_BASE)];
  static const Tables t = build_tables();
  return t.nbtab[kind][k];
}

}  // namespace mapa

// =================================================================== ABI

extern "C" {

const char *mapa_last_error(void) { return mapa::last_error(); }

int32_t mapa_ctx_create(int32_t device, size_t enum_buffer_bytes, mapa_ctx **out) {
  if (!out) return fail(MAPA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  mapa_ctx *c = new (std::nothrow) mapa_ctx();
  if (!c) return fail(MAPA_ERR_OOM, "context allocation failed");
  c->pat_nbtab.assign(MAPA_MAX_PATTERNS, 0);
  c->pat_k.assign(MAPA_MAX_PATTERNS, 0);
  c->enum_bytes = enum_buffer_bytes ? enum_buffer_bytes : kDefaultEnumBytes;
  if (device < 0) {  // validation-only context
    *out = c;
    return MAPA_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
    delete c;
    return fail(MAPA_ERR_NO_DEVICE, "HIP device %d not available (%d devices)", device, ndev);
  }
  c->device = device;
  c->has_device = true;
  auto bail = [&](int32_t rc) {
    mapa_ctx_destroy(c);
    return rc;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(fail(MAPA_ERR_DEVICE, "hipSetDevice failed"));
  if (int32_t rc0 = noalloc_setup(device)) return bail(rc0);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return bail(fail(MAPA_ERR_DEVICE, "hipGetDeviceProperties failed"));
  c->cu_count = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->internal, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->last, hipEventDisableTiming) != hipSuccess)
    return bail(fail(MAPA_ERR_DEVICE, "stream/event creation failed"));
  if (hipEventRecord(c->last, c->internal) != hipSuccess)
    return bail(fail(MAPA_ERR_DEVICE, "hipEventRecord failed"));
  const Tables t = build_tables();
  if (upload_tables(t) != hipSuccess) return bail(fail(MAPA_ERR_DEVICE, "table upload failed"));
  int32_t rc = ws_create(c->ws, c->enum_bytes);
  if (rc) return bail(rc);
  rc = upload_split_table(c);
  if (rc) return bail(rc);
  rc = upload_effbw_tables(c);
  if (rc) return bail(rc);
  if (dev_alloc(&c->d_flag, 1) != hipSuccess) return bail(fail(MAPA_ERR_OOM, "flag allocation failed"));
  if (dev_alloc(&c->d_pat_nbtab, MAPA_MAX_PATTERNS) != hipSuccess ||
      dev_alloc(&c->d_pat_k, MAPA_MAX_PATTERNS) != hipSuccess ||
      dev_alloc(&c->d_pat_nbtab_ord, MAPA_MAX_PATTERNS) != hipSuccess ||
      dev_alloc(&c->d_pat_order, MAPA_MAX_PATTERNS) != hipSuccess)
    return bail(fail(MAPA_ERR_OOM, "pattern table allocation failed"));
  if (hipMemset(c->d_pat_nbtab, 0, MAPA_MAX_PATTERNS * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(c->d_pat_k, 0, MAPA_MAX_PATTERNS) != hipSuccess)
    return bail(fail(MAPA_ERR_DEVICE, "pattern table initialisation failed"));
  if (hipDeviceSynchronize() != hipSuccess) return bail(fail(MAPA_ERR_DEVICE, "device init failed"));
  *out = c;
  return MAPA_OK;
}

int32_t mapa_ctx_destroy(mapa_ctx *c) {
  if (!c) return MAPA_OK;
  serve_teardown(c);
  if (c->has_device) {
    (void)hipSetDevice(c->device);
    if (c->last) (void)hipEventSynchronize(c->last);
    (void)hipDeviceSynchronize();
    for (auto *v : {&c->prof, &c->prof_free})
      for (auto &e : *v) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
      }
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    dev_free(c->d_pat_nbtab);
    dev_free(c->d_pat_k);
    dev_free(c->d_pat_nbtab_ord);
    dev_free(c->d_pat_order);
    dev_free(c->d_wide_rows);
    if (c->wide_buf.d) (void)hipFree(c->wide_buf.d);
    c->wide_buf.d = nullptr;
    dev_free(c->d_topo_n);
    dev_free(c->d_topo_W);
    dev_free(c->d_rows);
    dev_free(c->d_server_topo);
    dev_free(c->d_busy);
    dev_free(c->d_commit_slot);
    ws_destroy(c->ws);
    dev_free(c->d_ids);
    dev_free(c->d_masks);
    dev_free(c->d_handles);
    dev_free(c->d_flag);
    dev_free(c->d_split);
    dev_free(c->d_topo_maxw);
    dev_free(c->d_eff_rank);
    dev_free(c->d_eff_key);
    if (c->h_fq) (void)hipHostFree(c->h_fq);
    if (c->h_fres) (void)hipHostFree(c->h_fres);
    if (c->last) (void)hipEventDestroy(c->last);
    if (c->internal) (void)hipStreamDestroy(c->internal);
  }
  delete c;
  return MAPA_OK;
}

int32_t mapa_create_topology(mapa_ctx *c, int32_t n, const uint8_t *W, int32_t num_servers,
                             int32_t *topo_id, int32_t *first_server) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_create_topology")) return rc;
  if (n < 1) return fail(MAPA_ERR_INVALID_ARG, "n=%d < 1", n);
  if (n > MAPA_MAX_N_WIDE) return fail(MAPA_ERR_UNSUPPORTED, "n=%d > %d", n, MAPA_MAX_N_WIDE);
  if (!W) return fail(MAPA_ERR_INVALID_ARG, "W is NULL");
  if (num_servers < 0) return fail(MAPA_ERR_INVALID_ARG, "num_servers=%d < 0", num_servers);
  for (int i = 0; i < n; ++i) {
    if (W[i * n + i] != 0) return fail(MAPA_ERR_INVALID_ARG, "W[%d][%d] != 0", i, i);
    for (int j = 0; j < n; ++j)
      if (W[i * n + j] != W[j * n + i])
        return fail(MAPA_ERR_INVALID_ARG, "W not symmetric at (%d,%d)", i, j);
  }
  if (c->topo_n.size() >= 65535) return fail(MAPA_ERR_UNSUPPORTED, "too many topologies");
  if (c->server_topo.size() + (size_t)num_servers > (size_t)INT32_MAX)
    return fail(MAPA_ERR_UNSUPPORTED, "too many servers");
  // the batch path keeps 16x16 weights (zero for wider servers, which only
  // the wide path queries); the wide path keeps every topology as 32x32
  std::array<uint8_t, 256> w16{};
  std::array<uint8_t, 1024> w32{};
  uint8_t maxw = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (n <= kMaxN) w16[i * 16 + j] = W[i * n + j];
      w32[i * 32 + j] = W[i * n + j];
      maxw = std::max(maxw, W[i * n + j]);
    }
  const int32_t tid = (int32_t)c->topo_n.size();
  const int32_t first = (int32_t)c->server_topo.size();
  if (c->has_device) {
    int32_t rc = sync_ctx(c);
    if (rc) return rc;
    drop_graphs(c);
    const int old_wpr = c->wpr;
    c->topo_n.push_back(n);
    c->topo_W.push_back(w16);
    c->wide_W.push_back(w32);
    c->topo_maxw.push_back(maxw);
    if (n <= kMaxN) c->wpr = std::max(c->wpr, weight_class(W, n));
    rc = upload_topologies(c, (size_t)tid, c->wpr != old_wpr);
    if (!rc) rc = grow_servers(c, first + (size_t)num_servers);
    if (rc) {
      c->topo_n.pop_back();
      c->topo_W.pop_back();
      c->wide_W.pop_back();
      c->topo_maxw.pop_back();
      c->wpr = old_wpr;
      return rc;
    }
    if (num_servers > 0) {
      std::vector<int32_t> ids(num_servers, tid);
      MAPA_HIPCHK(hipMemcpy(c->d_server_topo + first, ids.data(), num_servers * sizeof(int32_t),
                            hipMemcpyHostToDevice));
      MAPA_HIPCHK(hipMemset(c->d_busy + first, 0, num_servers * sizeof(uint32_t)));
    }
  } else {
    c->topo_n.push_back(n);
    c->topo_W.push_back(w16);
    c->wide_W.push_back(w32);
    c->topo_maxw.push_back(maxw);
  }
  c->server_topo.insert(c->server_topo.end(), (size_t)num_servers, tid);
  if (topo_id) *topo_id = tid;
  if (first_server) *first_server = first;
  return MAPA_OK;
}

int32_t mapa_create_pattern(mapa_ctx *c, int32_t k, int32_t num_edges, const uint8_t *edges,
                            int32_t *kind_out) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (k > kMaxK) return fail(MAPA_ERR_UNSUPPORTED, "pattern of %d vertices > %d", k, kMaxK);
  if (k < 1) return fail(MAPA_ERR_INVALID_ARG, "pattern of %d vertices", k);
  if (num_edges < 0 || num_edges > k * (k - 1) / 2)
    return fail(MAPA_ERR_INVALID_ARG, "%d edges on %d vertices", num_edges, k);
  if (num_edges > 0 && !edges) return fail(MAPA_ERR_INVALID_ARG, "edges is NULL");
  if (c->npat >= MAPA_MAX_PATTERNS)
    return fail(MAPA_ERR_STATE, "all %d pattern slots are taken", MAPA_MAX_PATTERNS);
  // back-neighbour table: edge (u, v) with u < v makes u an earlier neighbour of v
  uint8_t nb[kMaxK] = {};
  for (int e = 0; e < num_edges; ++e) {
    const int u = edges[2 * e], v = edges[2 * e + 1];
    if (u >= k || v >= k || u == v)
      return fail(MAPA_ERR_INVALID_ARG, "edge %d = (%d, %d) on a pattern of %d vertices", e, u, v, k);
    const int lo = std::min(u, v), hi = std::max(u, v);
    if (nb[hi] & (1u << lo)) return fail(MAPA_ERR_INVALID_ARG, "edge (%d, %d) given twice", lo, hi);
    nb[hi] |= (uint8_t)(1u << lo);
  }
  unsigned long long tab = 0;
  for (int p = 0; p < k; ++p) tab |= (unsigned long long)nb[p] << (8 * p);
  // matching order for LINKED search (Sec. 3.3: a match must keep pattern
  // adjacency, so a candidate is pruned as soon as it misses an edge to an
  // already placed neighbour): the vertex of largest degree first, then
  // repeatedly the unplaced vertex with the most placed neighbours (ties:
  // larger degree, then smaller number), so every placed vertex after the
  // first of its connected component has an earlier neighbour
  uint8_t adj[kMaxK] = {};
  for (int v = 0; v < k; ++v)
    for (int u = 0; u < v; ++u)
      if ((nb[v] >> u) & 1u) {
        adj[v] |= (uint8_t)(1u << u);
        adj[u] |= (uint8_t)(1u << v);
      }
  uint32_t placed = 0, order = 0;
  int pos_of[kMaxK] = {};
  for (int p = 0; p < k; ++p) {
    int best = -1, best_links = -1, best_deg = -1;
    for (int v = 0; v < k; ++v) {
      if ((placed >> v) & 1u) continue;
      const int links = __builtin_popcount(adj[v] & placed), deg = __builtin_popcount(adj[v]);
      if (links > best_links || (links == best_links && deg > best_deg)) {
        best = v;
        best_links = links;
        best_deg = deg;
      }
    }
    placed |= 1u << best;
    order |= (uint32_t)best << (4 * p);
    pos_of[best] = p;
  }
  for (int p = k; p < 8; ++p) order |= (uint32_t)p << (4 * p);  // unused digits: identity
  unsigned long long tab_ord = 0;
  for (int p = 0; p < k; ++p) {
    const int v = (order >> (4 * p)) & 15;
    uint32_t m = 0;
    for (int u = 0; u < k; ++u)
      if (((adj[v] >> u) & 1u) && pos_of[u] < p) m |= 1u << pos_of[u];
    tab_ord |= (unsigned long long)m << (8 * p);
  }
  const int id = c->npat;
  if (c->has_device) {
    if (hipSetDevice(c->device) != hipSuccess) return fail(MAPA_ERR_DEVICE, "hipSetDevice failed");
    // the tables first, then k: a slot is valid to the kernels once its k matches
    const uint8_t kk = (uint8_t)k;
    MAPA_HIPCHK(hipMemcpy(c->d_pat_nbtab + id, &tab, sizeof tab, hipMemcpyHostToDevice));
    MAPA_HIPCHK(hipMemcpy(c->d_pat_nbtab_ord + id, &tab_ord, sizeof tab_ord, hipMemcpyHostToDevice));
    MAPA_HIPCHK(hipMemcpy(c->d_pat_order + id, &order, sizeof order, hipMemcpyHostToDevice));
    MAPA_HIPCHK(hipMemcpy(c->d_pat_k + id, &kk, 1, hipMemcpyHostToDevice));
  }
  c->pat_nbtab[id] = tab;
  c->pat_k[id] = (uint8_t)k;
  c->npat = id + 1;
  if (kind_out) *kind_out = MAPA_PATTERN_BASE + id;
  return MAPA_OK;
}

int32_t mapa_set_busy(mapa_ctx *c, int32_t count, const int32_t *ids, const uint32_t *masks,
                      uint32_t flags, void *stream) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_set_busy")) return rc;
  if (count < 0) return fail(MAPA_ERR_INVALID_ARG, "count < 0");
  if (count == 0) return MAPA_OK;
  if (!ids || !masks) return fail(MAPA_ERR_INVALID_ARG, "NULL array");
  const bool dev = flags & MAPA_DEVICE_PTRS;
  if (!dev) {
    for (int32_t i = 0; i < count; ++i) {
      const int32_t s = ids[i];
      if (s < 0 || (size_t)s >= c->server_topo.size())
        return fail(MAPA_ERR_UNKNOWN_SERVER, "entry %d: unknown server %d", i, s);
      const int n = c->topo_n[c->server_topo[s]];
      if (n < 32 && (masks[i] >> n) != 0)
        return fail(MAPA_ERR_INVALID_ARG, "entry %d: busy bit >= n=%d", i, n);
    }
  }
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  MAPA_HIPCHK(hipSetDevice(c->device));
  hipStream_t s = as_stream(stream);
  const int32_t *d_ids = ids;
  const uint32_t *d_masks = masks;
  if (!dev) {
    int32_t rc = ensure_small(c, count);
    if (rc) return rc;
    MAPA_HIPCHK(begin_call(c, s));
    MAPA_HIPCHK(hipMemcpyAsync(c->d_ids, ids, count * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MAPA_HIPCHK(hipMemcpyAsync(c->d_masks, masks, count * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    d_ids = c->d_ids;
    d_masks = c->d_masks;
  } else {
    MAPA_HIPCHK(begin_call(c, s));
  }
  MAPA_HIPCHK(launch_set_busy(d_ids, d_masks, count, (int32_t)c->server_topo.size(),
                              c->d_server_topo, c->d_topo_n, c->d_busy, s));
  MAPA_HIPCHK(end_call(c, s));
  if (!dev) MAPA_HIPCHK(hipStreamSynchronize(s));
  return MAPA_OK;
}

int32_t mapa_get_busy(mapa_ctx *c, int32_t count, const int32_t *ids, uint32_t *out) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_get_busy")) return rc;
  if (count < 0) return fail(MAPA_ERR_INVALID_ARG, "count < 0");
  if (count == 0) return MAPA_OK;
  if (!ids || !out) return fail(MAPA_ERR_INVALID_ARG, "NULL array");
  for (int32_t i = 0; i < count; ++i)
    if (ids[i] < 0 || (size_t)ids[i] >= c->server_topo.size())
      return fail(MAPA_ERR_UNKNOWN_SERVER, "entry %d: unknown server %d", i, ids[i]);
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  MAPA_HIPCHK(hipSetDevice(c->device));
  int32_t rc = ensure_small(c, count);
  if (rc) return rc;
  hipStream_t s = c->internal;
  MAPA_HIPCHK(begin_call(c, s));
  MAPA_HIPCHK(hipMemcpyAsync(c->d_ids, ids, count * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MAPA_HIPCHK(launch_get_busy(c->d_ids, count, c->d_busy, c->d_masks, s));
  MAPA_HIPCHK(hipMemcpyAsync(out, c->d_masks, count * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MAPA_HIPCHK(end_call(c, s));
  MAPA_HIPCHK(hipStreamSynchronize(s));
  return MAPA_OK;
}

int32_t mapa_query_batch(mapa_ctx *c, const mapa_query *q, int32_t nq, mapa_result *res,
                         uint32_t flags, void *stream) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_query_batch")) return rc;
  if (nq < 0) return fail(MAPA_ERR_INVALID_ARG, "nq < 0");
  if (nq == 0) return MAPA_OK;
  if (!q || !res) return fail(MAPA_ERR_INVALID_ARG, "NULL array");
  const bool dev = flags & MAPA_DEVICE_PTRS;
  if (!dev)
    for (int32_t i = 0; i < nq; ++i) {
      int32_t rc = validate_query(c, q[i], i);
      if (rc) return rc;
    }
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  if ((unsigned long long)nq + kPadReserve > c->ws.cap_items)
    return fail(MAPA_ERR_ADMISSION, "batch of %d queries exceeds the enumeration buffer (%llu items)",
                nq, c->ws.cap_items);
  if (c->server_topo.empty()) return fail(MAPA_ERR_UNKNOWN_SERVER, "no servers created");
  MAPA_HIPCHK(hipSetDevice(c->device));
  int32_t rc = ensure_batch_capacity(c, nq);
  if (rc) return rc;
  hipStream_t s = as_stream(stream);
  const bool use_graph = dev && (flags & MAPA_USE_GRAPH) && !c->profile;
  if (use_graph) {
    mapa_ctx::Graph *g = nullptr;
    for (auto &e : c->graphs)
      if (e.q == q && e.res == res && e.nq == nq && e.stream == s && e.version == c->version) g = &e;
    if (!g) {
      if (c->graphs.size() >= 16) drop_graphs(c);
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      MAPA_HIPCHK(hipStreamBeginCapture(c->internal, hipStreamCaptureModeRelaxed));
      const int32_t ecap = enqueue_batch(c, c->ws, q, res, nq, c->internal);
      const hipError_t eend = hipStreamEndCapture(c->internal, &graph);
      if (ecap != MAPA_OK || eend != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return ecap != MAPA_OK ? ecap
                               : fail(MAPA_ERR_DEVICE, "graph capture: %s", hipGetErrorString(eend));
      }
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return fail(MAPA_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(ei));
      c->graphs.push_back({q, res, nq, s, c->version, exec});
      g = &c->graphs.back();
    }
    MAPA_HIPCHK(begin_call(c, s));
    MAPA_HIPCHK(hipGraphLaunch(g->exec, s));
    MAPA_HIPCHK(end_call(c, s));
    ++c->batches;
    return MAPA_OK;
  }
  if (!dev && !(flags & MAPA_PIPELINE) && nq <= kFusedMaxQueries) {
    // small batch, one query per server: one fused launch on pinned staging
    unsigned long long total = 0;
    bool small = true;
    for (int32_t i = 0; i < nq && small; ++i) {
      const unsigned long long e = perm_leaves(c->topo_n[c->server_topo[q[i].server]], q[i].k);
      small = e <= kFusedMaxQueryLeaves;
      total += e;
    }
    if (small && total <= kFusedMaxLeaves && distinct_servers(c, q, nq)) {
      if (!c->h_fq) {
        MAPA_HIPCHK(hipHostMalloc((void **)&c->h_fq, kFusedMaxQueries * sizeof(mapa_query),
                                  hipHostMallocDefault));
        MAPA_HIPCHK(hipHostMalloc((void **)&c->h_fres, kFusedMaxQueries * sizeof(mapa_result),
                                  hipHostMallocDefault));
      }
      std::memcpy(c->h_fq, q, nq * sizeof(mapa_query));
      MAPA_HIPCHK(begin_call(c, s));
      if (int32_t rc2 = enqueue_fused(c, c->ws, c->h_fq, c->h_fres, nq, s)) return rc2;
      MAPA_HIPCHK(end_call(c, s));
      ++c->batches;
      MAPA_HIPCHK(hipStreamSynchronize(s));
      std::memcpy(res, c->h_fres, nq * sizeof(mapa_result));
      return MAPA_OK;
    }
  }
  MAPA_HIPCHK(begin_call(c, s));
  const mapa_query *dq = q;
  mapa_result *dr = res;
  if (!dev) {
    MAPA_HIPCHK(hipMemcpyAsync(c->ws.d_q, q, nq * sizeof(mapa_query), hipMemcpyHostToDevice, s));
    dq = c->ws.d_q;
    dr = c->ws.d_res;
  }
  BatchArgs a;
  std::memset(&a, 0, sizeof a);
  fill_args(c, c->ws, a);
  a.nq = nq;
  a.q = dq;
  a.res = dr;
  MAPA_HIPCHK(launch_batch_front(a, s));
  ProfEvents ev{};
  if (c->profile)
    if (int32_t rc2 = prof_start(c, s, ev)) return rc2;
  MAPA_HIPCHK(launch_enumerate(a, s));
  if (c->profile)
    if (int32_t rc2 = prof_stop(c, s, ev)) return rc2;
  MAPA_HIPCHK(launch_finalize(a, s));
  if (!dev) MAPA_HIPCHK(hipMemcpyAsync(res, c->ws.d_res, nq * sizeof(mapa_result), hipMemcpyDeviceToHost, s));
  MAPA_HIPCHK(end_call(c, s));
  ++c->batches;
  if (!dev) MAPA_HIPCHK(hipStreamSynchronize(s));
  return MAPA_OK;
}

int32_t mapa_release(mapa_ctx *c, int32_t count, const int64_t *handles, int32_t stride,
                     uint32_t flags, void *stream) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_release")) return rc;
  if (count < 0) return fail(MAPA_ERR_INVALID_ARG, "count < 0");
  if (count == 0) return MAPA_OK;
  if (!handles) return fail(MAPA_ERR_INVALID_ARG, "handles is NULL");
  const bool dev = flags & MAPA_DEVICE_PTRS;
  if (stride == 0) stride = sizeof(int64_t);
  if (stride < (int32_t)sizeof(int64_t) || stride % (int32_t)sizeof(int64_t) != 0)
    return fail(MAPA_ERR_INVALID_ARG, "stride %d is not a positive multiple of 8", stride);
  std::vector<int64_t> h;
  if (!dev) {
    // host handles: full validation, all-or-nothing
    std::vector<std::pair<int32_t, uint32_t>> seen;
    for (int32_t i = 0; i < count; ++i) {
      const int64_t x = *(const int64_t *)((const char *)handles + (size_t)i * stride);
      if (x == -1) continue;
      const int32_t s = (int32_t)(x >> 32);
      const uint32_t m = (uint32_t)x;
      if (x < 0 || s < 0 || (size_t)s >= c->server_topo.size())
        return fail(MAPA_ERR_UNKNOWN_SERVER, "handle %d: unknown server %d", i, s);
      const int n = c->topo_n[c->server_topo[s]];
      if (m == 0 || (n < 32 && (m >> n) != 0))
        return fail(MAPA_ERR_INVALID_ARG, "handle %d: vertex mask 0x%x invalid for n=%d", i, m, n);
      seen.push_back({s, m});
      h.push_back(x);
    }
    std::sort(seen.begin(), seen.end());
    for (size_t i = 1; i < seen.size(); ++i)
      if (seen[i].first == seen[i - 1].first) {
        uint32_t acc = 0;
        size_t j = i - 1;
        while (j > 0 && seen[j - 1].first == seen[i].first) --j;
        for (; j < i; ++j) acc |= seen[j].second;
        if (acc & seen[i].second)
          return fail(MAPA_ERR_NOT_BUSY, "two handles release the same vertex of server %d",
                      seen[i].first);
      }
  }
  if (!dev && h.empty()) return MAPA_OK;
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  MAPA_HIPCHK(hipSetDevice(c->device));
  if (dev) {
    hipStream_t s = as_stream(stream);
    MAPA_HIPCHK(begin_call(c, s));
    MAPA_HIPCHK(launch_release_apply(handles, stride, count, (int32_t)c->server_topo.size(),
                                     c->d_busy, s));
    MAPA_HIPCHK(end_call(c, s));
    return MAPA_OK;
  }
  int32_t rc = ensure_small(c, h.size());
  if (rc) return rc;
  hipStream_t s = c->internal;
  uint32_t flag = 0;
  MAPA_HIPCHK(begin_call(c, s));
  MAPA_HIPCHK(hipMemcpyAsync(c->d_handles, h.data(), h.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  MAPA_HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(uint32_t), s));
  MAPA_HIPCHK(launch_release_check(c->d_handles, 8, (int32_t)h.size(), c->d_busy, c->d_flag, s));
  MAPA_HIPCHK(hipMemcpyAsync(&flag, c->d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MAPA_HIPCHK(hipStreamSynchronize(s));
  if (flag) {
    MAPA_HIPCHK(end_call(c, s));
    return fail(MAPA_ERR_NOT_BUSY, "a released vertex is not busy; nothing released");
  }
  MAPA_HIPCHK(launch_release_apply(c->d_handles, 8, (int32_t)h.size(), (int32_t)c->server_topo.size(),
                                   c->d_busy, s));
  MAPA_HIPCHK(end_call(c, s));
  MAPA_HIPCHK(hipStreamSynchronize(s));
  return MAPA_OK;
}

int32_t mapa_get_tuning(mapa_ctx *c, mapa_tuning *out) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (out) *out = c->tuning;
  return MAPA_OK;
}

int32_t mapa_set_tuning(mapa_ctx *c, const mapa_tuning *in) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_set_tuning")) return rc;
  if (!in) return MAPA_OK;
  if (in->min_leaves_per_item < 1 || in->min_leaves_per_item > (1 << 20))
    return fail(MAPA_ERR_INVALID_ARG, "min_leaves_per_item outside 1..2^20");
  if (in->mean_item_leaves < 1 || in->mean_item_leaves > (1 << 30))
    return fail(MAPA_ERR_INVALID_ARG, "mean_item_leaves outside 1..2^30");
  if (in->blocks_per_cu < 0 || in->blocks_per_cu > 64)
    return fail(MAPA_ERR_INVALID_ARG, "blocks_per_cu outside 0..64");
  if (in->threads_per_block < 64 || in->threads_per_block > 256 || in->threads_per_block % 64)
    return fail(MAPA_ERR_INVALID_ARG, "threads_per_block must be 64, 128, 192 or 256");
  if (in->pair_width != 0 && in->pair_width != -1 && in->pair_width != 6 && in->pair_width != 12)
    return fail(MAPA_ERR_INVALID_ARG, "pair_width must be 0, -1, 6 or 12");
  c->tuning = *in;
  if (c->has_device) {
    int32_t rc = sync_ctx(c);
    if (rc) return rc;
    drop_graphs(c);
    rc = upload_split_table(c);
    if (rc) return rc;
  }
  return MAPA_OK;
}

int32_t mapa_profile(mapa_ctx *c, int32_t enable) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  c->profile = enable != 0;
  return MAPA_OK;
}

int32_t mapa_get_stats(mapa_ctx *c, mapa_stats *out) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(MAPA_ERR_INVALID_ARG, "out is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_get_stats")) return rc;
  std::memset(out, 0, sizeof *out);
  out->num_servers = (int32_t)c->server_topo.size();
  out->num_topologies = (int32_t)c->topo_n.size();
  out->batches = c->batches;
  out->cu_count = c->cu_count;
  if (c->has_device) {
    int32_t rc = sync_ctx(c);
    if (rc) return rc;
    for (auto &e : c->prof) {
      float ms = 0;
      MAPA_HIPCHK(hipEventElapsedTime(&ms, e.start, e.stop));
      c->prof_ms += ms;
      ++c->prof_launches;
      c->prof_free.push_back(e);
    }
    c->prof.clear();
    Counters h;
    MAPA_HIPCHK(hipMemcpy(&h, c->ws.d_ctr, sizeof h, hipMemcpyDeviceToHost));
    out->last_items = (int64_t)h.last_total_items;
    out->last_split = (int32_t)h.chosen_split;
    out->self_check_failures = h.self_check_failures;
  }
  out->enum_launches = c->prof_launches;
  out->enum_ms = c->prof_ms;
  return MAPA_OK;
}

int32_t mapa_reset_stats(mapa_ctx *c) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_reset_stats")) return rc;
  int32_t rc = sync_ctx(c);
  if (rc) return rc;
  for (auto &e : c->prof) c->prof_free.push_back(e);
  c->prof.clear();
  c->prof_ms = 0;
  c->prof_launches = 0;
  c->batches = 0;
  return MAPA_OK;
}

int32_t mapa_measure_alu_peak(mapa_ctx *c, double *ops_per_s) {
  if (!c || !ops_per_s) return fail(MAPA_ERR_INVALID_ARG, "NULL argument");
  if (int32_t rc = not_while_serving(c, "mapa_measure_alu_peak")) return rc;
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  int32_t rc = sync_ctx(c);
  if (rc) return rc;
  const int blocks = std::max(1, c->cu_count) * 16;  // 16 waves per CU
  const int iters = 4096;
  uint32_t *d_out = nullptr;
  if (dev_alloc(&d_out, blocks) != hipSuccess) return fail(MAPA_ERR_OOM, "probe buffer");
  hipEvent_t e0, e1;
  MAPA_HIPCHK(hipEventCreate(&e0));
  MAPA_HIPCHK(hipEventCreate(&e1));
  MAPA_HIPCHK(launch_valu_probe(d_out, blocks, iters, c->internal));  // warm-up
  MAPA_HIPCHK(hipEventRecord(e0, c->internal));
  MAPA_HIPCHK(launch_valu_probe(d_out, blocks, iters, c->internal));
  MAPA_HIPCHK(hipEventRecord(e1, c->internal));
  MAPA_HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  MAPA_HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(d_out);
  MAPA_HIPCHK(hipEventRecord(c->last, c->internal));
  const double lane_ops = (double)blocks * 256.0 * iters * valu_probe_ops_per_iter();
  *ops_per_s = ms > 0 ? lane_ops / (ms * 1e-3) : 0.0;
  return MAPA_OK;
}

int32_t mapa_sync(mapa_ctx *c) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (int32_t rc = not_while_serving(c, "mapa_sync")) return rc;
  return sync_ctx(c);
}

}  // extern "C"
