// Host side of mapa_query_batch_wide: validation, weight bit-planes of every
// topology as 32-bit rows, per-query plans (free set, b*W(R), pattern
// neighbour masks, prefix depth, block share), the launches and the copy back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "ctx.h"

namespace mapa {

namespace {

unsigned long long perm_wide(int F, int d) {  // F!/(F-d)!, 0 if d > F
  if (d > F) return 0;
  unsigned long long v = 1;
  for (int i = 0; i < d; ++i) v *= (unsigned long long)(F - i);
  return v;
}

// Upload the planes of topologies added since the last wide call.
int32_t upload_wide_rows(mapa_ctx *c) {
  const size_t T = c->wide_W.size();
  if (T == c->wide_uploaded) return MAPA_OK;
  size_t first = c->wide_uploaded;
  if (T > c->cap_wide) {
    size_t cap = std::max<size_t>(16, c->cap_wide);
    while (cap < T) cap *= 2;
    dev_free(c->d_wide_rows);
    c->cap_wide = 0;
    if (dev_alloc(&c->d_wide_rows, cap * kWidePlanes * 32) != hipSuccess)
      return fail(MAPA_ERR_OOM, "wide topology rows: device allocation failed");
    c->cap_wide = cap;
    first = 0;
  }
  std::vector<uint32_t> rows((T - first) * kWidePlanes * 32, 0u);
  for (size_t t = first; t < T; ++t) {
    const uint8_t *W = c->wide_W[t].data();
    uint32_t *r = &rows[(t - first) * kWidePlanes * 32];
    for (int v = 0; v < kWideN; ++v)
      for (int u = 0; u < kWideN; ++u) {
        const uint8_t x = W[v * kWideN + u];
        for (int b = 0; b < 8; ++b)
          if ((x >> b) & 1u) r[b * 32 + v] |= 1u << u;
        if (x) r[(kWidePlanes - 1) * 32 + v] |= 1u << u;
      }
  }
  MAPA_HIPCHK(hipMemcpy(c->d_wide_rows + first * kWidePlanes * 32, rows.data(),
                        rows.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  c->wide_uploaded = T;
  return MAPA_OK;
}

int32_t validate_wide(const mapa_ctx *c, const mapa_query &q, int32_t i) {
  if (q.server < 0 || (size_t)q.server >= c->server_topo.size())
    return fail(MAPA_ERR_UNKNOWN_SERVER, "query %d: unknown server %d", i, q.server);
  if (q.k > kWideK) return fail(MAPA_ERR_UNSUPPORTED, "query %d: k=%d > %d", i, q.k, kWideK);
  if (q.k < 1) return fail(MAPA_ERR_INVALID_ARG, "query %d: k=%d < 1", i, q.k);
  if (q.kind > MAPA_TREE) {
    const int id = q.kind - MAPA_PATTERN_BASE;
    if (id < 0 || id >= c->npat || c->pat_k[id] != q.k)
      return fail(MAPA_ERR_INVALID_ARG, "query %d: kind=%d with k=%d is neither a pattern kind "
                  "nor a registered pattern of that size", i, q.kind, q.k);
  }
  if (q.mode > 1) return fail(MAPA_ERR_INVALID_ARG, "query %d: mode=%d", i, q.mode);
  if (q.commit > 1) return fail(MAPA_ERR_INVALID_ARG, "query %d: commit=%d", i, q.commit);
  if (q.a < 0 || q.a > MAPA_MAX_AB || q.b < 0 || q.b > MAPA_MAX_AB)
    return fail(MAPA_ERR_INVALID_ARG, "query %d: key weights (%d,%d) outside 0..%d", i, q.a, q.b,
                MAPA_MAX_AB);
  if (q.metric == MAPA_METRIC_EFFBW)
    return fail(MAPA_ERR_UNSUPPORTED, "query %d: the wide path scores a*AggBW + b*PreservedBW only", i);
  if (q.metric != MAPA_METRIC_WEIGHTED) return fail(MAPA_ERR_INVALID_ARG, "query %d: metric=%d", i, q.metric);
  return MAPA_OK;
}

// earlier pattern neighbours of each position (bit j of nb[p]: j < p neighbours p)
void wide_neighbours(const mapa_ctx *c, int kind, int k, uint16_t *nb) {
  for (int p = 0; p < kWideK; ++p) nb[p] = 0;
  if (kind >= MAPA_PATTERN_BASE) {
    const unsigned long long tab = c->pat_nbtab[kind - MAPA_PATTERN_BASE];
    for (int p = 0; p < k; ++p) nb[p] = (uint16_t)((tab >> (8 * p)) & 0xFFu);
    return;
  }
  for (int p = 1; p < k; ++p) {
    if (kind == MAPA_RING) {
      nb[p] = (uint16_t)(1u << (p - 1));
      if (p == k - 1 && k >= 3) nb[p] |= 1u;
    } else if (kind == MAPA_ALL_TO_ALL) {
      nb[p] = (uint16_t)((1u << p) - 1u);
    } else {
      nb[p] = (uint16_t)(1u << ((p - 1) / 2));
    }
  }
}

}  // namespace

}  // namespace mapa

using namespace mapa;

extern "C" int32_t mapa_query_batch_wide(mapa_ctx *c, const mapa_query *q, int32_t nq,
                                         mapa_result_wide *res) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (c->serve) return fail(MAPA_ERR_STATE, "mapa_query_batch_wide: the serving loop owns the context");
  if (nq < 0) return fail(MAPA_ERR_INVALID_ARG, "nq=%d < 0", nq);
  if (nq > 0 && (!q || !res)) return fail(MAPA_ERR_INVALID_ARG, "queries or results NULL");
  for (int32_t i = 0; i < nq; ++i)
    if (int32_t rc = validate_wide(c, q[i], i)) return rc;
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  if (nq == 0) return MAPA_OK;
  if (hipSetDevice(c->device) != hipSuccess) return fail(MAPA_ERR_DEVICE, "hipSetDevice failed");
  if (int32_t rc = sync_ctx(c)) return rc;
  if (int32_t rc = upload_wide_rows(c)) return rc;

  // busy masks at the call's start
  std::vector<uint32_t> busy(c->server_topo.size());
  if (!busy.empty())
    MAPA_HIPCHK(hipMemcpy(busy.data(), c->d_busy, busy.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));

  std::vector<WidePlan> plans((size_t)nq);
  std::vector<uint32_t> blk_q;
  std::unordered_map<int32_t, int32_t> first_commit;  // server -> first committing query
  unsigned long long leaves = 0;
  for (int32_t i = 0; i < nq; ++i) {
    const mapa_query &qq = q[i];
    WidePlan &p = plans[(size_t)i];
    std::memset(&p, 0, sizeof p);
    const int t = c->server_topo[qq.server];
    const int n = c->topo_n[t];
    const uint32_t all = n >= 32 ? 0xFFFFFFFFu : (1u << n) - 1u;
    const uint32_t R = ~busy[qq.server] & all;
    const int F = __builtin_popcount(R);
    const uint8_t *W = c->wide_W[t].data();
    int WR = 0;
    for (int u = 0; u < n; ++u)
      for (int v = u + 1; v < n; ++v)
        if (((R >> u) & 1u) && ((R >> v) & 1u)) WR += W[u * kWideN + v];
    int B = 1;
    while (B < 8 && (c->topo_maxw[t] >> B)) ++B;
    p.R = R;
    p.kp0 = qq.b * WR;
    p.server = qq.server;
    wide_neighbours(c, qq.kind, qq.k, p.nb);
    p.nb_all = qq.kind == MAPA_ALL_TO_ALL ? 1 : 0;
    p.k = qq.k;
    p.mode = qq.mode;
    p.B = (uint8_t)B;
    p.F = (uint8_t)F;
    p.a = qq.a;
    p.b = qq.b;
    p.topo = (uint16_t)t;
    p.commit = qq.commit;
    if (qq.commit && first_commit.emplace(qq.server, i).second) p.owner = 1;
    if (qq.k > F) {
      p.status = kPlanNofit;
      continue;
    }
    p.status = kPlanOk;
    leaves += perm_wide(F, qq.k);
    if (leaves > kWideMaxLeaves)
      return fail(MAPA_ERR_ADMISSION, "wide batch exceeds %llu embeddings at query %d", kWideMaxLeaves, i);
    int d = 0;
    while (d < qq.k - 1 && perm_wide(F, d) < kWideMinItems) ++d;
    p.d = (uint8_t)d;
    p.items = (uint32_t)perm_wide(F, d);
    const unsigned long long want = (p.items + kWideThreads - 1) / kWideThreads;
    p.nblocks = (uint32_t)std::min<unsigned long long>(std::max<unsigned long long>(want, 1),
                                                       kWideMaxBlocksPerQuery);
    p.block0 = (uint32_t)blk_q.size();
    blk_q.insert(blk_q.end(), p.nblocks, (uint32_t)i);
  }
  const size_t blocks = blk_q.size();

  // one device buffer: plans | block table | partials | results
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_plan = 0, o_blk = align(o_plan + plans.size() * sizeof(WidePlan));
  const size_t o_part = align(o_blk + blocks * sizeof(uint32_t));
  const size_t o_res = align(o_part + blocks * sizeof(WidePartial));
  const size_t bytes = align(o_res + (size_t)nq * sizeof(mapa_result_wide));
  if (bytes > c->wide_buf.cap) {
    if (c->wide_buf.d) (void)hipFree(c->wide_buf.d);
    c->wide_buf.d = nullptr;
    c->wide_buf.cap = 0;
    if (hipMalloc(&c->wide_buf.d, bytes) != hipSuccess)
      return fail(MAPA_ERR_OOM, "wide batch buffer: device allocation failed");
    c->wide_buf.cap = bytes;
  }
  char *base = static_cast<char *>(c->wide_buf.d);
  WideArgs w;
  w.plan = reinterpret_cast<WidePlan *>(base + o_plan);
  w.nq = nq;
  w.blk_q = reinterpret_cast<uint32_t *>(base + o_blk);
  w.part = reinterpret_cast<WidePartial *>(base + o_part);
  w.rows = c->d_wide_rows;
  w.busy = c->d_busy;
  w.res = reinterpret_cast<mapa_result_wide *>(base + o_res);
  w.self_check_failures = &c->ws.d_ctr->self_check_failures;
  hipStream_t s = c->internal;
  MAPA_HIPCHK(hipMemcpyAsync(const_cast<WidePlan *>(w.plan), plans.data(), plans.size() * sizeof(WidePlan),
                             hipMemcpyHostToDevice, s));
  if (blocks)
    MAPA_HIPCHK(hipMemcpyAsync(const_cast<uint32_t *>(w.blk_q), blk_q.data(), blocks * sizeof(uint32_t),
                               hipMemcpyHostToDevice, s));
  ProfEvents ev{};
  if (c->profile && blocks)  // the search kernel's time counts as enumeration time
    if (int32_t rc2 = prof_start(c, s, ev)) return rc2;
  MAPA_HIPCHK(launch_wide_search(w, (int32_t)blocks, s));
  if (c->profile && blocks)
    if (int32_t rc2 = prof_stop(c, s, ev)) return rc2;
  MAPA_HIPCHK(launch_wide_finalize(w, s));
  MAPA_HIPCHK(hipMemcpyAsync(res, w.res, (size_t)nq * sizeof(mapa_result_wide), hipMemcpyDeviceToHost, s));
  MAPA_HIPCHK(hipEventRecord(c->last, s));
  MAPA_HIPCHK(hipStreamSynchronize(s));
  c->batches += 1;
  return MAPA_OK;
}
