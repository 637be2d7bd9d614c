// Host side of mapa_query_batch_wide: validation and admission of host
// batches, weight bit-planes of every topology as 32-bit rows, the call's
// device buffer, the launches (plan, search, finalize) and the copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "wide.h"

namespace mapa {

namespace {

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
  if (q.metric != MAPA_METRIC_WEIGHTED && q.metric != MAPA_METRIC_EFFBW)
    return fail(MAPA_ERR_INVALID_ARG, "query %d: metric=%d", i, q.metric);
  if (q.metric == MAPA_METRIC_EFFBW && c->topo_maxw[c->server_topo[q.server]] > 2)
    return fail(MAPA_ERR_UNSUPPORTED,
                "query %d: effective bandwidth needs link weights 0, 1, 2 (PCIe, single, double NVLink)", i);
  return MAPA_OK;
}

}  // namespace

unsigned long long wide_embeddings(int F, int k) {
  if (k > F) return 0;
  unsigned long long v = 1;
  for (int i = 0; i < k; ++i) v *= (unsigned long long)(F - i);
  return v;
}

int32_t wide_upload(mapa_ctx *c) {
  if (c->wide_uploaded == c->wide_W.size()) return MAPA_OK;
  if (int32_t rc = sync_ctx(c)) return rc;
  return upload_wide_rows(c);
}

void wide_ctx_args(const mapa_ctx *c, WideArgs &w) {
  w.rows = c->d_wide_rows;
  w.server_topo = c->d_server_topo;
  w.topo_n = c->d_topo_n;
  w.topo_maxw = c->d_topo_maxw;
  w.nservers = (int32_t)c->server_topo.size();
  w.ntopo_wide = (int32_t)c->wide_uploaded;
  w.pat_nbtab = c->d_pat_nbtab;
  w.pat_k = c->d_pat_k;
  w.eff_rank = c->d_eff_rank;
  w.eff_key = c->d_eff_key;
  w.busy = c->d_busy;
  w.commit_slot = c->d_commit_slot;
}

namespace {
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

size_t wide_scratch_bytes(int32_t nq) {
  return align256(256 + align256((size_t)nq * sizeof(WidePlan)) +
                  (size_t)nq * kWideMaxBlocksPerQuery * sizeof(WidePartial));
}

void wide_scratch_args(void *base, int32_t nq, WideArgs &w) {
  char *b = static_cast<char *>(base);
  w.total = reinterpret_cast<unsigned long long *>(b);
  w.plan = reinterpret_cast<WidePlan *>(b + 256);
  w.part = reinterpret_cast<WidePartial *>(b + 256 + align256((size_t)nq * sizeof(WidePlan)));
}

}  // namespace mapa

using namespace mapa;

extern "C" int32_t mapa_query_batch_wide(mapa_ctx *c, const mapa_query *q, int32_t nq,
                                         mapa_result_wide *res, uint32_t flags, void *stream) {
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (c->serve) return fail(MAPA_ERR_STATE, "mapa_query_batch_wide: the serving loop owns the context");
  if (nq < 0) return fail(MAPA_ERR_INVALID_ARG, "nq=%d < 0", nq);
  if (nq > kWideMaxQueries)
    return fail(MAPA_ERR_ADMISSION, "wide batch of %d queries exceeds %d", nq, kWideMaxQueries);
  if (nq > 0 && (!q || !res)) return fail(MAPA_ERR_INVALID_ARG, "queries or results NULL");
  const bool dev = flags & MAPA_DEVICE_PTRS;
  if (!dev)
    for (int32_t i = 0; i < nq; ++i)
      if (int32_t rc = validate_wide(c, q[i], i)) return rc;
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  if (nq == 0) return MAPA_OK;
  if (c->server_topo.empty()) return fail(MAPA_ERR_UNKNOWN_SERVER, "no servers created");
  if (hipSetDevice(c->device) != hipSuccess) return fail(MAPA_ERR_DEVICE, "hipSetDevice failed");
  if (!dev) {
    if (int32_t rc = sync_ctx(c)) return rc;
  }
  if (int32_t rc = wide_upload(c)) return rc;
  if (!dev) {
    // admission: the embeddings of the whole call, on the free sets at its start
    std::vector<uint32_t> busy(c->server_topo.size());
    MAPA_HIPCHK(hipMemcpy(busy.data(), c->d_busy, busy.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    unsigned long long leaves = 0;
    for (int32_t i = 0; i < nq; ++i) {
      const int n = c->topo_n[c->server_topo[q[i].server]];
      const uint32_t all = n >= 32 ? 0xFFFFFFFFu : (1u << n) - 1u;
      leaves += wide_embeddings(__builtin_popcount(~busy[q[i].server] & all), q[i].k);
      if (leaves > kWideMaxLeaves)
        return fail(MAPA_ERR_ADMISSION, "wide batch exceeds %llu embeddings at query %d", kWideMaxLeaves, i);
    }
  }

  // one device buffer: scratch (embedding total, plans, partials) | (host form) queries | results
  const size_t o_q = wide_scratch_bytes(nq);
  const size_t o_res = o_q + (dev ? 0 : ((size_t)nq * sizeof(mapa_query) + 255) / 256 * 256);
  const size_t bytes = o_res + (dev ? 0 : (size_t)nq * sizeof(mapa_result_wide));
  if (bytes > c->wide_buf.cap) {
    if (int32_t rc = sync_ctx(c)) return rc;  // earlier calls may still use the old buffer
    if (c->wide_buf.d) (void)hipFree(c->wide_buf.d);
    c->wide_buf.d = nullptr;
    c->wide_buf.cap = 0;
    if (hipMalloc(&c->wide_buf.d, bytes) != hipSuccess)
      return fail(MAPA_ERR_OOM, "wide batch buffer: device allocation failed");
    c->wide_buf.cap = bytes;
  }
  char *base = static_cast<char *>(c->wide_buf.d);
  WideArgs w;
  wide_ctx_args(c, w);
  wide_scratch_args(base, nq, w);
  w.q = dev ? q : reinterpret_cast<const mapa_query *>(base + o_q);
  w.nq = nq;
  w.res = dev ? res : reinterpret_cast<mapa_result_wide *>(base + o_res);
  w.self_check_failures = &c->ws.d_ctr->self_check_failures;
  hipStream_t s = dev ? reinterpret_cast<hipStream_t>(stream) : c->internal;
  MAPA_HIPCHK(hipStreamWaitEvent(s, c->last, 0));
  if (!dev)
    MAPA_HIPCHK(hipMemcpyAsync(const_cast<mapa_query *>(w.q), q, (size_t)nq * sizeof(mapa_query),
                               hipMemcpyHostToDevice, s));
  MAPA_HIPCHK(launch_wide_plan(w, s));
  ProfEvents ev{};
  if (c->profile)  // the search kernel's time counts as enumeration time
    if (int32_t rc2 = prof_start(c, s, ev)) return rc2;
  MAPA_HIPCHK(launch_wide_search(w, s));
  if (c->profile)
    if (int32_t rc2 = prof_stop(c, s, ev)) return rc2;
  MAPA_HIPCHK(launch_wide_finalize(w, s));
  if (!dev)
    MAPA_HIPCHK(hipMemcpyAsync(res, w.res, (size_t)nq * sizeof(mapa_result_wide), hipMemcpyDeviceToHost, s));
  MAPA_HIPCHK(hipEventRecord(c->last, s));
  if (!dev) MAPA_HIPCHK(hipStreamSynchronize(s));
  c->batches += 1;
  return MAPA_OK;
}
