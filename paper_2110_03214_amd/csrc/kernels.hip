// HIP kernels of the MAPA allocation hot path, written for gfx950 (CDNA4,
// wave64).  Integer-only: every match is enumerated and scored exactly.
//
// Batch pipeline (one launch each, all on the caller's stream):
//   k_front      few fat blocks, each over a share of the queries: per query
//                validate, free set R, constant key term b*W(R), commit
//                claim; the block's own prefix split from its share's item
//                totals; per query prefix depth d, shape bucket, offset
//                inside the bucket.  The last block to finish lays the
//                buckets out (largest items first) and resets the per-batch
//                counters.
//   k_expand     fills every query's work-list slots with (query, item index)
//                and pads each bucket to whole 64-item chunks; k_enumerate
//                turns the index into the prefix tuple.
//   k_enumerate  persistent: each wave takes a 64-item chunk; each lane
//                expands its prefix depth-first over the remaining pattern
//                positions, scoring every match incrementally, and keeps a
//                count and its best (key, mapping).  Lanes of one chunk share
//                the subtree shape, so their loops run in lock step.
//   k_finalize   per query: decode the best mapping, recompute AggBW and
//                PreservedBW from it, apply the batch's commits.
//
// Scoring (Eq. 1 and Eq. 3).  For a mapping phi with vertex set S inside the
// free set R:
//   key = a*AggBW + b*PreservedBW
//       = b*W(R) + sum_p [ a*sum_{j in Nb(p)} W[phi_j][phi_p]
//                          - b*sum_{u in R \ {phi_0..phi_{p-1}}} W[phi_p][u] ]
// where Nb(p) are the pattern neighbours of position p that precede it and
// W(X) is the total weight inside X.  The second form removes the chosen
// vertices from R one at a time (each removal drops the weight from that
// vertex to what is still left), so every tree node adds one term and a leaf
// costs two masked weighted popcounts.
//
// Weighted popcounts use bit-planes: row v of a topology holds, for each
// weight bit t, the mask of neighbours u with bit t of W[v][u] set; two planes
// share one 32-bit word (plane 2w in the low half, 2w+1 in the high half), so
// sum_{u in X} W[v][u] = sum_w 4^w * (popc(row_w & X2) + popc((row_w & X2) >> 16))
// with X2 = X | X << 16.
#include <algorithm>

#include "device.h"

namespace mapa {

hipError_t upload_tables_front(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

// ------------------------------------------------------------------- front

constexpr int kFatBlock = 1024;  // threads of a k_front block

// Lay the buckets out (largest items first, each rounded up to whole 64-item
// chunks) and reset the per-batch counters.  Run by the last k_front block
// to finish, once every block's counts are in.
__device__ void layout_buckets(const BatchArgs &a) {
  __shared__ uint32_t s_pad[kNumBuckets];
  __shared__ uint32_t s_cnt[kNumBuckets];
  __shared__ uint32_t s_start[kNumBuckets];
  __shared__ unsigned long long s_items;  // items of the batch (before padding)
  const int t = threadIdx.x;
  if (t == 0) s_items = 0;
  // loops over the buckets have a fixed stride (one 1024-thread block), so
  // they unroll and each thread's loads are in flight together.  The counts
  // are loaded in bucket order (into s_start, free until the scan) beside
  // the rank table, then gathered into rank order through LDS.
  constexpr int kPer = (kNumBuckets + kFatBlock - 1) / kFatBlock;
  int rank_b[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int i = t + e * kFatBlock;
    if (i < kNumBuckets) {
      rank_b[e] = c_tab.rank_bucket[i];
      s_start[i] = __hip_atomic_load(&a.ctr->bucket_items[i][0], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int r = t + e * kFatBlock;
    if (r < kNumBuckets) {
      const uint32_t cnt = s_start[rank_b[e]];
      if (cnt) atomicAdd(&s_items, (unsigned long long)cnt);
      s_cnt[r] = cnt;
      s_pad[r] = (cnt + (kChunk - 1)) & ~(uint32_t)(kChunk - 1);
    }
  }
  __syncthreads();
  {
    // exclusive scan of the padded sizes in rank order over the whole block:
    // thread t owns kPerT consecutive ranks; wave scans, then a scan of the
    // wave totals
    constexpr int kPerT = (kNumBuckets + kFatBlock - 1) / kFatBlock;
    __shared__ uint32_t s_wave[kFatBlock / 64];
    const int lane = t & 63, wave = t >> 6;
    uint32_t v[kPerT];
    uint32_t sum = 0;
#pragma unroll
    for (int e = 0; e < kPerT; ++e) {
      const int r = t * kPerT + e;
      v[e] = r < kNumBuckets ? s_pad[r] : 0u;
      sum += v[e];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    if (t < 64) {
      const uint32_t w = t < kFatBlock / 64 ? s_wave[t] : 0u;
      uint32_t wi = w;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(wi, off, 64);
        if (lane >= off) wi += o;
      }
      if (t < kFatBlock / 64) s_wave[t] = wi - w;  // exclusive
      if (t == kFatBlock / 64 - 1) a.ctr->total_chunks = wi / kChunk;
    }
    __syncthreads();
    uint32_t run = s_wave[wave] + incl - sum;
#pragma unroll
    for (int e = 0; e < kPerT; ++e) {
      const int r = t * kPerT + e;
      if (r < kNumBuckets) s_start[r] = run;
      run += v[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int r = t + e * kFatBlock;
    if (r >= kNumBuckets) break;
    const int b = rank_b[e];  // loaded above for the same r
    a.ctr->bucket_start[b] = s_start[r];
    a.ctr->bucket_count[b] = s_cnt[r];
    a.ctr->bucket_items[b][0] = 0;
  }
  // the enumeration's waves take their first chunks by wave id, except in
  // the twelve-wide instances (see chunk_loop): every queue's claims start
  // past them
  if (t < kQueues)
    a.ctr->queue_ctr[t][0] = enum_twelve_wide(a)
                                 ? 0u
                                 : (uint32_t)(a.enum_blocks * (a.enum_threads / 64)) / (uint32_t)kQueues;
  if (t == 0) a.ctr->last_total_items = s_items;
}

// Few, fat blocks, each over a share of the queries.  A block plans its
// queries (validation, free set R, the commit claim; the key's constant term
// b*W(R) is left to k_expand, whose loads it then overlaps), counts those
// that fit by (F, k), and from those counts picks its own prefix split: the
// item totals of every candidate split follow from the (F, k) counts, and
// the rule below is applied to the block's share of the work-list and of the
// resident lanes.  A split changes how a query's work is cut, never its
// result, so blocks need not agree, and each block's items fit its share of
// the work-list, so the batch's fit.  Then per query the prefix depth, the
// shape bucket and the offset inside it: an LDS histogram, then one global
// atomic per bucket per block, so every global counter sees only a handful
// of atomics.  The last block to finish (by a counter taken after its
// atomics are done) lays the buckets out, which needs every block's counts;
// no block waits for another.
__global__ __launch_bounds__(1024) void k_front(BatchArgs a) {
  __shared__ int s_split;
  __shared__ uint32_t s_cnt[kNumBuckets];
  __shared__ uint32_t s_base[kNumBuckets];
  __shared__ uint32_t s_h[kFkBins];
  __shared__ unsigned long long s_perm[kFkBins];  // F!/(F-d)! at F * (kMaxK + 1) + d
  __shared__ uint8_t s_sd[kSplitTable];           // the split table, see kSplitTable
  __shared__ unsigned long long s_tot[kNumSplits + 1];
  const int t = threadIdx.x;
#pragma unroll
  for (int b = t; b < kNumBuckets; b += kFatBlock) s_cnt[b] = 0;
  if (t < kFkBins) s_h[t] = 0;
  if (t <= kNumSplits) s_tot[t] = 0;
  // the tables are loaded before the planning and stored to LDS after it,
  // so their loads overlap the planning's
  constexpr int kSdPer = (kSplitTable + kFatBlock - 1) / kFatBlock;
  uint8_t sd[kSdPer];
#pragma unroll
  for (int e = 0; e < kSdPer; ++e)
    sd[e] = t + e * kFatBlock < kSplitTable ? a.split_d[t + e * kFatBlock] : 0;
  const unsigned long long perm = t < kFkBins ? c_tab.perm[t / (kMaxK + 1)][t % (kMaxK + 1)] : 0ull;
  const int per_block = (a.nq + gridDim.x - 1) / gridDim.x;
  const int q0 = blockIdx.x * per_block;
  const int q1 = min(a.nq, q0 + per_block);
  constexpr int kMaxPerThread = 16;
  // per query of this thread: F | k << 8 | bucket fields << 16, or ~0u when
  // the query does not fit (the plan itself goes to memory once)
  uint32_t shape[kMaxPerThread];
#pragma unroll
  for (int r = 0; r < kMaxPerThread; ++r) {
    const int i = q0 + t + r * kFatBlock;
    shape[r] = ~0u;
    if (i < q1) {
      const mapa_query q = a.q[i];
      const Plan p = make_plan(q, a.nservers, a.server_topo, a.topo_n, a.topo_maxw, a.busy, a.rows,
                               a.wpr, a.pat_nbtab, a.pat_k, a.pat_nbtab_ord, a.pat_order, false);
      if (p.status == kPlanOk)
        shape[r] = (uint32_t)p.F | (uint32_t)p.k << 8 | (uint32_t)p.kind << 16 |
                   (uint32_t)p.mode << 20 | (uint32_t)p.metric << 24;
      if (p.status != kPlanInvalid && p.commit)
        atomicMin(&a.commit_slot[p.server], (unsigned long long)i);
      a.plan[i] = p;
      a.acc_count[i] = 0;
      a.acc_best[i] = 0;
    }
  }
#pragma unroll
  for (int e = 0; e < kSdPer; ++e)
    if (t + e * kFatBlock < kSplitTable) s_sd[t + e * kFatBlock] = sd[e];
  if (t < kFkBins) s_perm[t] = perm;
  __syncthreads();
  // the share's queries that fit, by (F, k)
#pragma unroll
  for (int r = 0; r < kMaxPerThread; ++r)
    if (shape[r] != ~0u) atomicAdd(&s_h[(shape[r] & 0xFF) * (kMaxK + 1) + ((shape[r] >> 8) & 0xFF)], 1u);
  __syncthreads();
  // The share's totals: for each (bin, split) pair h * (items per query of
  // that split), and at j = kNumSplits h * F!/(F-k)!.
#pragma unroll
  for (int e = t; e < kFkBins * (kNumSplits + 1); e += kFatBlock) {
    const int bin = e / (kNumSplits + 1), j = e % (kNumSplits + 1);
    const uint32_t h = s_h[bin];
    if (h) {
      const int F = bin / (kMaxK + 1), kk = bin % (kMaxK + 1);
      const int d = j < kNumSplits ? (int)s_sd[bin * kNumSplits + j] : kk;
      atomicAdd(&s_tot[j], (unsigned long long)h * s_perm[F * (kMaxK + 1) + d]);
    }
  }
  __syncthreads();
  if (t < 64) {
    // Items get finer (more, smaller) as j falls.  Finer items balance the
    // lanes better but each costs a fixed setup, so take the finest split
    // that fits the share of the work-list, gives every resident lane of the
    // share an item and keeps the mean item at mean_leaves embeddings or
    // more.  Failing that: the coarsest split that still gives every such
    // lane an item; for a share too small for that, the finest split that
    // fits.  Only the splits above the coarsest one that does not fit count
    // as fitting.  Whole queries (one item each) always fit: the batch's
    // queries fit the work-list beside its padding, and the share is at
    // least whole queries' worth of it.  One lane per split, then ballots.
    const uint32_t nb = (uint32_t)max(q1 - q0, 0);
    const unsigned long long room = a.cap_items - kPadReserve;
    const uint32_t room32 = room > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)room;
    const unsigned long long cap = (unsigned long long)(room32 / (uint32_t)a.nq) * nb;
    const unsigned long long lanes =
        (unsigned long long)ceil((double)a.lanes * (double)nb / (double)a.nq);
    const unsigned long long leaves = s_tot[kNumSplits];
    const bool in = t <= kSplitWhole;
    const unsigned long long n = in ? s_tot[t] : 0ull;
    const unsigned long long nofit = __ballot(in && n > cap);
    const unsigned long long fill = __ballot(in && n >= lanes);
    const unsigned long long big = __ballot(in && leaves >= n * (unsigned long long)a.mean_leaves);
    constexpr unsigned long long kAll = (1ull << (kSplitWhole + 1)) - 1ull;
    const unsigned long long fits = nofit ? kAll & ~((2ull << (63 - __builtin_clzll(nofit))) - 1ull) : kAll;
    const unsigned long long best = fits & fill & big, busy = fits & fill;
    const int j = best   ? __builtin_ctzll(best)
                  : busy ? 63 - __builtin_clzll(busy)
                  : fits ? __builtin_ctzll(fits)
                         : kSplitWhole;
    if (t == 0) {
      s_split = j;
      if (blockIdx.x == 0) a.ctr->chosen_split = (uint32_t)j;
    }
  }
  __syncthreads();
  const int j = s_split;
  uint32_t local[kMaxPerThread];
  int bk[kMaxPerThread];
#pragma unroll
  for (int r = 0; r < kMaxPerThread; ++r) {
    const int i = q0 + t + r * kFatBlock;
    bk[r] = -1;
    local[r] = 0;
    if (shape[r] != ~0u) {
      const int F = shape[r] & 0xFF, kk = (shape[r] >> 8) & 0xFF;
      const int kind = (shape[r] >> 16) & 0xF, mode = (shape[r] >> 20) & 0xF;
      const int metric = shape[r] >> 24;
      const int d = s_sd[(F * (kMaxK + 1) + kk) * kNumSplits + j];
      const uint32_t nitems = (uint32_t)s_perm[F * (kMaxK + 1) + d];
      const int b = bucket_id(metric, mode, kind, kk - d, F - d);
      a.plan[i].d = (uint8_t)d;
      a.plan[i].bucket = (uint16_t)b;
      a.plan[i].nitems = nitems;
      bk[r] = b;
      local[r] = atomicAdd(&s_cnt[b], nitems);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = t; c < kNumBuckets; c += kFatBlock)
    s_base[c] = s_cnt[c] ? atomicAdd(&a.ctr->bucket_items[c][0], s_cnt[c]) : 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kMaxPerThread; ++r) {
    const int i = q0 + t + r * kFatBlock;
    if (bk[r] >= 0) a.plan[i].item_off = s_base[bk[r]] + local[r];
  }
  // Every count this block added came back from its atomic (s_base) before
  // the barrier, so it is in place before the block takes its turn; the
  // last block reads the counts with device-scope atomic loads.  No fence:
  // a device-scope fence writes back the whole L2, which cost more than a
  // separate launch.
  __shared__ bool s_last;
  __syncthreads();
  if (t == 0) s_last = atomicAdd(&a.ctr->bucketize_done, 1u) == gridDim.x - 1u;
  __syncthreads();
  if (s_last) {
    layout_buckets(a);
    if (t == 0) a.ctr->bucketize_done = 0;
  }
}

// ------------------------------------------------------------------ expand

// Prefix item x of a query (0 <= x < F!/(F-d)!) is the x-th injective
// d-tuple of free vertices in lexicographic order (k_enumerate unranks it).
//
// Each query's plan also gets its key's constant term b*W(R) here.
//
// Work-list fill: slot bucket_start + item_off + x of a query holds
// (query, x).  A group of bpg blocks owns qpb <= 256 consecutive queries: a
// scan of their item counts lays their items end to end and the group's
// threads write that sequence in order (block g of the group takes every
// bpg-th run of 256 slots), so consecutive threads fill consecutive slots of
// one query; each finds its slot's query by binary search over the scan.
// Small batches take one query per group and several blocks per query.  The
// query whose items end its bucket also writes the bucket's padding (invalid
// items up to a whole chunk), from the group's first block.
constexpr int kExpandThreads = 256;
__global__ __launch_bounds__(kExpandThreads) void k_expand(BatchArgs a, int qpb, int bpg) {
  __shared__ uint32_t s_end[kExpandThreads];  // inclusive scan of the item counts
  __shared__ uint32_t s_dst[kExpandThreads];  // each query's first slot
  __shared__ uint32_t s_wave[kExpandThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = (int)blockIdx.x % bpg;
  const int q0 = ((int)blockIdx.x / bpg) * qpb;
  const int nloc = min(qpb, a.nq - q0);
  uint32_t n = 0, dst = 0;
  if (t < nloc) {
    const Plan &p = a.plan[q0 + t];
    if (p.status == kPlanOk) {
      const uint32_t start = a.ctr->bucket_start[p.bucket];
      const uint32_t cnt = a.ctr->bucket_count[p.bucket];
      // the key's constant term (k_front leaves it out): its row loads
      // overlap the bucket loads above
      if (g == 0) a.plan[q0 + t].kp0 = plan_kp0(p, a.rows, a.wpr);
      n = p.nitems;
      dst = start + p.item_off;
      if (g == 0 && p.item_off + n == cnt) {
        const uint32_t pad = (cnt + (kChunk - 1)) & ~(uint32_t)(kChunk - 1);
        for (uint32_t x = cnt; x < pad; ++x) a.items[start + x] = make_uint2(kInvalidItem, 0u);
      }
    }
  }
  uint32_t incl = n;  // scan: within each wave, then the wave totals
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  for (int w = 0; w < wave; ++w) incl += s_wave[w];
  s_end[t] = incl;
  s_dst[t] = dst;
  __syncthreads();
  const uint32_t total = s_end[nloc - 1];
  for (uint32_t r = (uint32_t)(g * kExpandThreads + t); r < total; r += (uint32_t)(bpg * kExpandThreads)) {
    int lo = 0, hi = nloc - 1;  // the first query whose items end after slot r
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_end[mid] > r)
        hi = mid;
      else
        lo = mid + 1;
    }
    const uint32_t x = r - (lo ? s_end[lo - 1] : 0u);
    a.items[s_dst[lo] + x] = make_uint2((uint32_t)(q0 + lo), x);
  }
}

// ---------------------------------------------------------------- finalize

__global__ __launch_bounds__(256) void k_finalize(BatchArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nq) return;
  const Plan p = a.plan[i];
  Outcome o = decode_best(p, a.acc_count[i], a.acc_best[i], a.rows + (size_t)p.topo * kTopoWords * a.wpr,
                          a.wpr, a.eff_rank, a.eff_key, a.pat_order, &a.ctr->self_check_failures);
  a.acc_count[i] = 0;  // leave the accumulators clean for the next batch
  a.acc_best[i] = 0;
  if (p.status != kPlanInvalid && p.commit) {
    if (a.commit_slot[p.server] == (unsigned long long)i) {
      if (o.status == MAPA_RES_OK) {
        atomicOr(&a.busy[p.server], o.S);
        o.handle = ((int64_t)p.server << 32) | (int64_t)o.S;
      }
      a.commit_slot[p.server] = kSlotFree;
    } else if (o.status == MAPA_RES_OK) {
      o.status = MAPA_RES_CONFLICT;
    }
  }
  store_result(a.res + i, o);
}

// ------------------------------------------------------------- state kernels

__global__ void k_set_busy(const int32_t *ids, const uint32_t *masks, int32_t count,
                           int32_t nservers, const int32_t *server_topo, const int32_t *topo_n,
                           uint32_t *busy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int s = ids[i];
  if (s < 0 || s >= nservers) return;
  const int n = topo_n[server_topo[s]];
  busy[s] = masks[i] & (n >= 32 ? 0xFFFFFFFFu : (1u << n) - 1u);
}

__global__ void k_get_busy(const int32_t *ids, int32_t count, const uint32_t *busy,
                           uint32_t *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = busy[ids[i]];
}

__device__ __forceinline__ int64_t load_handle(const int64_t *h, int32_t stride, int i) {
  return *(const int64_t *)((const char *)h + (size_t)i * stride);
}

__global__ void k_release_check(const int64_t *h, int32_t stride, int32_t count,
                                const uint32_t *busy, uint32_t *flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t x = load_handle(h, stride, i);
  if (x == -1) return;
  const uint32_t m = (uint32_t)x;
  if ((busy[(int32_t)(x >> 32)] & m) != m) atomicOr(flag, 1u);
}

__global__ void k_release_apply(const int64_t *h, int32_t stride, int32_t count,
                                int32_t nservers, uint32_t *busy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t x = load_handle(h, stride, i);
  if (x == -1) return;
  const int32_t s = (int32_t)(x >> 32);
  if (s < 0 || s >= nservers) return;
  atomicAnd(&busy[s], ~(uint32_t)x);
}

// ---------------------------------------------------------- ALU peak probe

// Integer VALU throughput probe: eight independent chains per lane, each
// step applying the enumeration kernel's instruction mix (and, popcount with
// accumulate, shift, 24-bit multiply-add, max, add) to all eight chains in
// turn, so consecutive instructions never depend on each other and issue,
// not latency, limits the rate.  Written as inline VALU instructions so that
// every iteration is exactly kProbeOpsPerIter ops per lane.
constexpr int kProbeOpsPerIter = 8 * 6;

#define MAPA_PROBE_STEP(OP)                                                     \
  _Pragma("unroll") for (int c = 0; c < 8; ++c) asm volatile(OP : "+v"(x[c]) : "v"(m), "v"(k));

__global__ __launch_bounds__(256) void k_valu_probe(uint32_t *out, int iters, uint32_t seed) {
  uint32_t x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = seed * (threadIdx.x + 7u * c + 1u) + blockIdx.x;
  const uint32_t m = seed | 0x00FF00FFu;
  const uint32_t k = seed >> 7;
  for (int i = 0; i < iters; ++i) {
    MAPA_PROBE_STEP("v_and_b32 %0, %0, %1")
    MAPA_PROBE_STEP("v_bcnt_u32_b32 %0, %0, %2")
    MAPA_PROBE_STEP("v_lshrrev_b32 %0, 3, %0")
    MAPA_PROBE_STEP("v_mad_u32_u24 %0, %0, 3, %2")
    MAPA_PROBE_STEP("v_max_u32 %0, %0, %2")
    MAPA_PROBE_STEP("v_add_u32 %0, %0, %1")
  }
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) r ^= x[c];
  if (r == 0x12345678u) out[blockIdx.x] = r;  // keeps the chains alive
}

#undef MAPA_PROBE_STEP

hipError_t launch_valu_probe(uint32_t *out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_valu_probe, dim3(blocks), dim3(256), 0, s, out, iters, 0x2545F491u);
  return hipGetLastError();
}

int valu_probe_ops_per_iter() { return kProbeOpsPerIter; }

// ---------------------------------------------------------------- launchers


hipError_t launch_batch_front(const BatchArgs &a, hipStream_t s) {
  // 1024-thread blocks, up to 16 queries per thread, at most 64 blocks
  unsigned gb = blocks_for(a.nq, 1024 * 16);
  if (gb < 64) gb = std::min<unsigned>(64, blocks_for(a.nq, 1024));
  if (gb < 1) gb = 1;
  hipLaunchKernelGGL(k_front, dim3(gb), dim3(kFatBlock), 0, s, a);
  // about 2048 blocks: groups of up to 256 queries, or for a batch of fewer
  // than 2048 queries up to 64 blocks per query
  int qpb = (int)((a.nq + 2047) / 2048);
  qpb = std::max(1, std::min(qpb, kExpandThreads));
  const int bpg = qpb == 1 ? std::max(1, std::min(64, 2048 / std::max(1, a.nq))) : 1;
  hipLaunchKernelGGL(k_expand, dim3(blocks_for(a.nq, qpb) * bpg), dim3(kExpandThreads), 0, s, a, qpb,
                     bpg);
  return hipGetLastError();
}

hipError_t launch_enumerate(const BatchArgs &a, hipStream_t s) {
  if (enum_twelve_wide(a))
    return a.rows_in_lds ? launch_enum_pair12_lds(a, s) : launch_enum_pair12_glb(a, s);
  if (a.wpr == 1 && a.pair >= 6) return launch_enum_pair6(a, s);
  return launch_enum_plain(a, s);
}

int enumerate_occupancy(int wpr, int rows_in_lds, int pair, int threads, size_t lds_bytes) {
  if (wpr == 1 && pair >= 12)
    return rows_in_lds ? occ_enum_pair12_lds(threads, lds_bytes) : occ_enum_pair12_glb(threads, lds_bytes);
  if (wpr == 1 && pair >= 6) return occ_enum_pair6(rows_in_lds, threads, lds_bytes);
  return occ_enum_plain(wpr, rows_in_lds, threads, lds_bytes);
}

// every translation unit holds its own copy of the constant tables
hipError_t upload_tables(const Tables &t) {
  hipError_t e = upload_tables_front(t);
  if (e == hipSuccess) e = upload_tables_fused(t);
  if (e == hipSuccess) e = upload_tables_enum_pair12_lds(t);
  if (e == hipSuccess) e = upload_tables_enum_pair12_glb(t);
  if (e == hipSuccess) e = upload_tables_enum_pair6(t);
  if (e == hipSuccess) e = upload_tables_enum_plain(t);
  return e;
}

hipError_t launch_finalize(const BatchArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(blocks_for(a.nq, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_set_busy(const int32_t *ids, const uint32_t *masks, int32_t count,
                           int32_t nservers, const int32_t *server_topo, const int32_t *topo_n,
                           uint32_t *busy, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_busy, dim3(blocks_for(count, 256)), dim3(256), 0, s, ids, masks,
                     count, nservers, server_topo, topo_n, busy);
  return hipGetLastError();
}

hipError_t launch_get_busy(const int32_t *ids, int32_t count, const uint32_t *busy,
                           uint32_t *out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_get_busy, dim3(blocks_for(count, 256)), dim3(256), 0, s, ids, count,
                     busy, out);
  return hipGetLastError();
}

hipError_t launch_release_check(const int64_t *h, int32_t stride, int32_t count,
                                const uint32_t *busy, uint32_t *flag, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_release_check, dim3(blocks_for(count, 256)), dim3(256), 0, s, h, stride,
                     count, busy, flag);
  return hipGetLastError();
}

hipError_t launch_release_apply(const int64_t *h, int32_t stride, int32_t count,
                                int32_t nservers, uint32_t *busy, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_release_apply, dim3(blocks_for(count, 256)), dim3(256), 0, s, h, stride,
                     count, nservers, busy);
  return hipGetLastError();
}

}  // namespace mapa
