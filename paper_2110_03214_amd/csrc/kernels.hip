// HIP kernels of the MAPA allocation hot path, written for gfx950 (CDNA4,
// wave64).  Integer-only: every match is enumerated and scored exactly.
//
// Batch pipeline (one launch each, all on the caller's stream):
//   k_prepare    per query: validate, free set R, constant key term b*W(R),
//                per-split prefix depths and item totals, commit claim.
//   k_bucketize  choose one split for the batch; per query: prefix depth d,
//                shape bucket, offset inside the bucket.
//   k_layout     one block: lays the buckets out (largest items first), pads
//                each to whole 64-item chunks, resets the per-batch counters.
//   k_expand     fills every query's work-list slots with (query, item index);
//                k_enumerate turns the index into the prefix tuple.
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

#include "mapa_internal.h"

namespace mapa {

__constant__ Tables c_tab;

hipError_t upload_tables(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ unsigned long long perm64(int F, int k) {
  unsigned long long p = 1;
  for (int i = 0; i < k; ++i) p *= (unsigned long long)(F - i);
  return p;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Commit arbitration: every committing query of a batch claims its server's
// slot with atomicMin(query index); the holder of the minimum (the first
// committing query in array order) is the only one allowed to commit, and it
// resets the slot to "free" (all ones) in k_finalize, so slots are free
// between batches and concurrent batches on disjoint servers never interact.
constexpr unsigned long long kSlotFree = ~0ull;

// Weighted popcount over a bit-plane row with a runtime number of words:
// sum_{u in X} W[v][u] for row r of vertex v and X2 = X | X << 16.
__device__ __forceinline__ int wsum_rt(const uint32_t *r, int wpr, uint32_t m2) {
  int s = 0;
  for (int w = wpr - 1; w >= 0; --w) {
    const uint32_t x = r[w] & m2;
    s = s * 4 + __popc(x) + __popc(x >> 16);
  }
  return s;
}

// W(X): total weight of the pairs inside X (each pair seen from both ends).
__device__ __forceinline__ int set_weight(const uint32_t *trow, int wpr, uint32_t X) {
  const uint32_t X2 = X | (X << 16);
  int s = 0;
  if (wpr == 1) {
    // the 16 rows as four 16-byte loads issued together
    const uint4 *r4 = reinterpret_cast<const uint4 *>(trow);
    const uint4 q0 = r4[0], q1 = r4[1], q2 = r4[2], q3 = r4[3];
    const uint32_t row[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                              q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t x = row[v] & X2;
      s += ((X >> v) & 1u) ? (int)(__popc(x) + __popc(x >> 16)) : 0;
    }
    return s >> 1;
  }
  for (uint32_t m = X; m; m &= m - 1) s += wsum_rt(trow + (__builtin_ctz(m)) * wpr, wpr, X2);
  return s >> 1;
}

// ----------------------------------------------------------------- prepare

// Plan of one query against the busy mask now in memory: validation, free
// set R, the key's constant term b*W(R), the pattern's back-neighbour table.
__device__ __forceinline__ Plan make_plan(const mapa_query &q, int32_t nservers,
                                          const int32_t *server_topo, const int32_t *topo_n,
                                          const uint8_t *topo_maxw, const uint32_t *busy,
                                          const uint32_t *rows, int wpr) {
  Plan p = {};
  p.server = q.server;
  p.kind = q.kind;
  p.k = q.k;
  p.mode = q.mode;
  p.a = q.a;
  p.b = q.b;
  p.commit = q.commit;
  const bool ok = q.server >= 0 && q.server < nservers && q.kind <= 2 && q.k >= 1 &&
                  q.k <= kMaxK && q.mode <= 1 && q.commit <= 1 && q.a >= 0 &&
                  q.a <= MAPA_MAX_AB && q.b >= 0 && q.b <= MAPA_MAX_AB &&
                  (q.metric == MAPA_METRIC_WEIGHTED || q.metric == MAPA_METRIC_EFFBW);
  if (!ok) {
    p.status = kPlanInvalid;
    return p;
  }
  const int t = server_topo[q.server];
  p.metric = (uint8_t)q.metric;
  if (q.metric == MAPA_METRIC_EFFBW && topo_maxw[t] > 2) {  // no link class in Eq. 2
    p.status = kPlanInvalid;
    return p;
  }
  const int n = topo_n[t];
  const uint32_t R = ~busy[q.server] & ((1u << n) - 1u);
  const int F = __popc(R);
  p.topo = (uint16_t)t;
  p.n = (uint8_t)n;
  p.R = R;
  p.F = (uint8_t)F;
  // the search's running score starts from b * W(R); for Eq. 2 it is the
  // link mix of the edges placed so far, which starts empty
  p.kp0 = q.metric == MAPA_METRIC_EFFBW ? 0
                                        : (int32_t)q.b * set_weight(rows + (size_t)t * kTopoWords * wpr, wpr, R);
  p.nbtab = c_tab.nbtab[q.kind][q.k];
  p.status = q.k > F ? kPlanNofit : kPlanOk;
  return p;
}

__global__ __launch_bounds__(256) void k_prepare(BatchArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long leaves = 0;
  unsigned long long items[kNumSplits];
#pragma unroll
  for (int j = 0; j < kNumSplits; ++j) items[j] = 0;

  if (i < a.nq) {
    const mapa_query q = a.q[i];
    const Plan p = make_plan(q, a.nservers, a.server_topo, a.topo_n, a.topo_maxw, a.busy, a.rows,
                             a.wpr);
    if (p.status == kPlanOk) {
      leaves = c_tab.perm[p.F][p.k];
      const uint8_t *sd = a.split_d + ((size_t)p.F * (kMaxK + 1) + p.k) * kNumSplits;
#pragma unroll
      for (int j = 0; j < kNumSplits; ++j) items[j] = c_tab.perm[p.F][sd[j]];
    }
    if (p.status != kPlanInvalid && p.commit)
      atomicMin(&a.commit_slot[p.server], (unsigned long long)i);
    a.plan[i] = p;
    a.acc_count[i] = 0;
    a.acc_best[i] = 0;
  }
  // wave sums -> block sums in LDS -> one global atomic per block and counter
  __shared__ unsigned long long s_tot[kNumSplits + 1];
  if (threadIdx.x <= kNumSplits) s_tot[threadIdx.x] = 0;
  __syncthreads();
  leaves = wave_sum_u64(leaves);
#pragma unroll
  for (int j = 0; j < kNumSplits; ++j) items[j] = wave_sum_u64(items[j]);
  if ((threadIdx.x & 63) == 0) {
    if (leaves) atomicAdd(&s_tot[kNumSplits], leaves);
#pragma unroll
    for (int j = 0; j < kNumSplits; ++j)
      if (items[j]) atomicAdd(&s_tot[j], items[j]);
  }
  __syncthreads();
  if (threadIdx.x <= kNumSplits && s_tot[threadIdx.x])
    atomicAdd(&a.ctr->totals[blockIdx.x % kTotCopies][threadIdx.x][0], s_tot[threadIdx.x]);
}

// --------------------------------------------------------------- bucketize

constexpr int kFatBlock = 1024;  // threads of k_bucketize and k_layout blocks

// Lay the buckets out (largest items first), pad each to whole 64-item
// chunks with invalid items, and reset the per-batch counters.  Run by the
// one block of k_layout, once every k_bucketize block's counts are in.
__device__ void layout_buckets(const BatchArgs &a) {
  __shared__ uint32_t s_pad[kNumBuckets];
  __shared__ uint32_t s_cnt[kNumBuckets];
  __shared__ uint32_t s_start[kNumBuckets];
  const int t = threadIdx.x;
  // loops over the buckets have a fixed stride (one 1024-thread block), so
  // they unroll and each thread's loads are in flight together
#pragma unroll
  for (int r = t; r < kNumBuckets; r += kFatBlock) {
    const int b = c_tab.rank_bucket[r];
    const uint32_t cnt = __hip_atomic_load(&a.ctr->bucket_items[b][0], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    s_cnt[r] = cnt;
    s_pad[r] = (cnt + (kChunk - 1)) & ~(uint32_t)(kChunk - 1);
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
  for (int r = t; r < kNumBuckets; r += kFatBlock) {
    const int b = c_tab.rank_bucket[r];
    a.ctr->bucket_start[b] = s_start[r];
    for (uint32_t x = s_cnt[r]; x < s_pad[r]; ++x) a.items[s_start[r] + x] = make_uint2(kInvalidItem, 0u);
    a.ctr->bucket_items[b][0] = 0;
  }
  if (t < kQueues) a.ctr->queue_ctr[t][0] = 0;
  for (int e = t; e < kTotCopies * (kNumSplits + 1); e += blockDim.x)
    a.ctr->totals[e / (kNumSplits + 1)][e % (kNumSplits + 1)][0] = 0;
}

// One block, after k_bucketize: the bucket layout (the counts it needs are
// final only once every k_bucketize block has added its own).
__global__ __launch_bounds__(1024) void k_layout(BatchArgs a) { layout_buckets(a); }

// Few, fat blocks: each block histograms many queries in LDS and then adds
// one total per bucket to the global counters, so every global counter sees
// only a handful of atomics.
__global__ __launch_bounds__(1024) void k_bucketize(BatchArgs a) {
  __shared__ int s_split;
  __shared__ uint32_t s_cnt[kNumBuckets];
  __shared__ uint32_t s_base[kNumBuckets];
  __shared__ unsigned long long s_part[kTotCopies * (kNumSplits + 1)];
  __shared__ unsigned long long s_tot[kNumSplits + 1];
#pragma unroll
  for (int b = threadIdx.x; b < kNumBuckets; b += kFatBlock) s_cnt[b] = 0;
  // the batch totals: every copy loaded at once (one load per thread), then summed
  if (threadIdx.x < kTotCopies * (kNumSplits + 1))
    s_part[threadIdx.x] =
        a.ctr->totals[threadIdx.x / (kNumSplits + 1)][threadIdx.x % (kNumSplits + 1)][0];
  __syncthreads();
  if (threadIdx.x <= kNumSplits) {
    unsigned long long v = 0;
    for (int c = 0; c < kTotCopies; ++c) v += s_part[c * (kNumSplits + 1) + threadIdx.x];
    s_tot[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // The split is a pure function of batch totals, so every block picks the
    // same one.  Items get finer (more, smaller) as j falls.  Finer items
    // balance the lanes better but each costs a fixed setup, so take the
    // finest split that fits the work-list, gives every resident lane an
    // item and keeps the mean item at mean_leaves embeddings or more.
    // Failing that: the coarsest split that still gives every lane an item;
    // for a batch too small for that, the finest split that fits.  Whole
    // queries (one item each) always fit.
    const unsigned long long leaves = s_tot[kNumSplits];
    int best = -1, busy = -1, finest = kSplitWhole;
    for (int c = kSplitWhole; c >= 0; --c) {
      const unsigned long long n = s_tot[c];
      if (n + kPadReserve > a.cap_items) break;
      finest = c;
      if (n >= a.lanes) {
        if (busy < 0) busy = c;
        if (leaves >= n * (unsigned long long)a.mean_leaves) best = c;
      }
    }
    const int j = best >= 0 ? best : busy >= 0 ? busy : finest;
    s_split = j;
    if (blockIdx.x == 0) {
      a.ctr->chosen_split = (uint32_t)j;
      a.ctr->last_total_items = s_tot[j];
    }
  }
  __syncthreads();
  const int j = s_split;
  const int per_block = (a.nq + gridDim.x - 1) / gridDim.x;
  const int q0 = blockIdx.x * per_block;
  const int q1 = min(a.nq, q0 + per_block);
  constexpr int kMaxPerThread = 16;
  uint32_t local[kMaxPerThread];
  int bk[kMaxPerThread];
#pragma unroll
  for (int r = 0; r < kMaxPerThread; ++r) {
    const int i = q0 + threadIdx.x + r * (int)blockDim.x;
    bk[r] = -1;
    local[r] = 0;
    if (i < q1) {
      const Plan &p = a.plan[i];
      if (p.status == kPlanOk) {
        const int d = a.split_d[((size_t)p.F * (kMaxK + 1) + p.k) * kNumSplits + j];
        const uint32_t nitems = (uint32_t)c_tab.perm[p.F][d];
        const int b = bucket_id(p.metric, p.mode, p.kind, p.k - d, p.F - d);
        a.plan[i].d = (uint8_t)d;
        a.plan[i].bucket = (uint16_t)b;
        a.plan[i].nitems = nitems;
        bk[r] = b;
        local[r] = atomicAdd(&s_cnt[b], nitems);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = threadIdx.x; c < kNumBuckets; c += kFatBlock)
    s_base[c] = s_cnt[c] ? atomicAdd(&a.ctr->bucket_items[c][0], s_cnt[c]) : 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kMaxPerThread; ++r) {
    const int i = q0 + threadIdx.x + r * (int)blockDim.x;
    if (bk[r] >= 0) a.plan[i].item_off = s_base[bk[r]] + local[r];
  }
}

// ------------------------------------------------------------------ expand

// Prefix item x of a query (0 <= x < F!/(F-d)!) is the x-th injective
// d-tuple of free vertices in lexicographic order: digit t of x in the mixed
// radix (F, F-1, ..., F-d+1) picks the digit-th smallest still-unused vertex.
// Returns the tuple with the vertex of position t at bits 4t..4t+3.
// Position of the r-th (from 0) set bit of a 16-bit mask that has more than
// r set bits: a branch-free binary search on popcounts.
__device__ __forceinline__ int select_bit(uint32_t m, uint32_t r) {
  int pos = 0;
  uint32_t c = __popc(m & 0xFFu);
  bool up = r >= c;
  r -= up ? c : 0u;
  pos += up ? 8 : 0;
  c = __popc((m >> pos) & 0xFu);
  up = r >= c;
  r -= up ? c : 0u;
  pos += up ? 4 : 0;
  c = __popc((m >> pos) & 0x3u);
  up = r >= c;
  r -= up ? c : 0u;
  pos += up ? 2 : 0;
  c = (m >> pos) & 1u;
  pos += r >= c ? 1 : 0;
  return pos;
}

// Prefix x of depth d: x is a mixed-radix number whose digit t (radix F - t,
// most significant first) picks the position-t vertex among the free
// vertices not yet chosen, in increasing order, so consecutive x are
// consecutive prefixes in lexicographic order.  Digits come off the least
// significant end by multiply-high division (x < 2^28); the vertices then
// follow in order.  Returns the prefix's mapping code (vertex of position t
// at bits 4t..4t+3).
__device__ __forceinline__ uint32_t unrank_prefix(uint32_t x, int d, int F, uint32_t R) {
  uint32_t digits = 0;
  for (int t = d - 1; t >= 0; --t) {
    const uint32_t m = (uint32_t)(F - t);
    const uint32_t q = m > 1 ? __umulhi(x, c_tab.inv[m]) : x;
    digits |= (x - q * m) << (4 * t);
    x = q;
  }
  uint32_t avail = R, code = 0;
  for (int t = 0; t < d; ++t) {
    const int v = select_bit(avail, (digits >> (4 * t)) & 15u);
    avail &= ~(1u << v);
    code |= (uint32_t)v << (4 * t);
  }
  return code;
}

constexpr uint32_t kExpandSmall = 16;  // a lane writes up to this many items itself

// Work-list fill: item slot base+x of a query holds (query, x).  One-wave
// blocks own a range of queries; a lane fills a small query's items, the
// whole wave a large one's.
__global__ __launch_bounds__(64) void k_expand(BatchArgs a, int qpb) {
  __shared__ int s_big[64];
  __shared__ int s_nbig;
  const int q0 = blockIdx.x * qpb;
  const int q1 = min(a.nq, q0 + qpb);
  if (threadIdx.x == 0) s_nbig = 0;
  __syncthreads();
  for (int i = q0 + threadIdx.x; i < q1; i += blockDim.x) {
    const Plan &p = a.plan[i];
    if (p.status != kPlanOk) continue;
    if (p.nitems > kExpandSmall) {
      s_big[atomicAdd(&s_nbig, 1)] = i;
      continue;
    }
    uint2 *dst = a.items + a.ctr->bucket_start[p.bucket] + p.item_off;
    for (uint32_t x = 0; x < p.nitems; ++x) dst[x] = make_uint2((uint32_t)i, x);
  }
  __syncthreads();
  const int nbig = s_nbig;
  for (int bi = 0; bi < nbig; ++bi) {
    const int i = s_big[bi];
    const Plan &p = a.plan[i];
    uint2 *dst = a.items + a.ctr->bucket_start[p.bucket] + p.item_off;
    for (uint32_t x = threadIdx.x; x < p.nitems; x += blockDim.x) dst[x] = make_uint2((uint32_t)i, x);
  }
}

// --------------------------------------------------------------- enumerate

struct LaneState {
  const uint32_t *trow;  // this lane's topology rows [16][WPR]
  uint32_t R;            // free set
  int a, b;
  int k;
  int linked;
  unsigned long long nbtab;  // byte p: pattern neighbours of position p that precede it
  uint32_t count;        // matches seen
  // best leaf so far: bpk = ((key + 1) << 4) | (15 - last vertex) of the best
  // leaf-parent node (0: none), bcode = that node's mapping of positions < k-1
  uint32_t bpk;
  uint32_t bcode;
  // Eq. 2 (bandwidth-sensitive queries): rank table and this pattern's block
  const uint16_t *erank;
  int eoff, e1;
};

template <int WPR>
__device__ __forceinline__ int wsum(const uint32_t *r, uint32_t m2) {
  int s = 0;
#pragma unroll
  for (int w = WPR - 1; w >= 0; --w) {
    const uint32_t x = r[w] & m2;
    s = s * 4 + __popc(x) + __popc(x >> 16);
  }
  return s;
}

template <int WPR>
__device__ __forceinline__ uint32_t adjacency(const uint32_t *r) {
  uint32_t x = 0;
#pragma unroll
  for (int w = 0; w < WPR; ++w) x |= r[w] | (r[w] >> 16);
  return x & 0xFFFFu;
}

// Vertices at the pattern neighbours of position p that precede it, and the
// candidate set for position p.
//   ALL mode: computed per pattern kind (wave-uniform): ring -> the previous
//   vertex, plus vertex 0 at the closing position; tree -> the parent
//   (heap numbering); all-to-all -> every chosen vertex.  Candidates: every
//   free vertex not chosen yet.
//   LINKED mode: from the back-neighbour table; candidates must also be
//   adjacent to each of those vertices.
//   KIND >= 0 fixes the pattern kind at compile time (ALL mode inside the
//   search, where it is wave-uniform); KIND < 0 reads it from `kind`.
template <int WPR, bool LINKED, bool LAST, int KIND = -1>
__device__ __forceinline__ void node_masks(const LaneState &s, int kind, uint32_t rest,
                                           uint32_t code, int p, uint32_t prev, uint32_t &nbm,
                                           uint32_t &cand) {
  cand = rest;
  if constexpr (!LINKED) {
    const int kd = KIND >= 0 ? KIND : kind;
    if (kd == MAPA_ALL_TO_ALL) {
      nbm = s.R & ~rest;
    } else if (kd == MAPA_RING) {
      nbm = p > 0 ? (1u << prev) : 0u;
      if (LAST && s.k >= 3) nbm |= 1u << (code & 15u);
    } else {
      nbm = p > 0 ? (1u << ((code >> (4 * ((p - 1) >> 1))) & 15u)) : 0u;
    }
  } else {
    const uint32_t nbpos = (uint32_t)(s.nbtab >> (8 * p)) & 0xFFu;
    nbm = 0;
    for (uint32_t m = nbpos; m; m &= m - 1) {
      const int v = (code >> (4 * __builtin_ctz(m))) & 15;
      nbm |= 1u << v;
      cand &= adjacency<WPR>(s.trow + v * WPR);
    }
  }
}

// The last two pattern positions in ALL mode, with the N = M + 1 free
// vertices left (c_0 < ... < c_M) and M wave-uniform: every ordered pair
// (c_i at position p = k-2, c_j at position k-1) is a match.  With
//   D_j = w(c_j, rest)               weight to every vertex still free,
//   X_j = w(c_j, fixed neighbours of position k-1, i.e. those other than c_i),
//   Y_i = w(c_i, neighbours of position p),
// the leaf key of (c_i, c_j) is
//   kp + a*Y_i - b*D_i + a*(X_j + alpha*W[c_j][c_i]) - b*(D_j - W[c_j][c_i])
// where alpha says whether position p neighbours position k-1.  Per node the
// N values P_j = 16a*X_j - 16b*D_j - c_j are computed once; a leaf is then
// one packed-weight field, one multiply-add and a max.  The inner loop is
// unrolled over N, so the per-candidate values stay in registers.  Leaves
// come in lexicographic order (c_i, then c_j, ascending) as in level().
// Rows of one word (weights up to 3): the packed weight of u is 2 bits at 2u.
template <int M, int KIND, bool PRES>
__device__ __forceinline__ void pair_level(LaneState &s, uint32_t rest, uint32_t code, int kp,
                                           int p, uint32_t prev) {
  constexpr int N = M + 1;
  uint32_t nbm, cand;
  node_masks<1, false, false, KIND>(s, KIND, rest, code, p, prev, nbm, cand);
  // fixed neighbours of position k-1 and whether position p is one of them
  uint32_t fixm = 0;
  bool alpha = true;
  if constexpr (KIND == MAPA_ALL_TO_ALL) {
    fixm = s.R & ~rest;
  } else if constexpr (KIND == MAPA_RING) {
    if (s.k >= 3) fixm = 1u << (code & 15u);
  } else {
    const int parent = (s.k - 2) >> 1;  // heap parent of position k-1
    alpha = parent == p;
    if (!alpha) fixm = 1u << ((code >> (4 * parent)) & 15u);
  }
  const uint32_t nb2 = nbm | (nbm << 16), rest2 = rest | (rest << 16), fix2 = fixm | (fixm << 16);
  const uint32_t *prow = s.trow + 16;  // packed-weight rows
  uint32_t sh2[N];                     // 2 * c_j: bit offset of c_j's packed weight
  int P[N];
  uint32_t r = rest;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const uint32_t c = (uint32_t)__builtin_ctz(r);
    r &= r - 1;
    sh2[j] = 2 * c;
    const uint32_t *row = s.trow + c;
    P[j] = __mul24(16 * s.a, wsum<1>(row, fix2)) - (int)c;
    if constexpr (PRES) P[j] -= __mul24(16 * s.b, wsum<1>(row, rest2));
  }
  const int gamma = (alpha ? 16 * s.a : 0) + (PRES ? 16 * s.b : 0);
  s.count += (uint32_t)(N * M);
  const int sh = 4 * p;
  uint32_t ri = rest;
  for (int i = 0; i < N; ++i) {
    const uint32_t ci = (uint32_t)__builtin_ctz(ri);
    ri &= ri - 1;
    const uint32_t *row = s.trow + ci;
    int kp2 = kp + __mul24(s.a, wsum<1>(row, nb2));
    if constexpr (PRES) kp2 -= __mul24(s.b, wsum<1>(row, rest2));
    const int base = 16 * kp2 + 31;
    const uint32_t wp = prow[ci];
    const uint32_t si = 2 * ci;
    uint32_t pb = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int w = (int)((wp >> sh2[j]) & 3u);
      const uint32_t pk = (uint32_t)(base + P[j] + __mul24(gamma, w));
      pb = (pk > pb && sh2[j] != si) ? pk : pb;  // c_j = c_i is no match
    }
    const bool better = pb > (s.bpk | 15u);
    s.bpk = better ? pb : s.bpk;
    s.bcode = better ? (code | (ci << sh)) : s.bcode;
  }
}

// pair_level for N = 2 .. PAIRN free vertices at the last two positions (rows
// of one word); other shapes take the general per-level loops.
template <int KIND, int PAIRN, bool PRES>
__device__ __forceinline__ bool pair_dispatch(LaneState &s, uint32_t rest, uint32_t code, int kp,
                                              int p, uint32_t prev, int mu) {
  switch (mu) {
    case 2:
      if constexpr (PAIRN >= 2) {
        pair_level<1, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 3:
      if constexpr (PAIRN >= 3) {
        pair_level<2, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 4:
      if constexpr (PAIRN >= 4) {
        pair_level<3, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 5:
      if constexpr (PAIRN >= 5) {
        pair_level<4, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 6:
      if constexpr (PAIRN >= 6) {
        pair_level<5, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 7:
      if constexpr (PAIRN >= 7) {
        pair_level<6, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 8:
      if constexpr (PAIRN >= 8) {
        pair_level<7, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 9:
      if constexpr (PAIRN >= 9) {
        pair_level<8, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 10:
      if constexpr (PAIRN >= 10) {
        pair_level<9, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 11:
      if constexpr (PAIRN >= 11) {
        pair_level<10, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    case 12:
      if constexpr (PAIRN >= 12) {
        pair_level<11, KIND, PRES>(s, rest, code, kp, p, prev);
        return true;
      }
      return false;
    default: return false;
  }
}

// One pattern position: expand every candidate vertex c, scoring it with
//   a * (weight from c to the vertices at its earlier pattern neighbours)
//   - b * (weight from c to the free vertices not yet chosen)
// and recurse; at the last position keep the node's best leaf.
//
// The chain is entered at its top for every item: a level above the item's
// run of positions (Lrun) passes straight through, so each level exists once
// per instantiation.  In ALL mode every lane of a wave holds an item of the
// same bucket, so all lanes have the same number of candidates mu at every
// node and the loops are counted on the scalar unit; the last two positions
// go to pair_level.  The leaf loop keeps the node's best as one u32,
// ((key + 1) << 4) | (15 - c), so one max() picks the largest key and, among
// equal keys, the smallest vertex; the node then replaces the lane's best only
// on a strictly larger key (leaves arrive in lexicographic order).
template <int L, int WPR, bool LINKED, int KIND, int PAIR, bool PRES = true>
__device__ __forceinline__ void level(LaneState &s, int kind, uint32_t rest, uint32_t code,
                                      int kp, int p, uint32_t prev, int mu, int Lrun) {
  if constexpr (L > 1) {
    if (Lrun < L) {
      level<L - 1, WPR, LINKED, KIND, PAIR, PRES>(s, kind, rest, code, kp, p, prev, mu, Lrun);
      return;
    }
  }
  if constexpr (PAIR > 0 && L == 2 && !LINKED && KIND >= 0 && WPR == 1) {
    if (pair_dispatch<KIND, PAIR, PRES>(s, rest, code, kp, p, prev, mu)) return;
  }
  uint32_t nbm, cand;
  node_masks<WPR, LINKED, L == 1, KIND>(s, kind, rest, code, p, prev, nbm, cand);
  const uint32_t nb2 = nbm | (nbm << 16);
  const uint32_t rest2 = rest | (rest << 16);
  const int m = LINKED ? __popc(cand) : mu;
  if constexpr (L == 1) {
    s.count += (uint32_t)m;
    // ((key + 1) << 4) | (15 - c)  ==  16*(kp + 1) + 15 + 16a*nb - 16b*dr - c
    const int base = 16 * kp + 31;
    const int a16 = 16 * s.a, b16 = 16 * s.b;
    uint32_t pb = 0;
#pragma unroll 2
    for (int t = 0; t < m; ++t) {
      const int c = __builtin_ctz(cand);
      cand &= cand - 1;
      const uint32_t *rc = s.trow + c * WPR;
      int v = base + __mul24(a16, wsum<WPR>(rc, nb2)) - c;
      if constexpr (PRES) v -= __mul24(b16, wsum<WPR>(rc, rest2));
      const uint32_t pk = (uint32_t)v;
      pb = pk > pb ? pk : pb;
    }
    // strictly larger key <=> pb > (bpk | 15)
    const bool better = pb > (s.bpk | 15u);
    s.bpk = better ? pb : s.bpk;
    s.bcode = better ? code : s.bcode;
  } else {
    const int sh = 4 * p;
    for (int t = 0; t < m; ++t) {
      const int c = __builtin_ctz(cand);
      cand &= cand - 1;
      const uint32_t *rc = s.trow + c * WPR;
      int kp2 = kp + __mul24(s.a, wsum<WPR>(rc, nb2));
      if constexpr (PRES) kp2 -= __mul24(s.b, wsum<WPR>(rc, rest2));
      level<L - 1, WPR, LINKED, KIND, PAIR, PRES>(s, kind, rest & ~(1u << c), code | ((uint32_t)c << sh),
                                            kp2, p + 1, (uint32_t)c, mu - 1, L - 1);
    }
  }
}

template <int WPR, bool LINKED, int KIND, int PAIR, bool PRES = true>
__device__ __forceinline__ void expand(LaneState &s, int kind, int L, uint32_t rest,
                                       uint32_t code, int kp, int d, uint32_t prev, int mu) {
  if (L > 0) level<kMaxK, WPR, LINKED, KIND, PAIR, PRES>(s, kind, rest, code, kp, d, prev, mu, L);
}

// Bandwidth-sensitive queries (Eq. 2, sensitive branch of Alg. 1).  The
// search carries the link mix of the pattern edges placed so far, packed as
// x << 8 | y (x double NVLinks, y single NVLinks; z follows from the edge
// count), and a leaf's key is the rank of its mix's predicted effective
// bandwidth.  The mix added by placing c: among the vertices at the
// position's earlier pattern neighbours, those joined to c by weight 2 (high
// bit-plane only) and by weight 1 (low bit-plane only); such topologies have
// no higher planes.
template <int WPR>
__device__ __forceinline__ uint32_t link_mix(const uint32_t *rc, uint32_t nbm) {
  const uint32_t lo = rc[0] & 0xFFFFu, hi = rc[0] >> 16;
  return ((uint32_t)__popc(hi & ~lo & nbm) << 8) + (uint32_t)__popc(lo & ~hi & nbm);
}

template <int L, int WPR, bool LINKED>
__device__ __forceinline__ void level_eff(LaneState &s, int kind, uint32_t rest, uint32_t code,
                                          uint32_t mix, int p, uint32_t prev, int mu, int Lrun) {
  if constexpr (L > 1) {
    if (Lrun < L) {
      level_eff<L - 1, WPR, LINKED>(s, kind, rest, code, mix, p, prev, mu, Lrun);
      return;
    }
  }
  uint32_t nbm, cand;
  node_masks<WPR, LINKED, L == 1>(s, kind, rest, code, p, prev, nbm, cand);
  const int m = LINKED ? __popc(cand) : mu;
  if constexpr (L == 1) {
    s.count += (uint32_t)m;
    uint32_t pb = 0;
    for (int t = 0; t < m; ++t) {
      const int c = __builtin_ctz(cand);
      cand &= cand - 1;
      const uint32_t mx = mix + link_mix<WPR>(s.trow + c * WPR, nbm);
      const uint32_t rank = s.erank[s.eoff + (int)(mx >> 8) * s.e1 + (int)(mx & 255u)];
      const uint32_t pk = 16 * rank + 31 - (uint32_t)c;  // ((rank + 1) << 4) | (15 - c)
      pb = pk > pb ? pk : pb;
    }
    const bool better = pb > (s.bpk | 15u);
    s.bpk = better ? pb : s.bpk;
    s.bcode = better ? code : s.bcode;
  } else {
    const int sh = 4 * p;
    for (int t = 0; t < m; ++t) {
      const int c = __builtin_ctz(cand);
      cand &= cand - 1;
      level_eff<L - 1, WPR, LINKED>(s, kind, rest & ~(1u << c), code | ((uint32_t)c << sh),
                                    mix + link_mix<WPR>(s.trow + c * WPR, nbm), p + 1,
                                    (uint32_t)c, mu - 1, L - 1);
    }
  }
}

// One prefix item: prefix x (of depth p.d) of query plan *pp, expanded over
// the remaining positions.  pp == nullptr: the lane holds no item.  Returns
// the item's match count and its best as one u64 (key high, inverted
// lexicographic mapping code low, so max() takes the largest key and then
// the smallest mapping; 0: no match).  trow: the topology's rows.
template <int WPR, int PAIR>
__device__ __forceinline__ void item_search(const Plan *pp, const uint32_t *trow, uint32_t x,
                                            const uint16_t *erank, unsigned long long &cnt_out,
                                            unsigned long long &best_out) {
  const bool valid = pp != nullptr;
  LaneState s;
  s.count = 0;
  s.bpk = 0;
  s.bcode = 0;
  s.k = 0;
  s.linked = 0;
  s.erank = erank;
  s.eoff = 0;
  s.e1 = 1;
  uint32_t rest = 0, code = 0, prev = 0;
  int kp = 0, L = 0, d = 0, kind = 0, fp = 0, metric = 0;
  if (valid) {
    const Plan &p = *pp;
    s.trow = trow;
    s.R = p.R;
    s.a = p.a;
    s.b = p.b;
    s.k = p.k;
    s.linked = p.mode;
    s.nbtab = p.nbtab;
    metric = p.metric;
    if (metric) {
      const int E = __popcll(p.nbtab);  // pattern edges: one back-neighbour bit each
      s.eoff = eff_off(E);
      s.e1 = E + 1;
    }
    kind = p.kind;
    d = p.d;
    fp = p.F - d;
    rest = p.R;
    kp = p.kp0;
    bool ok = true;
    const uint32_t prefix = unrank_prefix(x, d, p.F, p.R);
    for (int pos = 0; pos < d; ++pos) {
      const int v = (prefix >> (4 * pos)) & 15;
      uint32_t nbm, cand;
      if (s.linked)
        node_masks<WPR, true, false>(s, kind, rest, code, pos, prev, nbm, cand);
      else if (pos == s.k - 1)
        node_masks<WPR, false, true>(s, kind, rest, code, pos, prev, nbm, cand);
      else
        node_masks<WPR, false, false>(s, kind, rest, code, pos, prev, nbm, cand);
      ok = ok && ((cand >> v) & 1u);
      const uint32_t *rv = s.trow + v * WPR;
      if (metric)
        kp += (int)link_mix<WPR>(rv, nbm);
      else
        kp += __mul24(s.a, wsum<WPR>(rv, nbm | (nbm << 16))) -
              __mul24(s.b, wsum<WPR>(rv, rest | (rest << 16)));
      rest &= ~(1u << v);
      code |= (uint32_t)v << (4 * pos);
      prev = (uint32_t)v;
    }
    L = ok ? (int)p.k - d : 0;
  }
  // Items of one chunk share a bucket: the mode, the pattern kind and (ALL
  // mode) the number of free vertices below the prefix are wave-uniform
  // (lane 0 holds a real item whenever any lane does).
  const int kind_w = __builtin_amdgcn_readfirstlane(kind);
  const int fp_w = __builtin_amdgcn_readfirstlane(fp);
  if (__builtin_amdgcn_readfirstlane(metric)) {
    if (L > 0) {
      if (__builtin_amdgcn_readfirstlane(s.linked))
        level_eff<kMaxK, WPR, true>(s, kind_w, rest, code, (uint32_t)kp, d, prev, 0, L);
      else
        level_eff<kMaxK, WPR, false>(s, kind_w, rest, code, (uint32_t)kp, d, prev, fp_w, L);
    }
  } else if (__builtin_amdgcn_readfirstlane(s.linked))
    expand<WPR, true, -1, PAIR>(s, kind_w, L, rest, code, kp, d, prev, 0);
  else if (__builtin_amdgcn_readfirstlane(L) >= fp_w - 1) {
    // The item's remaining positions leave at most one free vertex unused, so
    // every match below it preserves nothing (Eq. 3 over no pair): take the
    // preserved weight of its free vertices out of the running key once and
    // score the subtree by AggBW alone.
    if (L > 0) kp -= __mul24(s.b, set_weight(s.trow, WPR, rest));
    if (kind_w == MAPA_RING)
      expand<WPR, false, MAPA_RING, PAIR, false>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
    else if (kind_w == MAPA_ALL_TO_ALL)
      expand<WPR, false, MAPA_ALL_TO_ALL, PAIR, false>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
    else
      expand<WPR, false, MAPA_TREE, PAIR, false>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  } else if (kind_w == MAPA_RING)
    expand<WPR, false, MAPA_RING, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  else if (kind_w == MAPA_ALL_TO_ALL)
    expand<WPR, false, MAPA_ALL_TO_ALL, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  else
    expand<WPR, false, MAPA_TREE, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);

  int bkey = -1;
  uint32_t bcode = 0;
  if (s.bpk) {
    bkey = (int)(s.bpk >> 4) - 1;
    bcode = s.bcode | ((15u - (s.bpk & 15u)) << (4 * (s.k - 1)));
  }
  unsigned long long best = 0;
  if (bkey >= 0) {
    uint32_t lex = 0;
    for (int i = 0; i < s.k; ++i) lex = (lex << 4) | ((bcode >> (4 * i)) & 15u);
    best = ((unsigned long long)(uint32_t)bkey << 32) | (0xFFFFFFFFu - lex);
  }
  cnt_out = s.count;
  best_out = best;
}

template <int WPR, int PAIR>
__device__ __forceinline__ void run_item(const BatchArgs &a, const uint32_t *rows, uint2 it) {
  const int lane = threadIdx.x & 63;
  const bool valid = it.x != kInvalidItem;
  const Plan *pp = valid ? &a.plan[it.x] : nullptr;
  const uint32_t *trow = valid ? rows + (uint32_t)pp->topo * (kTopoWords * WPR) : rows;
  unsigned long long cnt, best;
  item_search<WPR, PAIR>(pp, trow, it.y, a.eff_rank, cnt, best);
  const int qi = valid ? (int)it.x : -1;
  const int q0 = __builtin_amdgcn_readfirstlane(qi);
  const bool same = __ballot(valid && qi != q0) == 0ull;
  if (same) {
    cnt = wave_sum_u64(cnt);
    best = wave_max_u64(best);
    if (lane == 0 && q0 >= 0) {
      atomicAdd(&a.acc_count[q0], cnt);
      if (best) atomicMax(&a.acc_best[q0], best);
    }
  } else {
    // The items of one query sit in consecutive lanes of a chunk: fold each
    // run of equal query ids onto its first lane, which alone issues the
    // atomics (one per query and chunk instead of one per item).
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int oq = __shfl_down(qi, off, 64);
      const unsigned long long oc = __shfl_down(cnt, off, 64);
      const unsigned long long ob = __shfl_down(best, off, 64);
      if (lane + off < 64 && oq == qi) {
        cnt += oc;
        best = ob > best ? ob : best;
      }
    }
    const int pq = __shfl_up(qi, 1, 64);
    if (valid && (lane == 0 || pq != qi)) {
      if (cnt) atomicAdd(&a.acc_count[qi], cnt);
      if (best) atomicMax(&a.acc_best[qi], best);
    }
  }
}

template <int WPR, int PAIR>
__device__ __forceinline__ void chunk_loop(const BatchArgs &a, const uint32_t *rows) {
  const int lane = threadIdx.x & 63;
  const uint32_t nchunks = *(volatile const uint32_t *)&a.ctr->total_chunks;
  // Home queue: consecutive blocks land on different XCDs, so the waves of
  // one queue mostly share an XCD.  A wave whose queue runs dry looks at
  // every queue's counter at once (one lane each) and moves to the next one,
  // counting from its home, that still holds chunks.
  const uint32_t home = blockIdx.x % kQueues;
  uint32_t qu = home;
  for (;;) {
    uint32_t c = 0;
    if (lane == 0) c = qu + atomicAdd(&a.ctr->queue_ctr[qu][0], 1u) * (uint32_t)kQueues;
    c = __shfl(c, 0, 64);
    if (c >= nchunks) {
      bool left = false;
      if (lane < kQueues) {
        const uint32_t pos = __hip_atomic_load(&a.ctr->queue_ctr[lane][0], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        left = (unsigned long long)lane + (unsigned long long)pos * kQueues < nchunks;
      }
      const unsigned long long m = __ballot(left);
      if (!m) break;
      // first queue with chunks left at or after home, cyclically
      const unsigned long long hi = m & (~0ull << home);
      qu = (uint32_t)__builtin_ctzll(hi ? hi : m);
      continue;
    }
    const uint2 it = a.items[(size_t)c * kChunk + lane];
    run_item<WPR, PAIR>(a, rows, it);
  }
}

// PAIR > 0: the last two positions of one-word-row topologies with up to PAIR
// free vertices go through pair_level (faster per match, more registers, so
// fewer waves per SIMD).
template <int WPR, bool ROWS_LDS, int PAIR>
// At most 128 VGPRs, so four waves share each SIMD: the values this forces
// to scratch belong to the outer levels of the search, which run rarely.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_enumerate(BatchArgs a) {
  if constexpr (ROWS_LDS) {
    extern __shared__ uint32_t s_rows[];
    const int words = a.ntopo * kTopoWords * WPR;
    for (int i = threadIdx.x; i < words; i += blockDim.x) s_rows[i] = a.rows[i];
    __syncthreads();
    chunk_loop<WPR, PAIR>(a, s_rows);
  } else {
    chunk_loop<WPR, PAIR>(a, a.rows);
  }
}

// ---------------------------------------------------------------- finalize

// A query's result from its plan, match count and best u64: the mapping,
// AggBW (Eq. 1) and PreservedBW (Eq. 3) recomputed from the mapping, checked
// against the key the search kept.  No commit yet (handle -1).
struct Outcome {
  int64_t count;
  int32_t status, key, agg, pres;
  uint32_t S, map_lo, map_hi;
  int32_t links;  // Eq. 2 queries: x | y << 8 | z << 16 of the chosen match
  int64_t handle;
};

__device__ __forceinline__ Outcome decode_best(const Plan &p, unsigned long long cnt,
                                               unsigned long long best, const uint32_t *trow,
                                               int wpr, const uint16_t *eff_rank,
                                               const int32_t *eff_key,
                                               uint32_t *self_check_failures) {
  Outcome o;
  o.count = 0;
  o.status = MAPA_RES_NOFIT;
  o.key = INT32_MIN;
  o.agg = o.pres = 0;
  o.S = 0;
  o.map_lo = o.map_hi = 0xFFFFFFFFu;
  o.links = 0;
  o.handle = -1;
  int32_t &status = o.status, &agg = o.agg, &pres = o.pres;
  uint32_t &S = o.S, &map_lo = o.map_lo, &map_hi = o.map_hi;
  if (p.status == kPlanInvalid) {
    status = MAPA_RES_INVALID;
  } else if (p.status == kPlanOk) {
    o.count = (int64_t)cnt;
    if (cnt > 0) {
      const int k = p.k;
      const uint32_t lex = 0xFFFFFFFFu - (uint32_t)best;
      uint32_t phi_code = 0;  // vertex of position t at bits 4t..4t+3
      for (int t = 0; t < k; ++t) {
        const uint32_t v = (lex >> (4 * (k - 1 - t))) & 15u;
        phi_code |= v << (4 * t);
        S |= 1u << v;
        if (t < 4) map_lo = (map_lo & ~(0xFFu << (8 * t))) | (v << (8 * t));
        else map_hi = (map_hi & ~(0xFFu << (8 * (t - 4)))) | (v << (8 * (t - 4)));
      }
      // AggBW (Eq. 1) from the mapping: each position against its earlier
      // pattern neighbours; PreservedBW (Eq. 3): weight left inside R \ S
      const bool eff = p.metric == MAPA_METRIC_EFFBW;
      int lx = 0, ly = 0, lz = 0;  // link mix of the mapped pattern edges (Eq. 2)
      for (int t = 1; t < k; ++t) {
        const uint32_t *rt = trow + ((phi_code >> (4 * t)) & 15u) * wpr;
        uint32_t nbm = 0;
        for (uint32_t m = (uint32_t)(p.nbtab >> (8 * t)) & 0xFFu; m; m &= m - 1) {
          const uint32_t v = (phi_code >> (4 * __builtin_ctz(m))) & 15u;
          nbm |= 1u << v;
          if (eff) {
            const int w = wsum_rt(rt, wpr, (1u << v) | (1u << (v + 16)));
            lx += w == 2;
            ly += w == 1;
            lz += w == 0;
          }
        }
        agg += wsum_rt(rt, wpr, nbm | (nbm << 16));
      }
      pres = set_weight(trow, wpr, p.R & ~S);
      status = MAPA_RES_OK;
      if (eff) {
        const int E = lx + ly + lz;
        const int at = eff_off(E) + lx * (E + 1) + ly;
        o.key = eff_key[at];
        o.links = lx | (ly << 8) | (lz << 16);
        if ((uint32_t)eff_rank[at] != (uint32_t)(best >> 32)) atomicAdd(self_check_failures, 1u);
      } else {
        o.key = (int32_t)(best >> 32);
        if ((int32_t)p.a * agg + (int32_t)p.b * pres != o.key) atomicAdd(self_check_failures, 1u);
      }
    }
  }
  return o;
}

// 48-byte result as three 16-byte stores
__device__ __forceinline__ void store_result(mapa_result *res, const Outcome &o) {
  int4 *dst = reinterpret_cast<int4 *>(res);
  dst[0] = make_int4((int32_t)(uint32_t)o.count, (int32_t)(o.count >> 32), o.status, o.key);
  dst[1] = make_int4(o.agg, o.pres, (int32_t)o.S, (int32_t)o.map_lo);
  dst[2] = make_int4((int32_t)o.map_hi, o.links, (int32_t)(uint32_t)o.handle, (int32_t)(o.handle >> 32));
}

__global__ __launch_bounds__(256) void k_finalize(BatchArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nq) return;
  const Plan p = a.plan[i];
  Outcome o = decode_best(p, a.acc_count[i], a.acc_best[i], a.rows + (size_t)p.topo * kTopoWords * a.wpr,
                          a.wpr, a.eff_rank, a.eff_key, &a.ctr->self_check_failures);
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

// ------------------------------------------------------------ fused batch

// Small batches whose queries all name different servers, in one launch:
// bpq blocks per query each build the query's plan, take every bpq-th group
// of prefix items (enough items for every thread of the query's blocks),
// expand them and add their count and best to the query's accumulators; the
// last block of a query to finish decodes the result, commits directly (no
// other query of the batch can claim the server) and clears the
// accumulators.  Queries and results may live in pinned host memory.
template <int WPR>
__global__ __launch_bounds__(256) void k_fused(FusedArgs f) {
  __shared__ Plan s_plan;
  __shared__ uint32_t s_rows[kTopoWords * WPR];
  __shared__ unsigned long long s_cnt[4], s_best[4];
  __shared__ bool s_last;
  const int i = blockIdx.x / f.bpq;
  const int j = blockIdx.x % f.bpq;
  const int tid = threadIdx.x;
  const uint32_t span = (uint32_t)f.bpq * blockDim.x;
  if (tid == 0) {
    const mapa_query q = f.q[i];
    Plan p = make_plan(q, f.nservers, f.server_topo, f.topo_n, f.topo_maxw, f.busy, f.rows, WPR);
    if (p.status == kPlanOk) {
      int d = 0;
      while (d < p.k - 1 && c_tab.perm[p.F][d] < (unsigned long long)span) ++d;
      p.d = (uint8_t)d;
      p.nitems = (uint32_t)c_tab.perm[p.F][d];
    }
    s_plan = p;
  }
  __syncthreads();
  const int status = s_plan.status;
  const uint32_t nitems = status == kPlanOk ? s_plan.nitems : 0u;
  if (status != kPlanInvalid && tid < kTopoWords * WPR)
    s_rows[tid] = f.rows[(size_t)s_plan.topo * kTopoWords * WPR + tid];
  __syncthreads();
  unsigned long long cnt = 0, best = 0;
  for (uint32_t base = (uint32_t)j * blockDim.x; base < nitems; base += span) {
    const uint32_t x = base + (uint32_t)tid;
    unsigned long long c1, b1;
    item_search<WPR, 0>(x < nitems ? &s_plan : nullptr, s_rows, x, f.eff_rank, c1, b1);
    cnt += c1;
    best = b1 > best ? b1 : best;
  }
  cnt = wave_sum_u64(cnt);
  best = wave_max_u64(best);
  if ((tid & 63) == 0) {
    s_cnt[tid >> 6] = cnt;
    s_best[tid >> 6] = best;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      cnt += s_cnt[w];
      best = s_best[w] > best ? s_best[w] : best;
    }
    bool last = true;
    if (f.bpq > 1) {
      if (cnt) atomicAdd(&f.acc_count[i], cnt);
      if (best) atomicMax(&f.acc_best[i], best);
      __threadfence();
      last = atomicAdd(&f.done[i], 1u) == (uint32_t)f.bpq - 1;
      if (last) {
        __threadfence();
        cnt = __hip_atomic_load(&f.acc_count[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        best = __hip_atomic_load(&f.acc_best[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        f.acc_count[i] = 0;
        f.acc_best[i] = 0;
        f.done[i] = 0;
      }
    }
    s_last = last;
  }
  __syncthreads();
  if (tid == 0 && s_last) {
    const Plan p = s_plan;
    Outcome o = decode_best(p, cnt, best, s_rows, WPR, f.eff_rank, f.eff_key, f.self_check_failures);
    if (p.status != kPlanInvalid && p.commit && o.status == MAPA_RES_OK) {
      atomicOr(&f.busy[p.server], o.S);
      o.handle = ((int64_t)p.server << 32) | (int64_t)o.S;
    }
    store_result(f.res + i, o);
  }
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
  busy[s] = masks[i] & ((1u << n) - 1u);
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

static inline unsigned blocks_for(long long n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

hipError_t launch_batch_front(const BatchArgs &a, hipStream_t s) {
  const unsigned g = blocks_for(a.nq, 256);
  hipLaunchKernelGGL(k_prepare, dim3(g), dim3(256), 0, s, a);
  // 1024-thread blocks, up to 16 queries per thread, at most 64 blocks
  unsigned gb = blocks_for(a.nq, 1024 * 16);
  if (gb < 64) gb = std::min<unsigned>(64, blocks_for(a.nq, 1024));
  if (gb < 1) gb = 1;
  hipLaunchKernelGGL(k_bucketize, dim3(gb), dim3(kFatBlock), 0, s, a);
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(kFatBlock), 0, s, a);
  // one-wave blocks of at most 64 queries, and at least ~2048 blocks
  int qpb = 64;
  if (blocks_for(a.nq, qpb) < 2048) qpb = (int)((a.nq + 2047) / 2048);
  if (qpb < 1) qpb = 1;
  hipLaunchKernelGGL(k_expand, dim3(blocks_for(a.nq, qpb)), dim3(64), 0, s, a, qpb);
  return hipGetLastError();
}

template <int WPR, bool LDS, int PAIR>
static hipError_t launch_enum_t(const BatchArgs &a, hipStream_t s) {
  const size_t lds = LDS ? (size_t)a.ntopo * kTopoWords * WPR * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL((k_enumerate<WPR, LDS, PAIR>), dim3(a.enum_blocks), dim3(a.enum_threads), lds, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_enumerate(const BatchArgs &a, hipStream_t s) {
  const bool lds = a.rows_in_lds != 0;
  switch (a.wpr) {
    case 1:
      if (a.pair >= 12) return lds ? launch_enum_t<1, true, 12>(a, s) : launch_enum_t<1, false, 12>(a, s);
      if (a.pair >= 8) return lds ? launch_enum_t<1, true, 8>(a, s) : launch_enum_t<1, false, 8>(a, s);
      return lds ? launch_enum_t<1, true, 0>(a, s) : launch_enum_t<1, false, 0>(a, s);
    case 2: return lds ? launch_enum_t<2, true, 0>(a, s) : launch_enum_t<2, false, 0>(a, s);
    default: return lds ? launch_enum_t<4, true, 0>(a, s) : launch_enum_t<4, false, 0>(a, s);
  }
}

template <int WPR, bool LDS, int PAIR>
static int occ_t(int threads, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_enumerate<WPR, LDS, PAIR>, threads, lds) !=
      hipSuccess)
    return 0;
  return nb;
}

int enumerate_occupancy(int wpr, int rows_in_lds, int pair, int threads, size_t lds_bytes) {
  const bool l = rows_in_lds != 0;
  switch (wpr) {
    case 1:
      if (pair >= 12) return l ? occ_t<1, true, 12>(threads, lds_bytes) : occ_t<1, false, 12>(threads, 0);
      if (pair >= 8) return l ? occ_t<1, true, 8>(threads, lds_bytes) : occ_t<1, false, 8>(threads, 0);
      return l ? occ_t<1, true, 0>(threads, lds_bytes) : occ_t<1, false, 0>(threads, 0);
    case 2: return l ? occ_t<2, true, 0>(threads, lds_bytes) : occ_t<2, false, 0>(threads, 0);
    default: return l ? occ_t<4, true, 0>(threads, lds_bytes) : occ_t<4, false, 0>(threads, 0);
  }
}

hipError_t launch_fused(const FusedArgs &f, hipStream_t s) {
  if (f.nq <= 0) return hipSuccess;
  if (f.bpq < 1 || f.bpq > kFusedMaxBlocksPerQuery) return hipErrorInvalidValue;
  switch (f.wpr) {
    case 1: hipLaunchKernelGGL(k_fused<1>, dim3(f.nq * f.bpq), dim3(kFusedThreads), 0, s, f); break;
    case 2: hipLaunchKernelGGL(k_fused<2>, dim3(f.nq * f.bpq), dim3(kFusedThreads), 0, s, f); break;
    default: hipLaunchKernelGGL(k_fused<4>, dim3(f.nq * f.bpq), dim3(kFusedThreads), 0, s, f); break;
  }
  return hipGetLastError();
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
