// Internal layout shared by the host core (host.cpp) and the kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mapa.h"

namespace mapa {

constexpr int kMaxN = MAPA_MAX_N;
constexpr int kMaxK = MAPA_MAX_K;

// Prefix-split candidates.  Split j < kSplitWhole aims at items of at most
// min_leaves * 2^j embeddings; split kSplitWhole keeps every query whole.
constexpr int kNumSplits = 17;
constexpr int kSplitWhole = kNumSplits - 1;

// Shape buckets: (metric, mode, pattern kind, L = positions left below the
// prefix, F' = free vertices left below the prefix).  Every item of one
// bucket runs the same scoring code and expands a subtree of the same pattern
// kind, and in ALL mode of the same shape, so the 64 lanes of a wave run in
// lock step.
constexpr int kFp = kMaxN + 1;                      // F' in 0..16
constexpr int kKinds = 4;        // ring, all-to-all, tree, registered pattern
constexpr int kKindPattern = 3;  // bucket and template kind of every registered pattern
constexpr int kNumBuckets = 2 * 2 * kKinds * kMaxK * kFp;  // 2176
constexpr int kChunk = 64;                          // items per wave-chunk (one per lane)
constexpr int kPadReserve = (kChunk - 1) * kNumBuckets;
constexpr uint32_t kInvalidItem = 0xFFFFFFFFu;

__host__ __device__ inline int bucket_id(int metric, int mode, int kind, int L, int Fp) {
  return (((metric * 2 + mode) * kKinds + kind) * kMaxK + (L - 1)) * kFp + Fp;
}

// Eq. 2 tables, one block per pattern edge count E = 0..28: entry
// eff_off(E) + x * (E + 1) + y holds, for the mix of x double NVLinks, y
// single NVLinks and z = E - x - y PCIe links, the dense rank of its
// predicted effective bandwidth among the mixes of E edges (0 = lowest) and
// round(1000 * EffBW).  eff_off(E) = 1^2 + ... + E^2.
constexpr int kMaxEdges = kMaxK * (kMaxK - 1) / 2;  // 28
__host__ __device__ constexpr int eff_off(int E) { return E * (E + 1) * (2 * E + 1) / 6; }
constexpr int kEffEntries = eff_off(kMaxEdges + 1);  // 8555

// Per-query plan, written by k_front (the key's constant term by k_expand).
struct Plan {
  uint32_t R;          // free vertex mask at batch start
  int32_t kp0;         // b * W(R): the key's constant term
  int32_t server;
  uint16_t topo;
  uint8_t n, k;
  uint8_t kind, mode, F, status;  // status: kPlanOk / kPlanNofit / kPlanInvalid
  int16_t a, b;
  uint8_t d;           // chosen prefix depth
  uint8_t commit;
  uint16_t bucket;
  uint32_t nitems;     // prefix items of the chosen split
  uint32_t item_off;   // offset of the first item inside its bucket
  uint8_t metric;      // MAPA_METRIC_*
  uint8_t pat;         // registered pattern id (kind kKindPattern)
  uint8_t ord;         // 1: positions are placed in the pattern's matching order
  uint8_t pad;
  uint64_t nbtab;      // byte p: pattern neighbours of position p that precede it
};
static_assert(sizeof(Plan) == 48, "Plan layout");

constexpr uint8_t kPlanOk = 0, kPlanNofit = 1, kPlanInvalid = 3;

// Matching order of a registered pattern for LINKED search: the pattern
// vertex placed at search position p is digit p (bits 4p..4p+3) of the order
// word.  The pattern's own numbering is the identity word.
constexpr uint32_t kIdentityOrder = 0x76543210u;

// Per-batch counters (device).  Zeroed at allocation; the block of
// k_front that lays the buckets out re-zeroes what the batch consumed so
// the next batch starts clean.
// Counters hit by atomics from many blocks each own a 128-byte line, so their
// atomics spread over L2 channels instead of queueing on one.
constexpr int kLine = 32;  // u32 per 128-byte line

// A topology's device block, per word of row format (wpr words per row):
// 16 bit-plane rows (vertex v: for each weight bit t, the mask of neighbours
// u with bit t of W[v][u] set; planes 2w and 2w+1 share word w, low and high
// half) followed by 16 packed-weight rows (vertex v: W[v][u] in field u, 2,
// 4 or 8 bits wide for wpr = 1, 2, 4).  kTopoWords * wpr u32 per topology.
constexpr int kTopoWords = 32;
// The chunk list is dealt round-robin into kQueues queues (chunk c goes to
// queue c % kQueues), each with its own claim counter, so the claims of the
// persistent waves spread over many addresses instead of serializing on one.
constexpr int kQueues = 32;
// bins of a (free vertices F, pattern size k) histogram, bin F * (kMaxK + 1) + k
constexpr int kFkBins = (kMaxN + 1) * (kMaxK + 1);
struct Counters {
  uint32_t bucket_items[kNumBuckets][kLine];              // [b][0] used
  uint32_t queue_ctr[kQueues][kLine];                     // next chunk of each queue
  uint32_t bucket_start[kNumBuckets];
  uint32_t bucket_count[kNumBuckets];  // items of each bucket (before padding)
  uint32_t bucketize_done;             // k_front blocks finished (the last one lays out)
  uint32_t total_chunks;
  uint32_t chosen_split;
  uint32_t self_check_failures;
  unsigned long long last_total_items;
};

struct Tables {          // uploaded once per device into __constant__ memory
  unsigned long long perm[kMaxN + 1][kMaxK + 1];  // F!/(F-d)!
  unsigned long long nbtab[3][kMaxK + 1];  // byte p: back-neighbour position mask of p
  uint8_t nb[3][kMaxK + 1][kMaxK];         // the same masks, one per entry
  uint16_t rank_bucket[kNumBuckets];       // bucket laid out at rank r (largest items first)
  uint32_t inv[kMaxN + 1];                 // ceil(2^32 / m), m >= 2: x / m = umulhi(x, inv[m])
                                           // for every x < 2^28
};

// Prefix depth of split j for a query with F free vertices and k pattern
// positions: the smallest d <= k-1 with (F-d)!/(F-k)! <= min_leaves * 2^j
// (j < kSplitWhole), and d = 0 for j = kSplitWhole.  Built on the host per
// context (it depends on the tuning), indexed [F][k][j].
constexpr int kSplitTable = (kMaxN + 1) * (kMaxK + 1) * kNumSplits;

// kernels.hip
hipError_t upload_tables(const Tables &t);

struct BatchArgs {
  const mapa_query *q;
  mapa_result *res;
  int32_t nq;
  Plan *plan;
  unsigned long long *acc_count;
  unsigned long long *acc_best;
  uint2 *items;
  unsigned long long cap_items;
  Counters *ctr;
  // context state
  const int32_t *server_topo;
  uint32_t *busy;
  unsigned long long *commit_slot;
  int32_t nservers;
  const int32_t *topo_n;
  const uint8_t *topo_W;  // [T][16][16]
  const uint32_t *rows;   // [T][kTopoWords][wpr], see kTopoWords
  const uint8_t *topo_maxw;  // [T] largest weight of each topology
  const uint16_t *eff_rank;  // [kEffEntries], see eff_off
  const int32_t *eff_key;    // [kEffEntries]
  int32_t ntopo;
  int32_t wpr;
  const uint8_t *split_d;  // [F][k][j], see kSplitTable
  const unsigned long long *pat_nbtab;  // [MAPA_MAX_PATTERNS] registered patterns
  const uint8_t *pat_k;                 // [MAPA_MAX_PATTERNS] their k (0: free slot)
  const unsigned long long *pat_nbtab_ord;  // [MAPA_MAX_PATTERNS] the same in matching order
  const uint32_t *pat_order;            // [MAPA_MAX_PATTERNS] matching order, see kIdentityOrder
  // tuning
  unsigned long long lanes;  // resident enumeration lanes
  uint32_t mean_leaves;      // smallest mean item size the split may take
  int32_t enum_blocks;
  int32_t enum_threads;
  int32_t rows_in_lds;
  int32_t pair;  // k_enumerate variant: widest pair_level (0: none)
};

// Whether a batch runs the twelve-wide k_enumerate instance (one-word rows,
// pair level up to 12 free vertices); the others take their first chunks by
// wave id, and the front end sets the chunk queues up for that.
__host__ __device__ inline bool enum_twelve_wide(const BatchArgs &a) {
  return a.wpr == 1 && a.pair >= 12;
}

// Fused path for small batches with one query per server (k_fused).
constexpr int kFusedThreads = 256;
constexpr int kFusedMaxBlocksPerQuery = 16;
constexpr int32_t kFusedMaxQueries = 4096;
constexpr unsigned long long kFusedMaxQueryLeaves = 1ull << 20;  // per query
constexpr unsigned long long kFusedMaxLeaves = 1ull << 24;       // per batch

struct FusedArgs {
  const mapa_query *q;  // device or pinned host memory
  mapa_result *res;     // device or pinned host memory
  int32_t nq;
  const int32_t *server_topo;
  uint32_t *busy;
  int32_t nservers;
  const int32_t *topo_n;
  const uint32_t *rows;
  int32_t wpr;
  const uint8_t *topo_maxw;
  const uint16_t *eff_rank;
  const int32_t *eff_key;
  const unsigned long long *pat_nbtab;
  const uint8_t *pat_k;
  const unsigned long long *pat_nbtab_ord;
  const uint32_t *pat_order;
  uint32_t *self_check_failures;
  unsigned long long *acc_count, *acc_best;  // per query, zero on entry and exit
  uint32_t *done;                            // per query, zero on entry and exit
  int32_t bpq;                               // blocks per query
};

hipError_t launch_fused(const FusedArgs &f, hipStream_t s);

// per translation unit: constant-table upload, enumeration launch and occupancy
hipError_t upload_tables_front(const Tables &t);
hipError_t upload_tables_fused(const Tables &t);
hipError_t upload_tables_enum_pair12_lds(const Tables &t);
hipError_t upload_tables_enum_pair12_glb(const Tables &t);
hipError_t upload_tables_enum_pair6(const Tables &t);
hipError_t upload_tables_enum_plain(const Tables &t);
hipError_t launch_enum_pair12_lds(const BatchArgs &a, hipStream_t s);
hipError_t launch_enum_pair12_glb(const BatchArgs &a, hipStream_t s);
hipError_t launch_enum_pair6(const BatchArgs &a, hipStream_t s);
hipError_t launch_enum_plain(const BatchArgs &a, hipStream_t s);
int occ_enum_pair12_lds(int threads, size_t lds_bytes);
int occ_enum_pair12_glb(int threads, size_t lds_bytes);
int occ_enum_pair6(int rows_in_lds, int threads, size_t lds_bytes);
int occ_enum_plain(int wpr, int rows_in_lds, int threads, size_t lds_bytes);
hipError_t launch_batch_front(const BatchArgs &a, hipStream_t s);   // prepare .. expand
hipError_t launch_enumerate(const BatchArgs &a, hipStream_t s);
hipError_t launch_finalize(const BatchArgs &a, hipStream_t s);
int enumerate_occupancy(int wpr, int rows_in_lds, int pair, int threads, size_t lds_bytes);

hipError_t launch_valu_probe(uint32_t *out, int blocks, int iters, hipStream_t s);
int valu_probe_ops_per_iter();

hipError_t launch_set_busy(const int32_t *ids, const uint32_t *masks, int32_t count,
                           int32_t nservers, const int32_t *server_topo, const int32_t *topo_n,
                           uint32_t *busy, hipStream_t s);
hipError_t launch_get_busy(const int32_t *ids, int32_t count, const uint32_t *busy,
                           uint32_t *out, hipStream_t s);
hipError_t launch_release_check(const int64_t *handles, int32_t stride, int32_t count,
                                const uint32_t *busy, uint32_t *flag, hipStream_t s);
hipError_t launch_release_apply(const int64_t *handles, int32_t stride, int32_t count,
                                int32_t nservers, uint32_t *busy, hipStream_t s);

}  // namespace mapa
