// Wide path (mapa_query_batch_wide): servers of up to 32 accelerators and
// patterns of up to 12 vertices.  Layout shared by the host side (wide.cpp)
// and the kernels (wide.hip); not part of the public ABI.
#pragma once

#include "mapa_internal.h"

namespace mapa {

constexpr int kWideN = MAPA_MAX_N_WIDE;
constexpr int kWideK = MAPA_MAX_K_WIDE;
constexpr int kWidePlanes = 9;  // rows per topology: weight bit-planes 0..7, then adjacency
constexpr int kWideThreads = 256;
// Open positions on a thread's LDS stack: the search keeps positions d .. top-1
// there, where the prefix depth d >= 1 whenever k >= 2 (the plan extends the
// prefix while it has fewer than kWideMinItems items, and one item never
// does) and top <= k - 2 <= 10, so position p sits at entry p - 1 < 9.
constexpr int kWideStack = kWideK - 3;
// Every query owns this many consecutive blocks of the search grid; a query
// that needs fewer leaves the rest idle (they write an empty partial).
constexpr int kWideMaxBlocksPerQuery = 128;
constexpr uint32_t kWideMinItems = 16384;             // prefix items a query is split into, at least
constexpr unsigned long long kWideMaxLeaves = 1ull << 36;  // embeddings per call
constexpr int kWideMaxQueries = MAPA_MAX_WIDE_QUERIES;
// Eq. 2 tables (layout of eff_off) are built up to this many pattern edges,
// a 12-vertex all-to-all; the batch path reads the first kEffEntries.
constexpr int kWideMaxEdges = kWideK * (kWideK - 1) / 2;  // 66
constexpr int kEffEntriesWide = eff_off(kWideMaxEdges + 1);
constexpr int kWideEffTab = (kWideMaxEdges + 1) * (kWideMaxEdges + 1);  // one edge count's block, at most

// Per-query plan, written by k_wide_plan from the query and the busy mask at
// the call's start.
struct WidePlan {
  uint32_t R;            // free vertex mask at the call's start
  int32_t kp0;           // b * W(R)
  int32_t server;
  uint16_t nb[kWideK];   // positions j < p that neighbour position p in the pattern
  uint8_t k, mode, d, B; // positions, match mode, prefix depth, weight bit-planes in use
  uint8_t F, status, commit, nb_all;  // nb_all: every earlier position neighbours each one
  int16_t a, b;
  uint16_t topo;
  uint8_t metric;        // MAPA_METRIC_WEIGHTED or MAPA_METRIC_EFFBW
  uint8_t E;             // pattern edges (Eq. 2 table block)
  uint32_t items;        // F!/(F-d)! prefixes
  uint32_t nblocks;      // blocks of the query's share that have items
};

struct WidePartial {     // one block's share of a query
  unsigned long long count;
  unsigned long long code;  // best mapping, position p in bits 5*(11-p) .. +4
  int32_t key;              // best key, -1: none
  int32_t pad;
};

struct WideArgs {
  const mapa_query *q;    // [nq] device or pinned memory
  int32_t nq;
  WidePlan *plan;         // [nq]
  WidePartial *part;      // [nq][kWideMaxBlocksPerQuery]
  const uint32_t *rows;   // [T][kWidePlanes][32]: bit u of row (t, v) = bit t of W[v][u]
  const int32_t *server_topo;
  const int32_t *topo_n;
  const uint8_t *topo_maxw;
  int32_t nservers;
  int32_t ntopo_wide;     // topologies whose rows are uploaded
  const unsigned long long *pat_nbtab;  // registered patterns
  const uint8_t *pat_k;
  const uint16_t *eff_rank;  // [kEffEntriesWide] Eq. 2 dense ranks, layout of eff_off
  const int32_t *eff_key;    // [kEffEntriesWide] round(1000 * EffBW)
  uint32_t *busy;
  unsigned long long *commit_slot;  // first committing query per server, all ones when free
  mapa_result_wide *res;  // [nq] device or pinned memory
  uint32_t *self_check_failures;
  unsigned long long *total;  // embeddings of the call (each query's share capped at 2^37)
};

// Host side (wide.cpp), for mapa_query_batch_wide and the serving loop:
// upload the rows of topologies added since the last upload (waits for the
// context's work first); the context's part of the arguments (rows,
// topologies, patterns, Eq. 2 tables, busy masks, commit claims); and the
// call's device scratch: embedding total | plans | partials of nq queries.
int32_t wide_upload(mapa_ctx *c);
void wide_ctx_args(const mapa_ctx *c, WideArgs &w);
size_t wide_scratch_bytes(int32_t nq);
void wide_scratch_args(void *base, int32_t nq, WideArgs &w);
unsigned long long wide_embeddings(int F, int k);  // F!/(F-k)!, 0 if k > F

hipError_t launch_wide_plan(const WideArgs &w, hipStream_t s);  // clears total, then plans
hipError_t launch_wide_search(const WideArgs &w, hipStream_t s);  // nq * kWideMaxBlocksPerQuery blocks
hipError_t launch_wide_finalize(const WideArgs &w, hipStream_t s);

}  // namespace mapa
