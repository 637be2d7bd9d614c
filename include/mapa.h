/*
 * mapa.h -- C ABI of the MI355X-native MAPA allocation hot path.
 *
 * MAPA (Multi-Accelerator Pattern Allocation, SC'21) places a job's
 * communication pattern on the free accelerators of a multi-GPU server:
 *   - the server is a weighted hardware graph G whose vertices are
 *     accelerators and whose edge label is the highest link bandwidth
 *     between two of them (Sec. 3.2);
 *   - the job is a small pattern graph P: a ring, an all-to-all or a binary
 *     tree on k accelerators (Sec. 3.1);
 *   - a match is a one-to-one map of V(P) into the free vertices of G
 *     (Sec. 3.3, subgraph isomorphism);
 *   - every match is scored with AggBW (Eq. 1) and PreservedBW (Eq. 3), and the
 *     best one is selected (Alg. 1; the Greedy policy of Sec. 4 uses AggBW);
 *   - allocation and release remove and add back vertices of G (Sec. 3.6).
 *
 * This library enumerates every match on the GPU, scores every match with
 * exact integer arithmetic, and returns the match count, the best key and the
 * chosen vertex set with a fixed tie-break.  All compute runs in hand-written
 * HIP kernels for gfx950; there is no CPU fallback: without a GPU every
 * compute entry point returns MAPA_ERR_NO_DEVICE after validating its
 * arguments.
 *
 * Conventions
 *   - Every function returns int32_t status: MAPA_OK (0) or a negative
 *     MAPA_ERR_* code.  Nothing aborts.  mapa_last_error() gives a
 *     human-readable message for the last error raised on the calling thread.
 *   - On error, no device state changes and no output is written, except
 *     where a function states otherwise.
 *   - A context is used by one host thread at a time.  Calls on one context
 *     are executed on the device in the order they are issued, whatever
 *     streams they name.
 *   - "Host pointer": ordinary CPU memory.  "Device pointer": memory from
 *     hipMalloc (for example a torch tensor on a ROCm device), on the
 *     context's device.
 */
#ifndef MAPA_H
#define MAPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- limits -------------------------------------------------------------- */
#define MAPA_MAX_N 16     /* accelerators per server, mapa_query_batch          */
#define MAPA_MAX_K 8      /* accelerators per job (pattern vertices), same      */
#define MAPA_MAX_N_WIDE 32 /* accelerators per server, mapa_create_topology and
                              mapa_query_batch_wide                           */
#define MAPA_MAX_K_WIDE 12 /* pattern vertices, mapa_query_batch_wide          */
#define MAPA_MAX_AB 1024  /* largest key weight a, b                             */

/* ---- status codes -------------------------------------------------------- */
#define MAPA_OK 0
#define MAPA_ERR_INVALID_ARG (-1)    /* malformed argument (see each function)  */
#define MAPA_ERR_UNSUPPORTED (-2)    /* a size beyond the call's limits        */
#define MAPA_ERR_OOM (-3)            /* device or host allocation failed       */
#define MAPA_ERR_DEVICE (-4)         /* a HIP call failed                      */
#define MAPA_ERR_NOT_BUSY (-5)       /* release of a vertex that is not busy   */
#define MAPA_ERR_UNKNOWN_SERVER (-6) /* server id not created                  */
#define MAPA_ERR_ADMISSION (-7)      /* batch does not fit the enumeration buffer */
#define MAPA_ERR_NO_DEVICE (-8)      /* context was created without a device   */
#define MAPA_ERR_STATE (-9)          /* call not allowed in the current state  */

/* ---- pattern kinds (Sec. 3.1) ----------------------------------------------
 * Pattern vertex i is position i of the mapping tuple.
 *   MAPA_RING:       k=1 no edge; k=2 the edge (0,1); k>=3 edges (i, i+1 mod k)
 *   MAPA_ALL_TO_ALL: every pair i<j
 *   MAPA_TREE:       binary heap, vertex i>0 joined to (i-1)/2
 *   MAPA_PATTERN_BASE + id: the application graph registered by
 *                    mapa_create_pattern under that id (0 <= id <
 *                    MAPA_MAX_PATTERNS); kinds 3 .. MAPA_PATTERN_BASE - 1 are
 *                    invalid                                                  */
#define MAPA_RING 0
#define MAPA_ALL_TO_ALL 1
#define MAPA_TREE 2
#define MAPA_PATTERN_BASE 16
#define MAPA_MAX_PATTERNS 240

/* ---- match modes (Sec. 3.2 / 3.3) -------------------------------------------
 * MAPA_ALL_INJECTIVE: the hardware graph is taken as fully connected (every
 *   pair of accelerators can talk through the host), so every injective map
 *   of the pattern into the free vertices is a match.  A pair with weight 0
 *   contributes 0 bandwidth.
 * MAPA_LINKED: a match must map every pattern edge onto a pair with weight > 0
 *   (subgraph isomorphism over the direct links; induced-ness not required). */
#define MAPA_ALL_INJECTIVE 0
#define MAPA_LINKED 1

/* ---- per-query result status ------------------------------------------------ */
#define MAPA_RES_OK 0        /* at least one match; best fields are valid         */
#define MAPA_RES_NOFIT 1     /* no match (k > free vertices, or none linked)      */
#define MAPA_RES_CONFLICT 2  /* asked to commit, but an earlier query of the same
                                batch already owns this server's commit; result
                                fields are valid, nothing was committed           */
#define MAPA_RES_INVALID 3   /* malformed query (device-pointer batches only;
                                host-pointer batches are rejected up front)       */
#define MAPA_RES_REFUSED 4   /* beyond the wide kernels' embedding limit (a
                                device-pointer wide batch, or a served request):
                                nothing was evaluated or committed                */

/* ---- flags ------------------------------------------------------------------ */
#define MAPA_DEVICE_PTRS 1u  /* array arguments are device pointers; the call is
                                asynchronous on the given stream                 */
#define MAPA_PIPELINE 4u     /* host pointers: always run the multi-kernel batch
                                pipeline, never the fused small-batch launch     */
#define MAPA_USE_GRAPH 2u    /* with MAPA_DEVICE_PTRS: capture the batch's launch
                                sequence into a HIP graph on first use for this
                                (queries, results, nq, stream) and replay it on
                                later calls with the same arguments; the graph is
                                rebuilt after topologies, servers, tuning or
                                capacity change.  Results are identical.  Ignored
                                while kernel timing (mapa_profile) is on.        */

typedef struct mapa_ctx mapa_ctx; /* opaque; owns all device memory it uses */

/* One allocation query: place pattern (kind, k) on server `server`.
 * 16 bytes, no padding. */
typedef struct {
  int32_t server;   /* server id from mapa_create_topology                      */
  uint8_t kind;     /* MAPA_RING / MAPA_ALL_TO_ALL / MAPA_TREE, or
                       MAPA_PATTERN_BASE + id of a registered pattern            */
  uint8_t k;        /* pattern vertices, 1..8 (a registered pattern's own k)    */
  uint8_t mode;     /* MAPA_ALL_INJECTIVE or MAPA_LINKED                        */
  uint8_t commit;   /* 1: on MAPA_RES_OK mark the chosen vertices busy          */
  int16_t a;        /* key = a*AggBW + b*PreservedBW, 0 <= a, b <= 1024.        */
  int16_t b;        /*   (1,0): Greedy; (0,1): Alg. 1 insensitive branch;
                         (1,1): both terms                                      */
  int32_t metric;   /* MAPA_METRIC_WEIGHTED: the key above.  MAPA_METRIC_EFFBW:
                       the bandwidth-sensitive branch of Alg. 1, key = predicted
                       effective bandwidth (Eq. 2) of the mapped pattern edges'
                       link mix; a, b unused; the server's topology must have
                       weights 0, 1, 2 only (PCIe, single, double NVLink), else
                       MAPA_ERR_UNSUPPORTED (host batches) / MAPA_RES_INVALID  */
} mapa_query;

#define MAPA_METRIC_WEIGHTED 0
#define MAPA_METRIC_EFFBW 1

/* Result of one query.  48 bytes. */
typedef struct {
  int64_t count;        /* number of matches (every one was scored)              */
  int32_t status;       /* MAPA_RES_*                                            */
  int32_t key;          /* key of the chosen match; INT32_MIN if none            */
  int32_t agg;          /* AggBW of the chosen match (Eq. 1)                     */
  int32_t pres;         /* PreservedBW of the chosen match (Eq. 3)               */
  uint32_t vertex_mask; /* bit v set iff accelerator v is chosen; 0 if none     */
  uint8_t mapping[8];   /* mapping[i] = accelerator of pattern vertex i;
                           0xFF beyond k or if none                              */
  int32_t links;        /* MAPA_METRIC_EFFBW: x | y << 8 | z << 16, the numbers of
                           the chosen match's pattern edges on double NVLinks,
                           single NVLinks and PCIe (Eq. 2); else 0               */
  int64_t alloc_handle; /* (server << 32) | vertex_mask if committed, else -1    */
} mapa_result;

/* Selection rule (Alg. 1, strict improvement): the chosen match has the
 * largest key; among equal keys, the lexicographically smallest mapping tuple
 * (mapping[0], ..., mapping[k-1]) wins.  With MAPA_METRIC_EFFBW the key
 * compared is Eq. 2's value in double precision (coefficients of Table
 * "Values of Coefficients"), and `key` reports round(1000 * EffBW).  PreservedBW of a match M is the total
 * weight of pairs u<v of free vertices that M leaves unused (Eq. 3); busy
 * vertices never contribute.  AggBW is the total weight of the pattern edges
 * under the mapping (Eq. 1). */

/* Message for the last error raised on the calling thread ("" if none). */
const char *mapa_last_error(void);

/* Create a context on HIP device `device` (>= 0), or a validation-only
 * context with device = -1 (argument checks run; compute calls then return
 * MAPA_ERR_NO_DEVICE).  enum_buffer_bytes sizes the prefix work-list of one
 * in-flight batch (0 = default 256 MiB); a batch of nq queries needs at least
 * 8 * (nq + 137088) bytes of it, else MAPA_ERR_ADMISSION.  *out receives the
 * context. */
int32_t mapa_ctx_create(int32_t device, size_t enum_buffer_bytes, mapa_ctx **out);

/* Wait for outstanding work, free every device and host resource.  NULL-safe. */
int32_t mapa_ctx_destroy(mapa_ctx *ctx);

/* Register a hardware graph (Sec. 3.2) and create num_servers servers of it,
 * all free.
 *   n:  1..32 accelerators (n > 32: MAPA_ERR_UNSUPPORTED); servers of more
 *       than 16 are queried with mapa_query_batch_wide only
 *   W:  host pointer, n*n uint8 row-major, W[i][j] = link weight of the pair,
 *       symmetric, W[i][i] = 0, 0 = no direct link.  Copied; caller keeps it.
 *   num_servers: >= 0.
 * Outputs (host pointers, may be NULL): *topo_id = the topology index,
 * *first_server = id of the first new server; the new servers are
 * first_server .. first_server + num_servers - 1. */
int32_t mapa_create_topology(mapa_ctx *ctx, int32_t n, const uint8_t *W, int32_t num_servers,
                             int32_t *topo_id, int32_t *first_server);

/* Register an application graph that is not one of the canonical shapes
 * (Sec. 3.1: a union of them, or a graph derived from a program's
 * communication), for use as mapa_query.kind / mapa_request.kind.
 *   k:         1..8 pattern vertices (k > 8: MAPA_ERR_UNSUPPORTED), numbered
 *              0..k-1; vertex i is position i of the mapping tuple, so the
 *              tie-break is lexicographic in this numbering, and positions
 *              are placed in this order (for MAPA_LINKED a numbering in which
 *              every vertex after the first has an earlier neighbour prunes
 *              soonest).
 *   num_edges: 0 .. k(k-1)/2.
 *   edges:     host pointer, 2 * num_edges uint8 values, pairs (u, v) with
 *              u, v < k, u != v, each unordered pair at most once (else
 *              MAPA_ERR_INVALID_ARG).  Copied; caller keeps it.
 * *kind_out (host pointer, may be NULL) receives MAPA_PATTERN_BASE + id, ids
 * counting up from 0 per context; MAPA_ERR_STATE once MAPA_MAX_PATTERNS are
 * registered.  Registered patterns are immutable; the call may run while
 * batches or the serving loop are in flight (earlier ids are not touched). */
int32_t mapa_create_pattern(mapa_ctx *ctx, int32_t k, int32_t num_edges, const uint8_t *edges,
                            int32_t *kind_out);

/* Overwrite the busy masks of `count` servers (bit v set = accelerator v is
 * allocated; Sec. 3.6).  server_ids / busy_masks: host pointers (synchronous
 * call, fully validated: unknown server -> MAPA_ERR_UNKNOWN_SERVER, a bit >= n
 * -> MAPA_ERR_INVALID_ARG), or device pointers with MAPA_DEVICE_PTRS
 * (asynchronous on hip_stream; entries with an unknown server are skipped and
 * bits >= n are cleared). */
int32_t mapa_set_busy(mapa_ctx *ctx, int32_t count, const int32_t *server_ids,
                      const uint32_t *busy_masks, uint32_t flags, void *hip_stream);

/* Read the busy masks of `count` servers into busy_out (host pointers;
 * synchronous). */
int32_t mapa_get_busy(mapa_ctx *ctx, int32_t count, const int32_t *server_ids,
                      uint32_t *busy_out);

/* Run nq allocation queries (Sec. 3.3-3.5) as one batch.
 *   q:   nq queries; res: nq results (same index).
 *   Host pointers (flags = 0): the batch is validated first (bad field ->
 *     MAPA_ERR_INVALID_ARG, k > 8 or a server of more than 16 accelerators
 *     -> MAPA_ERR_UNSUPPORTED, unknown server -> MAPA_ERR_UNKNOWN_SERVER;
 *     nothing runs on error), then the call blocks
 *     until res is filled.  A small batch (at most 4096 queries, each on a
 *     different server, at most 2^20 embeddings per query and 2^24 in all,
 *     counted on the whole topology) runs as one fused launch that reads and
 *     writes pinned staging memory; MAPA_PIPELINE forces the pipeline.
 *     Results are identical either way.
 *   MAPA_DEVICE_PTRS: q and res are device pointers (16-byte aligned); the
 *     call returns once the work is queued on hip_stream (a hipStream_t,
 *     NULL = the default stream); malformed queries get status
 *     MAPA_RES_INVALID.
 * Semantics: every query is evaluated against the busy masks as they are when
 * the batch starts.  Then commits are applied: for each server, only the first
 * query of the batch (in array order) with commit = 1 may commit, and does so
 * if its status is MAPA_RES_OK; later committing queries of that server get
 * MAPA_RES_CONFLICT.  The caller owns q and res. */
int32_t mapa_query_batch(mapa_ctx *ctx, const mapa_query *q, int32_t nq, mapa_result *res,
                         uint32_t flags, void *hip_stream);

/* ---- allocation-free batch ---------------------------------------------------
 * For callers that cannot allocate device memory during a call: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same queries, results, semantics and kernels as
 * mapa_query_batch with MAPA_DEVICE_PTRS; the batch's workspace (per-query
 * plans and accumulators, counters, prefix work-list) is a fixed device
 * array of MAPA_NOALLOC_SCRATCH_MIB MiB that each device the library runs on
 * holds from context creation until the process ends, instead of memory the
 * context allocates.  The call allocates and frees nothing.
 *   q, res: device pointers (16-byte aligned), nq entries each; the call
 *     returns once the work is queued on hip_stream (NULL = default stream).
 *   nq > MAPA_NOALLOC_MAX_QUERIES -> MAPA_ERR_ADMISSION, nothing runs.
 *   Malformed queries get status MAPA_RES_INVALID, as with device pointers.
 *   A batch whose finest prefix split does not fit the array's work-list
 *   runs with a coarser split; results are identical, only speed differs.
 * Every call on one device shares that device's array: calls on one context
 * are ordered (as every call on a context), but calls from different
 * contexts on the same device that overlap in time race and give undefined
 * results.  Self-check failures of these calls are not added to
 * mapa_get_stats. */
#define MAPA_NOALLOC_MAX_QUERIES 65536
#define MAPA_NOALLOC_SCRATCH_MIB 32
int32_t mapa_query_batch_noalloc(mapa_ctx *ctx, const mapa_query *q, int32_t nq,
                                 mapa_result *res, void *hip_stream);

/* Result of one wide query: as mapa_result, with room for 16 mapping
 * entries.  56 bytes. */
typedef struct {
  int64_t count;
  int32_t status, key, agg, pres;
  uint32_t vertex_mask;
  uint8_t mapping[16];  /* mapping[i] = accelerator of pattern vertex i; 0xFF beyond k */
  int32_t links;        /* MAPA_METRIC_EFFBW: x | y << 8 | z << 16, as in
                           mapa_result; else 0                                  */
  int64_t alloc_handle; /* (server << 32) | vertex_mask if committed, else -1 */
} mapa_result_wide;

/* The same query semantics (Sec. 3.3-3.5, Alg. 1, reading of batches as in
 * mapa_query_batch) for the sizes beyond the batch path, the jobs of 9
 * accelerators and more on larger hardware graphs whose scheduling cost
 * Sec. 5.4 discusses: servers of up to 32 accelerators and patterns
 * of up to 12 vertices (ring, all-to-all and tree of any k <= 12, or a
 * registered pattern), key a*AggBW + b*PreservedBW or, with
 * MAPA_METRIC_EFFBW, the predicted effective bandwidth of Eq. 2 on the link
 * mix of the mapped pattern edges (up to 66 of them; topologies of weights
 * 0, 1, 2 only, as on the batch path).  Any server may be queried this way.
 *   nq: 0 .. MAPA_MAX_WIDE_QUERIES (more -> MAPA_ERR_ADMISSION, nothing runs).
 *   Host pointers (flags = 0): q, res hold nq entries each; the call is
 *     validated as mapa_query_batch's host form (k > 12 ->
 *     MAPA_ERR_UNSUPPORTED) and blocks until res is filled.  A batch of more
 *     than 2^36 embeddings in all (summed over its queries, on their free
 *     vertices at the batch's start) is refused with MAPA_ERR_ADMISSION
 *     before anything runs.
 *   MAPA_DEVICE_PTRS: q and res are device pointers (16-byte aligned); the
 *     call returns once the work is queued on hip_stream (NULL = the default
 *     stream).  Queries are validated and planned on the device: malformed
 *     ones get MAPA_RES_INVALID; a batch beyond the same 2^36 embeddings
 *     gets MAPA_RES_REFUSED in every well-formed query, and nothing of it
 *     is committed.
 * Every embedding is enumerated and scored, as on the batch path; the work
 * of each query is split over blocks by a prefix of its first positions. */
#define MAPA_MAX_WIDE_QUERIES 16384
int32_t mapa_query_batch_wide(mapa_ctx *ctx, const mapa_query *q, int32_t nq,
                              mapa_result_wide *res, uint32_t flags, void *hip_stream);

/* Release committed allocations (Sec. 3.6: add the vertices back).
 * Handles equal to -1 are ignored.
 *   Host pointers: synchronous and all-or-nothing: if any handle names an
 *     unknown server (MAPA_ERR_UNKNOWN_SERVER), a vertex that is not busy or
 *     two handles overlap (MAPA_ERR_NOT_BUSY), nothing is released.
 *   MAPA_DEVICE_PTRS: handles is a device array whose entries may be read at
 *     any int64 stride: entry i is at byte offset i * stride_bytes
 *     (stride_bytes = 8 for a plain array, 48 to release the alloc_handle
 *     fields of a mapa_result array in place).  Asynchronous on hip_stream;
 *     each handle is applied on its own: its vertices become free. */
int32_t mapa_release(mapa_ctx *ctx, int32_t count, const int64_t *handles, int32_t stride_bytes,
                     uint32_t flags, void *hip_stream);

/* ---- job-trace simulation (Sec. 5.2) ------------------------------------------
 * The paper's simulation framework, run on the library's allocation path.  A
 * job file lists jobs with their arrival cycle, execution time, pattern and
 * bandwidth sensitivity; a dispatcher puts arriving jobs into a first-in
 * first-out queue; whenever the head of the queue fits in the free
 * accelerators, the simulation's allocation policy places it and marks its
 * accelerators busy; once its execution time has elapsed the Job Finished
 * Signal frees them again.  The engine is cycle based.  Within one cycle:
 * finished jobs free their accelerators, then arrivals join the queue, then
 * the head is placed again and again while it fits (a blocked head blocks
 * the queue).  Every match is an injective map into the free accelerators
 * (MAPA_ALL_INJECTIVE); ties go to the lexicographically smallest mapping.
 * The log records, per job, its start and finish cycles, the accelerators it
 * got and, scored at its start cycle, AggBW (Eq. 1), PreservedBW (Eq. 3)
 * and its predicted effective bandwidth (Eq. 2). */
#define MAPA_POLICY_PRESERVE 0 /* Alg. 1: bandwidth-sensitive jobs take the match of
                                  largest predicted effective bandwidth (Eq. 2), the
                                  others the match of largest PreservedBW (Eq. 3)   */
#define MAPA_POLICY_GREEDY 1   /* the match of largest AggBW (Eq. 1)                   */
#define MAPA_POLICY_BASELINE 2 /* the lowest free accelerator ids, pattern vertex i on
                                  the i-th lowest (the comparison policy of Sec. 5.1) */

typedef struct {          /* 16 bytes */
  int32_t id;             /* caller's job id, echoed in the log                       */
  int32_t arrival;        /* cycle at which the dispatcher queues the job, >= 0,
                             non-decreasing within one simulation                     */
  int32_t duration;       /* execution cycles, >= 1                                   */
  uint8_t kind;           /* pattern, as mapa_query.kind                              */
  uint8_t k;              /* accelerators requested, 1..8                             */
  uint8_t sensitive;      /* 1: bandwidth-sensitive                                   */
  uint8_t reserved;       /* must be 0                                                */
} mapa_job;

typedef struct {          /* 48 bytes */
  int32_t id;
  int32_t status;         /* MAPA_RES_OK; MAPA_RES_NOFIT: the job needs more accelerators
                             than the server ever has free, it is logged when it arrives
                             and leaves the queue                                      */
  int32_t start, finish;  /* cycles (finish = start + duration); -1 if not placed     */
  uint32_t vertex_mask;   /* accelerators the job ran on                              */
  uint8_t mapping[8];     /* mapping[i] = accelerator of pattern vertex i; 0xFF beyond k */
  int32_t agg, pres;      /* AggBW and PreservedBW of the placement at its start      */
  int32_t effbw_milli;    /* round(1000 * predicted effective bandwidth)              */
  int32_t links;          /* x | y << 8 | z << 16: the placement's pattern edges on double
                             NVLinks, single NVLinks and PCIe                         */
  int32_t reserved;
} mapa_job_log;

typedef struct {
  int64_t cycles;         /* last cycle simulated                                     */
  int64_t event_cycles;   /* cycles with an arrival or a finish                       */
  int64_t rounds;         /* placement rounds (one scoring launch each)               */
  int64_t device_batches; /* allocation-query batches                                 */
  int64_t jobs_placed;
} mapa_sim_stats;

/* Run nsim independent simulations together.  Simulation i runs the jobs
 * jobs[job_offsets[i] .. job_offsets[i+1]) on server servers[i] under policy
 * policies[i] and writes their logs at the same indices of logs.
 *   servers: distinct servers of at most 16 accelerators whose topologies have
 *     link weights 0, 1, 2 only (PCIe, single, double NVLink; Eq. 2), else
 *     MAPA_ERR_UNSUPPORTED.  A server's accelerators that are busy when the
 *     call starts stay reserved throughout; every other one is free at cycle 0
 *     and free again when the call returns.
 *   All arrays are host pointers; job_offsets has nsim + 1 entries, starting
 *   at 0.  stats (may be NULL) receives counters of the run.  The call is
 *   synchronous and validates everything before it starts (bad field ->
 *   MAPA_ERR_INVALID_ARG, nothing runs). */
int32_t mapa_simulate(mapa_ctx *ctx, int32_t nsim, const int32_t *servers, const int32_t *policies,
                      const int32_t *job_offsets, const mapa_job *jobs, mapa_job_log *logs,
                      mapa_sim_stats *stats);

/* ---- tuning and measurement ---------------------------------------------- */

typedef struct {
  int32_t min_leaves_per_item;  /* smallest prefix-item size considered (64);
                                   sizes min_leaves_per_item * 2^j, j < 16,
                                   and whole queries are the candidates      */
  int32_t mean_item_leaves;     /* the batch takes the finest split whose
                                   items still average this many embeddings
                                   and give every resident GPU lane one
                                   (128); a batch too small to fill the lanes
                                   takes the finest split that fits          */
  int32_t blocks_per_cu;        /* persistent enumeration blocks per CU (0=auto) */
  int32_t threads_per_block;    /* 64..256, multiple of 64 (256)                 */
  int32_t pair_width;           /* widest number of free vertices whose last two
                                   positions are scored from per-candidate
                                   tables: 6 or 12; -1 none; 0 auto (12 when the
                                   context has a topology of 10 or more
                                   vertices, else 6)                          */
} mapa_tuning;

/* Read or replace the context's tuning knobs (NULL out/in allowed).  Results
 * never depend on tuning; only speed does. */
int32_t mapa_get_tuning(mapa_ctx *ctx, mapa_tuning *out);
int32_t mapa_set_tuning(mapa_ctx *ctx, const mapa_tuning *in);

typedef struct {
  mapa_tuning tuning;
  double ms;              /* mean time of one batch with this tuning (HIP events) */
} mapa_tune_trial;

/* Autotuner: time candidate tunings on a representative batch and keep the
 * fastest.  q: nq host queries, validated as by mapa_query_batch; they run
 * without commits, so no server state changes.  Starting from the current
 * tuning, the knobs are searched one at a time (coordinate descent, at most
 * two passes): min_leaves_per_item in {16, 64, 256, 1024, 4096},
 * mean_item_leaves in {32, 128, 512, 2048, 8192}, threads_per_block in
 * {64, 128, 192, 256}, blocks_per_cu in {0, 1, 2, 4, 8} and, for contexts
 * whose weights fit 2 bits, pair_width in {0, -1, 6, 12}; a candidate runs
 * one warm-up batch and `reps` (1..100) timed ones, and its results must
 * equal the first candidate's byte for byte (else MAPA_ERR_DEVICE and the
 * starting tuning is restored).  A change is kept only if it is at least 1 %
 * faster.  On success the context keeps the fastest tuning, *best (may be
 * NULL) receives it, trials[0 .. min(cap, *ntrials)) the candidates in the
 * order timed (trials may be NULL with cap = 0) and *ntrials (may be NULL)
 * their number.  Synchronous. */
int32_t mapa_autotune(mapa_ctx *ctx, const mapa_query *q, int32_t nq, int32_t reps,
                      mapa_tuning *best, mapa_tune_trial *trials, int32_t cap, int32_t *ntrials);

typedef struct {
  int64_t batches;         /* query batches run                                */
  int64_t enum_launches;   /* enumeration-kernel launches timed                */
  double enum_ms;          /* summed enumeration-kernel time (HIP events)      */
  int64_t last_items;      /* prefix items of the last batch (0 if unknown)    */
  int32_t last_split;      /* split size chosen by the last batch's first block */
  int64_t self_check_failures; /* results whose key disagreed with the AggBW and
                                  PreservedBW recomputed from the chosen mapping
                                  (always 0 unless something is broken)        */
  int32_t cu_count;        /* compute units of the device                      */
  int32_t num_servers;
  int32_t num_topologies;
} mapa_stats;

/* Enable (1) or disable (0) HIP-event timing of the enumeration kernel on the
 * stream it is launched on.  mapa_get_stats synchronises the context and
 * fills *out; mapa_reset_stats zeroes the counters. */
int32_t mapa_profile(mapa_ctx *ctx, int32_t enable);
int32_t mapa_get_stats(mapa_ctx *ctx, mapa_stats *out);
int32_t mapa_reset_stats(mapa_ctx *ctx);

/* Block until all work issued on the context has finished. */
int32_t mapa_sync(mapa_ctx *ctx);

/* Measure the device's integer vector-ALU throughput: a probe kernel of
 * independent integer chains (the enumeration kernel's instruction mix) runs
 * on every compute unit.  *ops_per_s receives 32-bit lane operations per
 * second (host pointer).  Synchronous; changes no context state. */
int32_t mapa_measure_alu_peak(mapa_ctx *ctx, double *ops_per_s);

/* ---- serving loop (continuous batching) -------------------------------------
 * A context can run one serving loop: a host thread owned by the context that
 * takes allocation requests as they arrive, answers each one against the
 * device-resident busy masks of its server (Sec. 3.3-3.5), marks granted
 * accelerators busy, holds them for the requested time and then adds them
 * back (Sec. 3.6).  While the loop runs it owns the context: every other call
 * except mapa_serve_* and mapa_last_error returns MAPA_ERR_STATE.
 *
 * Scheduling.  Requests of one server are answered one at a time in arrival
 * order (first in, first out per server), each against the busy mask left by
 * every earlier request and release of that server.  Requests of different
 * servers are batched together.  Up to `inflight` device batches run at once,
 * each on its own stream and workspace, so requests that arrive while a batch
 * is on the GPU join the next one as soon as a slot frees up.  A request joins
 * a batch only while the batch's prefix work-list estimate fits the admission
 * budget; otherwise it waits for the next batch (at the head of the line).  A
 * request asking for more accelerators than its server has free is answered
 * MAPA_RES_NOFIT on the host at once.  Requests the batch path does not take
 * (a server of more than 16 accelerators, or k > 8) run in the same dispatch
 * as a second device batch on the kernels of mapa_query_batch_wide, up to 256
 * of them and 2^34 embeddings per dispatch (a single larger one runs alone);
 * one of more than 2^36 embeddings on its free accelerators is answered
 * MAPA_RES_REFUSED on the host.  Every completion reports the busy mask it
 * was evaluated against, so each answer can be reproduced alone. */

typedef struct {
  int32_t max_batch;       /* queries per device batch, 1..65536 (0: 4096)            */
  int32_t inflight;        /* device batches in flight, 1 or 2 (0: 2)                  */
  double time_unit_us;     /* wall-clock microseconds per trace time unit; trace time 0
                              is when the run's first mapa_serve_submit returns.  0:
                              every request is due when it is submitted               */
  int64_t admission_items; /* prefix-item budget of one batch (0: the work-list buffer) */
  int32_t item_leaves;     /* embeddings per prefix item assumed by admission (0: 4096) */
  int32_t reserved;        /* must be 0                                                 */
} mapa_serve_opts;

typedef struct {           /* 40 bytes */
  int64_t id;              /* caller's request id, echoed in the completion            */
  double t_arrival;        /* arrival time in trace units, non-decreasing              */
  double hold;             /* a granted allocation is released `hold` trace units after
                              it is granted; < 0: held until mapa_serve_stop          */
  int32_t server;
  uint8_t kind, k, mode;   /* as in mapa_query                                         */
  uint8_t metric;          /* as in mapa_query                                         */
  int16_t a, b;            /* key weights, as in mapa_query                            */
  int32_t reserved1;       /* must be 0                                                */
} mapa_request;

typedef struct {           /* 88 bytes */
  int64_t id;
  int64_t count;           /* matches scored                                           */
  int64_t alloc_handle;    /* (server << 32) | vertex_mask if granted, else -1         */
  double latency_us;       /* completion time minus scheduled arrival time             */
  double wait_us;          /* queue wait: dispatch of its batch (or its host answer)
                              minus scheduled arrival; latency_us - wait_us is the
                              batch's turnaround                                       */
  int32_t status;          /* MAPA_RES_OK, MAPA_RES_NOFIT or MAPA_RES_REFUSED          */
  int32_t key, agg, pres;
  uint32_t vertex_mask;
  uint32_t busy_before;    /* the server's busy mask this request was answered against */
  int32_t batch;           /* device batch index; -1 if answered on the host           */
  int32_t server;
  uint8_t mapping[16];     /* accelerator of each pattern vertex; 0xFF beyond k       */
} mapa_completion;

typedef struct {
  int64_t requests, completed, granted, nofit;
  int64_t host_nofit;      /* answered on the host without a device batch              */
  int64_t batches, releases, embeddings, admission_waits;
  double wall_s;           /* from the first submission to the last completion         */
  double requests_per_s, embeddings_per_s;
  double p50_us, p99_us, p999_us, max_us;  /* request latency percentiles            */
  double mean_batch;       /* mean queries per device batch                            */
  double mean_batch_us;    /* mean time from a batch's dispatch to its results on the host */
  int64_t fused_batches;   /* batches run as one fused launch (small batches)    */
  double wait_p50_us, wait_p99_us;        /* queue wait percentiles                     */
  double turnaround_p50_us, turnaround_p99_us;  /* latency minus queue wait           */
  double mean_dispatch_us; /* host time to build and enqueue one device batch          */
  double mean_gpu_us;      /* device time of one batch's kernels (HIP events on one batch in 8) */
  double mean_harvest_us;  /* host time to turn one batch's results into completions   */
} mapa_serve_stats;

/* Start the loop.  opts may be NULL (defaults).  MAPA_ERR_STATE if a loop is
 * already running; MAPA_ERR_NO_DEVICE without a device. */
int32_t mapa_serve_start(mapa_ctx *ctx, const mapa_serve_opts *opts);

/* Queue n requests (host array, copied).  All-or-nothing validation: unknown
 * server -> MAPA_ERR_UNKNOWN_SERVER, malformed field or an arrival earlier
 * than the previous one -> MAPA_ERR_INVALID_ARG, k > 12 -> MAPA_ERR_UNSUPPORTED. */
int32_t mapa_serve_submit(mapa_ctx *ctx, const mapa_request *reqs, int32_t n);

/* Move up to cap finished requests into out (host array); *n_out = how many. */
int32_t mapa_serve_poll(mapa_ctx *ctx, mapa_completion *out, int32_t cap, int32_t *n_out);

/* Answer every submitted request, release every allocation still held, stop
 * the loop and fill *out (may be NULL).  Completions not yet polled are
 * dropped.  The context is usable by the other calls again afterwards. */
int32_t mapa_serve_stop(mapa_ctx *ctx, mapa_serve_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* MAPA_H */
