// Device code shared by the kernel translation units of the MAPA library
// (kernels.hip: the batch pipeline around the search; enum_*.hip: the
// enumeration kernel's variants; fused.hip: the one-launch small-batch
// path).  Each unit includes it and gets its own copy of the constant
// tables, which the host uploads to every unit.
#pragma once

#include <algorithm>
#include <climits>

#include "mapa_internal.h"

namespace mapa {

static __constant__ Tables c_tab;

static inline unsigned blocks_for(long long n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
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

// The key's constant term of a plan, b*W(R) (0 for Eq. 2, whose running
// score is the link mix of the edges placed so far and starts empty).
__device__ __forceinline__ int32_t plan_kp0(const Plan &p, const uint32_t *rows, int wpr) {
  return p.metric == MAPA_METRIC_EFFBW
             ? 0
             : (int32_t)p.b * set_weight(rows + (size_t)p.topo * kTopoWords * wpr, wpr, p.R);
}

// Plan of one query against the busy mask now in memory: validation, free
// set R, the pattern's back-neighbour table and, with with_kp0, the key's
// constant term b*W(R) (else 0, to be set with plan_kp0 before the search).
__device__ __forceinline__ Plan make_plan(const mapa_query &q, int32_t nservers,
                                          const int32_t *server_topo, const int32_t *topo_n,
                                          const uint8_t *topo_maxw, const uint32_t *busy,
                                          const uint32_t *rows, int wpr,
                                          const unsigned long long *pat_nbtab,
                                          const uint8_t *pat_k,
                                          const unsigned long long *pat_nbtab_ord,
                                          const uint32_t *pat_order, bool with_kp0 = true) {
  Plan p = {};
  p.server = q.server;
  const bool registered = q.kind >= MAPA_PATTERN_BASE;
  p.kind = registered ? (uint8_t)kKindPattern : q.kind;
  p.k = q.k;
  p.mode = q.mode;
  p.a = q.a;
  p.b = q.b;
  p.commit = q.commit;
  // a registered pattern's slot holds its k (0 while the slot is free)
  const bool kind_ok = q.kind <= MAPA_TREE || (registered && pat_k[q.kind - MAPA_PATTERN_BASE] == q.k);
  const bool ok = q.server >= 0 && q.server < nservers && kind_ok && q.k >= 1 &&
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
  if (n > kMaxN) {  // servers of more than 16 accelerators take the wide path
    p.status = kPlanInvalid;
    return p;
  }
  const uint32_t R = ~busy[q.server] & ((1u << n) - 1u);
  const int F = __popc(R);
  p.topo = (uint16_t)t;
  p.n = (uint8_t)n;
  p.R = R;
  p.F = (uint8_t)F;
  if (with_kp0) p.kp0 = plan_kp0(p, rows, wpr);
  p.nbtab = registered ? pat_nbtab[q.kind - MAPA_PATTERN_BASE] : c_tab.nbtab[q.kind][q.k];
  if (registered) {
    // LINKED search of a registered pattern places its vertices in the
    // pattern's matching order (weighted key; the tie-break stays
    // lexicographic in the pattern's own numbering)
    const int id = q.kind - MAPA_PATTERN_BASE;
    p.pat = (uint8_t)id;
    const uint32_t digits = q.k >= 8 ? 0xFFFFFFFFu : ((1u << (4 * q.k)) - 1u);
    if (q.mode == MAPA_LINKED && q.metric == MAPA_METRIC_WEIGHTED &&
        ((pat_order[id] ^ kIdentityOrder) & digits) != 0) {
      p.ord = 1;
      p.nbtab = pat_nbtab_ord[id];
    }
  }
  p.status = q.k > F ? kPlanNofit : kPlanOk;
  return p;
}

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
  // Eq. 2 (bandwidth-sensitive queries): rank table and this pattern's block.
  // LINKED search of a registered pattern in its matching order (weighted key
  // only) reuses these words: e1 = 0 marks it and eoff holds the order word
  // (digit p = pattern vertex at position p); the lane's best is then the
  // u64 (bpk, bcode) = (key, inverted lexicographic code in the pattern's
  // numbering), so equal keys are decided by that code.
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
//   (heap numbering); all-to-all -> every chosen vertex; a registered pattern
//   -> the vertices at the positions its back-neighbour table names.
//   Candidates: every free vertex not chosen yet.
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
    } else if (kd == MAPA_TREE) {
      nbm = p > 0 ? (1u << ((code >> (4 * ((p - 1) >> 1))) & 15u)) : 0u;
    } else {  // registered pattern: its back-neighbour table
      nbm = 0;
      for (uint32_t m = (uint32_t)(s.nbtab >> (8 * p)) & 0xFFu; m; m &= m - 1)
        nbm |= 1u << ((code >> (4 * __builtin_ctz(m))) & 15u);
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
// N values P_j = 16a*X_j - 16b*D_j - c_j (and, for long rows, the row terms
// Q_i = a*Y_i - b*D_i) are computed once; a leaf is then one packed-weight
// field, one multiply-add and a max.  The inner loop is
// unrolled over N, so the per-candidate values stay in registers.  Leaves
// come in lexicographic order (c_i, then c_j, ascending) as in level().
// Rows of one word (weights up to 3): the packed weight of u is 2 bits at 2u.
#ifndef MAPA_PAIR_MAX_FIRST
#define MAPA_PAIR_MAX_FIRST 9
#endif
constexpr int kPairMaxFirst = MAPA_PAIR_MAX_FIRST;  // N from which rows take the max first

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
  } else if constexpr (KIND == MAPA_TREE) {
    const int parent = (s.k - 2) >> 1;  // heap parent of position k-1
    alpha = parent == p;
    if (!alpha) fixm = 1u << ((code >> (4 * parent)) & 15u);
  } else {  // registered pattern: back-neighbours of position k-1 from its table
    const uint32_t nbl = (uint32_t)(s.nbtab >> (8 * (s.k - 1))) & 0xFFu;
    alpha = (nbl >> p) & 1u;
    for (uint32_t m = nbl & ~(1u << p); m; m &= m - 1)
      fixm |= 1u << ((code >> (4 * __builtin_ctz(m))) & 15u);
  }
  const uint32_t nb2 = nbm | (nbm << 16), rest2 = rest | (rest << 16), fix2 = fixm | (fixm << 16);
  const uint32_t *prow = s.trow + 16;  // packed-weight rows
  // Long rows (N >= kPairMaxFirst) also take the row term a*Y_i - b*D_i from
  // the per-candidate pass (Q_i) and unroll over i, so Q stays in registers.
  constexpr bool kLong = N >= kPairMaxFirst;
  // ring and tree: the neighbours of position p and the fixed neighbours of
  // position k-1 are at most one vertex each, whose packed-weight row gives
  // the weight to every candidate as one field
  constexpr bool kSingle = KIND == MAPA_RING || KIND == MAPA_TREE;
  uint32_t pnb = 0, pfix = 0;
  if constexpr (kSingle) {
    pnb = nbm ? prow[__builtin_ctz(nbm)] : 0u;
    pfix = fixm ? prow[__builtin_ctz(fixm)] : 0u;
  }
  if constexpr (M == 1) {
    // Two free vertices c0 < c1, two leaves.  Both still-free weights are
    // w01 = W[c0][c1], so the leaf keys are kp + a*(Y_i + X_j) + (a*alpha -
    // b*PRES) * w01 and the pair placing c0 first wins unless strictly worse.
    const uint32_t c0 = (uint32_t)__builtin_ctz(rest);
    const uint32_t c1 = (uint32_t)__builtin_ctz(rest & (rest - 1u));
    const int w01 = (int)((prow[c0] >> (2 * c1)) & 3u);
    int X0, X1, Y0, Y1;
    if constexpr (kSingle) {
      X0 = (int)((pfix >> (2 * c0)) & 3u);
      X1 = (int)((pfix >> (2 * c1)) & 3u);
      Y0 = (int)((pnb >> (2 * c0)) & 3u);
      Y1 = (int)((pnb >> (2 * c1)) & 3u);
    } else {
      X0 = wsum<1>(s.trow + c0, fix2);
      X1 = wsum<1>(s.trow + c1, fix2);
      if constexpr (KIND == MAPA_ALL_TO_ALL) {
        Y0 = X0;
        Y1 = X1;
      } else {
        Y0 = wsum<1>(s.trow + c0, nb2);
        Y1 = wsum<1>(s.trow + c1, nb2);
      }
    }
    const int kA = __mul24(s.a, Y0 + X1), kB = __mul24(s.a, Y1 + X0);
    const bool first = kA >= kB;
    const int key = kp + (first ? kA : kB) + __mul24((alpha ? s.a : 0) - (PRES ? s.b : 0), w01);
    const uint32_t cf = first ? c0 : c1, cl = first ? c1 : c0;
    const uint32_t pb = ((uint32_t)(key + 1) << 4) | (15u - cl);
    const bool better = pb > (s.bpk | 15u);
    s.bpk = better ? pb : s.bpk;
    s.bcode = better ? (code | (cf << (4 * p))) : s.bcode;
    s.count += 2u;
    return;
  }
  uint32_t sh2[N];  // 2 * c_j: bit offset of c_j's packed weight
  int P[N];
  int Q[kLong ? N : 1];
  uint32_t r = rest;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const uint32_t c = (uint32_t)__builtin_ctz(r);
    r &= r - 1;
    sh2[j] = 2 * c;
    const uint32_t *row = s.trow + c;
    int X;
    if constexpr (kSingle)
      X = (int)((pfix >> (2 * c)) & 3u);
    else
      X = wsum<1>(row, fix2);
    const int D = PRES ? wsum<1>(row, rest2) : 0;
    P[j] = __mul24(16 * s.a, X) - (int)c;
    if constexpr (PRES) P[j] -= __mul24(16 * s.b, D);
    if constexpr (kLong) {
      int Y;
      if constexpr (kSingle)
        Y = (int)((pnb >> (2 * c)) & 3u);
      else if constexpr (KIND == MAPA_ALL_TO_ALL)
        Y = X;  // every chosen vertex neighbours both positions
      else
        Y = wsum<1>(row, nb2);
      Q[j] = __mul24(s.a, Y) - (PRES ? __mul24(s.b, D) : 0);
    }
  }
  const int gamma = (alpha ? 16 * s.a : 0) + (PRES ? 16 * s.b : 0);
  s.count += (uint32_t)(N * M);
  const int sh = 4 * p;
  uint32_t ri = rest;
  if constexpr (kLong) {
    // the leaf values are base_i + P[j] + gamma * w with base_i shared by the
    // row: take the max over j first and add base_i once (every leaf value is
    // > 0); with i unrolled the j == i exclusion costs nothing
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const uint32_t ci = (uint32_t)__builtin_ctz(ri);
      ri &= ri - 1;
      const uint32_t wp = prow[ci];
      int tb = INT_MIN;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (j == i) continue;  // c_j = c_i is no match (both loops take one order)
        const int w = (int)((wp >> sh2[j]) & 3u);
        const int t = P[j] + __mul24(gamma, w);
        tb = t > tb ? t : tb;
      }
      const uint32_t pb = (uint32_t)(16 * (kp + Q[i]) + 31 + tb);
      const bool better = pb > (s.bpk | 15u);
      s.bpk = better ? pb : s.bpk;
      s.bcode = better ? (code | (ci << sh)) : s.bcode;
    }
  } else {
    // short rows keep the exclusion test per leaf and the row term per row:
    // with few leaves per row this uses fewer registers (measured faster)
    for (int i = 0; i < N; ++i) {
      const uint32_t ci = (uint32_t)__builtin_ctz(ri);
      ri &= ri - 1;
      const uint32_t *row = s.trow + ci;
      int kp2 = kp + __mul24(s.a, wsum<1>(row, nb2));
      if constexpr (PRES) kp2 -= __mul24(s.b, wsum<1>(row, rest2));
      const uint32_t wp = prow[ci];
      const int base = 16 * kp2 + 31;
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
template <int L, int WPR, bool LINKED, int KIND, int PAIR, bool PRES = true, bool ORD = false>
__device__ __forceinline__ void level(LaneState &s, int kind, uint32_t rest, uint32_t code,
                                      int kp, int p, uint32_t prev, int mu, int Lrun) {
  if constexpr (L > 1) {
    if (Lrun < L) {
      level<L - 1, WPR, LINKED, KIND, PAIR, PRES, ORD>(s, kind, rest, code, kp, p, prev, mu, Lrun);
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
  if constexpr (L == 1 && LINKED && ORD) {
    {
      // code digit t is the vertex at position t; in the pattern's numbering
      // it is vertex ordw[t], lexicographic digit k - 1 - ordw[t]
      const uint32_t ordw = (uint32_t)s.eoff;
      uint32_t lexn = 0;
      for (int t = 0; t < p; ++t)
        lexn |= ((code >> (4 * t)) & 15u) << (4 * (s.k - 1 - (int)((ordw >> (4 * t)) & 15u)));
      const int shl = 4 * (s.k - 1 - (int)((ordw >> (4 * p)) & 15u));
      s.count += (uint32_t)m;
      unsigned long long b64 = ((unsigned long long)s.bpk << 32) | s.bcode;
      for (int t = 0; t < m; ++t) {
        const int c = __builtin_ctz(cand);
        cand &= cand - 1;
        const uint32_t *rc = s.trow + c * WPR;
        int key = kp + __mul24(s.a, wsum<WPR>(rc, nb2));
        if constexpr (PRES) key -= __mul24(s.b, wsum<WPR>(rc, rest2));
        const uint32_t lex = lexn | ((uint32_t)c << shl);
        const unsigned long long v = ((unsigned long long)(uint32_t)key << 32) | (0xFFFFFFFFu - lex);
        b64 = v > b64 ? v : b64;
      }
      s.bpk = (uint32_t)(b64 >> 32);
      s.bcode = (uint32_t)b64;
      return;
    }
  }
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
      level<L - 1, WPR, LINKED, KIND, PAIR, PRES, ORD>(s, kind, rest & ~(1u << c),
                                                 code | ((uint32_t)c << sh), kp2, p + 1, (uint32_t)c,
                                                 mu - 1, L - 1);
    }
  }
}

template <int WPR, bool LINKED, int KIND, int PAIR, bool PRES = true, bool ORD = false>
__device__ __forceinline__ void expand(LaneState &s, int kind, int L, uint32_t rest,
                                       uint32_t code, int kp, int d, uint32_t prev, int mu) {
  if (L > 0) level<kMaxK, WPR, LINKED, KIND, PAIR, PRES, ORD>(s, kind, rest, code, kp, d, prev, mu, L);
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
                                            const uint16_t *erank, const uint32_t *pat_order,
                                            unsigned long long &cnt_out,
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
    // LINKED weighted search of a registered pattern: matching order (the
    // identity when the pattern's numbering is kept) and the u64 best
    if (p.mode == MAPA_LINKED && p.kind == kKindPattern && p.metric == MAPA_METRIC_WEIGHTED) {
      s.e1 = 0;
      s.eoff = (int)(p.ord ? pat_order[p.pat] : kIdentityOrder);
    }
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
  } else if (__builtin_amdgcn_readfirstlane(s.linked)) {
    // registered patterns (bucket kind) in matching order, with the best
    // compared by (key, lexicographic code in the pattern's numbering)
    if (kind_w == kKindPattern)
      expand<WPR, true, -1, PAIR, true, true>(s, kind_w, L, rest, code, kp, d, prev, 0);
    else
      expand<WPR, true, -1, PAIR>(s, kind_w, L, rest, code, kp, d, prev, 0);
  }
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
    else if (kind_w == MAPA_TREE)
      expand<WPR, false, MAPA_TREE, PAIR, false>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
    else
      expand<WPR, false, kKindPattern, PAIR, false>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  } else if (kind_w == MAPA_RING)
    expand<WPR, false, MAPA_RING, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  else if (kind_w == MAPA_ALL_TO_ALL)
    expand<WPR, false, MAPA_ALL_TO_ALL, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  else if (kind_w == MAPA_TREE)
    expand<WPR, false, MAPA_TREE, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);
  else
    expand<WPR, false, kKindPattern, PAIR>(s, kind_w, L, rest, code, kp, d, prev, fp_w);

  int bkey = -1;
  uint32_t bcode = 0;
  if (s.bpk) {
    bkey = (int)(s.bpk >> 4) - 1;
    bcode = s.bcode | ((15u - (s.bpk & 15u)) << (4 * (s.k - 1)));
  }
  unsigned long long best = 0;
  if (s.e1 == 0) {
    best = ((unsigned long long)s.bpk << 32) | s.bcode;
  } else if (bkey >= 0) {
    uint32_t lex = 0;
    for (int i = 0; i < s.k; ++i) lex = (lex << 4) | ((bcode >> (4 * i)) & 15u);
    best = ((unsigned long long)(uint32_t)bkey << 32) | (0xFFFFFFFFu - lex);
  }
  cnt_out = s.count;
  best_out = best;
}

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
                                               const int32_t *eff_key, const uint32_t *pat_order,
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
      // a plan in matching order lists back-neighbours by search position:
      // the vertex at search position t is the mapping's entry ordw[t]
      if (p.ord) {
        const uint32_t ordw = pat_order[p.pat];
        uint32_t placed = 0;
        for (int t = 0; t < k; ++t)
          placed |= ((phi_code >> (4 * ((ordw >> (4 * t)) & 15u))) & 15u) << (4 * t);
        phi_code = placed;
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

}  // namespace mapa
