// Wide path: servers of up to 32 accelerators and patterns of up to 12
// vertices (the paper's jobs of 9 GPUs and more).  The same definitions as
// the batch path: every injective embedding (ALL mode) or every one whose
// pattern edges land on direct links (LINKED), AggBW (Eq. 1) and PreservedBW
// (Eq. 3) through the scoring identity
//   key = b*W(R) + sum_p [ a*w(phi_p, earlier neighbours) - b*w(phi_p, still free) ],
// the first maximum in lexicographic order (Alg. 1 with strict improvement).
//
// k_wide_plan: per query, on the device (so the call also takes device
// pointers): validation, the free set R from the busy mask at the call's
// start, b*W(R), the pattern's neighbour masks, the prefix depth and block
// share, the server's commit claim, and the call's embedding total.
// k_wide_search: every query owns kWideMaxBlocksPerQuery consecutive blocks
// of the grid, of which its plan's share search; its threads take the query's
// prefixes of depth d (F!/(F-d)! of them, in lexicographic order of their
// index) in a loop strided over the share and expand each depth-first, keeping a count
// and their best (key, mapping).  The search is iterative: each thread keeps
// the candidates left, the running key and the neighbour mask of every open
// position in an LDS stack, so nothing spills and no call frames are built.
// The last two positions are one step: in ALL mode every ordered pair of the
// N free vertices left is a match, and its key is a sum of per-candidate
// terms tabulated once per node plus one pair weight (see pair_table).
// Weighted sums are popcounts over 32-bit weight bit-planes staged in LDS.
// The lanes of a wave hold prefixes of one query, so in ALL mode they open
// the same number of candidates at every position and run in lock step.
// The block reduces to one partial.
// k_wide_finalize: per query, the partials of its blocks, the mapping, a
// recomputation of AggBW and PreservedBW from it (self-check) and the commit.
#include "wide.h"

namespace mapa {

// sum of W[v][u] over u in X, from the B weight bit-planes of row v
__device__ __forceinline__ int wsum_wide(const uint32_t *rows, int B, int v, uint32_t X) {
  int s = 0;
  for (int t = 0; t < B; ++t) s += __popc(rows[t * 32 + v] & X) << t;
  return s;
}

// Position of the r-th (from 0) set bit of m (m has more than r set bits).
__device__ __forceinline__ int select_bit32(uint32_t m, uint32_t r) {
  int pos = 0;
  for (int w = 16; w >= 1; w >>= 1) {
    const uint32_t c = __popc((m >> pos) & ((1u << w) - 1u));
    if (r >= c) {
      r -= c;
      pos += w;
    }
  }
  return pos;
}

__device__ __forceinline__ int vertex_at(unsigned long long code, int pos) {
  return (int)((code >> (5 * (kWideK - 1 - pos))) & 31ull);
}


// key of a leaf, packed so one unsigned max picks the largest key and, among
// equal keys, the smallest last vertex: ((key + 1) << 5) | (31 - c).  Keys
// stay below 2^27 (weights <= 255, n <= 32, a, b <= 1024: at most 465 pairs
// of one of the two sums), so the packed value fits 32 bits.
__device__ __forceinline__ uint32_t pack_leaf(int key, int c) {
  return ((uint32_t)(key + 1) << 5) | (31u - (uint32_t)c);
}

// sum of W[v][u] over u in X from B (1, 2, or any up to 8) bit-planes
template <int B>
__device__ __forceinline__ int wsum_b(const uint32_t *rows, int Bn, int v, uint32_t X) {
  if constexpr (B == 1) {
    return __popc(rows[v] & X);
  } else if constexpr (B == 2) {
    return __popc(rows[v] & X) + 2 * __popc(rows[32 + v] & X);
  } else {
    int s = 0;
    for (int t = 0; t < Bn; ++t) s += __popc(rows[t * 32 + v] & X) << t;
    return s;
  }
}

// W[u][v] from the bit-planes
template <int B>
__device__ __forceinline__ int wpair_b(const uint32_t *rows, int Bn, int u, int v) {
  if constexpr (B == 1) {
    return (int)((rows[u] >> v) & 1u);
  } else if constexpr (B == 2) {
    return (int)((rows[u] >> v) & 1u) + 2 * (int)((rows[32 + u] >> v) & 1u);
  } else {
    int s = 0;
    for (int t = 0; t < Bn; ++t) s += (int)((rows[t * 32 + u] >> v) & 1u) << t;
    return s;
  }
}

struct WideCtx {
  const uint32_t *rows;  // LDS: [kWidePlanes][32]
  const uint16_t *erank; // LDS: Eq. 2 dense ranks of the query's edge count, [x * e1 + y]
  const uint32_t *pw;    // LDS: [32][2] packed 2-bit weights (weights <= 3): W[v][u] at
                         // bit 2 * (u % 16) of word 2 * v + u / 16
  const uint16_t *nb;    // LDS: back-neighbour position masks of the pattern
  uint32_t R;
  int Bn, a, b, k, linked, nb_all, e1;
};

// The score a search carries, fixed per query by the template argument B:
// B = kEffB scores by Eq. 2 (the running value is the link mix of the
// pattern edges placed so far, x << 8 | y with x double and y single
// NVLinks, and a leaf's key is the mix's dense rank among the mixes of the
// query's edge count); any other B by a*AggBW + b*PreservedBW through the
// identity above, from B weight bit-planes (0: as many as the topology has).
constexpr int kEffB = -1;

// running value after placing c at a position whose earlier pattern
// neighbours sit on nbm, with `rest` free before c is placed
template <int B>
__device__ __forceinline__ int step_key(const WideCtx &s, int kp, int c, uint32_t nbm, uint32_t rest) {
  if constexpr (B == kEffB) {
    // weights 0, 1, 2 only: plane 1 marks the double NVLinks, plane 0 the single ones
    return kp + (__popc(s.rows[32 + c] & nbm) << 8) + __popc(s.rows[c] & nbm);
  } else {
    return kp + s.a * wsum_b<B>(s.rows, s.Bn, c, nbm) - s.b * wsum_b<B>(s.rows, s.Bn, c, rest);
  }
}

// key of a leaf whose running value is v
template <int B>
__device__ __forceinline__ int leaf_key(const WideCtx &s, int v) {
  if constexpr (B == kEffB)
    return (int)s.erank[(v >> 8) * s.e1 + (v & 255)];
  else
    return v;
}

// vertices at the earlier pattern neighbours of position pos (except the
// positions in `skip`), and the candidates for pos (in LINKED mode adjacent
// to each of them)
__device__ __forceinline__ void wide_masks(const WideCtx &s, unsigned long long code, int pos,
                                           uint32_t rest, uint32_t skip, uint32_t &nbm,
                                           uint32_t &cand) {
  cand = rest;
  if (s.nb_all && !s.linked && !skip) {  // all-to-all: every vertex chosen so far
    nbm = s.R & ~rest;
    return;
  }
  nbm = 0;
  for (uint32_t m = (uint32_t)s.nb[pos] & ~skip; m; m &= m - 1) {
    const int v = vertex_at(code, __builtin_ctz(m));
    nbm |= 1u << v;
    if (s.linked) cand &= s.rows[(kWidePlanes - 1) * 32 + v];
  }
}

// Lane state of the search
struct WideLane {
  unsigned long long count;
  uint32_t bpk;            // best packed leaf of the best node (0: none)
  unsigned long long bcode;  // that node's mapping of the positions before the leaf
  int bsh;                 // shift of the leaf position in the code
};

__device__ __forceinline__ void keep_best(WideLane &L, uint32_t pk, unsigned long long code, int sh) {
  // nodes come in lexicographic order: a node replaces the best only with a
  // strictly larger key
  if (pk > (L.bpk | 31u)) {
    L.bpk = pk;
    L.bcode = code;
    L.bsh = sh;
  }
}

// One position left (pos = k - 1): every candidate is a leaf.
template <int B>
__device__ __forceinline__ void leaf_level(const WideCtx &s, WideLane &L, uint32_t rest,
                                           unsigned long long code, int kp, int pos) {
  uint32_t nbm, cand;
  wide_masks(s, code, pos, rest, 0u, nbm, cand);
  L.count += (unsigned long long)__popc(cand);
  uint32_t best = 0;
  for (uint32_t m = cand; m; m &= m - 1) {
    const int c = __builtin_ctz(m);
    const uint32_t pk = pack_leaf(leaf_key<B>(s, step_key<B>(s, kp, c, nbm, rest)), c);
    best = pk > best ? pk : best;
  }
  if (best) keep_best(L, best, code, 5 * (kWideK - 1 - pos));
}

// The last two positions p = k - 2 and k - 1 in ALL mode with N free
// vertices c_0 < ... < c_{N-1} (N wave-uniform): every ordered pair
// (c_i at p, c_j at k - 1), i != j, is a leaf, with key
//   kp + [a Y_i - b D_i] + [a X_j - b D_j] + (a alpha + b) W[c_i][c_j]
// where D = weight to every free vertex, Y = weight to the vertices at the
// earlier neighbours of p, X = weight to those of k - 1 other than p, and
// alpha = whether p neighbours k - 1 (placing c_i first takes W[c_i][c_j]
// out of c_j's preserved weight and, if alpha, adds it to its AggBW).  The
// per-candidate terms are tabulated once, so a leaf is one pair weight, one
// multiply-add and a max.  Rows come in ascending c_i and each row's max
// takes the smallest c_j among equal keys: lexicographic order.
template <int N, int B>
__device__ __forceinline__ void pair_table(const WideCtx &s, WideLane &L, uint32_t rest,
                                           unsigned long long code, int kp, int p) {
  uint32_t nbm, cand, fixm, unused;
  wide_masks(s, code, p, rest, 0u, nbm, cand);
  const uint32_t nbq = (uint32_t)s.nb[p + 1];
  const int alpha = (int)((nbq >> p) & 1u);
  if (s.nb_all)
    fixm = s.R & ~rest;  // all-to-all: the chosen vertices neighbour both positions
  else
    wide_masks(s, code, p + 1, rest, 1u << p, fixm, unused);
  int c[N], P[N], Q[N];
  uint32_t sh2[N];  // bit offset of c_j's field in its packed-weight word
  bool hi[N];       // c_j's field is in the second word
  uint32_t r = rest;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    c[j] = __builtin_ctz(r);
    r &= r - 1;
    sh2[j] = 2u * ((uint32_t)c[j] & 15u);
    hi[j] = c[j] >= 16;
    const int D = wsum_b<B>(s.rows, s.Bn, c[j], rest);
    const int X = wsum_b<B>(s.rows, s.Bn, c[j], fixm);
    const int Y = s.nb_all ? X : wsum_b<B>(s.rows, s.Bn, c[j], nbm);
    P[j] = 32 * (s.a * X - s.b * D) - c[j];
    Q[j] = s.a * Y - s.b * D;
  }
  const int g32 = 32 * (s.a * alpha + s.b);
  const uint32_t base = (uint32_t)(32 * kp + 63);
  L.count += (unsigned long long)(N * (N - 1));
  const int sh = 5 * (kWideK - 1 - p);
  uint32_t sbest = 0;  // the step's best leaf and its row, as in triple_table
  int sci = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int tb = INT_MIN;
    if constexpr (B == 1 || B == 2) {
      // weights <= 3: one 2-bit field of c_i's packed row per leaf
      const uint32_t w0 = s.pw[2 * c[i]], w1 = s.pw[2 * c[i] + 1];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        const int w = (int)(((hi[j] ? w1 : w0) >> sh2[j]) & 3u);
        const int t = P[j] + g32 * w;
        tb = t > tb ? t : tb;
      }
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        const int t = P[j] + g32 * wpair_b<B>(s.rows, s.Bn, c[i], c[j]);
        tb = t > tb ? t : tb;
      }
    }
    const uint32_t pk = base + (uint32_t)(32 * Q[i]) + (uint32_t)tb;
    const bool up = pk > (sbest | 31u);
    sbest = up ? pk : sbest;
    sci = up ? c[i] : sci;
  }
  keep_best(L, sbest, code | ((unsigned long long)sci << sh), sh - 5);
}

// The last two positions without the table (LINKED mode, or more free
// vertices than the table is built for): position p, then a leaf level.
template <int B>
__device__ __forceinline__ void pair_plain(const WideCtx &s, WideLane &L, uint32_t rest,
                                           unsigned long long code, int kp, int p) {
  uint32_t nbm, cand;
  wide_masks(s, code, p, rest, 0u, nbm, cand);
  const int sh = 5 * (kWideK - 1 - p);
  for (uint32_t m = cand; m; m &= m - 1) {
    const int c = __builtin_ctz(m);
    const int kp2 = step_key<B>(s, kp, c, nbm, rest);
    leaf_level<B>(s, L, rest & ~(1u << c), code | ((unsigned long long)c << sh), kp2, p + 1);
  }
}

template <int B>
__device__ __forceinline__ void last_two(const WideCtx &s, WideLane &L, uint32_t rest,
                                         unsigned long long code, int kp, int p, int nfree) {
  if constexpr (B != kEffB) {  // Eq. 2 keys are not sums of per-candidate terms
    if (!s.linked) {
      switch (nfree) {
        case 2: pair_table<2, B>(s, L, rest, code, kp, p); return;
        case 3: pair_table<3, B>(s, L, rest, code, kp, p); return;
        case 4: pair_table<4, B>(s, L, rest, code, kp, p); return;
        case 5: pair_table<5, B>(s, L, rest, code, kp, p); return;
        case 6: pair_table<6, B>(s, L, rest, code, kp, p); return;
        case 7: pair_table<7, B>(s, L, rest, code, kp, p); return;
        case 8: pair_table<8, B>(s, L, rest, code, kp, p); return;
        default: break;
      }
    }
  }
  pair_plain<B>(s, L, rest, code, kp, p);
}

// Expand one prefix: positions d .. k - 3 by an iterative depth-first search
// whose open positions live in the LDS stack (column `tid`), then the last
// two positions in one step.
// The last three positions a = k - 3, p = k - 2, q = k - 1 in ALL mode
// with N3 free vertices (weights <= 3; N3 wave-uniform).  For every choice
// c_a at a, the last two positions are the step of pair_table on the other
// N = N3 - 1 vertices, and its per-candidate terms differ from terms
// tabulated once for all N3 vertices only by the weight to c_a:
//   D_j = D3_j - W[c_j][c_a]                 (c_a is no longer free)
//   Y_j = Yb_j + [a neighbours p] W[c_j][c_a]
//   X_j = Xb_j + [a neighbours q] W[c_j][c_a]
// where D3 is the weight to every free vertex, Yb the weight to p's earlier
// neighbours before a and Xb to q's earlier neighbours before a; c_a itself
// adds a * (weight to a's earlier neighbours) - b * D3_a.  A child's tables
// then cost one packed-weight field and a few adds per candidate.  Choices
// of c_a, rows and columns all come in ascending order: lexicographic.
template <int N3>
__device__ __forceinline__ void triple_table(const WideCtx &s, WideLane &L, uint32_t rest3,
                                             unsigned long long code, int kp, int a) {
  constexpr int N = N3 - 1;
  const int p = a + 1, q = a + 2;
  uint32_t nbm_a, nbm_pb, fix_b, unused;
  wide_masks(s, code, a, rest3, 0u, nbm_a, unused);
  if (s.nb_all) {
    nbm_pb = fix_b = s.R & ~rest3;  // all-to-all: the vertices chosen before a
  } else {
    wide_masks(s, code, p, rest3, 1u << a, nbm_pb, unused);
    wide_masks(s, code, q, rest3, (1u << a) | (1u << p), fix_b, unused);
  }
  const int by = (int)((s.nb[p] >> a) & 1u), bx = (int)((s.nb[q] >> a) & 1u);
  const int alpha = (int)((s.nb[q] >> p) & 1u);
  int c3[N3], D3[N3], Yb[N3], Xb[N3], KA[N3];
  uint32_t sh3[N3];
  bool hi3[N3];
  uint32_t r = rest3;
#pragma unroll
  for (int j = 0; j < N3; ++j) {
    c3[j] = __builtin_ctz(r);
    r &= r - 1;
    sh3[j] = 2u * ((uint32_t)c3[j] & 15u);
    hi3[j] = c3[j] >= 16;
    D3[j] = wsum_b<2>(s.rows, 2, c3[j], rest3);
    Xb[j] = wsum_b<2>(s.rows, 2, c3[j], fix_b);
    Yb[j] = s.nb_all ? Xb[j] : wsum_b<2>(s.rows, 2, c3[j], nbm_pb);
    KA[j] = kp + s.a * wsum_b<2>(s.rows, 2, c3[j], nbm_a) - s.b * D3[j];
  }
  // The weights among the N3 candidates as one word per candidate: field m
  // (bits 2m, 2m+1) of lw[j] = W[c_j][c_m].  Each pair is read once from the
  // packed rows and entered in both words; every later read is a field at a
  // fixed offset.
  uint32_t lw[N3];
#pragma unroll
  for (int j = 0; j < N3; ++j) lw[j] = 0;
#pragma unroll
  for (int j = 0; j < N3; ++j) {
    const uint32_t w0 = s.pw[2 * c3[j]], w1 = s.pw[2 * c3[j] + 1];
#pragma unroll
    for (int m = j + 1; m < N3; ++m) {
      const uint32_t f = ((hi3[m] ? w1 : w0) >> sh3[m]) & 3u;
      lw[j] |= f << (2 * m);
      lw[m] |= f << (2 * j);
    }
  }
  const int g32 = 32 * (s.a * alpha + s.b);
  L.count += (unsigned long long)(N3 * N * (N - 1));
  const int sha = 5 * (kWideK - 1 - a), shp = sha - 5;
  // The two-position terms before c_a is chosen, and what one unit of
  // W[c_j][c_a] adds to them: D loses it, X and Y gain it where a
  // neighbours q or p, so P gains 32 (a bx + b) and Q gains a by + b per unit.
  int P3[N3], Q3[N3];
#pragma unroll
  for (int j = 0; j < N3; ++j) {
    P3[j] = 32 * (s.a * Xb[j] - s.b * D3[j]) - c3[j];
    Q3[j] = s.a * Yb[j] - s.b * D3[j];
  }
  const int dP = 32 * (s.a * bx + s.b), dQ = s.a * by + s.b;
  // the step's best leaf and its first two vertices; rows come in
  // lexicographic order, so a row replaces it only with a strictly larger
  // key (as keep_best), and the lane's best is updated once at the end
  uint32_t sbest = 0;
  int sca = 0, sci = 0;
#pragma unroll
  for (int ia = 0; ia < N3; ++ia) {
    // tables of the last two positions over the candidates other than c_a
    int P[N3], Q[N3];
#pragma unroll
    for (int j = 0; j < N3; ++j) {
      if (j == ia) continue;
      const int w = (int)((lw[ia] >> (2 * j)) & 3u);  // W[c_a][c_j]
      P[j] = P3[j] + dP * w;
      Q[j] = Q3[j] + dQ * w;
    }
    const uint32_t base = (uint32_t)(32 * KA[ia] + 63);
#pragma unroll
    for (int i = 0; i < N3; ++i) {
      if (i == ia) continue;
      int tb = INT_MIN;
#pragma unroll
      for (int j = 0; j < N3; ++j) {
        if (j == i || j == ia) continue;
        const int t = P[j] + g32 * (int)((lw[i] >> (2 * j)) & 3u);
        tb = t > tb ? t : tb;
      }
      const uint32_t pk = base + (uint32_t)(32 * Q[i]) + (uint32_t)tb;
      const bool up = pk > (sbest | 31u);
      sbest = up ? pk : sbest;
      sca = up ? c3[ia] : sca;
      sci = up ? c3[i] : sci;
    }
  }
  keep_best(L, sbest, code | ((unsigned long long)sca << sha) | ((unsigned long long)sci << shp), shp - 5);
}

// The step that finishes a prefix from position `at`: the three-position
// table (ALL mode, weights <= 3, 3..6 free vertices; with 7 the tables
// spilled 200 bytes per lane at the same speed) or the last two.
template <int B>
__device__ __forceinline__ void final_step(const WideCtx &s, WideLane &L, uint32_t rest,
                                           unsigned long long code, int kp, int at, int nfree,
                                           bool triple) {
  if constexpr (B == 1 || B == 2) {
    if (triple) {
      switch (nfree) {
        case 3: triple_table<3>(s, L, rest, code, kp, at); return;
        case 4: triple_table<4>(s, L, rest, code, kp, at); return;
        case 5: triple_table<5>(s, L, rest, code, kp, at); return;
        case 6: triple_table<6>(s, L, rest, code, kp, at); return;
        default: break;
      }
    }
  }
  last_two<B>(s, L, rest, code, kp, at, nfree);
}

template <int B>
__device__ __forceinline__ void expand_prefix(const WideCtx &s, WideLane &L, uint32_t *stk_cand,
                                              int *stk_kp, uint32_t *stk_nbm, int tid,
                                              uint32_t rest, unsigned long long code, int kp,
                                              int d, int F) {
  const int k = s.k;
  if (k - d == 1) {
    leaf_level<B>(s, L, rest, code, kp, d);
    return;
  }
  // position at which the finishing step takes over: k - 3 for the
  // three-position table, else k - 2
  const int nf3 = F - (k - 3);
  const bool triple = (B == 1 || B == 2) && !s.linked && d <= k - 3 && nf3 >= 3 && nf3 <= 6;
  const int top = triple ? k - 3 : k - 2;
  if (d == top) {
    final_step<B>(s, L, rest, code, kp, top, F - top, triple);
    return;
  }
  // open position d
  {
    uint32_t nbm, cand;
    wide_masks(s, code, d, rest, 0u, nbm, cand);
    stk_cand[(d - 1) * kWideThreads + tid] = cand;
    stk_kp[(d - 1) * kWideThreads + tid] = kp;
    stk_nbm[(d - 1) * kWideThreads + tid] = nbm;
  }
  int pos = d;
  for (;;) {
    const uint32_t cand = stk_cand[(pos - 1) * kWideThreads + tid];
    if (cand == 0) {  // position exhausted: back to the previous one
      if (pos == d) break;
      --pos;
      const int v = vertex_at(code, pos);
      rest |= 1u << v;
      code &= ~(31ull << (5 * (kWideK - 1 - pos)));
      continue;
    }
    const int c = __builtin_ctz(cand);
    stk_cand[(pos - 1) * kWideThreads + tid] = cand & (cand - 1);
    const uint32_t nbm = stk_nbm[(pos - 1) * kWideThreads + tid];
    const int kpc = step_key<B>(s, stk_kp[(pos - 1) * kWideThreads + tid], c, nbm, rest);
    rest &= ~(1u << c);
    code |= (unsigned long long)c << (5 * (kWideK - 1 - pos));
    if (pos + 1 == top) {
      final_step<B>(s, L, rest, code, kpc, top, F - top, triple);
      rest |= 1u << c;  // undo the choice, stay at pos
      code &= ~(31ull << (5 * (kWideK - 1 - pos)));
      continue;
    }
    ++pos;
    uint32_t nbm2, cand2;
    wide_masks(s, code, pos, rest, 0u, nbm2, cand2);
    stk_cand[(pos - 1) * kWideThreads + tid] = cand2;
    stk_kp[(pos - 1) * kWideThreads + tid] = kpc;
    stk_nbm[(pos - 1) * kWideThreads + tid] = nbm2;
  }
}

// (k1, c1) better than (k2, c2): larger key, then the smaller mapping
__device__ __forceinline__ bool wide_better(int k1, unsigned long long c1, int k2,
                                            unsigned long long c2) {
  return k1 > k2 || (k1 == k2 && c1 < c2);
}

template <int B>
__device__ __forceinline__ void wide_search_items(const WidePlan *p, const WideCtx &s, WideLane &L,
                                                  uint32_t *stk_cand, int *stk_kp, uint32_t *stk_nbm,
                                                  int tid, uint32_t bi) {
  const int d = p->d, F = p->F;
  const uint32_t stride = p->nblocks * (uint32_t)kWideThreads;
  for (uint32_t x0 = bi * kWideThreads + tid; x0 < p->items; x0 += stride) {
    // prefix x0: mixed-radix digits (radix F - t at position t, position 0
    // most significant), each picking among the vertices still free; the
    // digits are unpacked least significant first into 5-bit fields
    uint32_t x = x0;
    unsigned long long digits = 0;
    for (int t = d - 1; t >= 0; --t) {
      const uint32_t m = (uint32_t)(F - t);
      digits |= (unsigned long long)(x % m) << (5 * t);
      x /= m;
    }
    uint32_t rest = p->R;
    unsigned long long code = 0;
    int kp = p->kp0;
    bool ok = true;
    for (int t = 0; t < d; ++t) {
      const int v = select_bit32(rest, (uint32_t)((digits >> (5 * t)) & 31ull));
      uint32_t nbm, cand;
      wide_masks(s, code, t, rest, 0u, nbm, cand);
      ok = ok && ((cand >> v) & 1u);
      kp = step_key<B>(s, kp, v, nbm, rest);
      rest &= ~(1u << v);
      code |= (unsigned long long)v << (5 * (kWideK - 1 - t));
    }
    if (ok) expand_prefix<B>(s, L, stk_cand, stk_kp, stk_nbm, tid, rest, code, kp, d, F);
  }
}

// The call's embedding total starts from zero (a kernel, not a memset, so
// the launch sequence may be captured into a graph).
__global__ void k_wide_clear(unsigned long long *total) {
  if (threadIdx.x == 0) *total = 0;
}

// Plan of one query from the busy mask in memory (the call's start): the
// checks of the host form (malformed -> kPlanInvalid), free set R,
// b * W(R) (0 for Eq. 2), the pattern's earlier-neighbour masks and edge
// count, weight bit-planes in use, prefix depth (the smallest with at least
// kWideMinItems prefixes), the blocks that have items, the claim of the
// server's commit (the first committing query of the batch, array order)
// and the query's embeddings added to the call's total.
__global__ __launch_bounds__(256) void k_wide_plan(WideArgs w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w.nq) return;
  const mapa_query q = w.q[i];
  WidePlan p;
  p.R = 0;
  p.kp0 = 0;
  p.server = q.server;
  for (int t = 0; t < kWideK; ++t) p.nb[t] = 0;
  p.k = q.k;
  p.mode = q.mode;
  p.d = 0;
  p.B = 1;
  p.F = 0;
  p.commit = q.commit;
  p.nb_all = q.kind == MAPA_ALL_TO_ALL;
  p.a = q.a;
  p.b = q.b;
  p.topo = 0;
  p.metric = q.metric;
  p.E = 0;
  p.items = 0;
  p.nblocks = 0;
  const int pid = (int)q.kind - MAPA_PATTERN_BASE;  // registered pattern id
  const bool registered = pid >= 0 && pid < MAPA_MAX_PATTERNS;
  const bool ok = q.server >= 0 && q.server < w.nservers && q.k >= 1 && q.k <= kWideK &&
                  (q.kind <= MAPA_TREE || (registered && w.pat_k[pid] == q.k)) &&
                  q.mode <= 1 && q.commit <= 1 && q.a >= 0 && q.a <= MAPA_MAX_AB && q.b >= 0 &&
                  q.b <= MAPA_MAX_AB &&
                  (q.metric == MAPA_METRIC_WEIGHTED || q.metric == MAPA_METRIC_EFFBW) &&
                  w.server_topo[q.server] < w.ntopo_wide &&
                  (q.metric == MAPA_METRIC_WEIGHTED || w.topo_maxw[w.server_topo[q.server]] <= 2);
  if (!ok) {
    p.status = kPlanInvalid;
    w.plan[i] = p;
    return;
  }
  const int t = w.server_topo[q.server];
  const int n = w.topo_n[t];
  const uint32_t R = ~w.busy[q.server] & (n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u));
  const int F = __popc(R);
  int B = 1;
  while (B < 8 && (w.topo_maxw[t] >> B)) ++B;
  const uint32_t *rows = w.rows + (size_t)t * kWidePlanes * 32;
  int wr2 = 0;  // twice W(R): every pair counted from both ends
  for (uint32_t m = R; m; m &= m - 1) wr2 += wsum_b<0>(rows, B, __builtin_ctz(m), R);
  p.topo = (uint16_t)t;
  p.R = R;
  p.F = (uint8_t)F;
  p.B = (uint8_t)B;
  p.kp0 = q.metric == MAPA_METRIC_EFFBW ? 0 : q.b * (wr2 / 2);  // Eq. 2 starts from no edges
  if (registered) {
    const unsigned long long tab = w.pat_nbtab[pid];
    for (int j = 0; j < q.k; ++j) p.nb[j] = (uint16_t)((tab >> (8 * j)) & 0xFFu);
  } else {
    for (int j = 1; j < q.k; ++j) {
      if (q.kind == MAPA_RING)
        p.nb[j] = (uint16_t)((1u << (j - 1)) | (j == q.k - 1 && q.k >= 3 ? 1u : 0u));
      else if (q.kind == MAPA_ALL_TO_ALL)
        p.nb[j] = (uint16_t)((1u << j) - 1u);
      else
        p.nb[j] = (uint16_t)(1u << ((j - 1) / 2));
    }
  }
  int E = 0;
  for (int j = 0; j < q.k; ++j) E += __popc(p.nb[j]);
  p.E = (uint8_t)E;
  if (q.commit) atomicMin(&w.commit_slot[q.server], (unsigned long long)i);
  if (q.k > F) {
    p.status = kPlanNofit;
    w.plan[i] = p;
    return;
  }
  p.status = kPlanOk;
  unsigned long long leaves = 1;  // F!/(F-k)! <= 32!/20! < 2^54
  for (int j = 0; j < q.k; ++j) leaves *= (unsigned long long)(F - j);
  atomicAdd(w.total, leaves < 2 * kWideMaxLeaves ? leaves : 2 * kWideMaxLeaves);
  int d = 0;
  unsigned long long items = 1;  // F!/(F-d)!
  while (d < q.k - 1 && items < kWideMinItems) {
    items *= (unsigned long long)(F - d);
    ++d;
  }
  p.d = (uint8_t)d;
  p.items = (uint32_t)items;
  const unsigned long long want = (items + kWideThreads - 1) / kWideThreads;
  p.nblocks = (uint32_t)(want < 1 ? 1 : want > kWideMaxBlocksPerQuery ? kWideMaxBlocksPerQuery : want);
  w.plan[i] = p;
}

// Four waves per SIMD: 128 VGPRs (135 uncapped), 37 KB of LDS per block
// (the nine-entry stack and the Eq. 2 ranks).  The cap leaves a few
// bytes per lane in scratch that stay in cache: the wide workload's HBM
// writes are the same 0.59 MB per call with and without it, and the call
// takes 3.37 instead of 3.53 ms.
__global__ __launch_bounds__(kWideThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_wide_search(WideArgs w) {
  __shared__ uint32_t s_rows[kWidePlanes * 32];
  __shared__ uint32_t s_pw[64];
  __shared__ uint16_t s_nb[kWideK];
  __shared__ uint32_t s_cand[kWideStack * kWideThreads];
  __shared__ int s_kp[kWideStack * kWideThreads];
  __shared__ uint32_t s_nbm[kWideStack * kWideThreads];
  __shared__ unsigned long long s_cnt[kWideThreads / 64], s_code[kWideThreads / 64];
  __shared__ int s_key[kWideThreads / 64];
  __shared__ uint16_t s_erank[kWideEffTab];
  // block b of query q's share: b = blockIdx.x % kWideMaxBlocksPerQuery
  const uint32_t q = blockIdx.x / kWideMaxBlocksPerQuery;
  const uint32_t bi = blockIdx.x % kWideMaxBlocksPerQuery;
  const WidePlan *p = w.plan + q;
  const int tid = threadIdx.x;
  // nothing to search (or the call is over its embedding limit): an empty partial
  if (p->status != kPlanOk || bi >= p->nblocks || *w.total > kWideMaxLeaves) {
    if (tid == 0) {
      WidePartial r;
      r.count = 0;
      r.code = ~0ull;
      r.key = -1;
      r.pad = 0;
      w.part[blockIdx.x] = r;
    }
    return;
  }
  for (int i = tid; i < kWidePlanes * 32; i += blockDim.x)
    s_rows[i] = w.rows[(size_t)p->topo * kWidePlanes * 32 + i];
  if (tid < kWideK) s_nb[tid] = p->nb[tid];
  const int e1 = p->E + 1;
  if (p->metric == MAPA_METRIC_EFFBW)  // the ranks of the query's edge count
    for (int i = tid; i < e1 * e1; i += blockDim.x) s_erank[i] = w.eff_rank[eff_off(p->E) + i];
  __syncthreads();
  if (tid < 64) {  // packed 2-bit weights from the two low planes
    const int v = tid >> 1, h = tid & 1;
    const uint32_t lo = s_rows[v] >> (16 * h), hb = s_rows[32 + v] >> (16 * h);
    uint32_t word = 0;
    for (int u = 0; u < 16; ++u) word |= (((lo >> u) & 1u) | (((hb >> u) & 1u) << 1)) << (2 * u);
    s_pw[tid] = word;
  }
  __syncthreads();
  WideCtx s;
  s.rows = s_rows;
  s.erank = s_erank;
  s.e1 = e1;
  s.pw = s_pw;
  s.nb = s_nb;
  s.R = p->R;
  s.Bn = p->B;
  s.a = p->a;
  s.b = p->b;
  s.k = p->k;
  s.linked = p->mode;
  s.nb_all = p->nb_all;
  WideLane L;
  L.count = 0;
  L.bpk = 0;
  L.bcode = 0;
  L.bsh = 0;
  if (p->metric == MAPA_METRIC_EFFBW)
    wide_search_items<kEffB>(p, s, L, s_cand, s_kp, s_nbm, tid, bi);
  else if (s.Bn == 1)
    wide_search_items<1>(p, s, L, s_cand, s_kp, s_nbm, tid, bi);
  else if (s.Bn == 2)
    wide_search_items<2>(p, s, L, s_cand, s_kp, s_nbm, tid, bi);
  else
    wide_search_items<0>(p, s, L, s_cand, s_kp, s_nbm, tid, bi);
  // this lane's best: the node's code plus its leaf vertex
  unsigned long long cnt = L.count, code = ~0ull;
  int key = -1;
  if (L.bpk) {
    key = (int)(L.bpk >> 5) - 1;
    code = L.bcode | ((unsigned long long)(31u - (L.bpk & 31u)) << L.bsh);
  }
  // block reduction: count sum; best = largest key, then smallest mapping
  for (int off = 32; off >= 1; off >>= 1) {
    cnt += __shfl_xor(cnt, off, 64);
    const int ok2 = __shfl_xor(key, off, 64);
    const unsigned long long oc = __shfl_xor(code, off, 64);
    if (wide_better(ok2, oc, key, code)) {
      key = ok2;
      code = oc;
    }
  }
  const int wave = tid >> 6;
  if ((tid & 63) == 0) {
    s_cnt[wave] = cnt;
    s_code[wave] = code;
    s_key[wave] = key;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      cnt += s_cnt[i];
      if (wide_better(s_key[i], s_code[i], key, code)) {
        key = s_key[i];
        code = s_code[i];
      }
    }
    WidePartial r;
    r.count = cnt;
    r.code = code;
    r.key = key;
    r.pad = 0;
    w.part[blockIdx.x] = r;
  }
}

// One wave per query: the lanes combine the query's block partials, then
// lane 0 builds the result.
__global__ __launch_bounds__(256) void k_wide_finalize(WideArgs w) {
  const int q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= w.nq) return;
  const WidePlan &p = w.plan[q];
  const bool refused = *w.total > kWideMaxLeaves;
  unsigned long long cnt = 0, code = ~0ull;
  int key = -1;
  if (p.status == kPlanOk && !refused) {
    for (uint32_t b = lane; b < p.nblocks; b += 64) {
      const WidePartial &pt = w.part[(size_t)q * kWideMaxBlocksPerQuery + b];
      cnt += pt.count;
      if (wide_better(pt.key, pt.code, key, code)) {
        key = pt.key;
        code = pt.code;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      cnt += __shfl_xor(cnt, off, 64);
      const int k2 = __shfl_xor(key, off, 64);
      const unsigned long long c2 = __shfl_xor(code, off, 64);
      if (wide_better(k2, c2, key, code)) {
        key = k2;
        code = c2;
      }
    }
  }
  if (lane != 0) return;
  mapa_result_wide r;
  r.count = (int64_t)cnt;
  r.status = MAPA_RES_NOFIT;
  r.key = INT32_MIN;
  r.agg = 0;
  r.pres = 0;
  r.vertex_mask = 0;
  for (int i = 0; i < 16; ++i) r.mapping[i] = 0xFF;
  r.links = 0;
  r.alloc_handle = -1;
  if (p.status == kPlanOk && !refused && cnt > 0 && key >= 0) {
    const uint32_t *rows = w.rows + (size_t)p.topo * kWidePlanes * 32;
    uint32_t S = 0;
    int agg = 0, lx = 0, ly = 0, lz = 0;
    for (int i = 0; i < p.k; ++i) {
      const int v = vertex_at(code, i);
      r.mapping[i] = (uint8_t)v;
      S |= 1u << v;
      for (uint32_t m = p.nb[i]; m; m &= m - 1) {  // Eq. 1 over the pattern edges
        const int wv = wsum_wide(rows, p.B, v, 1u << vertex_at(code, __builtin_ctz(m)));
        agg += wv;
        lx += wv == 2;  // Eq. 2's link classes
        ly += wv == 1;
        lz += wv == 0;
      }
    }
    const uint32_t left = p.R & ~S;  // Eq. 3 over the free vertices left
    int pres2 = 0;
    for (uint32_t m = left; m; m &= m - 1) pres2 += wsum_wide(rows, p.B, __builtin_ctz(m), left);
    r.status = MAPA_RES_OK;
    r.agg = agg;
    r.pres = pres2 / 2;
    r.vertex_mask = S;
    if (p.metric == MAPA_METRIC_EFFBW) {
      const int at = eff_off(p.E) + lx * (p.E + 1) + ly;
      r.key = w.eff_key[at];
      r.links = lx | (ly << 8) | (lz << 16);
      if ((int)w.eff_rank[at] != key || lx + ly + lz != p.E) atomicAdd(w.self_check_failures, 1u);
    } else {
      r.key = key;
      if ((int)p.a * agg + (int)p.b * r.pres != key) atomicAdd(w.self_check_failures, 1u);
    }
  }
  if (p.status == kPlanInvalid) {
    r.status = MAPA_RES_INVALID;
  } else if (refused) {  // nothing evaluated; a claim is only given back
    r.status = MAPA_RES_REFUSED;
    if (p.commit && w.commit_slot[p.server] == (unsigned long long)q) w.commit_slot[p.server] = ~0ull;
  } else if (p.commit) {
    // the server's first committing query commits (if it found a match) and
    // frees the claim; later committing queries of the server conflict
    if (w.commit_slot[p.server] == (unsigned long long)q) {
      if (r.status == MAPA_RES_OK) {
        atomicOr(&w.busy[p.server], r.vertex_mask);
        r.alloc_handle = ((int64_t)p.server << 32) | (int64_t)r.vertex_mask;
      }
      w.commit_slot[p.server] = ~0ull;
    } else if (r.status == MAPA_RES_OK) {
      r.status = MAPA_RES_CONFLICT;
    }
  }
  w.res[q] = r;
}

hipError_t launch_wide_plan(const WideArgs &w, hipStream_t s) {
  if (w.nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wide_clear, dim3(1), dim3(64), 0, s, w.total);
  hipLaunchKernelGGL(k_wide_plan, dim3((w.nq + 255) / 256), dim3(256), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_wide_search(const WideArgs &w, hipStream_t s) {
  if (w.nq > 0)
    hipLaunchKernelGGL(k_wide_search, dim3((unsigned)w.nq * kWideMaxBlocksPerQuery), dim3(kWideThreads), 0,
                       s, w);
  return hipGetLastError();
}

hipError_t launch_wide_finalize(const WideArgs &w, hipStream_t s) {
  if (w.nq > 0) hipLaunchKernelGGL(k_wide_finalize, dim3((w.nq + 3) / 4), dim3(256), 0, s, w);
  return hipGetLastError();
}

}  // namespace mapa
