// Wide path: servers of up to 32 accelerators and patterns of up to 12
// vertices (the paper's jobs of 9 GPUs and more).  The same definitions as
// the batch path: every injective embedding (ALL mode) or every one whose
// pattern edges land on direct links (LINKED), AggBW (Eq. 1) and PreservedBW
// (Eq. 3) through the scoring identity
//   key = b*W(R) + sum_p [ a*w(phi_p, earlier neighbours) - b*w(phi_p, still free) ],
// the first maximum in lexicographic order (Alg. 1 with strict improvement).
//
// k_wide_search: a block works on one query; its threads take the query's
// prefixes of depth d (F!/(F-d)! of them, in lexicographic order of their
// index) in a block-strided loop and expand each depth-first, keeping a count
// and their best (key, mapping).  Weighted sums are popcounts over 32-bit
// weight bit-planes staged in LDS.  The block reduces to one partial.
// k_wide_finalize: per query, the partials of its blocks, the mapping, a
// recomputation of AggBW and PreservedBW from it (self-check) and the commit.
#include "mapa_internal.h"

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

struct WideState {
  const uint32_t *rows;  // LDS: [kWidePlanes][32]
  const WidePlan *p;
  int B, a, b, k, linked, nb_all;
  unsigned long long count;
  int bkey;
  unsigned long long bcode;
};

// a * w(c, nbm) - b * w(c, rest): one pass over the weight planes; the
// common cases of one and two planes (weights up to 3) unrolled
__device__ __forceinline__ int wide_term(const WideState &s, int c, uint32_t nbm, uint32_t rest) {
  const uint32_t r0 = s.rows[c];
  int v = s.a * __popc(r0 & nbm) - s.b * __popc(r0 & rest);
  if (s.B == 1) return v;
  const uint32_t r1 = s.rows[32 + c];
  v += (s.a * __popc(r1 & nbm) - s.b * __popc(r1 & rest)) << 1;
  for (int t = 2; t < s.B; ++t) {
    const uint32_t r = s.rows[t * 32 + c];
    v += (s.a * __popc(r & nbm) - s.b * __popc(r & rest)) << t;
  }
  return v;
}

// vertices at the earlier pattern neighbours of position pos, and the
// candidates for pos (in LINKED mode adjacent to each of them)
__device__ __forceinline__ void wide_masks(const WideState &s, unsigned long long code, int pos,
                                           uint32_t rest, uint32_t &nbm, uint32_t &cand) {
  cand = rest;
  if (s.nb_all && !s.linked) {  // all-to-all: every vertex chosen so far
    nbm = s.p->R & ~rest;
    return;
  }
  nbm = 0;
  for (uint32_t m = s.p->nb[pos]; m; m &= m - 1) {
    const int v = vertex_at(code, __builtin_ctz(m));
    nbm |= 1u << v;
    if (s.linked) cand &= s.rows[(kWidePlanes - 1) * 32 + v];
  }
}

template <int L>
__device__ void wide_level(WideState &s, uint32_t rest, unsigned long long code, int kp, int pos) {
  uint32_t nbm, cand;
  wide_masks(s, code, pos, rest, nbm, cand);
  const int sh = 5 * (kWideK - 1 - pos);
  if constexpr (L == 1) {
    // every candidate is a leaf: scored as ((key + 1) << 5) | (31 - c), so
    // one max picks the node's largest key and, among equal keys, the first
    // leaf (keys stay below 2^27: weights <= 255, n <= 32, a, b <= 1024)
    s.count += (unsigned long long)__popc(cand);
    uint32_t best = 0;
    for (uint32_t m = cand; m; m &= m - 1) {
      const int c = __builtin_ctz(m);
      const int v = kp + 1 + wide_term(s, c, nbm, rest);
      const uint32_t pk = ((uint32_t)v << 5) | (31u - (uint32_t)c);
      best = pk > best ? pk : best;
    }
    const int key = (int)(best >> 5) - 1;
    if (best && key > s.bkey) {  // nodes come in lexicographic order: keep the first maximum
      s.bkey = key;
      s.bcode = code | ((unsigned long long)(31u - (best & 31u)) << sh);
    }
  } else {
    for (uint32_t m = cand; m; m &= m - 1) {
      const int c = __builtin_ctz(m);
      const int kp2 = kp + wide_term(s, c, nbm, rest);
      wide_level<L - 1>(s, rest & ~(1u << c), code | ((unsigned long long)c << sh), kp2, pos + 1);
    }
  }
}

__device__ void wide_expand(WideState &s, int L, uint32_t rest, unsigned long long code, int kp,
                            int pos) {
  switch (L) {
    case 1: wide_level<1>(s, rest, code, kp, pos); break;
    case 2: wide_level<2>(s, rest, code, kp, pos); break;
    case 3: wide_level<3>(s, rest, code, kp, pos); break;
    case 4: wide_level<4>(s, rest, code, kp, pos); break;
    case 5: wide_level<5>(s, rest, code, kp, pos); break;
    case 6: wide_level<6>(s, rest, code, kp, pos); break;
    case 7: wide_level<7>(s, rest, code, kp, pos); break;
    case 8: wide_level<8>(s, rest, code, kp, pos); break;
    case 9: wide_level<9>(s, rest, code, kp, pos); break;
    case 10: wide_level<10>(s, rest, code, kp, pos); break;
    case 11: wide_level<11>(s, rest, code, kp, pos); break;
    case 12: wide_level<12>(s, rest, code, kp, pos); break;
    default: break;
  }
}

// (k1, c1) better than (k2, c2): larger key, then the smaller mapping
__device__ __forceinline__ bool wide_better(int k1, unsigned long long c1, int k2,
                                            unsigned long long c2) {
  return k1 > k2 || (k1 == k2 && c1 < c2);
}

// 8 waves per SIMD (at most 64 VGPRs): on the wide workload 14.4 ms per
// call against 14.7 at 6 and 18.5 at 4 (the compiler's own choice)
__global__ __launch_bounds__(kWideThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_wide_search(
    WideArgs w) {
  __shared__ uint32_t s_rows[kWidePlanes * 32];
  __shared__ unsigned long long s_cnt[kWideThreads / 64], s_code[kWideThreads / 64];
  __shared__ int s_key[kWideThreads / 64];
  const uint32_t q = w.blk_q[blockIdx.x];
  const WidePlan *p = w.plan + q;
  const int tid = threadIdx.x;
  for (int i = tid; i < kWidePlanes * 32; i += blockDim.x)
    s_rows[i] = w.rows[(size_t)p->topo * kWidePlanes * 32 + i];
  __syncthreads();
  WideState s;
  s.rows = s_rows;
  s.p = p;
  s.B = p->B;
  s.a = p->a;
  s.b = p->b;
  s.k = p->k;
  s.linked = p->mode;
  s.nb_all = p->nb_all;
  s.count = 0;
  s.bkey = -1;
  s.bcode = ~0ull;
  const int d = p->d, F = p->F;
  const uint32_t bi = blockIdx.x - p->block0;
  const uint32_t stride = p->nblocks * (uint32_t)blockDim.x;
  for (uint32_t x0 = bi * blockDim.x + tid; x0 < p->items; x0 += stride) {
    // prefix x0: mixed-radix digits (radix F - t at position t, position 0
    // most significant), each picking among the vertices still free
    uint32_t x = x0, digits[kWideK];
    for (int t = d - 1; t >= 0; --t) {
      const uint32_t m = (uint32_t)(F - t);
      digits[t] = x % m;
      x /= m;
    }
    uint32_t rest = p->R;
    unsigned long long code = 0;
    int kp = p->kp0;
    bool ok = true;
    for (int t = 0; t < d; ++t) {
      const int v = select_bit32(rest, digits[t]);
      uint32_t nbm, cand;
      wide_masks(s, code, t, rest, nbm, cand);
      ok = ok && ((cand >> v) & 1u);
      kp += s.a * wsum_wide(s_rows, s.B, v, nbm) - s.b * wsum_wide(s_rows, s.B, v, rest);
      rest &= ~(1u << v);
      code |= (unsigned long long)v << (5 * (kWideK - 1 - t));
    }
    if (ok) wide_expand(s, s.k - d, rest, code, kp, d);
  }
  // block reduction: count sum; best = largest key, then smallest mapping
  unsigned long long cnt = s.count, code = s.bcode;
  int key = s.bkey;
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

__global__ __launch_bounds__(256) void k_wide_finalize(WideArgs w) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= w.nq) return;
  const WidePlan &p = w.plan[q];
  mapa_result_wide r;
  r.count = 0;
  r.status = MAPA_RES_NOFIT;
  r.key = INT32_MIN;
  r.agg = 0;
  r.pres = 0;
  r.vertex_mask = 0;
  for (int i = 0; i < 16; ++i) r.mapping[i] = 0xFF;
  r.reserved = 0;
  r.alloc_handle = -1;
  if (p.status == kPlanOk) {
    unsigned long long cnt = 0, code = ~0ull;
    int key = -1;
    for (uint32_t b = 0; b < p.nblocks; ++b) {
      const WidePartial &pt = w.part[p.block0 + b];
      cnt += pt.count;
      if (wide_better(pt.key, pt.code, key, code)) {
        key = pt.key;
        code = pt.code;
      }
    }
    r.count = (int64_t)cnt;
    if (cnt > 0 && key >= 0) {
      const uint32_t *rows = w.rows + (size_t)p.topo * kWidePlanes * 32;
      uint32_t S = 0;
      int agg = 0;
      for (int i = 0; i < p.k; ++i) {
        const int v = vertex_at(code, i);
        r.mapping[i] = (uint8_t)v;
        S |= 1u << v;
        for (uint32_t m = p.nb[i]; m; m &= m - 1)  // Eq. 1 over the pattern edges
          agg += wsum_wide(rows, p.B, v, 1u << vertex_at(code, __builtin_ctz(m)));
      }
      const uint32_t left = p.R & ~S;  // Eq. 3 over the free vertices left
      int pres2 = 0;
      for (uint32_t m = left; m; m &= m - 1) pres2 += wsum_wide(rows, p.B, __builtin_ctz(m), left);
      r.status = MAPA_RES_OK;
      r.key = key;
      r.agg = agg;
      r.pres = pres2 / 2;
      r.vertex_mask = S;
      if ((int)p.a * agg + (int)p.b * r.pres != key) atomicAdd(w.self_check_failures, 1u);
      if (p.commit) {
        if (p.owner) {
          w.busy[p.server] |= S;
          r.alloc_handle = ((int64_t)p.server << 32) | (int64_t)S;
        } else {
          r.status = MAPA_RES_CONFLICT;
        }
      }
    }
  }
  w.res[q] = r;
}

hipError_t launch_wide_search(const WideArgs &w, int32_t blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_wide_search, dim3(blocks), dim3(kWideThreads), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_wide_finalize(const WideArgs &w, hipStream_t s) {
  if (w.nq > 0) hipLaunchKernelGGL(k_wide_finalize, dim3((w.nq + 255) / 256), dim3(256), 0, s, w);
  return hipGetLastError();
}

}  // namespace mapa
