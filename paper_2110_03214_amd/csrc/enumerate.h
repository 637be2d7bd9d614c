// The persistent enumeration kernel (template); the enum_*.hip units
// instantiate its variants.
#pragma once

#include "device.h"

namespace mapa {

template <int WPR, int PAIR>
__device__ __forceinline__ void run_item(const BatchArgs &a, const uint32_t *rows, uint2 it) {
  const int lane = threadIdx.x & 63;
  const bool valid = it.x != kInvalidItem;
  const Plan *pp = valid ? &a.plan[it.x] : nullptr;
  const uint32_t *trow = valid ? rows + (uint32_t)pp->topo * (kTopoWords * WPR) : rows;
  unsigned long long cnt, best;
  item_search<WPR, PAIR>(pp, trow, it.y, a.eff_rank, a.pat_order, cnt, best);
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

template <int WPR, bool LDS, int PAIR>
static hipError_t launch_enum_t(const BatchArgs &a, hipStream_t s) {
  const size_t lds = LDS ? (size_t)a.ntopo * kTopoWords * WPR * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL((k_enumerate<WPR, LDS, PAIR>), dim3(a.enum_blocks), dim3(a.enum_threads), lds, s,
                     a);
  return hipGetLastError();
}

template <int WPR, bool LDS, int PAIR>
static int occ_t(int threads, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_enumerate<WPR, LDS, PAIR>, threads, lds) !=
      hipSuccess)
    return 0;
  return nb;
}

}  // namespace mapa
