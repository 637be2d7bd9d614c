// The persistent enumeration kernel (template); the enum_*.hip units
// instantiate its variants.
#pragma once

#include "device.h"

namespace mapa {

// The lane id, opaque to the compiler at each use.  Taken once per chunk, it
// keeps the cross-lane source addresses of the reductions below (and the
// lane's work-list address) from being hoisted out of the persistent loop:
// hoisted, they outlived the register budget and were spilled, 76 bytes per
// lane written to scratch by every thread of the grid at each launch (the
// batched config's kernel: 4.2 instead of 21.7 MiB written per launch, 4 %
// faster).  The twelve-wide instances keep the hoisted form, measured 2 %
// faster on the large config.
template <int PAIR>
__device__ __forceinline__ int chunk_lane() {
  int lane = (int)(threadIdx.x & 63u);
  if constexpr (PAIR < 12) __asm__ volatile("" : "+v"(lane));
  return lane;
}

// v of lane src (0 <= src < 64 for a defined value)
__device__ __forceinline__ unsigned long long lane_read_u64(int src, unsigned long long v) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(v >> 32));
  return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int WPR, int PAIR>
__device__ __forceinline__ void run_item(const BatchArgs &a, const uint32_t *rows, uint2 it,
                                         int lane) {
  const bool valid = it.x != kInvalidItem;
  const Plan *pp = valid ? &a.plan[it.x] : nullptr;
  const uint32_t *trow = valid ? rows + (uint32_t)pp->topo * (kTopoWords * WPR) : rows;
  unsigned long long cnt, best;
  item_search<WPR, PAIR>(pp, trow, it.y, a.eff_rank, a.pat_order, cnt, best);
  const int qi = valid ? (int)it.x : -1;
  const int q0 = __builtin_amdgcn_readfirstlane(qi);
  const bool same = __ballot(valid && qi != q0) == 0ull;
  if (same) {
    if constexpr (PAIR >= 12) {
      cnt = wave_sum_u64(cnt);
      best = wave_max_u64(best);
    } else {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        cnt += lane_read_u64(lane ^ off, cnt);
        const unsigned long long ob = lane_read_u64(lane ^ off, best);
        best = ob > best ? ob : best;
      }
    }
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
      const int src = lane + off;  // beyond lane 63 the value read is not used
      int oq;
      unsigned long long oc, ob;
      if constexpr (PAIR >= 12) {
        oq = __shfl_down(qi, off, 64);
        oc = __shfl_down(cnt, off, 64);
        ob = __shfl_down(best, off, 64);
      } else {
        oq = __builtin_amdgcn_ds_bpermute(src << 2, qi);
        oc = lane_read_u64(src, cnt);
        ob = lane_read_u64(src, best);
      }
      if (src < 64 && oq == qi) {
        cnt += oc;
        best = ob > best ? ob : best;
      }
    }
    int pq;  // not used on lane 0
    if constexpr (PAIR >= 12)
      pq = __shfl_up(qi, 1, 64);
    else
      pq = __builtin_amdgcn_ds_bpermute((lane - 1) << 2, qi);
    if (valid && (lane == 0 || pq != qi)) {
      if (cnt) atomicAdd(&a.acc_count[qi], cnt);
      if (best) atomicMax(&a.acc_best[qi], best);
    }
  }
}

template <int WPR, int PAIR>
__device__ __forceinline__ void chunk_loop(const BatchArgs &a, const uint32_t *rows) {
  const uint32_t nchunks = *(volatile const uint32_t *)&a.ctr->total_chunks;
  // Home queue: consecutive blocks land on different XCDs, so the waves of
  // one queue mostly share an XCD.  A wave whose queue runs dry looks at
  // every queue's counter at once (one lane each) and moves to the next one,
  // counting from its home, that still holds chunks.
  const uint32_t home = blockIdx.x % kQueues;
  uint32_t qu = home;
  if constexpr (PAIR >= 12) {
    // the twelve-wide instances claim every chunk (their first chunks by
    // wave id, below, measured 5 % slower on the large config: a different
    // register allocation of the whole loop)
    for (;;) {
      const int lane = chunk_lane<PAIR>();
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
      run_item<WPR, PAIR>(a, rows, it, lane);
    }
  } else {
    // First chunks by wave id: with S the grid's waves rounded down to whole
    // rounds of the queues, wave w < S starts on chunk w without a claim (the
    // front end starts every queue's counter past those S chunks), so no wave
    // waits on an atomic before its first loads.
    const uint32_t waves = gridDim.x * (blockDim.x / 64u);
    const uint32_t w = blockIdx.x * (blockDim.x / 64u) + threadIdx.x / 64u;
    constexpr uint32_t kClaim = ~0u;
    uint32_t c = w < waves / kQueues * kQueues ? w : kClaim;
    for (;;) {
      const int lane = chunk_lane<PAIR>();
      if (c == kClaim) {
        if (lane == 0) c = qu + atomicAdd(&a.ctr->queue_ctr[qu][0], 1u) * (uint32_t)kQueues;
        c = __shfl(c, 0, 64);
      }
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
        c = kClaim;
        continue;
      }
      const uint2 it = a.items[(size_t)c * kChunk + lane];
      run_item<WPR, PAIR>(a, rows, it, lane);
      c = kClaim;
    }
  }
}

// PAIR > 0: the last two positions of one-word-row topologies with up to PAIR
// free vertices go through pair_level (faster per match, more registers, so
// fewer waves per SIMD).
template <int WPR, bool ROWS_LDS, int PAIR>
// At most 128 VGPRs, so four waves share each SIMD.
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
