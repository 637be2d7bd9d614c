// The fused small-batch kernel (one launch per batch of distinct servers).
#include "device.h"

namespace mapa {

hipError_t upload_tables_fused(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
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
    Plan p = make_plan(q, f.nservers, f.server_topo, f.topo_n, f.topo_maxw, f.busy, f.rows, WPR,
                       f.pat_nbtab, f.pat_k, f.pat_nbtab_ord, f.pat_order);
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
    item_search<WPR, 0>(x < nitems ? &s_plan : nullptr, s_rows, x, f.eff_rank, f.pat_order, c1, b1);
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
    Outcome o = decode_best(p, cnt, best, s_rows, WPR, f.eff_rank, f.eff_key, f.pat_order,
                            f.self_check_failures);
    if (p.status != kPlanInvalid && p.commit && o.status == MAPA_RES_OK) {
      atomicOr(&f.busy[p.server], o.S);
      o.handle = ((int64_t)p.server << 32) | (int64_t)o.S;
    }
    store_result(f.res + i, o);
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

}  // namespace mapa
