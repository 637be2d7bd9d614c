// Job-trace simulation (mapa_simulate), device part: one kernel that turns
// a round of placements into log entries.  A round holds at most one job
// per simulation (its FIFO head); jobs under the Preserve and Greedy
// policies were placed by the query batch that ran just before on the same
// stream, jobs under the lowest-id policy are placed here.  For every job
// the kernel scores the mapping at its start cycle: AggBW (Eq. 1) and the
// link mix over the mapped pattern edges, PreservedBW (Eq. 3) over the free
// accelerators left, and the predicted effective bandwidth (Eq. 2) of the
// mix from the context's table.
#include "simulate.h"

namespace mapa {

__global__ __launch_bounds__(256) void k_sim_place(SimPlaceArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const SimEntry e = a.entries[i];
  const int t = a.server_topo[e.server];
  const int n = a.topo_n[t];
  const uint8_t *W = a.topo_W + (size_t)t * 256;
  const uint32_t full = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
  const uint32_t R = ~e.busy_before & full;
  SimOut o;
  o.mask = 0;
  for (int p = 0; p < 8; ++p) o.mapping[p] = 0xFF;
  o.agg = o.pres = o.effbw_milli = o.links = 0;
  if (e.qi < 0) {
    // lowest free ids: pattern vertex p on the p-th lowest free accelerator
    uint32_t m = R;
    for (int p = 0; p < e.k; ++p) {
      const int v = __builtin_ctz(m);
      m &= m - 1u;
      o.mapping[p] = (uint8_t)v;
      o.mask |= 1u << v;
    }
    a.busy[e.server] |= o.mask;
  } else {
    const mapa_result &r = a.qres[e.qi];
    if (r.status != MAPA_RES_OK) {  // cannot happen for a job that fits: report it
      a.out[i] = o;
      return;
    }
    o.mask = r.vertex_mask;
    for (int p = 0; p < 8; ++p) o.mapping[p] = r.mapping[p];
  }
  int x = 0, y = 0, z = 0, agg = 0;
  for (int p = 1; p < e.k; ++p)
    for (uint32_t m = (uint32_t)(e.nbtab >> (8 * p)) & 0xFFu; m; m &= m - 1u) {
      const int w = W[o.mapping[p] * 16 + o.mapping[__builtin_ctz(m)]];
      agg += w;
      x += w == 2;
      y += w == 1;
      z += w == 0;
    }
  const uint32_t left = R & ~o.mask;
  int pres = 0;
  for (uint32_t m = left; m; m &= m - 1u) {
    const int u = __builtin_ctz(m);
    for (uint32_t m2 = left & ~((2u << u) - 1u); m2; m2 &= m2 - 1u) pres += W[u * 16 + __builtin_ctz(m2)];
  }
  const int E = x + y + z;
  o.agg = agg;
  o.pres = pres;
  o.links = x | (y << 8) | (z << 16);
  o.effbw_milli = a.eff_key[eff_off(E) + x * (E + 1) + y];
  if (e.qi >= 0) {  // the query's own scores must agree with the recomputation
    const mapa_result &r = a.qres[e.qi];
    if (r.agg != agg || r.pres != pres) atomicAdd(a.self_check_failures, 1u);
  }
  a.out[i] = o;
}

hipError_t launch_sim_place(const SimPlaceArgs &a, hipStream_t s) {
  if (a.n > 0) hipLaunchKernelGGL(k_sim_place, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mapa
