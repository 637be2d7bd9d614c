// Job-trace simulation (mapa_simulate): the layout shared by its host loop
// (simulate.cpp) and its scoring kernel (simulate.hip).  Not part of the
// public ABI.
#pragma once

#include "mapa_internal.h"

namespace mapa {

// One round of placements.
struct SimEntry {          // one simulation's queue head, placed this round
  int32_t server;
  int32_t qi;              // its result in the round's query batch; -1: lowest free ids
  uint32_t busy_before;    // the server's busy mask before the placement
  uint8_t k, pad[3];
  unsigned long long nbtab;  // byte p: pattern positions before p that neighbour it
};
struct SimOut {            // the placement and its scores at its start
  uint32_t mask;
  uint8_t mapping[8];
  int32_t agg, pres, effbw_milli, links;
};
struct SimPlaceArgs {
  const SimEntry *entries;  // pinned host memory
  int32_t n;
  const mapa_result *qres;  // pinned host memory
  SimOut *out;              // pinned host memory
  const int32_t *server_topo;
  const int32_t *topo_n;
  const uint8_t *topo_W;    // [T][16][16]
  const int32_t *eff_key;   // [kEffEntries], see eff_off
  uint32_t *busy;
  uint32_t *self_check_failures;
};
hipError_t launch_sim_place(const SimPlaceArgs &a, hipStream_t s);

}  // namespace mapa
