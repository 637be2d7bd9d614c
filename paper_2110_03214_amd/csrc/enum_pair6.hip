// k_enumerate for one-word rows with pair_level up to 6 free vertices (the
// contexts of topologies of at most 9 vertices: wider pair levels are rare
// there and their registers cost the whole kernel more than they save).
#include "enumerate.h"

namespace mapa {

hipError_t upload_tables_enum_pair6(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

hipError_t launch_enum_pair6(const BatchArgs &a, hipStream_t s) {
  return a.rows_in_lds ? launch_enum_t<1, true, 6>(a, s) : launch_enum_t<1, false, 6>(a, s);
}

int occ_enum_pair6(int rows_in_lds, int threads, size_t lds_bytes) {
  return rows_in_lds ? occ_t<1, true, 6>(threads, lds_bytes) : occ_t<1, false, 6>(threads, 0);
}

}  // namespace mapa
