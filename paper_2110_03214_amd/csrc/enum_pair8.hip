// k_enumerate for one-word rows with pair_level up to 8 free vertices.
#include "enumerate.h"

namespace mapa {

hipError_t upload_tables_enum_pair8(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

hipError_t launch_enum_pair8(const BatchArgs &a, hipStream_t s) {
  return a.rows_in_lds ? launch_enum_t<1, true, 8>(a, s) : launch_enum_t<1, false, 8>(a, s);
}

int occ_enum_pair8(int rows_in_lds, int threads, size_t lds_bytes) {
  return rows_in_lds ? occ_t<1, true, 8>(threads, lds_bytes) : occ_t<1, false, 8>(threads, 0);
}

}  // namespace mapa
