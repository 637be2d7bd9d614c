// k_enumerate for one-word rows with pair_level up to 12 free vertices.
#include "enumerate.h"

namespace mapa {

hipError_t upload_tables_enum_pair12(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

hipError_t launch_enum_pair12(const BatchArgs &a, hipStream_t s) {
  return a.rows_in_lds ? launch_enum_t<1, true, 12>(a, s) : launch_enum_t<1, false, 12>(a, s);
}

int occ_enum_pair12(int rows_in_lds, int threads, size_t lds_bytes) {
  return rows_in_lds ? occ_t<1, true, 12>(threads, lds_bytes) : occ_t<1, false, 12>(threads, 0);
}

}  // namespace mapa
