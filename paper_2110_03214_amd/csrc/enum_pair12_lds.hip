// k_enumerate for one-word rows with pair_level up to 12 free vertices,
// topology rows staged in LDS.
#include "enumerate.h"

namespace mapa {

hipError_t upload_tables_enum_pair12_lds(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

hipError_t launch_enum_pair12_lds(const BatchArgs &a, hipStream_t s) {
  return launch_enum_t<1, true, 12>(a, s);
}

int occ_enum_pair12_lds(int threads, size_t lds_bytes) {
  return occ_t<1, true, 12>(threads, lds_bytes);
}

}  // namespace mapa
