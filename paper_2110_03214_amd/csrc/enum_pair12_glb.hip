// k_enumerate for one-word rows with pair_level up to 12 free vertices,
// topology rows read from global memory.
#include "enumerate.h"

namespace mapa {

hipError_t upload_tables_enum_pair12_glb(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

hipError_t launch_enum_pair12_glb(const BatchArgs &a, hipStream_t s) {
  return launch_enum_t<1, false, 12>(a, s);
}

int occ_enum_pair12_glb(int threads, size_t lds_bytes) {
  (void)lds_bytes;
  return occ_t<1, false, 12>(threads, 0);
}

}  // namespace mapa
