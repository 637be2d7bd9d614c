// k_enumerate without pair_level: rows of 1, 2 or 4 words.
#include "enumerate.h"

namespace mapa {

hipError_t upload_tables_enum_plain(const Tables &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab), &t, sizeof(Tables));
}

hipError_t launch_enum_plain(const BatchArgs &a, hipStream_t s) {
  const bool lds = a.rows_in_lds != 0;
  switch (a.wpr) {
    case 1: return lds ? launch_enum_t<1, true, 0>(a, s) : launch_enum_t<1, false, 0>(a, s);
    case 2: return lds ? launch_enum_t<2, true, 0>(a, s) : launch_enum_t<2, false, 0>(a, s);
    default: return lds ? launch_enum_t<4, true, 0>(a, s) : launch_enum_t<4, false, 0>(a, s);
  }
}

int occ_enum_plain(int wpr, int rows_in_lds, int threads, size_t lds_bytes) {
  const bool l = rows_in_lds != 0;
  switch (wpr) {
    case 1: return l ? occ_t<1, true, 0>(threads, lds_bytes) : occ_t<1, false, 0>(threads, 0);
    case 2: return l ? occ_t<2, true, 0>(threads, lds_bytes) : occ_t<2, false, 0>(threads, 0);
    default: return l ? occ_t<4, true, 0>(threads, lds_bytes) : occ_t<4, false, 0>(threads, 0);
  }
}

}  // namespace mapa
