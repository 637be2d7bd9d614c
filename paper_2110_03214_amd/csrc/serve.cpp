// Serving loop of the MAPA allocation library (continuous batching).
#include "ctx.h"

namespace mapa {

void serve_teardown(mapa_ctx *c) { (void)c; }

}  // namespace mapa
