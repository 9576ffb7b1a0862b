// Serving loop (continuous batching of mapping jobs).
#include "em_runtime.h"

namespace em {

void serve_stop(Ctx &) {}

}  // namespace em
