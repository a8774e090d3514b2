// Serving loop (placeholder until the continuous-batching scheduler lands).
#include "runtime_internal.h"

namespace xs {

void serve_shutdown(Ctx*) {}

}  // namespace xs
