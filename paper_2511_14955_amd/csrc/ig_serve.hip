// Serving loop (continuous batching of featurize / count requests).
#include "ig_internal.h"

namespace ig {
void serve_teardown(ig_ctx *c) { (void)c; }
}  // namespace ig
