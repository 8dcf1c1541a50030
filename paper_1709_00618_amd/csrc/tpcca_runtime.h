// Hooks of the context runtime used by the server (GPU library internal).
#pragma once
#include <hip/hip_runtime.h>

#include "tpcca.h"

namespace tpcca {
hipStream_t ctx_stream(tpcca_ctx_t *c);
size_t ctx_allocated(tpcca_ctx_t *c);
}  // namespace tpcca
