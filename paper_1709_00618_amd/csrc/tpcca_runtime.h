// Hooks of the context runtime used by the server (GPU library internal).
#pragma once
#include <hip/hip_runtime.h>

#include "tpcca.h"

#include <mutex>

namespace tpcca {
hipStream_t ctx_stream(tpcca_ctx_t *c);
size_t ctx_allocated(tpcca_ctx_t *c);
// Held by every call that may synchronise the device (allocation, release,
// stream and context set-up) and by graph capture, so that no capture on
// one thread meets such a call from another.
std::recursive_mutex &device_ops_lock();
// The knob ranges tpcca_set_tuning accepts (n_rows bounds the row bands).
bool tuning_valid(const tpcca_tuning_t *t, int n_rows);
}  // namespace tpcca
