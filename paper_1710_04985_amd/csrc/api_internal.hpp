// Library-internal entry points shared between the C ABI sources.
#pragma once

#include <cstdint>

#include "sptrsv.h"

namespace sptrsv {

// sptrsv_solve with the position-ordered solution kept in the caller-side
// buffer xp (xp_bytes of device memory on the handle's device) instead of the
// handle's own, and no allocation of any kind: work tables that the current
// schedule needs and that do not exist yet give kErrNotSupported, a schedule
// that needs more than xp_bytes gives kErrTooLarge.  Serialized with the
// handle's other calls like sptrsv_solve.
int solve_external_scratch(sptrsv_handle_t h, const void* b, void* x, void* xp, int64_t xp_bytes,
                           hipStream_t s);

// Device the handle was analysed on.
int handle_device(sptrsv_handle_t h);

}  // namespace sptrsv
