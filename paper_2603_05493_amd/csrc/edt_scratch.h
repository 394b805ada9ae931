// Scratch array of the allocation-free distance transform (edt_scratch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace wb {

// Device address and size in bytes of the scratch array on the current
// device; the address is looked up once per device and cached.
hipError_t edt_scratch_address(int32_t **out, size_t *bytes);

}  // namespace wb
