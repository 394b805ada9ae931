// Launcher of the exact distance transform of a site grid (edt.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace wb {

// sites [nz][ny][nx] uint8; nearest [nz][ny][nx] packed sites (required:
// the last pass writes it); dist [nz][ny][nx] or null; A and B hold
// nx * ny * nz ints each.
hipError_t launch_edt(int nx, int ny, int nz, const uint8_t *sites, float voxel_size, int32_t *nearest, float *dist,
                      int32_t *A, int32_t *B, hipStream_t s);

}  // namespace wb
