// Host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "hpt_types.hpp"

namespace hpt {

hipError_t launch_raygen(const BatchDev &B, hipStream_t st);
// One interaction for every ray in queue q: closest hit, then shading into queue q^1.
hipError_t launch_bounce(const BatchDev &B, int q, hipStream_t st);
hipError_t launch_accumulate(const BatchDev &B, uint32_t tb, bool has_f64, bool has_f32, hipStream_t st);
hipError_t launch_cache_reduce(const BatchDev &B, hipStream_t st);
hipError_t launch_grf(double2 *spec, double2 *rows, float2 *table, uint32_t gw, uint32_t gh, uint32_t T,
                      uint64_t seed, double scale, hipStream_t st);

}  // namespace hpt
