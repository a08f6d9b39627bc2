// Host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "hpt_types.hpp"

namespace hpt {

hipError_t launch_raygen(const BatchDev &B, hipStream_t st);
// One interaction for every ray in queue q: closest hit (trace), then
// shading that compacts continuing rays into queue q^1 (shade).
// depth: the deepest BVH among the batch's scenes (sizes the LDS stack).
hipError_t launch_trace(const BatchDev &B, int q, bool count, uint32_t depth, hipStream_t st);
hipError_t launch_shade(const BatchDev &B, int q, hipStream_t st);
hipError_t launch_accumulate(const BatchDev &B, bool has_f64, bool has_f32, hipStream_t st);
hipError_t launch_cache_reduce(const BatchDev &B, hipStream_t st);
hipError_t launch_grf(double2 *spec, double2 *rows, float2 *table, uint32_t gw, uint32_t gh, uint32_t T,
                      uint64_t seed, double scale, hipStream_t st);

}  // namespace hpt
