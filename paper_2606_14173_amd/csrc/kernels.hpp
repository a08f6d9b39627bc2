// Host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "hpt_types.hpp"

namespace hpt {

// uni: the batch has one job and at most shade_lds_units() units
hipError_t launch_raygen(const BatchDev &B, bool uni, hipStream_t st);
// One interaction for every ray in queue q: closest hit (trace), then
// shading that compacts continuing rays into queue q^1 (shade).
// Fails (hipErrorInvalidValue) if the batch's stack spill is too small.
// dense: queue q is the first queue (ray generation order), else it is read
// through its index list.
hipError_t launch_trace(const BatchDev &B, int q, bool dense, bool count, hipStream_t st);
// After the shading pass over queue q: prefix sums of the per-chunk counts
// of queue q^1, its ray count and its index list.
hipError_t launch_compact(const BatchDev &B, int q, hipStream_t st);
// Workgroups and threads per workgroup of a traversal launch for a batch of
// n_paths (they size the stack spill).
uint32_t trace_grid(uint32_t n_paths);
uint32_t trace_block();
// first: queue from k_raygen; ext: the batch's jobs use next-event estimation
// or principled materials (extended shading kernel); uni: the batch has one
// job, at most shade_lds_mats() materials and at most shade_lds_units() units
// shading pass `pass` (0: the first, over ray generation's queue)
hipError_t launch_shade(const BatchDev &B, int q, uint32_t pass, bool ext, bool uni, hipStream_t st);
uint32_t shade_lds_mats();
uint32_t shade_lds_units();
// accumulation lanes [lane0, lane_end) of the batch
hipError_t launch_accumulate(const BatchDev &B, bool has_f64, bool has_f32, uint32_t lane0, uint32_t lane_end,
                             hipStream_t st);
hipError_t launch_cache_reduce(const BatchDev &B, hipStream_t st);
// Point-emitter terms of the batch's hologram units that start at sample 0
// (added to the field; run after the batch's accumulation, on its stream).
// max_pn: the largest pixel count of a unit in the batch.
hipError_t launch_points(const BatchDev &B, uint32_t max_pn, hipStream_t st);
hipError_t launch_grf(double2 *spec, double2 *rows, float2 *table, uint32_t gw, uint32_t gh, uint32_t T,
                      uint64_t seed, double scale, hipStream_t st);

}  // namespace hpt
