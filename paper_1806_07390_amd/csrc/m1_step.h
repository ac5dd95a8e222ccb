// m1_step.h -- tiling of the fused step kernel (m1_step.hip); internal to libfornax_m1.
#pragma once

#include <hip/hip_runtime.h>

#include "m1_internal.h"

namespace fm1 {

// Tile of TXB x TYB zone columns and GB groups per unit, TM planes along the march direction;
// in 1-D/2-D a unit is one wavefront (TXB = 64/GB, TYB = 1) and a block holds NW units.
// Returns a tile with nblocks = 0 when the combination is invalid (thread count, halo slots,
// LDS budget).
Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM, int GB, int NW, int V);
Tile choose_tile(const fornax_m1_desc& D, int V);
// Raise the dynamic LDS limit of every step-kernel instantiation (once per process).
int prepare_step_kernels();

// Launch the step kernel with the context's tile for these arguments (all groups per block
// when dE_matter is asked for; single groups per lane when an array is not aligned to two
// elements).
template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, hipStream_t st);

}  // namespace fm1
