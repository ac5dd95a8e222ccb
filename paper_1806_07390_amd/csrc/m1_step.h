// m1_step.h -- tiling of the fused step kernel (m1_step.hip); internal to libfornax_m1.
#pragma once

#include <hip/hip_runtime.h>

#include "m1_internal.h"

namespace fm1 {

// Tile of TXB x TYB zone columns (TYB = 1 unless 3-D) and GB groups per block, TM planes along
// the march direction.  Returns a tile with nblocks = 0 when the combination is invalid
// (thread count, halo slots, LDS budget).
Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM, int GB);
Tile choose_tile(const fornax_m1_desc& D, bool all_groups);
// Raise the dynamic LDS limit of every step-kernel instantiation (once per process).
int prepare_step_kernels();

template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, const Tile& tl, hipStream_t st);

}  // namespace fm1
