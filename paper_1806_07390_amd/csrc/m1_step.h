// m1_step.h -- tiling of the fused step kernel (m1_step.hip); internal to libfornax_m1.
#pragma once

#include <hip/hip_runtime.h>

#include "m1_internal.h"

namespace fm1 {

Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM);
bool halo_slots_fit(const Tile& tl, int dim);
Tile choose_tile(const fornax_m1_desc& D, size_t rsize);
size_t tile_lds_bytes(const Tile& tl, int dim, int G, size_t rsize, bool dz);

template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, const Tile& tl, hipStream_t st);

}  // namespace fm1
