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

// Launch the step kernel with the context's tile for these arguments (the whole-zone kernel
// when the context has one; single groups per lane when an array is not aligned to two
// elements).
template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, hipStream_t st);

// The 2-D, 16-group kernel with whole-zone transfers through LDS (m1_step_rows.hip): a tile
// with nblocks = 0 when the grid does not qualify (2-D Cartesian, 16 groups, arrays under
// 2 GiB; NWX = 1; TM >= 3).
RowsTile make_rows_tile(const fornax_m1_desc& D, int NWX, int TM);
RowsTile choose_rows_tile(const fornax_m1_desc& D, int cus);
template <typename S>
int launch_rows(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, hipStream_t st);

// The 3-D kernel with x neighbours by lane shifts and y neighbours through LDS
// (m1_step_3d.hip): a tile with nblocks = 0 when the grid does not qualify (3-D, groups a
// multiple of 4; Cartesian without inflow or axis boundaries, or spherical with inflow at the
// inner radius and polar axes over a periodic phi of even length; NR 6, 8 or 12 in double,
// 4, 8 or 16 in float, 8 (double) or 4, 8 and 12 (float) on spherical grids).
C3Tile make_c3_tile(const fornax_m1_desc& D, int NR, int TM);
// the step's tiling, and Step 1 of the velocity step's (planes per block from the CU count)
C3Tile choose_c3_tile(const fornax_m1_desc& D, int cus);
C3Tile choose_c3_vel_tile(const fornax_m1_desc& D, int cus);
template <typename S>
int launch_c3(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, hipStream_t st);
// Step 1 of the velocity step on the same kernel (3-D Cartesian grids it takes; StepArgs without
// interaction update or diagnostics); FORNAX_EUNSUPPORTED when the grid does not qualify.
template <typename S>
int launch_c3_vel(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, const VelArgs<S>& va, hipStream_t st);

}  // namespace fm1
