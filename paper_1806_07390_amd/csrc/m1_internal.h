// m1_internal.h -- types shared by the host side (m1_host.cpp) and the kernels (m1_kernels.hip)
// of libfornax_m1.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "fornax_m1.h"

namespace fm1 {

constexpr int NG = 2;            // ghost layers of linear reconstruction
constexpr int BLOCK = 256;       // threads per block of the zone-group kernels

// Geometry tables (device), per axis over the extended zone range e = i + NG,
// i in [-NG, n + NG); face tables over e in [0, n + 2 NG] (face e is x_{i-1/2}).
// Weights of the parabolic reconstruction per zone (spherical grids): face states of the
// parabola with the three averages (lower: 0..2, upper: 3..5, on q_{i-1}, q_i, q_{i+1}), its
// linear and quadratic coefficients (6..8, 9..11), those of the parabola through the face
// states and the average (12..14, 15..17, on v_lo, q_i, v_hi), and the reset face states with
// zero slope at the lower face (18, 19 on q_i, v_hi) and at the upper face (20, 21 on v_lo, q_i).
constexpr int PPM_TAB = 22;

template <typename R>
struct Geo {
  const R* idm[3];   // 1 / (X_i - X_{i-1}), X = volume centroid <x^d>
  const R* idp[3];   // 1 / (X_{i+1} - X_i)
  const R* dlo[3];   // x_{i-1/2} - X_i
  const R* dhi[3];   // x_{i+1/2} - X_i
  const R* iW[3];    // 1 / (integral of the x^d factor of sqrt(g) over the zone)
  const R* wf[3];    // x^d factor of sqrt(g) at face e (exactly 0 on a polar-axis face)
  const R* idc[3];   // 1 / (X_{i+1} - X_{i-1}) (MC limiter)
  const double* Wd[3];  // zone volume factors in double (energy accounting)
  // spherical (x1 = ln r, x2 = theta) only
  const R* rc;       // axis 0: r at the zone's coordinate centre
  const R* rf;       // axis 0: r at face e
  const R* hr;       // axis 0: sqrt(<r^2>) (cell-centred h_1 = h_2)
  const R* sc;       // axis 1: |sin theta| at the coordinate centre
  const R* sf;       // axis 1: |sin theta| at face e
  const R* hs;       // axis 1: sqrt(<sin^2 theta>)  (h_3 = hr * hs)
  const R* gam;      // axis 1, active zones j: <Gamma^3_23>, <Gamma^1_33>, <Gamma^2_33>, <Gamma^2_22>
  const R* irc;      // 1 / rc, 1 / rf, 1 / sc, 1 / sf (0 where sf = 0), 1 / hr, 1 / hs
  const R* irf;
  const R* isc;
  const R* isf;
  const R* ihr;
  const R* ihs;
  // spherical grids with the parabolic reconstruction: per axis and extended zone, PPM_TAB
  // weights in the zone's coordinate u = (x - x_i)/dx (see build_geometry), else null
  const R* ppm[3];
  R dx[3];           // coordinate spacing
  R idx[3];          // 1 / dx
};

// Host-side copy of the tables in double (the source of both device copies).
struct HostGeo {
  int n[3];
  std::vector<double> idm[3], idp[3], dlo[3], dhi[3], iW[3], W[3], wf[3], idc[3];
  std::vector<double> rc, rf, hr, sc, sf, hs, gam;
  std::vector<double> irc, irf, isc, isf, ihr, ihs;   // inverses (0 for a zero entry)
  std::vector<double> ppm[3];
  double dx[3];
};

struct StepArgsBase {
  int n[3];
  int G, ndim;
  int bc_lo[3], bc_hi[3];
  // ghost sources per axis for the indices -2, -1, n, n + 1: the source zone index and
  // flags (bit 0: flip the normal flux, bit 1: inflow state, bit 2: polar-axis copy)
  int gsrc[3][4], gfl[3][4];
  int limiter, closure;
  int wavespeed;             // FORNAX_WAVESPEED_*
  int zones_per_block;
  int64_t nzones;
  double c, dt;
  double f2_fp64;            // (f_fp64)^2, MIXED only
  const double* inflow;      // [G][1+ndim] or null
};

// Ghost rules (periodic wrap, outflow / inflow edge copy, reflect / axis mirror) of the two
// ghost layers on both sides of every axis.
inline void fill_ghost_table(StepArgsBase& a) {
  for (int d = 0; d < 3; ++d) {
    const int n = a.n[d];
    for (int k = 0; k < 4; ++k) {
      const int e = (k < 2) ? k - 2 : n + (k - 2);
      const bool low = e < 0;
      const int bc = low ? a.bc_lo[d] : a.bc_hi[d];
      int src = 0, fl = 0;
      if (bc == FORNAX_BC_PERIODIC) {
        src = low ? e + n : e - n;
        while (src < 0) src += n;
        while (src >= n) src -= n;
      } else if (bc == FORNAX_BC_OUTFLOW || bc == FORNAX_BC_INFLOW) {
        src = low ? 0 : n - 1;
        fl = (bc == FORNAX_BC_INFLOW) ? 2 : 0;
      } else {
        src = low ? -1 - e : 2 * n - 1 - e;
        if (src < 0) src = 0;
        if (src > n - 1) src = n - 1;
        fl = (bc == FORNAX_BC_AXIS) ? 5 : 1;
      }
      a.gsrc[d][k] = src;
      a.gfl[d][k] = fl;
    }
  }
}

template <typename S>
struct StepArgs : StepArgsBase {
  const S* E;
  const S* F[3];
  S* Eo;
  S* Fo[3];
  const S* kap;
  const S* sig;
  const S* B;
  double* dEm;               // per zone, nullable
  double* dzp;               // [group block][zone] partials of dE_matter (tiles with ngb > 1)
  // Runge-Kutta stages: src = 0 writes U^- itself (no interaction update); Ea, Fa (nullable)
  // replace U^- by (Ua + U^-) / 2 before the interaction update
  int src;
  const S* Ea;
  const S* Fa[3];
  // per-block partial reductions (null: no diagnostics), summed by a second launch
  double* p_energy;
  double* p_maxf2;
  int* p_nun;
  int* p_nnp;
};

// The prescribed velocity of the velocity step: coordinate components on the faces of each
// direction, the group edges; Fn (nullable): the flux components of U^n, given when the
// transport of Step 1 ran without the zone-local velocity terms of the flux rows, which the
// frequency step then adds.
template <typename S>
struct VelArgs {
  const S* v[3];      // [ND][faces_d]: coordinate components on the d-faces
  const double* nu;   // [G + 1] group edges
  const S* Fn[3];
};

}  // namespace fm1

namespace fm1 {
struct Tile {
  int TXB, TYB;        // zone columns per block in x and in y (y: 3-D only, else 1)
  int TM;              // planes per block along the march direction (1 for 1-D)
  bool row;            // 1-D/2-D wave rows (else one tile unit per block)
  int V;               // groups per lane (1, or 2: pairs of consecutive groups)
  int GB;              // groups per tile unit (a divisor of G; wave rows: a power of two)
  int NW;              // 1-D/2-D: wavefronts (tile units) per block, each a group subset; 3-D: 1
  int ntx, nty, ntm;   // tiles per direction
  int ngb;             // G / (GB NW): blocks per tile
  int nblocks;
  int xq, xr;          // nblocks = 8 xq + xr (XCD renumbering)
  int nthreads;        // 64 NW (1-D/2-D) or TXB * TYB * GB (3-D)
  size_t lds;          // dynamic LDS bytes per block (with the dE_matter buffer)
};
// Tiling of the 3-D Cartesian step kernel for group counts that are multiples of 4
// (m1_step_3d.hip): blocks of NR waves, one y row of 16 x columns by 4 groups each (rows 0 and
// NR - 1 and columns 0 and 15 are halo), TM planes along z, ngb = G / 4 blocks per tile.
struct C3Tile {
  int NR, TM;
  int ntx, nty, ntz, ngb, nblocks;
  int xq, xr;
};
// Tiling of the 2-D, 16-group step kernel that streams whole zones through LDS
// (m1_step_rows.hip): NWX wave rows of 16 zone columns (4 NWX waves), TM planes per block.
struct RowsTile {
  int NWX, TXB, TM;
  int ntx, ntm, nblocks;
  int xq, xr;
  int nthreads;
  size_t lds;          // static LDS bytes per block
};
}  // namespace fm1

struct fornax_m1_ctx {
  fornax_m1_desc desc;
  int device;
  fm1::HostGeo hgeo;
  fm1::Geo<double> geo_d;
  fm1::Geo<float> geo_f;
  void* geo_mem;              // one allocation holding every device table
  size_t geo_bytes;
  double max_dt1;             // max_dt(cfl = 1)
  fm1::Tile tile;              // tiling of the fused step kernel
  fm1::Tile tile_v1;           // one group per lane (arrays not aligned to pairs of groups)
  fm1::RowsTile rows;          // the whole-zone LDS kernel when nblocks > 0 (2-D, 16 groups)
  fm1::C3Tile c3;              // the 3-D Cartesian kernel when nblocks > 0
  fm1::C3Tile c3v;             // the same kernel's tiling for Step 1 of the velocity step
  int cus;                     // compute units of the device (0 if unknown)
  fm1::Tile last_tile[1];      // the tile of the last step launch (for inspection)
  // reduction scratch (one partial per block of the step kernel)
  int nblocks_step;
  size_t nb_partials;          // partials the step kernels may write (the most blocks of any)
  double* p_energy;
  double* p_maxf2;
  int* p_nun;
  int* p_nnp;
  // dE_matter partials of the group blocks of a tile, [ngb][zones] (null when every tile
  // holds all groups of a zone)
  double* dzp;
  // SSP-RK2: the first stage's state U* (E, F_1..F_ndim), null for the Euler push
  void* stage_mem;
  // adjoint: ghost-zone adjoint buffers per direction, [side][layer][plane][G][1+ndim+1]
  double* adj_gbuf[3];
  int adj_gplane[3];
  int adj_txb, adj_tm;        // adjoint tiling override (0: the default choice)
  // matter model (fornax_m1_set_matter_model): device tables nu_edge [G+1], nu_c [G], kg [G]
  double* mat_tab;
  double mat_a, mat_tol;
  int mat_maxn;
  // group edges of the velocity step (fornax_m1_set_group_edges): device table [G + 1]
  double* vel_nu;
};

// Scratch memory of one step launch: per-block diagnostics partials, the dE_matter partials of
// split group blocks, the first Runge-Kutta stage.
struct StepScratch {
  double* p_energy;
  double* p_maxf2;
  int* p_nun;
  int* p_nnp;
  double* dzp;
  void* stage;
};

// kernel launchers (m1_kernels.hip)
int fm1_launch_step(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                    const fornax_m1_coeffs* cf, const double* inflow, double dt,
                    const fornax_m1_diag* diag, hipStream_t stream);
// the same step with its scratch in the library's static device array (no allocation), whose
// address fornax_m1_create set up on the context's device
int fm1_launch_step_noalloc(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                            const fornax_m1_coeffs* cf, const double* inflow, double dt,
                            const fornax_m1_diag* diag, hipStream_t stream);
// address of the static scratch array on a device (hipGetSymbolAddress, once per device, the
// device current); FORNAX_OK or FORNAX_EDEVICE
int fm1_static_scratch_setup(int device);
int fm1_launch_flux(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_coeffs* cf,
                    const double* inflow, void* face_flux[3], hipStream_t stream);
int fm1_launch_source(fornax_m1_ctx* ctx, fornax_m1_state* inout, const fornax_m1_coeffs* cf,
                      double dt, double* dEm, hipStream_t stream);
int fm1_launch_adjoint(fornax_m1_ctx* ctx, const fornax_m1_state* Un, const fornax_m1_state* Unp1,
                       const fornax_m1_coeffs* cf,
                       const double* inflow, double dt, const fornax_m1_state* lam_np1,
                       fornax_m1_state* lam_n, void* dkappa, hipStream_t stream);
int fm1_launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t stream);
// the diagnostics totals of a step from nb per-block partials (fixed order, deterministic)
int fm1_launch_finalize(const double* p_energy, const double* p_maxf2, const int* p_nun, const int* p_nnp, int nb,
                        const fornax_m1_diag* diag, hipStream_t stream);
int fm1_launch_transport(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                         const fornax_m1_coeffs* cf, const double* inflow, double dt, hipStream_t stream);
// m1_velocity.hip
int fm1_launch_step_velocity(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                             const fornax_m1_coeffs* cf, const double* inflow, const fornax_m1_velocity* vel,
                             double dt, const fornax_m1_diag* diag, hipStream_t stream);
int fm1_launch_lab_frame(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_velocity* vel,
                         double* E_lab, double* const* F_lab, hipStream_t stream);
namespace fm1 {
// the kernel arguments common to every step launch (m1_kernels.hip)
template <typename S>
void fill_args(const fornax_m1_ctx* ctx, StepArgs<S>& a, const fornax_m1_coeffs* cf, const double* inflow,
               double dt);
}  // namespace fm1
// m1_matter.hip
int fm1_launch_matter_coeffs(fornax_m1_ctx* ctx, const fornax_m1_matter* m, void* kap, void* B,
                             hipStream_t stream);
int fm1_launch_matter_source(fornax_m1_ctx* ctx, fornax_m1_state* io, const void* sigma,
                             const fornax_m1_matter* m, double dt, double* dEm, int* iters,
                             hipStream_t stream);
