// m1_step_3d.hip -- the fused M1 step for 3-D grids whose group count is a multiple of 4: the
// Cartesian 192^3 x 12 workload's layout, and spherical (ln r, theta, phi) grids with an inflow
// inner boundary, polar axes and periodic phi (the 256 x 64 x 128 x 20 workload).
//
// Same method and arithmetic as k_step_tiled (eq:finite_vol with the reconstruction of
// eq:recon_constraints, the M1 closure, the HLL flux eq:hll with the correction eq:epsilon, the
// backward-Euler interaction update eq:be_update); what differs is how neighbours meet:
//   * a wave is one y row of 16 x columns by 4 consecutive groups, lane = 16 group + column:
//     the x neighbours of a lane are the lanes next to it in its 16-lane row, reached by DPP
//     row shifts (no LDS, no barrier).  Columns 0 and 15 are halo: their zones are
//     reconstructed (their face states close the tile) but not updated, and their own outer
//     neighbours are loaded by those two lanes;
//   * a block is NI waves stacked in y and one group quad.  Each row computes the flux at its
//     lower y face from its own reconstruction and that of the row below, both from the
//     plane's states in LDS.  With AR (all rows) the NI rows are updated and the top row also
//     computes the flux at the block's upper face (from the reconstruction of the row above;
//     two rows above the block in LDS); without (the float blocks of 8 and 16 rows, whose
//     register budget at four waves per SIMD has no room for the extra loads) the lower NI - 1
//     rows are updated and the top row only computes the flux at its lower face (its zones are
//     the next tile's first row; one row above the block in LDS).
//     The two rows below the block and those above it are loaded into LDS by all waves
//     together.  The fluxes pass through LDS;
//   * the block marches along z over TM planes with a register window: every z face is
//     computed once, from values each lane loads for its own column one plane ahead;
//   * x faces are computed once (by the lane above the face), y faces once per block (the
//     lower row's upper state is recomputed by the row above instead of exchanged), z faces
//     once; only the halo columns and the faces between tiles repeat work of the neighbouring
//     tiles.
// One block barrier per plane (after the states), which waits for LDS only: the loads of the
// next plane stay in flight.  The update of a plane follows the next plane's barrier.
// With VEL (Cartesian grids), Step 1 of the velocity step: the same transport without the
// interaction update, each face flux with the advective flux v^d U of the upwind face state
// added (the face's left state where v^d >= 0), from the normal velocity component on the face;
// the zone-local velocity terms of the flux rows follow in the frequency step.
// Spherical grids (SPH): the same structure with the geometry of the lane's zone from the
// per-axis tables (volume-coordinate slopes, face scale factors for the realizability checks and
// the fluxes, face weights and zone widths for the divergence, proper widths for the optical
// depth; the radial values of the block's columns staged in LDS once, the theta values of the
// wave's row read by scalar loads), the geometric source terms after the divergence, theta faces on the polar axis
// closed; a polar-axis ghost row takes the mirrored row of the plane n_phi/2 away (with F_theta
// and F_phi flipped), and an inflow ghost column the prescribed state with its own scale
// factors.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

constexpr int C3_TX = 16;   // x columns of a wave row (14 updated)

// the value of the lane one column lower (row_shr:1) / higher (row_shl:1) in the same 16-lane
// row; the lanes at the row's ends receive 0 (bound_ctrl: they never use it, and no register
// has to be cleared first)
template <typename R>
__device__ __forceinline__ R col_prev(R v) {
  return __builtin_amdgcn_update_dpp(R(0), v, 0x111, 0xf, 0xf, true);
}
template <typename R>
__device__ __forceinline__ R col_next(R v) {
  return __builtin_amdgcn_update_dpp(R(0), v, 0x101, 0xf, 0xf, true);
}

// v of this lane plus v of the lane 16 (S = 16) or 32 (S = 32) apart, by the row swaps of
// gfx950 (VALU; the lane sums are formed in the same order as a shuffle sum would)
template <int S>
__device__ __forceinline__ double lane_pair_sum(double v) {
  struct W {
    unsigned lo, hi;
  };
  const W w = __builtin_bit_cast(W, v);
  W a, b;
  if constexpr (S == 16) {
    const auto l = __builtin_amdgcn_permlane16_swap(w.lo, w.lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(w.hi, w.hi, false, false);
    a = W{l[0], h[0]};
    b = W{l[1], h[1]};
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(w.lo, w.lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(w.hi, w.hi, false, false);
    a = W{l[0], h[0]};
    b = W{l[1], h[1]};
  }
  return __builtin_bit_cast(double, a) + __builtin_bit_cast(double, b);
}

// the advective flux v U of the upwind face state added to a face flux (the left state where
// v >= 0)
template <typename R>
__device__ __forceinline__ void add_upwind(R v, const R qL[4], const R qR[4], R flux[4]) {
  const bool left = v >= R(0);
  for (int c = 0; c < 4; ++c) flux[c] += v * (left ? qL[c] : qR[c]);
}

// The ghost rules of one axis, taken from the launch's table at each use (measured: faster
// than copies of the table held in scalar registers for the whole kernel, which crowd out the
// other uniform values).
struct C3Axis {
  const StepArgsBase* a;
  int d;
};
template <int D>
__device__ __forceinline__ C3Axis c3_axis(const StepArgsBase& a) { return C3Axis{&a, D}; }
// Ghost rule of index e (clamped into -2 .. n + 1 first): source zone and flags (bit 0 flips
// the flux component along the axis), selected without indexing the table by a per-lane value.
__device__ __forceinline__ void c3_src(const C3Axis& ax, int e, int& src, int& fl) {
  const StepArgsBase& a = *ax.a;
  const int D = ax.d;
  const int n = a.n[D];
  e = e < -2 ? -2 : (e > n + 1 ? n + 1 : e);
  src = e;
  fl = 0;
  if (e < 0 || e >= n) {
    const int k = e < 0 ? e + 2 : e - n + 2;
    src = k == 0 ? a.gsrc[D][0] : k == 1 ? a.gsrc[D][1] : k == 2 ? a.gsrc[D][2] : a.gsrc[D][3];
    fl = k == 0 ? a.gfl[D][0] : k == 1 ? a.gfl[D][1] : k == 2 ? a.gfl[D][2] : a.gfl[D][3];
  }
}

// the sign rules: F_c flipped where bit c - 1 of the mask is set
template <typename R>
__device__ __forceinline__ void c3_fix(const R raw[4], int mask, R q[4]) {
  q[0] = raw[0];
  for (int c = 1; c < 4; ++c) q[c] = ((mask >> (c - 1)) & 1) ? -raw[c] : raw[c];
}

template <typename S, typename R>
__device__ __forceinline__ void c3_load(const StepArgs<S>& a, int off, R q[4]) {
  q[0] = R(a.E[off]);
  q[1] = R(a.F[0][off]);
  q[2] = R(a.F[1][off]);
  q[3] = R(a.F[2][off]);
}

// LDS barrier: waits for the wave's LDS operations only (the global loads of the next plane
// stay in flight); the empty asm statements keep the compiler from moving memory accesses
// across it
__device__ __forceinline__ void c3_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Rows of the plane held in LDS: the block's NI rows in slots 2 .. NI + 1, the two rows below
// in slots 0, 1 and those above in slots NI + 2 (and NI + 3 where every row is updated).  The
// outer rows are loaded by all waves together, one (slot, component) item per wave and load:
// the 4 state components of slot 0, the 4 state components, kappa and sigma of slot 1; above
// the block either those of slot NI + 2 and the 4 state components of NI + 3 (every row
// updated), or the 4 state components of slot NI + 2.
template <bool AR>
constexpr int c3_nitem() { return AR ? 20 : 14; }

// NI waves per block, W waves per SIMD (register budget 512 / W)
template <typename S, int NI, int W, int LIM, bool SPH, bool AR, bool VEL = false>
__global__ void __launch_bounds__(64 * NI) __attribute__((amdgpu_waves_per_eu(W)))
k_step_3d(StepArgs<S> a, Geo<S> geo, C3Tile tl, VelArgs<S> va) {
  using R = S;
  constexpr int TX = C3_TX;
  constexpr int NS = NI + (AR ? 4 : 3);                   // LDS row slots
  constexpr int NIT = c3_nitem<AR>();
  constexpr int NHI = (NIT + NI - 1) / NI;                // outer-row items per wave
  // double-buffered by plane parity: one barrier per plane (see the plane loop)
  __shared__ R QS[2][6][NS][64];    // E, F_x, F_y, F_z, kappa, sigma of the plane's rows
  __shared__ R FY[2][4][NI + AR][64];  // y flux at the lower face of each row (and the block's upper face)
  __shared__ double red_e[NI], red_m[NI];
  __shared__ int red_u[NI], red_p[NI];

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave = row (uniform)
  const int x = lane & (TX - 1), gq = lane >> 4;
  const int sw = w + 2;                                   // the wave's slot
  const bool top = w == NI - 1;
  const bool idle = !AR && top;          // a row that only computes its lower face flux

  // tile of the block (XCD-aware renumbering; the group quads of a tile adjacent)
  const int b = blockIdx.x;
  const int xcd = b & 7, sl = b >> 3;
  const int L = xcd * tl.xq + min(xcd, tl.xr) + sl;
  const int gb = L % tl.ngb;
  int rest = L / tl.ngb;
  const int tx = rest % tl.ntx;
  rest /= tl.ntx;
  const int ty = rest % tl.nty;
  const int tz = rest / tl.nty;

  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2], G = a.G;
  const int g = gb * 4 + gq;
  const int xz = tx * (TX - 2) + x - 1;          // zone of the lane's column
  const int y0 = ty * (AR ? NI : NI - 1);        // zone of slot 2
  const int yz = y0 + w;                         // zone of the wave's row
  const int mbeg = tz * tl.TM, mend = min(mbeg + tl.TM, n2);
  const bool upd = !idle && yz < n1 && x >= 1 && x <= TX - 2 && xz < n0;
  const int PL = n0 * n1 * G;                    // elements of a z plane

  const C3Axis ax0 = c3_axis<0>(a), ax1 = c3_axis<1>(a), ax2 = c3_axis<2>(a);
  // sources and sign rules of the lane's column and of its outer x neighbour (columns 0, 15)
  int xs, xf, ys, yf;
  c3_src(ax0, xz, xs, xf);
  c3_src(ax1, yz, ys, yf);
  const bool xedge = x == 0 || x == TX - 1;
  int xef;
  const int cb = (ys * n0 + xs) * G + g;
  int xeo;
  c3_src(ax0, x == 0 ? xz - 1 : xz + 1, xeo, xef);
  const int ceb = (ys * n0 + xeo) * G + g;
  // flip masks: bit c - 1 flips F_c; a polar-axis ghost row (flag bit 2) also flips F_phi
  const int lm = (xf & 1) | ((yf & 1) << 1) | (((yf >> 2) & 1) << 2);
  const int lme = (xef & 1) | ((yf & 1) << 1) | (((yf >> 2) & 1) << 2);
  // spherical grids: extended indices of the lane's zone for the geometry tables (clamped:
  // lanes outside the grid compute but never store), the phi shift of a polar-axis ghost row,
  // inflow ghosts (flag bit 1) of the lane's column and of its outer neighbour
  const int ex = SPH ? min(max(xz, -2), n0 + 1) + NG : 0;
  const int ey = SPH ? min(max(yz, -2), n1 + 1) + NG : 0;
  const int zsh = (SPH && ((yf >> 2) & 1)) ? n2 / 2 : 0;
  const bool xinf = SPH && ((xf >> 1) & 1), xinfe = SPH && ((xef >> 1) & 1);
  // B of the lane's own zone (clamped into the domain so every lane may load it)
  const int cbb = ((min(max(yz, 0), n1 - 1) * n0 + min(max(xz, 0), n0 - 1)) * G + g);
  // the wave's outer-row items: LDS slot and component (uniform), element offset within a
  // plane and flip of its row and column (per lane), the array (uniform)
  int hslot[NHI], hcomp[NHI], hoff[NHI], hmask[NHI], hsh[NHI], hey[NHI];
  const S* hsrc[NHI];
  for (int k = 0; k < NHI; ++k) {
    int it = w + k * NI;
    if (it >= NIT) it = -1;
    int slot = 0, comp = 0;
    if (it >= 0) {
      if (it < 4) { slot = 0; comp = it; }
      else if (it < 10) { slot = 1; comp = it - 4; }
      else if (!AR || it < 16) { slot = NI + 2; comp = it - 10; }
      else { slot = NI + 3; comp = it - 16; }
    }
    int hys, hyf;
    c3_src(ax1, y0 - 2 + slot, hys, hyf);
    hslot[k] = it >= 0 ? slot : -1;
    hcomp[k] = comp;
    hoff[k] = (hys * n0 + xs) * G + g;
    const int hm = (xf & 1) | ((hyf & 1) << 1) | (((hyf >> 2) & 1) << 2);
    hmask[k] = comp >= 1 && comp <= 3 ? ((hm >> (comp - 1)) & 1) : 0;
    hsh[k] = (SPH && ((hyf >> 2) & 1)) ? n2 / 2 : 0;
    hey[k] = min(max(y0 - 2 + slot, -2), n1 + 1) + NG;
    hsrc[k] = comp == 0 ? a.E : comp <= 3 ? a.F[comp - 1] : comp == 4 ? a.kap : a.sig;
  }
  // plane m (-2 .. n2 + 1, clamped): element offset and flip mask
  auto plane = [&](int m, int& pm) -> int {
    int zs, zf;
    c3_src(ax2, m, zs, zf);
    pm = (zf & 1) << 2;
    return zs * PL;
  };
  // plane m of a row shifted by sh in phi (a polar-axis ghost row: phi is periodic there)
  auto plane_s = [&](int m, int sh, int& pm) -> int {
    if (sh == 0) return plane(m, pm);
    pm = 0;
    int zz = (m + sh) % n2;
    if (zz < 0) zz += n2;
    return zz * PL;
  };
  // the inflow ghost state of zone (extended ex_, ey_): E and covariant F_k = h_k F^_k with the
  // ghost's own scale factors (spherical grids, inflow on x1 only)
  auto inflow_state = [&](int ex_, int ey_, R q[4]) {
    const double* in = a.inflow + g * 4;
    R h[3];
    cell_h<R, SPH>(geo, ex_, ey_, h);
    q[0] = R(in[0]);
    for (int c = 0; c < 3; ++c) q[1 + c] = h[c] * R(in[1 + c]);
  };

  const bool want_diag = a.p_energy != nullptr;
  ZoneDiag zd;
  const double cdt = a.c * a.dt;
  const R dtR = R(a.dt);
  const R idx0 = geo.idx[0], idx1 = geo.idx[1], idx2 = geo.idx[2];
  const R dx0 = geo.dx[0], dx1 = geo.dx[1], dx2 = geo.dx[2];
  const R hone[3] = {R(1), R(1), R(1)};
  const double Vz = want_diag ? (SPH ? geo.Wd[0][ex] * geo.Wd[1][ey] * geo.Wd[2][NG]
                                     : geo.Wd[0][NG] * geo.Wd[1][NG] * geo.Wd[2][NG])
                              : 0.0;
  // phi-face scale factors of the lane's column (the same for every plane) and the proper width
  // along phi; cell-centred h for the geometric source
  R hz[3] = {R(1), R(1), R(1)}, ihz[3] = {R(1), R(1), R(1)};
  R dlz = dx2;
  if constexpr (SPH) {
    face_h<R, SPH>(geo, 2, ex, ey, 0, hz);
    face_ih<R, SPH>(geo, 2, ex, ey, 0, ihz);
    dlz = proper_width<R, SPH>(geo, 2, ex, ey);
  }
  // spherical grids: the radial tables at the block's 16 columns, staged in LDS once (the first
  // plane's barrier orders the reads): the plane loop reads them from LDS rather than from the
  // tables (the theta tables, indexed by the wave's row, are scalar loads)
  enum { RG_IRC, RG_RC, RG_HR, RG_IHR, RG_IRF0, RG_IRF1, RG_RF, RG_IDM, RG_IDP, RG_DLO, RG_DHI, RG_IDC, RG_WF0,
         RG_WF1, RG_IW, RG_N };
  __shared__ R RGT[SPH ? RG_N : 1][TX];
  if constexpr (SPH) {
    if (w == 0 && gq == 0) {
      RGT[RG_IRC][x] = gld(geo.irc, ex);
      RGT[RG_RC][x] = gld(geo.rc, ex);
      RGT[RG_HR][x] = gld(geo.hr, ex);
      RGT[RG_IHR][x] = gld(geo.ihr, ex);
      RGT[RG_IRF0][x] = gld(geo.irf, ex);
      RGT[RG_IRF1][x] = gld(geo.irf, ex + 1);
      RGT[RG_RF][x] = gld(geo.rf, ex);
      RGT[RG_IDM][x] = gld(geo.idm[0], ex);
      RGT[RG_IDP][x] = gld(geo.idp[0], ex);
      RGT[RG_DLO][x] = gld(geo.dlo[0], ex);
      RGT[RG_DHI][x] = gld(geo.dhi[0], ex);
      RGT[RG_IDC][x] = gld(geo.idc[0], ex);
      RGT[RG_WF0][x] = gld(geo.wf[0], ex);
      RGT[RG_WF1][x] = gld(geo.wf[0], ex + 1);
      RGT[RG_IW][x] = gld(geo.iW[0], ex);
    }
  }
  auto rg = [&](int k) -> R { return RGT[SPH ? k : 0][x]; };

  // ---- register window along z: q(m), q(m + 1); the upper z face state of zone m and the
  // flux at m - 1/2; kappa and sigma of plane m ----
  R q0[4], q1[4], hiM[4], fPrev[4];
  R k0, s0;
  // values in flight: q(m + 2), the outer x neighbour (columns 0, 15) of plane m and the
  // wave's outer-row items of plane m, kappa, sigma of m + 1 (Pk, Ps) and B of m (PB), all
  // loaded at the top of the plane before (Pk2, Ps2, PB2: those of the next plane)
  R Pr[4], Po[4], Ph[NHI], Pk, Ps, PB, Pk2, Ps2, PB2;
  int Ppm, Popm;
  // the wave's outer-row items of plane m (element offset off of the unshifted plane m)
  auto load_items = [&](int off, int m) {
    for (int k = 0; k < NHI; ++k)
      if (hslot[k] >= 0) {
        int o = off;
        if (SPH && hsh[k] != 0) {
          int pmx;
          o = plane_s(m, hsh[k], pmx);
        }
        Ph[k] = R(hsrc[k][o + hoff[k]]);
        if (SPH && xinf && hcomp[k] <= 3) {
          R qi[4];
          inflow_state(ex, hey[k], qi);
          const int hc = hcomp[k];
          Ph[k] = hc == 0 ? qi[0] : hc == 1 ? qi[1] : hc == 2 ? qi[2] : qi[3];
        }
      }
  };
  // VEL: normal velocity components on the lane's faces (indices clamped into the face arrays:
  // lanes and rows outside the grid compute but never store).  x faces [n2][n1][n0 + 1], y faces
  // [n2][n1 + 1][n0] after the n0 (n1 + 1) n2 x components of v[1], z faces [n2 + 1][n1][n0]
  // after 2 n0 n1 (n2 + 1) components of v[2].
  const int64_t vxc = min(max(xz, 0), n0), vxz = min(max(xz, 0), n0 - 1);
  const int64_t vyr = min(max(yz, 0), n1 - 1), vyf = min(max(yz, 0), n1), vyt = min(max(yz + 1, 0), n1);
  const int64_t nfy = (int64_t)n0 * (n1 + 1) * n2, nfz = (int64_t)n0 * n1 * (n2 + 1);
  auto vel_z = [&](int f) -> R { return R(va.v[2][2 * nfz + ((int64_t)f * n1 + vyr) * n0 + vxz]); };
  R Ux = R(0), Uy = R(0), Uyt = R(0), Uz = R(0);   // face velocities of the plane
  {
    int pm;
    R raw[4], qa[4], qb[4];
    const int o0 = plane_s(mbeg, zsh, pm);
    c3_load<S, R>(a, o0 + cb, raw);
    c3_fix(raw, lm ^ pm, q0);
    k0 = R(a.kap[o0 + cb]);
    s0 = R(a.sig[o0 + cb]);
    const int o1 = plane_s(mbeg + 1, zsh, pm);
    c3_load<S, R>(a, o1 + cb, raw);
    c3_fix(raw, lm ^ pm, q1);
    int pa, pb;
    const int oa = plane_s(mbeg - 2, zsh, pa), ob = plane_s(mbeg - 1, zsh, pb);
    c3_load<S, R>(a, oa + cb, raw);
    c3_fix(raw, lm ^ pa, qa);
    c3_load<S, R>(a, ob + cb, raw);
    c3_fix(raw, lm ^ pb, qb);
    if (SPH && xinf) {
      inflow_state(ex, ey, q0);
      inflow_state(ex, ey, q1);
      inflow_state(ex, ey, qa);
      inflow_state(ex, ey, qb);
    }
    const R ksb = R(a.kap[ob + cb]) + R(a.sig[ob + cb]);
    // face mbeg - 1/2 from zones mbeg - 1 (upper state) and mbeg (lower state)
    for (int c = 0; c < 4; ++c) hiM[c] = fPrev[c] = R(0);
    if (!idle) {
      R lo[4], hiP[4];
      reconstruct<R, SPH, 3, LIM>(a, geo, 2, NG, qa, qb, q0, ihz, ihz, true, true, lo, hiP);
      reconstruct<R, SPH, 3, LIM>(a, geo, 2, NG, qb, q0, q1, ihz, ihz, true, true, lo, hiM);
      hll<R, SPH, 3, (LIM < 0)>(a, 2, hiP, lo, hz, ihz, epsilon_of(ksb, k0 + s0, dlz, dlz), fPrev);
      if constexpr (VEL) add_upwind(vel_z(mbeg), hiP, lo, fPrev);
    }
    // in flight into the first plane
    Pk = R(a.kap[o1 + cb]);
    Ps = R(a.sig[o1 + cb]);
    PB = R(a.B[mbeg * PL + cbb]);
    const int o2 = plane_s(mbeg + 2, zsh, Ppm);
    c3_load<S, R>(a, o2 + cb, Pr);
    plane_s(mbeg, zsh, Popm);
    c3_load<S, R>(a, o0 + ceb, Po);
    if (SPH && xinfe) inflow_state(ex - 1, ey, Po);
    int pmu;
    load_items(plane(mbeg, pmu), mbeg);
  }

  // The update of plane m needs the y flux that the row above computes for plane m: it runs
  // after the next plane's barrier, from values the lane keeps (the state, the x and z part of
  // the divergence and the flux at its lower y face, kappa, sigma, B).  With the LDS arrays
  // double-buffered by plane parity, the one barrier per plane orders every LDS access: a
  // buffer written for plane m was last read for plane m - 2, before the barrier of m - 1.
  R qU[4], accU[4], fyU[4], kU = R(0), sU = R(0), BU = R(0);
  for (int c = 0; c < 4; ++c) qU[c] = accU[c] = fyU[c] = R(0);
  for (int m = mbeg; m <= mend; ++m) {
    const int buf = m & 1;
    const bool live = m < mend;       // the last pass only updates plane mend - 1
    R q2[4], qo[4];
    if (live) {
      // ---- consume the values loaded one plane ago; the plane's rows to LDS ----
      c3_fix(Pr, lm ^ Ppm, q2);            // plane m + 2
      c3_fix(Po, lme ^ Popm, qo);          // outer x neighbour, plane m
      if (SPH && xinf) inflow_state(ex, ey, q2);
      if (SPH && xinfe) inflow_state(ex - 1, ey, qo);
      for (int c = 0; c < 4; ++c) QS[buf][c][sw][lane] = q0[c];
      QS[buf][4][sw][lane] = k0;
      QS[buf][5][sw][lane] = s0;
      for (int k = 0; k < NHI; ++k)
        if (hslot[k] >= 0) {
          const int zflip = (hcomp[k] == 3) ? (Popm >> 2) & 1 : 0;
          QS[buf][hcomp[k]][hslot[k]][lane] = (hmask[k] ^ zflip) ? -Ph[k] : Ph[k];
        }
      // ---- loads for the next plane: q(m + 3), outer neighbours of m + 1, kappa, sigma of
      // m + 2 and B of m + 1 (indices clamped into the ghost range; the last planes' are not
      // used) ----
      const int o3 = plane_s(min(m + 3, n2 + 1), zsh, Ppm);
      c3_load<S, R>(a, o3 + cb, Pr);
      const int oe = plane_s(min(m + 1, n2 + 1), zsh, Popm);
      if (xedge) c3_load<S, R>(a, oe + ceb, Po);
      int pmu;
      load_items(SPH ? plane(min(m + 1, n2 + 1), pmu) : oe, min(m + 1, n2 + 1));
      // kappa, sigma of m + 2 and B of m + 1 (they move into the window at the end of the plane:
      // loaded here, a plane before, so that no wait for the loads in flight falls there)
      const int ok = plane_s(min(m + 2, n2 + 1), zsh, pmu);
      Pk2 = R(a.kap[ok + cb]);
      Ps2 = R(a.sig[ok + cb]);
      PB2 = R(a.B[min(m + 1, n2 - 1) * PL + cbb]);
      if constexpr (VEL) {
        // this plane's face velocities (used after the barrier)
        Ux = R(va.v[0][((int64_t)m * n1 + vyr) * (n0 + 1) + vxc]);
        Uy = R(va.v[1][nfy + ((int64_t)m * (n1 + 1) + vyf) * n0 + vxz]);
        if (AR && top) Uyt = R(va.v[1][nfy + ((int64_t)m * (n1 + 1) + vyt) * n0 + vxz]);
        Uz = vel_z(m + 1);
      }
    }
    c3_barrier();
    // ---- update of plane m - 1 (every lane of the inner rows computes; the lanes that hold a
    // zone of the tile store) ----
    if (m > mbeg && !idle) {
      const int mu = m - 1;
      R acc[4];
      if constexpr (SPH) {
        const R wl = gld(geo.wf[1], ey), wh = gld(geo.wf[1], ey + 1), iW = gld(geo.iW[1], ey);
        for (int c = 0; c < 4; ++c) acc[c] = accU[c] + (wh * FY[buf ^ 1][c][w + 1][lane] - wl * fyU[c]) * iW;
      } else {
        for (int c = 0; c < 4; ++c) acc[c] = accU[c] + (FY[buf ^ 1][c][w + 1][lane] - fyU[c]) * idx1;
      }
      const int zg = upd ? (mu * n1 + yz) * n0 * G + xz * G + g : 0;
      R Um[4];
      for (int c = 0; c < 4; ++c) Um[c] = qU[c] - dtR * acc[c];
      if constexpr (SPH) {
        // geometric source terms of the covariant flux components (cell-centred h)
        R h[3], ih[3], P[9], Sg[3];
        h[0] = h[1] = rg(RG_HR);
        h[2] = rg(RG_HR) * gld(geo.hs, ey);
        ih[0] = ih[1] = rg(RG_IHR);
        ih[2] = rg(RG_IHR) * gld(geo.ihs, ey);
        closure_full<R, SPH, 3>(qU, ih, R(a.c), a.closure, P);
        geometric_source<R>(P, h, ih, geo.gam + 4 * min(max(yz, 0), n1 - 1), R(a.c), Sg);
        for (int cc = 0; cc < 3; ++cc) Um[1 + cc] += dtR * Sg[cc];
      }
      if (a.Ea) {
        // second Runge-Kutta stage: U^- = (U^n + U* + dt L(U*)) / 2
        Um[0] = R(0.5) * (R(a.Ea[zg]) + Um[0]);
        for (int c = 0; c < 3; ++c) Um[1 + c] = R(0.5) * (R(a.Fa[c][zg]) + Um[1 + c]);
      }
      S Eo, F1[3];
      double dz = 0.0;
      if (a.src) {
        const double ck = cdt * (double)kU;
        dz = source_zone<S, R, SPH, 3>(a, geo, xz, yz, Um, ck, cdt * ((double)kU + (double)sU), ck * (double)BU,
                                         want_diag && upd, Vz, zd, Eo, F1);
      } else {
        Eo = S(Um[0]);
        for (int c = 0; c < 3; ++c) F1[c] = S(Um[1 + c]);
      }
      if (upd) {
        a.Eo[zg] = Eo;
        for (int c = 0; c < 3; ++c) a.Fo[c][zg] = F1[c];
      }
      if (a.dEm) {
        // the zone's sum over the block's 4 groups (lanes 16 apart)
        dz = upd ? dz : 0.0;
        dz = lane_pair_sum<32>(lane_pair_sum<16>(dz));
        if (upd && gq == 0) {
          const int64_t zone = ((int64_t)mu * n1 + yz) * n0 + xz;
          if (tl.ngb == 1) a.dEm[zone] = -dz;
          else a.dzp[(int64_t)gb * a.nzones + zone] = dz;
        }
      }
    }
    if (!live) break;
    const R ks0 = k0 + s0;
    // ---- y: the flux at the lower y face of the row, from the reconstructions of the row
    // below (upper state) and of the row (lower state) ----
    R fy[4];
    {
      R qa[4], qb[4], qc[4], lo[4], hiP[4], hiY[4], loY[4];
      for (int c = 0; c < 4; ++c) {
        qa[c] = QS[buf][c][sw - 2][lane];
        qb[c] = QS[buf][c][sw - 1][lane];
      }
      const R ksb = QS[buf][4][sw - 1][lane] + QS[buf][5][sw - 1][lane];
      for (int c = 0; c < 4; ++c) qc[c] = QS[buf][c][sw + 1][lane];
      if constexpr (SPH) {
        // theta faces: scale factors at the face centres of the lane's column; a face on the
        // polar axis is closed (no flux, its face states not checked)
        // (theta faces: 1/h_r = 1/h_theta = 1/r at the column's centre, 1/h_phi with 1/sin theta
        // of the face)
        const R irc = rg(RG_IRC), rc = rg(RG_RC), dly = rg(RG_HR) * geo.dx[1];
        auto ih_th = [&](int ef, R ih[3]) {
          ih[0] = ih[1] = irc;
          ih[2] = irc * gld(geo.isf, ef);
        };
        auto h_th = [&](int ef, R h[3]) {
          h[0] = h[1] = rc;
          h[2] = rc * gld(geo.sf, ef);
        };
        R ihm[3], ih0[3], ih1[3];
        ih_th(ey - 1, ihm);
        ih_th(ey, ih0);
        ih_th(ey + 1, ih1);
        const bool om = gld(geo.wf[1], ey - 1) != R(0), o0f = gld(geo.wf[1], ey) != R(0), o1f = gld(geo.wf[1], ey + 1) != R(0);
        reconstruct<R, SPH, 3, LIM>(a, geo, 1, ey - 1, qa, qb, q0, ihm, ih0, om, o0f, lo, hiP);
        reconstruct<R, SPH, 3, LIM>(a, geo, 1, ey, qb, q0, qc, ih0, ih1, o0f, o1f, loY, hiY);
        for (int c = 0; c < 4; ++c) fy[c] = R(0);
        if (o0f) {
          R hf[3];
          h_th(ey, hf);
          hll<R, SPH, 3, (LIM < 0)>(a, 1, hiP, loY, hf, ih0, epsilon_of(ksb, ks0, dly, dly), fy);
        }
        if (AR && top && yz < n1) {
          // the block's upper face (ey + 1 <= n1 - 1 + NG + 1: inside the face tables)
          R qd[4], loA[4], hiA[4], ih2[3], fu[4];
          for (int c = 0; c < 4; ++c) qd[c] = QS[buf][c][sw + 2][lane];
          const R ksa = QS[buf][4][sw + 1][lane] + QS[buf][5][sw + 1][lane];
          ih_th(ey + 2, ih2);
          const bool o2f = gld(geo.wf[1], ey + 2) != R(0);
          reconstruct<R, SPH, 3, LIM>(a, geo, 1, ey + 1, q0, qc, qd, ih1, ih2, o1f, o2f, loA, hiA);
          for (int c = 0; c < 4; ++c) fu[c] = R(0);
          if (o1f) {
            R hf[3];
            h_th(ey + 1, hf);
            hll<R, SPH, 3, (LIM < 0)>(a, 1, hiY, loA, hf, ih1, epsilon_of(ks0, ksa, dly, dly), fu);
          }
          for (int c = 0; c < 4; ++c) FY[buf][c][NI][lane] = fu[c];
        }
      } else {
        reconstruct<R, false, 3, LIM>(a, geo, 1, 0, qa, qb, q0, hone, hone, true, true, lo, hiP);
        reconstruct<R, false, 3, LIM>(a, geo, 1, 0, qb, q0, qc, hone, hone, true, true, loY, hiY);
        hll<R, false, 3, (LIM < 0)>(a, 1, hiP, loY, hone, hone, epsilon_of(ksb, ks0, dx1, dx1), fy);
        if constexpr (VEL) add_upwind(Uy, hiP, loY, fy);
        if (AR && top && yz < n1) {
          // the block's upper face
          R qd[4], loA[4], hiA[4], fu[4];
          for (int c = 0; c < 4; ++c) qd[c] = QS[buf][c][sw + 2][lane];
          const R ksa = QS[buf][4][sw + 1][lane] + QS[buf][5][sw + 1][lane];
          reconstruct<R, false, 3, LIM>(a, geo, 1, 0, q0, qc, qd, hone, hone, true, true, loA, hiA);
          hll<R, false, 3, (LIM < 0)>(a, 1, hiY, loA, hone, hone, epsilon_of(ks0, ksa, dx1, dx1), fu);
          if constexpr (VEL) add_upwind(Uyt, hiY, loA, fu);
          for (int c = 0; c < 4; ++c) FY[buf][c][NI][lane] = fu[c];
        }
      }
      for (int c = 0; c < 4; ++c) FY[buf][c][w][lane] = fy[c];
    }
    R acc[4] = {R(0), R(0), R(0), R(0)};
    if (!idle) {
      // ---- x: reconstruction, the flux at the lower x face of the column (the upper state
      // of the column below by a lane shift), the x part of the divergence ----
      {
        R qm[4], qp[4], loX[4], hiX[4];
        for (int c = 0; c < 4; ++c) {
          const R pv = col_prev(q0[c]), nv = col_next(q0[c]);
          qm[c] = x == 0 ? qo[c] : pv;
          qp[c] = x == TX - 1 ? qo[c] : nv;
        }
        R qL[4], fx[4];
        if constexpr (SPH) {
          // r faces of the lane's zone; the flux at its lower face
          R ihl[3], ihr[3], hf[3];
          const R isc = gld(geo.isc, ey);
          ihl[0] = ihl[1] = rg(RG_IRF0);
          ihl[2] = rg(RG_IRF0) * isc;
          ihr[0] = ihr[1] = rg(RG_IRF1);
          ihr[2] = rg(RG_IRF1) * isc;
          const R vs[5] = {rg(RG_IDM), rg(RG_IDP), rg(RG_DLO), rg(RG_DHI), rg(RG_IDC)};
          reconstruct<R, SPH, 3, LIM>(a, geo, 0, ex, qm, q0, qp, ihl, ihr, true, true, loX, hiX, vs);
          for (int c = 0; c < 4; ++c) qL[c] = col_prev(hiX[c]);
          const R ksL = col_prev(ks0);
          const R dlx = rg(RG_HR) * geo.dx[0];
          const R dlL = col_prev(dlx);
          hf[0] = hf[1] = rg(RG_RF);
          hf[2] = rg(RG_RF) * gld(geo.sc, ey);
          hll<R, SPH, 3, (LIM < 0)>(a, 0, qL, loX, hf, ihl, epsilon_of(ksL, ks0, dlL, dlx), fx);
          const R wl = rg(RG_WF0), wh = rg(RG_WF1), iW = rg(RG_IW);
          for (int c = 0; c < 4; ++c) acc[c] = (wh * col_next(fx[c]) - wl * fx[c]) * iW;
        } else {
          reconstruct<R, false, 3, LIM>(a, geo, 0, 0, qm, q0, qp, hone, hone, true, true, loX, hiX);
          for (int c = 0; c < 4; ++c) qL[c] = col_prev(hiX[c]);
          const R ksL = col_prev(ks0);
          hll<R, false, 3, (LIM < 0)>(a, 0, qL, loX, hone, hone, epsilon_of(ksL, ks0, dx0, dx0), fx);
          if constexpr (VEL) add_upwind(Ux, qL, loX, fx);
          for (int c = 0; c < 4; ++c) acc[c] = (col_next(fx[c]) - fx[c]) * idx0;
        }
      }
      // ---- z: reconstruction of zone m + 1, the flux at m + 1/2; the window's face values
      // move on at once ----
      {
        R nLo[4], nHi[4], fNext[4];
        reconstruct<R, SPH, 3, LIM>(a, geo, 2, NG, q0, q1, q2, ihz, ihz, true, true, nLo, nHi);
        hll<R, SPH, 3, (LIM < 0)>(a, 2, hiM, nLo, hz, ihz, epsilon_of(ks0, Pk + Ps, dlz, dlz), fNext);
        if constexpr (VEL) add_upwind(Uz, hiM, nLo, fNext);
        for (int c = 0; c < 4; ++c) {
          acc[c] += (fNext[c] - fPrev[c]) * idx2;
          fPrev[c] = fNext[c];
          hiM[c] = nHi[c];
        }
      }
    }
    // ---- keep what the update of plane m needs; advance the window ----
    for (int c = 0; c < 4; ++c) {
      qU[c] = q0[c];
      accU[c] = acc[c];
      fyU[c] = fy[c];
      q0[c] = q1[c];
      q1[c] = q2[c];
    }
    kU = k0;
    sU = s0;
    BU = PB;
    k0 = Pk;
    s0 = Ps;
    Pk = Pk2;
    Ps = Ps2;
    PB = PB2;
  }

  if (!want_diag) return;
  // ---- block partials of the diagnostics ----
  double e = zd.energy, mf = zd.maxf2();
  int un = zd.nun, pnp = zd.nnp;
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off);
    mf = fmax(mf, __shfl_xor(mf, off));
    un += __shfl_xor(un, off);
    pnp += __shfl_xor(pnp, off);
  }
  if (lane == 0) {
    red_e[w] = e;
    red_m[w] = mf;
    red_u[w] = un;
    red_p[w] = pnp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double se = 0.0, sm = 0.0;
    int su = 0, sp = 0;
    for (int k = 0; k < NI; ++k) {
      se += red_e[k];
      sm = fmax(sm, red_m[k]);
      su += red_u[k];
      sp += red_p[k];
    }
    a.p_energy[blockIdx.x] = se;
    a.p_maxf2[blockIdx.x] = sm;
    a.p_nun[blockIdx.x] = su;
    a.p_nnp[blockIdx.x] = sp;
  }
}

// ------------------------------------------------------------------------------------------
// every row of a block updated: double blocks, and float blocks of 4 and 12 rows (three waves
// per SIMD)
static bool c3_all_rows(const fornax_m1_desc& D, int NR) { return D.precision == FORNAX_FP64 || NR == 4 || NR == 12; }

C3Tile make_c3_tile(const fornax_m1_desc& D, int NR, int TM) {
  C3Tile tl{};
  tl.nblocks = 0;
  if (D.ndim != 3 || D.ngroups % 4 != 0) return tl;
  const bool sph = D.coord == FORNAX_SPHERICAL_LOGR;
  if (!sph && D.coord != FORNAX_CARTESIAN) return tl;
  // the instantiated block heights: 6, 8 or 12 rows in double, 4, 8, 12 or 16 in float
  // (spherical grids: 8 rows, or 4, 8 or 12 in float)
  const bool dbl = D.precision == FORNAX_FP64;
  if (!(NR == 8 || (!dbl && (NR == 4 || NR == 12)) || (!sph && (NR == (dbl ? 6 : 4) || NR == (dbl ? 12 : 16)))))
    return tl;
  if (TM < 1) return tl;
  // inflow only on the lower x1 boundary of spherical grids; a polar axis (theta, spherical
  // grids) needs a periodic phi axis of even length
  for (int d = 0; d < 3; ++d) {
    if (D.bc_hi[d] == FORNAX_BC_INFLOW || (D.bc_lo[d] == FORNAX_BC_INFLOW && !(sph && d == 0))) return tl;
    if ((D.bc_lo[d] == FORNAX_BC_AXIS || D.bc_hi[d] == FORNAX_BC_AXIS) && !(sph && d == 1)) return tl;
  }
  if (sph && (D.bc_lo[1] == FORNAX_BC_AXIS || D.bc_hi[1] == FORNAX_BC_AXIS) &&
      (D.bc_lo[2] != FORNAX_BC_PERIODIC || D.bc_hi[2] != FORNAX_BC_PERIODIC || D.n[2] % 2 != 0))
    return tl;
  tl.NR = NR;
  tl.TM = TM;
  tl.ntx = (D.n[0] + C3_TX - 3) / (C3_TX - 2);
  // tiles of NR rows, or NR - 1 (the top row is the next tile's first)
  tl.nty = c3_all_rows(D, NR) ? (D.n[1] + NR - 1) / NR : (D.n[1] + NR - 2) / (NR - 1);
  tl.ntz = (D.n[2] + TM - 1) / TM;
  tl.ngb = D.ngroups / 4;
  const int64_t nb = (int64_t)tl.ntx * tl.nty * tl.ntz * tl.ngb;
  if (nb > (int64_t)1 << 30) return C3Tile{};
  tl.nblocks = (int)nb;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  return tl;
}

// Planes per block: a block walks its TM planes (and about three planes' worth of start-up: the
// first planes' loads and the face below its first plane, the last deferred update) one after
// the other, so the kernel takes about the number of rounds of block slots times TM + 3.  The
// tile of NR rows with the least such cost (ties: the longer tile), the slots from the shape's
// W waves per SIMD and the CU count.  Measured on MI355X this picks the fastest of the lengths
// tried in each case: 192 planes at 192^3 x 12 FP64 (one tile along z: 2.6 % faster than 64
// and 1 % than 96), 64 in MIXED (7 % faster than 96, 1 % than 32), 128 on the 256 x 64 x 128 x
// 20 spherical grid in FP64 (1 % faster than 32 and 64) and 32 in MIXED (12 % faster than 64).
static C3Tile c3_tile_by_rounds(const fornax_m1_desc& D, int NR, int W, int cus) {
  const int per_cu = std::max(1, 4 * W / NR);
  const long slots = (long)per_cu * (cus > 0 ? cus : 256);
  C3Tile best{};
  double best_cost = 0.0;
  for (int TM = std::min(8, D.n[2]); TM <= D.n[2]; ++TM) {
    const C3Tile t = make_c3_tile(D, NR, TM);
    if (t.nblocks <= 0) continue;
    const double cost = (double)((t.nblocks + slots - 1) / slots) * (TM + 3);
    if (best.nblocks <= 0 || cost <= best_cost) {
      best = t;
      best_cost = cost;
    }
  }
  return best;
}

C3Tile choose_c3_tile(const fornax_m1_desc& D, int cus) {
  // one y row per wave: 8 rows (spherical grids in float: 12, every row updated at three waves
  // per SIMD).  Measured at 192^3 x 12 (Cartesian) and 256 x 64 x 128 x 20 (spherical): float
  // Cartesian blocks of 12 or 4 rows at three waves per SIMD 3 % and 11 % slower than 8 rows;
  // spherical float 12 rows 9 % faster than 4 rows and 22 % faster than 8 rows at four waves
  // per SIMD, which spill registers.  Waves per SIMD as launch_c3 instantiates the shapes:
  // double 2, float Cartesian 4, float spherical 3.
  const bool dbl = D.precision == FORNAX_FP64;
  const bool sph = D.coord == FORNAX_SPHERICAL_LOGR;
  return c3_tile_by_rounds(D, (sph && !dbl) ? 12 : 8, dbl ? 2 : (sph ? 3 : 4), cus);
}

// Step 1 of the velocity step: 8 rows at two waves per SIMD in double, 12 rows at three in
// float (launch_c3_vel)
C3Tile choose_c3_vel_tile(const fornax_m1_desc& D, int cus) {
  const bool dbl = D.precision == FORNAX_FP64;
  if (D.coord != FORNAX_CARTESIAN) return C3Tile{};
  return c3_tile_by_rounds(D, dbl ? 8 : 12, dbl ? 2 : 3, cus);
}

template <typename S>
int launch_c3(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, hipStream_t st) {
  const C3Tile& tl = ctx->c3;
  if (tl.nblocks <= 0) return FORNAX_EUNSUPPORTED;
  if (a.dEm && tl.ngb > 1 && !a.dzp) return FORNAX_EUNSUPPORTED;
  // the minmod instantiation has the -+c bounds built in; the other takes both options at run time
  const bool mm = a.limiter == FORNAX_LIMITER_MINMOD && a.wavespeed == FORNAX_WAVESPEED_LIGHT;
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  dim3 grid(tl.nblocks), block(64 * tl.NR);
  const VelArgs<S> nova{};
#define FM1_C3(NRV, WV, SP, AR)                                                                                       \
  do {                                                                                                                \
    if (mm)                                                                                                           \
      hipLaunchKernelGGL((k_step_3d<S, NRV, WV, FORNAX_LIMITER_MINMOD, SP, AR>), grid, block, 0, st, a, geo, tl, nova); \
    else                                                                                                              \
      hipLaunchKernelGGL((k_step_3d<S, NRV, WV, -1, SP, AR>), grid, block, 0, st, a, geo, tl, nova);                    \
  } while (0)
  // waves per SIMD: the register budget of each shape (double: 168 or 256 VGPRs; float: 128,
  // or 168 for the 4- and 12-row blocks)
  if constexpr (sizeof(S) == 8) {
    if (sph) FM1_C3(8, 2, true, true);
    else if (tl.NR == 6) FM1_C3(6, 3, false, true);
    else if (tl.NR == 8) FM1_C3(8, 2, false, true);
    else FM1_C3(12, 3, false, true);
  } else {
    if (sph && tl.NR == 4) FM1_C3(4, 3, true, true);
    else if (sph && tl.NR == 12) FM1_C3(12, 3, true, true);
    else if (sph) FM1_C3(8, 4, true, false);
    else if (tl.NR == 4) FM1_C3(4, 3, false, true);
    else if (tl.NR == 8) FM1_C3(8, 4, false, false);
    else if (tl.NR == 12) FM1_C3(12, 3, false, true);
    else FM1_C3(16, 4, false, false);
  }
#undef FM1_C3
  Tile lt{};
  lt.nblocks = tl.nblocks;
  lt.ngb = tl.ngb;
  *ctx->last_tile = lt;
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template int launch_c3<double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&, hipStream_t);
template int launch_c3<float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, hipStream_t);

// Step 1 of the velocity step (transport with the advective fluxes, no interaction update, no
// diagnostics) on 3-D Cartesian grids of the kernel's kind: 8-row blocks in double, 12-row
// blocks (three waves per SIMD) in float, planes per block chosen at create.
template <typename S>
int launch_c3_vel(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, const VelArgs<S>& va, hipStream_t st) {
  const fornax_m1_desc& D = ctx->desc;
  if (D.coord != FORNAX_CARTESIAN || D.ndim != 3) return FORNAX_EUNSUPPORTED;
  if (a.src || a.dEm || a.p_energy || a.Ea) return FORNAX_EUNSUPPORTED;
  constexpr bool dbl = sizeof(S) == 8;
  const C3Tile tl = ctx->c3v;
  constexpr int NRV = dbl ? 8 : 12, WV = dbl ? 2 : 3;
  if (tl.nblocks <= 0 || tl.NR != NRV) return FORNAX_EUNSUPPORTED;
  const bool mm = a.limiter == FORNAX_LIMITER_MINMOD && a.wavespeed == FORNAX_WAVESPEED_LIGHT;
  dim3 grid(tl.nblocks), block(64 * tl.NR);
  if (mm)
    hipLaunchKernelGGL((k_step_3d<S, NRV, WV, FORNAX_LIMITER_MINMOD, false, true, true>), grid, block, 0, st, a, geo, tl,
                       va);
  else
    hipLaunchKernelGGL((k_step_3d<S, NRV, WV, -1, false, true, true>), grid, block, 0, st, a, geo, tl, va);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template int launch_c3_vel<double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&,
                                   const VelArgs<double>&, hipStream_t);
template int launch_c3_vel<float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, const VelArgs<float>&,
                                  hipStream_t);

}  // namespace fm1
