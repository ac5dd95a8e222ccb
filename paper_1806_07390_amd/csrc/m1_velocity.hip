// m1_velocity.hip -- the step with a prescribed velocity field: the velocity-dependent terms
// of the comoving-frame moment equations to first order in v/c (eq:rad_system), with the
// advective fluxes taken from the upwind face state and the volume-averaged velocity gradient
// of the Riemann Solvers subsection, the frequency advection of eq:freq_adv_system
// (Algorithmic Steps 1 and 2), then the interaction update (Steps 3 and 4); and the
// first-order lab-frame moments.
//
// Two launches per step:
//   k_vel_explicit  one thread per zone-group: Step 1, the static step's transport (HLL fluxes
//                   of the reconstructed face states, geometric sources) plus v^d U_upwind on
//                   every face and, in the flux rows, + <Gamma^l_{ik}> <v^i> F_l - <v^i_{;k}> F_i;
//                   writes U^(1) to the output state;
//                   On 3-D Cartesian grids of the whole-zone 3-D kernel's kind (groups a multiple
//                   of 4) Step 1 runs on that kernel instead (m1_step_3d.hip: the transport with
//                   the advective fluxes), and the zone-local velocity terms of the flux rows
//                   move to k_vel_freq, which reads F^n for them;
//   k_vel_freq      whole zones per block (BLOCK / G zones of G groups, lanes = groups): Step 2
//                   on U^(1) (the compression work, and the upwind intergroup fluxes of the
//                   energy and of the flux components from the minmod-reconstructed spectral
//                   densities, neighbours through LDS), then the interaction update, dE_matter
//                   and the diagnostics partials, in place.
// Readings shared with the CPU definition of the method: the intergroup flux of edge g-1/2
// takes, for each <v^i_{;j}>, the left (lower-group) spectral density where it is negative and
// the right one otherwise, which splits the contractions sum_ij <v^i_{;j}> P^j_i / dnu and
// sum_ik <v^i_{;k}> Q^k_{ji} / dnu into parts (-, +) that are reconstructed (linear in nu, minmod
// slopes over the group-centre distances, none in the first and last group); the frequency
// range is closed (no flux through its two ends); the third moment Q^ is the M1 interpolation
// A (n d + d n + ...) + B n n n, A = |F^| (1 - chi) 3/10 = |F^| (s - 1)/5,
// B = |F^| (3 chi - 1)/2 = |F^| (2 - s), s = sqrt(4 - 3 f^2), between the diffusion-limit form
// (c E / 5)(sym f) and the beam c E n n n; no local Q term in the flux rows.
//
// k_vel_explicit is bound by the per-thread recomputation of the face states (two faces per zone
// and direction) rather than HBM: the general path of the method's velocity terms.

#include <algorithm>
#include <type_traits>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

// coordinate component `comp` of the velocity on the lower (up = 0) or upper (up = 1) d-face of
// zone (i, j, k)
template <typename S, typename R>
__device__ __forceinline__ R face_v(const StepArgsBase& a, const VelArgs<S>& va, int d, int comp, int i, int j, int k,
                                    int up) {
  int m0 = a.n[0], m1 = a.n[1], m2 = a.n[2];
  if (d == 0) {
    m0 += 1;
    i += up;
  } else if (d == 1) {
    m1 += 1;
    j += up;
  } else {
    m2 += 1;
    k += up;
  }
  const int64_t nf = (int64_t)m0 * m1 * m2;
  return R(va.v[d][comp * nf + ((int64_t)k * m1 + j) * m0 + i]);
}

// Volume-averaged connection coefficients <Gamma^l_{km}> of a zone in row j (index 9 l + 3 k + m):
// zero on Cartesian grids; on spherical (ln r, theta, phi) grids the constants
// Gamma^1_11 = Gamma^2_12 = Gamma^3_13 = 1, Gamma^1_22 = -1 and the theta tables (with the
// paper's overrides) of the geometric sources.  Fully unrolled loops fold the zero entries.
template <typename R, bool SPH>
__device__ __forceinline__ void connection(const Geo<R>& geo, int j, R Gm[27]) {
  for (int t = 0; t < 27; ++t) Gm[t] = R(0);
  if constexpr (SPH) {
    const R* g = geo.gam + 4 * j;
    const R G323 = g[0], G133 = g[1], G233 = g[2], G222 = g[3];
    Gm[0] = R(1);                           // Gamma^1_11
    Gm[9 + 1] = Gm[9 + 3] = R(1);           // Gamma^2_12 = Gamma^2_21
    Gm[18 + 2] = Gm[18 + 6] = R(1);         // Gamma^3_13 = Gamma^3_31
    Gm[18 + 5] = Gm[18 + 7] = G323;         // Gamma^3_23 = Gamma^3_32
    Gm[4] = R(-1);                          // Gamma^1_22
    Gm[8] = G133;                           // Gamma^1_33
    Gm[9 + 8] = G233;                       // Gamma^2_33
    Gm[9 + 4] = G222;                       // Gamma^2_22
  } else {
    (void)geo;
    (void)j;
  }
}

// <v^i_{;j}> (Vg[3 i + j]) and <v^k> (vb) of zone (i, j, k): every coordinate component linear
// across the zone between its values on the two faces of each direction, so <v^i_{,j}> is their
// difference over dx^j and <v^k> the value of v^k's profile at the volume centroid <x^k>
// (x_{k-1/2} - <x^k> = dlo); then <v^i_{;j}> = <v^i_{,j}> + <Gamma^i_{jk}> <v^k>.
template <typename S, typename R, bool SPH, int ND>
__device__ __forceinline__ void vel_grad(const StepArgsBase& a, const Geo<R>& geo, const VelArgs<S>& va, int i, int j,
                                         int k, const R Gm[27], R Vg[9], R vb[3]) {
  const int ez[3] = {i + NG, j + NG, k + NG};
  R dv[9];
  for (int t = 0; t < 9; ++t) dv[t] = R(0);
  for (int t = 0; t < 3; ++t) vb[t] = R(0);
  // the zone's lower face in each direction's face array and the stride to the upper face
  // (the face arrays of direction d have one more entry along d), and each array's
  // component stride
  const int64_t n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const int64_t lo[3] = {((int64_t)k * n1 + j) * (n0 + 1) + i, ((int64_t)k * (n1 + 1) + j) * n0 + i,
                         ((int64_t)k * n1 + j) * n0 + i};
  const int64_t up[3] = {1, n0, n0 * n1};
  const int64_t nf[3] = {(n0 + 1) * n1 * n2, n0 * (n1 + 1) * n2, n0 * n1 * (n2 + 1)};
  for (int jd = 0; jd < ND; ++jd) {
    const R idx = geo.idx[jd];
    const R w = -gld(geo.dlo[jd], ez[jd]) * idx;   // (<x> - x_{-1/2}) / dx
    for (int ic = 0; ic < ND; ++ic) {
      const S* vp = va.v[jd] + ic * nf[jd] + lo[jd];
      const R vlo = R(vp[0]);
      const R vhi = R(vp[up[jd]]);
      dv[3 * ic + jd] = (vhi - vlo) * idx;
      if (ic == jd) vb[jd] = vlo + (vhi - vlo) * w;
    }
  }
  for (int ic = 0; ic < 3; ++ic)
    for (int jd = 0; jd < 3; ++jd) {
      R s = dv[3 * ic + jd];
      for (int kk = 0; kk < 3; ++kk) s += Gm[9 * ic + 3 * jd + kk] * vb[kk];
      Vg[3 * ic + jd] = s;
    }
}

// Flux through the d-face with index f of the row of zone (i, j): the static step's HLL flux of
// the reconstructed face states (q[] holds zones f-2 .. f+1, ksL, ksR the opacities of f-1 and
// f) plus the advective flux vd U_upwind, the left state for vd >= 0.  A face of zero area
// (polar axis) has no flux.
template <typename S, typename R, bool SPH, int ND>
__device__ __forceinline__ void face_flux_v(const StepArgs<S>& a, const Geo<R>& geo, int d, int f, int i, int j,
                                            const R (*q)[4], R ksL, R ksR, R vd, R flux[4]) {
  const int ef = f + NG;
  for (int c = 0; c < 4; ++c) flux[c] = R(0);
  if (SPH && geo.wf[d][ef] == R(0)) return;
  const int ei = i + NG, ej = j + NG;
  R ih0[3], h1[3], ih1[3], ih2[3];
  face_ih<R, SPH>(geo, d, ei, ej, ef - 1, ih0);
  face_h<R, SPH>(geo, d, ei, ej, ef, h1);
  face_ih<R, SPH>(geo, d, ei, ej, ef, ih1);
  face_ih<R, SPH>(geo, d, ei, ej, ef + 1, ih2);
  const bool o0 = !SPH || geo.wf[d][ef - 1] != R(0), o2 = !SPH || geo.wf[d][ef + 1] != R(0);
  R Llo[4], Lhi[4], Rlo[4], Rhi[4];
  reconstruct<R, SPH, ND>(a, geo, d, ef - 1, q[0], q[1], q[2], ih0, ih1, o0, true, Llo, Lhi);
  reconstruct<R, SPH, ND>(a, geo, d, ef, q[1], q[2], q[3], ih1, ih2, true, o2, Rlo, Rhi);
  const int eL = ef - 1;
  const R dlL = proper_width<R, SPH>(geo, d, d == 0 ? eL : ei, d == 1 ? eL : ej);
  const R dlR = proper_width<R, SPH>(geo, d, d == 0 ? ef : ei, d == 1 ? ef : ej);
  const R eps = epsilon_of(ksL, ksR, dlL, dlR);
  hll<R, SPH, ND, false>(a, d, Lhi, Rlo, h1, ih1, eps, flux);
  const R* qu = (vd >= R(0)) ? Lhi : Rlo;
  for (int c = 0; c <= ND; ++c) flux[c] += vd * qu[c];
}

// Coefficients of the third moment Q^ = A (n^k d^{ji} + n^j d^{ki} + n^i d^{kj}) + B n^k n^j n^i
// of the state q (physical components, unit direction n of F^, |F^| clamped to cE):
// A = |F^| (s - 1)/5, B = |F^| (2 - s), s = sqrt(4 - 3 f^2), written without cancellation
// (s - 1 = 3 (1 - f^2)/(1 + s), 2 - s = 3 f^2/(2 + s)); the Eddington closure gives A = |F^|/5,
// B = 0.  E <= 0 or F = 0: A = B = 0.
template <typename R, bool SPH, int ND>
__device__ __forceinline__ void third_moment(const R q[4], const R ih[3], R c, int eddington, R& A, R& B, R n[3]) {
  A = R(0);
  B = R(0);
  n[0] = n[1] = n[2] = R(0);
  const R E = q[0];
  if (!(E > R(0))) return;
  const R icE = rcp_(c * E);
  R f[3] = {R(0), R(0), R(0)};
  R f2 = R(0);
  for (int k = 0; k < ND; ++k) {
    f[k] = (SPH ? q[1 + k] * ih[k] : q[1 + k]) * icE;
    f2 += f[k] * f[k];
  }
  if (!(f2 > R(0))) return;
  const R fm = sqrt_(f2);
  const R ifm = rcp_(fm);
  for (int k = 0; k < ND; ++k) n[k] = f[k] * ifm;
  const R fa = (f2 > R(1)) ? R(1) : fm;
  const R f2c = (f2 > R(1)) ? R(1) : f2;
  const R Fa = c * E * fa;
  if (eddington) {
    A = Fa * R(0.2);
    return;
  }
  const R s = sqrt_(R(4) - R(3) * f2c);
  A = Fa * R(0.6) * (R(1) - f2c) * rcp_(R(1) + s);
  B = Fa * R(3) * f2c * rcp_(R(2) + s);
}

// ------------------------------------------------------------------------------------------
// Step 1 with the velocity terms, one thread per zone-group; U^(1) into a.Eo, a.Fo.
// ------------------------------------------------------------------------------------------
template <typename S, typename R, bool SPH, int ND>
__global__ void __launch_bounds__(BLOCK) k_vel_explicit(StepArgs<S> a, Geo<R> geo, VelArgs<S> va) {
  const int64_t id = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (id >= a.nzones * a.G) return;
  const int grp = (int)(id % a.G);
  const int64_t z = id / a.G;
  const int i = (int)(z % a.n[0]), j = (int)((z / a.n[0]) % a.n[1]), k = (int)(z / ((int64_t)a.n[0] * a.n[1]));
  const int iz[3] = {i, j, k};
  R q0[4], ks0;
  fetch<S, R, SPH, ND>(a, geo, 0, i, i, j, k, grp, q0, &ks0);
  R acc[4] = {R(0), R(0), R(0), R(0)};
  for (int d = 0; d < ND; ++d) {
    const int m = iz[d];
    R q[5][4], ks[3];
    for (int o = -2; o <= 2; ++o) {
      if (o == 0) {
        for (int c = 0; c < 4; ++c) q[2][c] = q0[c];
        ks[1] = ks0;
      } else {
        fetch<S, R, SPH, ND>(a, geo, d, m + o, i, j, k, grp, q[o + 2],
                             o == -1 ? &ks[0] : (o == 1 ? &ks[2] : nullptr));
      }
    }
    const R vlo = face_v<S, R>(a, va, d, d, i, j, k, 0), vhi = face_v<S, R>(a, va, d, d, i, j, k, 1);
    R flo[4], fhi[4];
    face_flux_v<S, R, SPH, ND>(a, geo, d, m, i, j, q, ks[0], ks[1], vlo, flo);
    face_flux_v<S, R, SPH, ND>(a, geo, d, m + 1, i, j, q + 1, ks[1], ks[2], vhi, fhi);
    R wl = R(1), wh = R(1), iW = geo.idx[d];
    if constexpr (SPH) {
      wl = geo.wf[d][m + NG];
      wh = geo.wf[d][m + NG + 1];
      iW = geo.iW[d][m + NG];
    }
    for (int c = 0; c <= ND; ++c) acc[c] += (wh * fhi[c] - wl * flo[c]) * iW;
  }
  const R dtR = R(a.dt), c = R(a.c);
  R Um[4];
  for (int cc = 0; cc < 4; ++cc) Um[cc] = (cc <= ND) ? q0[cc] - dtR * acc[cc] : R(0);
  if constexpr (SPH) {
    R h[3], ih[3], P[9], Sg[3];
    cell_h<R, SPH>(geo, i + NG, j + NG, h);
    cell_ih<R, SPH>(geo, i + NG, j + NG, ih);
    closure_full<R, SPH, ND>(q0, ih, c, a.closure, P);
    geometric_source<R>(P, h, ih, geo.gam + 4 * j, c, Sg);
    for (int cc = 0; cc < ND; ++cc) Um[1 + cc] += dtR * Sg[cc];
  }
  // velocity terms of the flux rows: + <Gamma^l_{ik}> <v^i> F_l - <v^i_{;k}> F_i
  R Gm[27], Vg[9], vb[3];
  connection<R, SPH>(geo, j, Gm);
  vel_grad<S, R, SPH, ND>(a, geo, va, i, j, k, Gm, Vg, vb);
  for (int kk = 0; kk < ND; ++kk) {
    R s = R(0);
    for (int ic = 0; ic < 3; ++ic)
      for (int l = 0; l < 3; ++l) s += Gm[9 * l + 3 * ic + kk] * vb[ic] * q0[1 + l];
    for (int ic = 0; ic < 3; ++ic) s -= Vg[3 * ic + kk] * q0[1 + ic];
    Um[1 + kk] += dtR * s;
  }
  const int64_t zg = id;
  a.Eo[zg] = S(Um[0]);
  for (int cc = 0; cc < ND; ++cc) a.Fo[cc][zg] = S(Um[1 + cc]);
}

// ------------------------------------------------------------------------------------------
// Step 2 and the interaction update, whole zones per block, in place on (a.E, a.F) = (a.Eo,
// a.Fo).  Blocks stride over the zones; the diagnostics partials are per block.
// ------------------------------------------------------------------------------------------
template <typename S, typename R, bool SPH, int ND>
__global__ void __launch_bounds__(BLOCK) k_vel_freq(StepArgs<S> a, Geo<R> geo, VelArgs<S> va, int want_diag) {
  // parts of the contractions: 0 = X- and 1 = X+ (energy row), 2 + 2 j = Y-_j and 3 + 2 j = Y+_j
  // (flux row j); the - parts are taken at a group's upper edge, the + parts at its lower edge
  constexpr int NP = 2 + 2 * ND;
  const int G = a.G;
  const int zpb = a.zones_per_block;
  const int t = threadIdx.x;
  const int lz = t / G, grp = t - lz * G;
  const bool lane_ok = lz < zpb;
  __shared__ R sV[NP][BLOCK], sEd[NP][BLOCK];
  __shared__ double sdz[BLOCK];
  // the group's frequency geometry (double)
  double nlo = 0.0, nhi = 1.0, cm = 0.0, cp = 0.0;
  if (lane_ok) {
    nlo = va.nu[grp];
    nhi = va.nu[grp + 1];
    if (grp > 0 && grp < G - 1) {
      cm = 0.5 * (va.nu[grp - 1] + nlo);
      cp = 0.5 * (nhi + va.nu[grp + 2]);
    }
  }
  const double nc = 0.5 * (nlo + nhi);
  const bool interior = lane_ok && grp > 0 && grp < G - 1;
  const R idm = interior ? R(1.0 / (nc - cm)) : R(0), idp = interior ? R(1.0 / (cp - nc)) : R(0);
  const R idnu = R(1.0 / (nhi - nlo)), half = R(0.5 * (nhi - nlo));
  const R Rnlo = R(nlo), Rnhi = R(nhi);
  const R dtR = R(a.dt), c = R(a.c);
  const double cdt = a.c * a.dt;
  ZoneDiag zd;
  for (int64_t zb = (int64_t)blockIdx.x * zpb; zb < a.nzones; zb += (int64_t)gridDim.x * zpb) {
    const int64_t z = zb + lz;
    const bool act = lane_ok && z < a.nzones;
    R U[4] = {R(0), R(0), R(0), R(0)};
    R vP = R(0);
    R val[NP];
    for (int pp = 0; pp < NP; ++pp) val[pp] = R(0);
    int i = 0, j = 0, k = 0;
    int64_t zg = 0;
    if (act) {
      zg = z * G + grp;
      i = (int)(z % a.n[0]);
      j = (int)((z / a.n[0]) % a.n[1]);
      k = (int)(z / ((int64_t)a.n[0] * a.n[1]));
      U[0] = R(a.E[zg]);
      for (int cc = 0; cc < ND; ++cc) U[1 + cc] = R(a.F[cc][zg]);
      R Gm[27], Vg[9], vb[3];
      connection<R, SPH>(geo, j, Gm);
      vel_grad<S, R, SPH, ND>(a, geo, va, i, j, k, Gm, Vg, vb);
      if (va.Fn[0]) {
        // Step 1 ran on the transport kernel: its zone-local velocity terms of the flux rows,
        // + <Gamma^l_{ik}> <v^i> F_l - <v^i_{;k}> F_i of U^n, are added here
        R Fn[3] = {R(0), R(0), R(0)};
        for (int cc = 0; cc < ND; ++cc) Fn[cc] = R(va.Fn[cc][zg]);
        for (int kk = 0; kk < ND; ++kk) {
          R sv = R(0);
          for (int ic = 0; ic < 3; ++ic)
            for (int l = 0; l < 3; ++l) sv += Gm[9 * l + 3 * ic + kk] * vb[ic] * Fn[l];
          for (int ic = 0; ic < 3; ++ic) sv -= Vg[3 * ic + kk] * Fn[ic];
          U[1 + kk] += dtR * sv;
        }
      }
      R h[3] = {R(1), R(1), R(1)}, ih[3] = {R(1), R(1), R(1)};
      if constexpr (SPH) {
        cell_h<R, SPH>(geo, i + NG, j + NG, h);
        cell_ih<R, SPH>(geo, i + NG, j + NG, ih);
      }
      // the gradient in the frame of the physical components, Vt_ik = <v^i_{;k}> h_i / h_k, split
      // by sign into Wm (< 0) and Wp (>= 0)
      R Wm[9], Wp[9];
      for (int ic = 0; ic < 3; ++ic)
        for (int kc = 0; kc < 3; ++kc) {
          const R v = SPH ? Vg[3 * ic + kc] * (h[ic] * ih[kc]) : Vg[3 * ic + kc];
          Wm[3 * ic + kc] = (Vg[3 * ic + kc] < R(0)) ? v : R(0);
          Wp[3 * ic + kc] = (Vg[3 * ic + kc] < R(0)) ? R(0) : v;
        }
      // energy row: sum_ij W_ij P^^{ji}
      R P[9];
      closure_full<R, SPH, ND>(U, ih, c, a.closure, P);
      R xm = R(0), xp = R(0);
      for (int ic = 0; ic < 3; ++ic)
        for (int jd = 0; jd < 3; ++jd) {
          xm += Wm[3 * ic + jd] * P[3 * jd + ic];
          xp += Wp[3 * ic + jd] * P[3 * jd + ic];
        }
      vP = xm + xp;
      val[0] = xm * idnu;
      val[1] = xp * idnu;
      // flux rows: h_j [A ((W n)_j + n_j tr W + (W^T n)_j) + B n_j (n W n)]
      R A, B, n[3];
      third_moment<R, SPH, ND>(U, ih, c, a.closure, A, B, n);
      for (int sd = 0; sd < 2; ++sd) {
        const R* W = sd == 0 ? Wm : Wp;
        R Wn[3], WTn[3];
        for (int r = 0; r < 3; ++r) {
          Wn[r] = W[3 * r] * n[0] + W[3 * r + 1] * n[1] + W[3 * r + 2] * n[2];
          WTn[r] = W[r] * n[0] + W[3 + r] * n[1] + W[6 + r] * n[2];
        }
        const R tr = W[0] + W[4] + W[8];
        const R nWn = n[0] * Wn[0] + n[1] * Wn[1] + n[2] * Wn[2];
        for (int jd = 0; jd < ND; ++jd) {
          const R y = A * (Wn[jd] + n[jd] * tr + WTn[jd]) + B * n[jd] * nWn;
          val[2 + 2 * jd + sd] = (SPH ? h[jd] * y : y) * idnu;
        }
      }
    }
    for (int pp = 0; pp < NP; ++pp) sV[pp][t] = val[pp];
    __syncthreads();
    // edge values: the - parts at the group's upper edge, the + parts at its lower edge
    R ed[NP];
    for (int pp = 0; pp < NP; ++pp) {
      R sl = R(0);
      if (act && interior) sl = minmod((val[pp] - sV[pp][t - 1]) * idm, (sV[pp][t + 1] - val[pp]) * idp);
      ed[pp] = (pp & 1) ? val[pp] - sl * half : val[pp] + sl * half;
      sEd[pp][t] = ed[pp];
    }
    __syncthreads();
    double dz = 0.0;
    if (act) {
      for (int r = 0; r <= ND; ++r) {
        const R flo = (grp > 0) ? Rnlo * (sEd[2 * r][t - 1] + ed[2 * r + 1]) : R(0);
        const R fhi = (grp < G - 1) ? Rnhi * (ed[2 * r] + sEd[2 * r + 1][t + 1]) : R(0);
        U[r] += dtR * ((fhi - flo) - (r == 0 ? vP : R(0)));
      }
      // Steps 3 and 4
      const double kd = (double)a.kap[zg], sd = (double)a.sig[zg], Bd = (double)a.B[zg];
      const double ck = cdt * kd, cks = cdt * (kd + sd), jB = ck * Bd;
      const double V = geo.Wd[0][i + NG] * geo.Wd[1][j + NG] * geo.Wd[2][k + NG];
      S E1, F1[3];
      dz = source_zone<S, R, SPH, ND>(a, geo, i, j, U, ck, cks, jB, want_diag != 0, V, zd, E1, F1);
      a.Eo[zg] = E1;
      for (int cc = 0; cc < ND; ++cc) a.Fo[cc][zg] = F1[cc];
    }
    if (a.dEm) {
      sdz[t] = dz;
      __syncthreads();
      if (act && grp == 0) {
        double s = 0.0;
        for (int g2 = 0; g2 < G; ++g2) s += sdz[t + g2];
        a.dEm[z] = -s;
      }
    }
    __syncthreads();
  }
  if (!want_diag) return;
  double e = zd.energy, mf = zd.maxf2();
  int un = zd.nun, p = zd.nnp;
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off);
    mf = fmax(mf, __shfl_xor(mf, off));
    un += __shfl_xor(un, off);
    p += __shfl_xor(p, off);
  }
  __shared__ double we[BLOCK / 64], wm[BLOCK / 64];
  __shared__ int wu[BLOCK / 64], wp[BLOCK / 64];
  const int wave = t >> 6, lane = t & 63;
  if (lane == 0) {
    we[wave] = e;
    wm[wave] = mf;
    wu[wave] = un;
    wp[wave] = p;
  }
  __syncthreads();
  if (t == 0) {
    double se = 0.0, sm = 0.0;
    int su = 0, sp = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
      se += we[w];
      sm = fmax(sm, wm[w]);
      su += wu[w];
      sp += wp[w];
    }
    a.p_energy[blockIdx.x] = se;
    a.p_maxf2[blockIdx.x] = sm;
    a.p_nun[blockIdx.x] = su;
    a.p_nnp[blockIdx.x] = sp;
  }
}

// ------------------------------------------------------------------------------------------
// Lab-frame moments, one thread per zone (groups in a loop), accumulated in double.
// ------------------------------------------------------------------------------------------
template <typename S, typename R, bool SPH, int ND>
__global__ void __launch_bounds__(BLOCK) k_lab_frame(StepArgs<S> a, Geo<R> geo, VelArgs<S> va, double* El,
                                                     double* Fl0, double* Fl1, double* Fl2) {
  const int64_t z = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (z >= a.nzones) return;
  const int i = (int)(z % a.n[0]), j = (int)((z / a.n[0]) % a.n[1]), k = (int)(z / ((int64_t)a.n[0] * a.n[1]));
  R Gm[27], Vg[9], vb[3];
  connection<R, SPH>(geo, j, Gm);
  vel_grad<S, R, SPH, ND>(a, geo, va, i, j, k, Gm, Vg, vb);
  R h[3] = {R(1), R(1), R(1)}, ih[3] = {R(1), R(1), R(1)};
  if constexpr (SPH) {
    cell_h<R, SPH>(geo, i + NG, j + NG, h);
    cell_ih<R, SPH>(geo, i + NG, j + NG, ih);
  }
  double v[3];
  for (int kk = 0; kk < 3; ++kk) v[kk] = (double)h[kk] * (double)vb[kk];
  const double cc = a.c;
  double el = 0.0, fl[3] = {0.0, 0.0, 0.0};
  for (int g = 0; g < a.G; ++g) {
    const int64_t zg = z * a.G + g;
    R q[4] = {R(a.E[zg]), R(0), R(0), R(0)};
    for (int c = 0; c < ND; ++c) q[1 + c] = R(a.F[c][zg]);
    R P[9];
    closure_full<R, SPH, ND>(q, ih, R(a.c), a.closure, P);
    double Fh[3];
    for (int c = 0; c < 3; ++c) Fh[c] = (double)q[1 + c] * (double)ih[c];
    const double E = (double)q[0];
    el += E + 2.0 * (v[0] * Fh[0] + v[1] * Fh[1] + v[2] * Fh[2]) / (cc * cc);
    for (int c = 0; c < 3; ++c)
      fl[c] += Fh[c] + v[c] * E + (v[0] * (double)P[c] + v[1] * (double)P[3 + c] + v[2] * (double)P[6 + c]);
  }
  El[z] = el;
  double* Fo[3] = {Fl0, Fl1, Fl2};
  for (int c = 0; c < ND; ++c) Fo[c][z] = fl[c];
}

}  // namespace fm1

using namespace fm1;

namespace {

template <typename S>
VelArgs<S> vel_args(const fornax_m1_ctx* ctx, const fornax_m1_velocity* vel) {
  VelArgs<S> va;
  for (int d = 0; d < 3; ++d) {
    va.v[d] = (d < ctx->desc.ndim) ? (const S*)vel->v[d] : nullptr;
    va.Fn[d] = nullptr;
  }
  va.nu = ctx->vel_nu;
  return va;
}

template <typename S, typename R, bool SPH, int ND>
int launch_vel_nd(fornax_m1_ctx* ctx, const Geo<R>& geo, StepArgs<S>& a, const VelArgs<S>& va,
                  const fornax_m1_diag* diag, hipStream_t st) {
  VelArgs<S> vf = va;
  bool fused = false;
  if constexpr (!SPH && ND == 3 && std::is_same<S, R>::value) {
    // Step 1 on the whole-zone 3-D kernel where the grid is of its kind: transport with the
    // advective fluxes; the flux rows' zone-local velocity terms move to the frequency step
    StepArgs<S> s1 = a;
    s1.src = 0;
    s1.Ea = nullptr;
    s1.dEm = nullptr;
    s1.p_energy = s1.p_maxf2 = nullptr;
    s1.p_nun = s1.p_nnp = nullptr;
    const int rc = launch_c3_vel<S>(ctx, geo, s1, va, st);
    if (rc == FORNAX_OK) {
      fused = true;
      for (int k = 0; k < 3; ++k) vf.Fn[k] = a.F[k];
    } else if (rc != FORNAX_EUNSUPPORTED) {
      return rc;
    }
  }
  if (!fused) {
    const int64_t nzg = a.nzones * a.G;
    hipLaunchKernelGGL((k_vel_explicit<S, R, SPH, ND>), dim3((unsigned)((nzg + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       st, a, geo, va);
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  // Step 2 and the interaction update, in place on the output
  StepArgs<S> b = a;
  b.E = b.Eo;
  for (int k = 0; k < 3; ++k) b.F[k] = b.Fo[k];
  const bool want = diag && (diag->energy_total || diag->max_f || diag->n_unrealizable || diag->n_nonpositive);
  b.dEm = diag ? diag->dE_matter : nullptr;
  const int64_t need = (a.nzones + a.zones_per_block - 1) / a.zones_per_block;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(need, std::min<int64_t>(ctx->nb_partials, 65536)));
  b.p_energy = ctx->p_energy;
  b.p_maxf2 = ctx->p_maxf2;
  b.p_nun = ctx->p_nun;
  b.p_nnp = ctx->p_nnp;
  hipLaunchKernelGGL((k_vel_freq<S, R, SPH, ND>), dim3(nb), dim3(BLOCK), 0, st, b, geo, vf, want ? 1 : 0);
  if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  if (want) return fm1_launch_finalize(ctx->p_energy, ctx->p_maxf2, ctx->p_nun, ctx->p_nnp, nb, diag, st);
  return FORNAX_OK;
}

template <typename S, typename R>
int launch_vel_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, fornax_m1_state* out,
                 const fornax_m1_coeffs* cf, const double* inflow, const fornax_m1_velocity* vel, double dt,
                 const fornax_m1_diag* diag, hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, inflow, dt);
  a.E = (const S*)in->E;
  a.Eo = (S*)out->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) {
    a.F[k] = (const S*)in->F[k];
    a.Fo[k] = (S*)out->F[k];
  }
  const VelArgs<S> va = vel_args<S>(ctx, vel);
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  switch (ctx->desc.ndim * 2 + (sph ? 1 : 0)) {
    case 2: return launch_vel_nd<S, R, false, 1>(ctx, geo, a, va, diag, st);
    case 3: return launch_vel_nd<S, R, true, 1>(ctx, geo, a, va, diag, st);
    case 4: return launch_vel_nd<S, R, false, 2>(ctx, geo, a, va, diag, st);
    case 5: return launch_vel_nd<S, R, true, 2>(ctx, geo, a, va, diag, st);
    case 6: return launch_vel_nd<S, R, false, 3>(ctx, geo, a, va, diag, st);
    default: return launch_vel_nd<S, R, true, 3>(ctx, geo, a, va, diag, st);
  }
}

template <typename S, typename R, bool SPH, int ND>
int launch_lab_nd(const Geo<R>& geo, const StepArgs<S>& a, const VelArgs<S>& va, double* El, double* const* Fl,
                  hipStream_t st) {
  hipLaunchKernelGGL((k_lab_frame<S, R, SPH, ND>), dim3((unsigned)((a.nzones + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                     st, a, geo, va, El, Fl[0], ND > 1 ? Fl[1] : nullptr, ND > 2 ? Fl[2] : nullptr);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template <typename S, typename R>
int launch_lab_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, const fornax_m1_velocity* vel,
                 double* El, double* const* Fl, hipStream_t st) {
  // coefficients are not read: point them at the state (fill_args needs non-null arrays)
  fornax_m1_coeffs cf{in->E, in->E, in->E};
  StepArgs<S> a;
  fill_args<S>(ctx, a, &cf, nullptr, 0.0);
  a.E = (const S*)in->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) a.F[k] = (const S*)in->F[k];
  const VelArgs<S> va = vel_args<S>(ctx, vel);
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  switch (ctx->desc.ndim * 2 + (sph ? 1 : 0)) {
    case 2: return launch_lab_nd<S, R, false, 1>(geo, a, va, El, Fl, st);
    case 3: return launch_lab_nd<S, R, true, 1>(geo, a, va, El, Fl, st);
    case 4: return launch_lab_nd<S, R, false, 2>(geo, a, va, El, Fl, st);
    case 5: return launch_lab_nd<S, R, true, 2>(geo, a, va, El, Fl, st);
    case 6: return launch_lab_nd<S, R, false, 3>(geo, a, va, El, Fl, st);
    default: return launch_lab_nd<S, R, true, 3>(geo, a, va, El, Fl, st);
  }
}

}  // namespace

int fm1_launch_step_velocity(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                             const fornax_m1_coeffs* cf, const double* inflow, const fornax_m1_velocity* vel,
                             double dt, const fornax_m1_diag* diag, hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_vel_t<double, double>(ctx, ctx->geo_d, in, out, cf, inflow, vel, dt, diag, stream);
  return launch_vel_t<float, float>(ctx, ctx->geo_f, in, out, cf, inflow, vel, dt, diag, stream);
}

int fm1_launch_lab_frame(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_velocity* vel, double* E_lab,
                         double* const* F_lab, hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_lab_t<double, double>(ctx, ctx->geo_d, in, vel, E_lab, F_lab, stream);
  return launch_lab_t<float, float>(ctx, ctx->geo_f, in, vel, E_lab, F_lab, stream);
}
