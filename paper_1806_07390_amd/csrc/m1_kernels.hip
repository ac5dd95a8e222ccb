// m1_kernels.hip -- gfx950 kernels of libfornax_m1 (one explicit transport + implicit
// interaction step of the multigroup M1 radiation moments, static medium).
//
// Method (Skinner et al. 2019, FORNAX):
//   finite-volume update, eq:finite_vol; linear reconstruction in the volume coordinate,
//   eq:recon_constraints with n = 1, minmod limited; M1 closure; HLL fluxes with the
//   asymptotic-diffusion correction of the energy flux, eq:hll / eq:epsilon; geometric source
//   terms of the covariant flux equation with the overrides eq:angmom / eq:grad2P;
//   backward-Euler interaction update eq:be_update and the flux update that follows it.
// Readings of details the paper leaves open (all shared with the library's documentation):
//   wavespeeds +-c (physical), i.e. +-c/h_d in x^d; tau_cell = mean (kappa + sigma) of the
//   two zones times their mean proper width; epsilon on the energy flux only; a zone whose
//   face state in direction d is not realizable (E <= 0 or |F^| > cE) is piecewise constant
//   in d; emissivity j = c kappa B; f^2 clamped to 1, Eddington value for E <= 0.
//
// Layout: structure of arrays, zone-group index ((k n1 + j) n0 + i) G + g, group innermost,
// so a block of whole zones reads and writes contiguous runs of every component.

#include <hip/hip_runtime.h>

#include "m1_internal.h"

namespace fm1 {

template <typename R>
__device__ __forceinline__ R minmod(R a, R b) {
  return (a * b <= R(0)) ? R(0) : (fabs(a) <= fabs(b) ? a : b);
}

// cell-centred scale factors sqrt(<g_kk>) at extended indices (ei, ej)
template <typename R, bool SPH>
__device__ __forceinline__ void cell_h(const Geo<R>& geo, int ei, int ej, R h[3]) {
  if constexpr (SPH) {
    R r = geo.hr[ei];
    h[0] = r;
    h[1] = r;
    h[2] = r * geo.hs[ej];
  } else {
    h[0] = h[1] = h[2] = R(1);
  }
}

// scale factors at the centre of a d-face with extended face index ef, zone row (ei, ej)
template <typename R, bool SPH>
__device__ __forceinline__ void face_h(const Geo<R>& geo, int d, int ei, int ej, int ef, R h[3]) {
  if constexpr (SPH) {
    R r = (d == 0) ? geo.rf[ef] : geo.rc[ei];
    R s = (d == 1) ? geo.sf[ef] : geo.sc[ej];
    h[0] = r;
    h[1] = r;
    h[2] = r * s;
  } else {
    h[0] = h[1] = h[2] = R(1);
  }
}

// Proper width h_d Delta x^d of the zone with extended indices (ei, ej) along d.
template <typename R, bool SPH>
__device__ __forceinline__ R proper_width(const Geo<R>& geo, int d, int ei, int ej) {
  if constexpr (SPH) {
    R r = geo.hr[ei];
    return (d == 2) ? r * geo.hs[ej] * geo.dx[2] : r * geo.dx[d];
  } else {
    return geo.dx[d];
  }
}

// State of the zone whose index along d is m (possibly a ghost) in the row of (i, j, k), and
// optionally its total opacity.  Ghost rules: periodic wrap, outflow copy, reflection with
// the normal flux flipped, prescribed inflow (E, physical F) with the ghost's own scale
// factors, and the polar-axis copy (mirror in theta, shift n2/2 in phi, flip F_theta, F_phi).
template <typename S, typename R, bool SPH>
__device__ __forceinline__ void fetch(const StepArgs<S>& a, const Geo<R>& geo, int d, int m, int i, int j, int k,
                                      int grp, R q[4], R* ks) {
  int mm[3] = {i, j, k};
  mm[d] = m;
  R sg[3] = {R(1), R(1), R(1)};
  bool infl = false;
  const int nd = a.n[d];
  if (m < 0 || m >= nd) {
    const bool low = m < 0;
    const int bc = low ? a.bc_lo[d] : a.bc_hi[d];
    if (bc == FORNAX_BC_PERIODIC) {
      mm[d] = ((m % nd) + nd) % nd;
    } else if (bc == FORNAX_BC_OUTFLOW) {
      mm[d] = low ? 0 : nd - 1;
    } else if (bc == FORNAX_BC_REFLECT) {
      mm[d] = low ? -1 - m : 2 * nd - 1 - m;
      sg[d] = R(-1);
    } else if (bc == FORNAX_BC_INFLOW) {
      mm[d] = low ? 0 : nd - 1;
      infl = true;
    } else {  // polar axis
      mm[d] = low ? -1 - m : 2 * nd - 1 - m;
      mm[2] = (mm[2] + a.n[2] / 2) % a.n[2];
      sg[1] = R(-1);
      sg[2] = R(-1);
    }
  }
  const int64_t zg = (((int64_t)mm[2] * a.n[1] + mm[1]) * a.n[0] + mm[0]) * a.G + grp;
  if (ks) *ks = R(a.kap[zg]) + R(a.sig[zg]);
  if (infl) {
    const double* in = a.inflow + grp * (1 + a.ndim);
    R h[3];
    cell_h<R, SPH>(geo, (d == 0 ? m : i) + NG, (d == 1 ? m : j) + NG, h);
    q[0] = R(in[0]);
    for (int c = 0; c < 3; ++c) q[1 + c] = (c < a.ndim) ? h[c] * R(in[1 + c]) : R(0);
  } else {
    q[0] = R(a.E[zg]);
    for (int c = 0; c < 3; ++c) q[1 + c] = (c < a.ndim) ? sg[c] * R(a.F[c][zg]) : R(0);
  }
}

// E > 0 and |F^| <= cE with F^_k = F_k / h_k
template <typename R>
__device__ __forceinline__ bool realizable(const R q[4], const R h[3], R c, int ndim) {
  if (!(q[0] > R(0))) return false;
  R F2 = R(0);
  for (int k = 0; k < ndim; ++k) {
    R fk = q[1 + k] / h[k];
    F2 += fk * fk;
  }
  R cE = c * q[0];
  return F2 <= cE * cE;
}

// Linear reconstruction of one zone along d (extended index e): face states at its lower
// and upper faces, with the piecewise-constant fallback when either is not realizable.
template <typename R, bool SPH>
__device__ __forceinline__ void reconstruct(const StepArgsBase& a, const Geo<R>& geo, int d, int e, const R qm[4],
                                            const R q0[4], const R qp[4], const R hlo[3], const R hhi[3],
                                            bool lo_open, bool hi_open, R lo[4], R hi[4]) {
  const R c = R(a.c);
  const R idm = geo.idm[d][e], idp = geo.idp[d][e], dl = geo.dlo[d][e], dh = geo.dhi[d][e];
  for (int cp = 0; cp < 4; ++cp) {
    R s = R(0);
    if (cp <= a.ndim) {
      if (a.limiter == FORNAX_LIMITER_MINMOD) {
        s = minmod((q0[cp] - qm[cp]) * idm, (qp[cp] - q0[cp]) * idp);
      } else if (a.limiter == FORNAX_LIMITER_MC) {
        R sa = (q0[cp] - qm[cp]) * idm, sb = (qp[cp] - q0[cp]) * idp, sc = (qp[cp] - qm[cp]) * geo.idc[d][e];
        s = minmod(R(2) * sa, minmod(R(2) * sb, sc));
      }
    }
    lo[cp] = q0[cp] + s * dl;
    hi[cp] = q0[cp] + s * dh;
  }
  const bool ok = (!lo_open || realizable(lo, hlo, c, a.ndim)) && (!hi_open || realizable(hi, hhi, c, a.ndim));
  if (!ok)
    for (int cp = 0; cp < 4; ++cp) lo[cp] = hi[cp] = q0[cp];
}

// M1 closure: P^ = E [ (1 - f^2)/(1 + s) I + 3/(2 + s) f f ], s = sqrt(4 - 3 f^2), f = F^/(cE)
// (algebraically the Levermore form chi = (3 + 4 f^2)/(5 + 2 s), written without
// cancellation as f -> 1).  Physical components; full tensor (row-major 3x3).
template <typename R>
__device__ __forceinline__ void closure_full(const R q[4], const R h[3], R c, int ndim, int eddington, R P[9]) {
  const R E = q[0];
  for (int t = 0; t < 9; ++t) P[t] = R(0);
  if (eddington || !(E > R(0))) {
    P[0] = P[4] = P[8] = E / R(3);
    return;
  }
  R Fh[3];
  for (int k = 0; k < 3; ++k) Fh[k] = (k < ndim) ? q[1 + k] / h[k] : R(0);
  const R F2 = Fh[0] * Fh[0] + Fh[1] * Fh[1] + Fh[2] * Fh[2];
  const R cE = c * E;
  R f2 = F2 / (cE * cE);
  R inv;
  if (f2 > R(1)) {
    f2 = R(1);
    inv = R(1) / sqrt(F2);
  } else {
    inv = R(1) / cE;
  }
  R f[3] = {Fh[0] * inv, Fh[1] * inv, Fh[2] * inv};
  const R s = sqrt(R(4) - R(3) * f2);
  const R r = R(1) / ((R(1) + s) * (R(2) + s));
  const R iso = E * (R(1) - f2) * (R(2) + s) * r;
  const R ani = E * R(3) * (R(1) + s) * r;
  for (int p = 0; p < 3; ++p)
    for (int q2 = 0; q2 < 3; ++q2) P[3 * p + q2] = ani * f[p] * f[q2];
  P[0] += iso;
  P[4] += iso;
  P[8] += iso;
}

// Row d of the closure, P^^{dk}, k < 3; in the MIXED path (R = float) the closure is evaluated
// in double where f^2 >= f2_fp64.
template <typename R>
__device__ __forceinline__ void closure_row(const R q[4], const R h[3], int d, R c, int ndim, int eddington,
                                            double f2_fp64, R P[3]) {
  if constexpr (sizeof(R) == 4) {
    R Fh2 = R(0);
    for (int k = 0; k < ndim; ++k) {
      R fk = q[1 + k] / h[k];
      Fh2 += fk * fk;
    }
    R cE = c * q[0];
    if (!eddington && q[0] > R(0) && (double)Fh2 >= f2_fp64 * (double)(cE * cE)) {
      double qd[4] = {q[0], q[1], q[2], q[3]}, hd[3] = {h[0], h[1], h[2]}, Pd[9];
      closure_full<double>(qd, hd, (double)c, ndim, 0, Pd);
      for (int k = 0; k < 3; ++k) P[k] = (R)Pd[3 * d + k];
      return;
    }
  }
  R Pf[9];
  closure_full<R>(q, h, c, ndim, eddington, Pf);
  for (int k = 0; k < 3; ++k) P[k] = Pf[3 * d + k];
}

// HLL flux (coordinate components) across a d-face with face scale factors h, left/right
// states qL, qR and the correction factor eps of the energy flux.
template <typename R, bool SPH>
__device__ __forceinline__ void hll(const StepArgsBase& a, int d, const R qL[4], const R qR[4], const R h[3], R eps,
                                    R flux[4]) {
  const R c = R(a.c);
  R PL[3], PR[3];
  closure_row<R>(qL, h, d, c, a.ndim, a.closure, a.f2_fp64, PL);
  closure_row<R>(qR, h, d, c, a.ndim, a.closure, a.f2_fp64, PR);
  R ihd = R(1), S = c;
  if constexpr (SPH) {
    ihd = R(1) / h[d];
    S = c * ihd;
  }
  const R half = R(0.5);
  // energy: F^d = F_d / h_d^2; S_R = -S_L = S
  flux[0] = half * ((qL[1 + d] + qR[1 + d]) * (ihd * ihd)) - half * eps * S * (qR[0] - qL[0]);
  // covariant flux components: c^2 P^d_k = c^2 P^^{dk} h_k / h_d
  for (int k = 0; k < 3; ++k) {
    if (k < a.ndim) {
      R hk = SPH ? h[k] * ihd : R(1);
      flux[1 + k] = half * c * c * (PL[k] + PR[k]) * hk - half * S * (qR[1 + k] - qL[1 + k]);
    } else {
      flux[1 + k] = R(0);
    }
  }
}

template <typename R>
__device__ __forceinline__ R epsilon_of(R ksL, R ksR, R dlL, R dlR) {
  const R tau = R(0.5) * (ksL + ksR) * (R(0.5) * (dlL + dlR));
  return (tau > R(1)) ? R(1) / tau : R(1);
}

// Flux through the d-face with index f (face f-1/2 of zone f along d) of the row (i, j, k),
// from the five zones f-3 .. f+1 ... computed from q[] holding zones f-2 .. f+1 (4 zones) and
// the opacities of zones f-1, f.  lo/hi open flags come from the area table.
template <typename S, typename R, bool SPH>
__device__ __forceinline__ void face_flux(const StepArgs<S>& a, const Geo<R>& geo, int d, int f, int i, int j,
                                          const R q[4][4], R ksL, R ksR, R flux[4]) {
  const int ef = f + NG;
  if (geo.wf[d][ef] == R(0)) {
    for (int c = 0; c < 4; ++c) flux[c] = R(0);
    return;
  }
  const int ei = i + NG, ej = j + NG;
  R h0[3], h1[3], h2[3];
  face_h<R, SPH>(geo, d, ei, ej, ef - 1, h0);
  face_h<R, SPH>(geo, d, ei, ej, ef, h1);
  face_h<R, SPH>(geo, d, ei, ej, ef + 1, h2);
  const bool o0 = geo.wf[d][ef - 1] != R(0), o2 = geo.wf[d][ef + 1] != R(0);
  R Llo[4], Lhi[4], Rlo[4], Rhi[4];
  reconstruct<R, SPH>(a, geo, d, ef - 1, q[0], q[1], q[2], h0, h1, o0, true, Llo, Lhi);
  reconstruct<R, SPH>(a, geo, d, ef, q[1], q[2], q[3], h1, h2, true, o2, Rlo, Rhi);
  const int eL = ef - 1;
  const R dlL = proper_width<R, SPH>(geo, d, d == 0 ? eL : ei, d == 1 ? eL : ej);
  const R dlR = proper_width<R, SPH>(geo, d, d == 0 ? ef : ei, d == 1 ? ef : ej);
  const R eps = epsilon_of(ksL, ksR, dlL, dlR);
  hll<R, SPH>(a, d, Lhi, Rlo, h1, eps, flux);
}

// geometric source c^2 sum_{l,m} <Gamma^l_{km}> P^m_l for the covariant flux components of a
// spherical (ln r, theta, phi) zone, P^m_l = P^^{ml} h_l / h_m with cell-centred h
template <typename R>
__device__ __forceinline__ void geometric_source(const R P[9], const R h[3], const R* gam, R c, R Sg[3]) {
  const R G323 = gam[0], G133 = gam[1], G233 = gam[2], G222 = gam[3];
  const R c2 = c * c;
  // F_1: Gamma^1_11 = Gamma^2_12 = Gamma^3_13 = 1
  Sg[0] = c2 * (P[0] + P[4] + P[8]);
  // F_2: Gamma^1_22 = -1, Gamma^2_21 = 1, <Gamma^2_22>, <Gamma^3_23>
  Sg[1] = c2 * (-P[3] * (h[0] / h[1]) + P[1] * (h[1] / h[0]) + G222 * P[4] + G323 * P[8]);
  // F_3: <Gamma^1_33>, <Gamma^2_33>, Gamma^3_31 = 1, <Gamma^3_32>
  Sg[2] = c2 * (G133 * P[6] * (h[0] / h[2]) + G233 * P[7] * (h[1] / h[2]) + P[2] * (h[2] / h[0]) +
                G323 * P[5] * (h[2] / h[1]));
}

// ------------------------------------------------------------------------------------------
// The fused step: one thread per zone-group; a block holds whole zones (BLOCK / G of them).
// ------------------------------------------------------------------------------------------
template <typename S, typename R, int DIM, bool SPH>
__global__ void __launch_bounds__(BLOCK) k_step(StepArgs<S> a, Geo<R> geo) {
  const int G = a.G;
  const int lz = threadIdx.x / G, grp = threadIdx.x - lz * G;
  const int64_t z = (int64_t)blockIdx.x * a.zones_per_block + lz;
  const bool act = (lz < a.zones_per_block) && (z < a.nzones);
  double e_c = 0.0, mf2 = 0.0, dz = 0.0;
  int nun = 0, nnp = 0;
  if (act) {
    const int i = (int)(z % a.n[0]);
    const int j = (int)((z / a.n[0]) % a.n[1]);
    const int k = (int)(z / ((int64_t)a.n[0] * a.n[1]));
    R q0[4];
    fetch<S, R, SPH>(a, geo, 0, i, i, j, k, grp, q0, nullptr);
    R acc[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int m = (d == 0) ? i : (d == 1 ? j : k);
      R q[5][4], ks[3];
      for (int o = -2; o <= 2; ++o)
        fetch<S, R, SPH>(a, geo, d, m + o, i, j, k, grp, q[o + 2], (o >= -1 && o <= 1) ? &ks[o + 1] : nullptr);
      R flo[4], fhi[4];
      face_flux<S, R, SPH>(a, geo, d, m, i, j, reinterpret_cast<const R(*)[4]>(&q[0][0]), ks[0], ks[1], flo);
      face_flux<S, R, SPH>(a, geo, d, m + 1, i, j, reinterpret_cast<const R(*)[4]>(&q[1][0]), ks[1], ks[2], fhi);
      const int e = m + NG;
      const R wlo = geo.wf[d][e], whi = geo.wf[d][e + 1], iW = geo.iW[d][e];
      for (int c = 0; c <= a.ndim; ++c) acc[c] += (whi * fhi[c] - wlo * flo[c]) * iW;
    }
    const R dtR = R(a.dt);
    R Um[4];
    for (int c = 0; c < 4; ++c) Um[c] = (c <= a.ndim) ? q0[c] - dtR * acc[c] : R(0);
    if constexpr (SPH) {
      R h[3], P[9], Sg[3];
      cell_h<R, SPH>(geo, i + NG, j + NG, h);
      closure_full<R>(q0, h, R(a.c), a.ndim, a.closure, P);
      geometric_source<R>(P, h, geo.gam + 4 * j, R(a.c), Sg);
      for (int c = 0; c < a.ndim; ++c) Um[1 + c] += dtR * Sg[c];
    }
    // implicit interaction update in double
    const int64_t zg = z * G + grp;
    const double kd = (double)a.kap[zg], sd = (double)a.sig[zg], Bd = (double)a.B[zg];
    const double c = a.c, dt = a.dt;
    const double Emd = (double)Um[0];
    const double E1 = (Emd + dt * (c * kd * Bd)) / (1.0 + (c * dt) * kd);
    const double fden = 1.0 + (c * dt) * (kd + sd);
    const S E1s = (S)E1;
    a.Eo[zg] = E1s;
    double F1s[3] = {0.0, 0.0, 0.0};
    for (int cc = 0; cc < a.ndim; ++cc) {
      const S v = (S)((double)Um[1 + cc] / fden);
      a.Fo[cc][zg] = v;
      F1s[cc] = (double)v;
    }
    if (a.p_energy || a.dEm) {
      const double E1d = (double)E1s;
      const double V = geo.Wd[0][i + NG] * geo.Wd[1][j + NG] * geo.Wd[2][k + NG];
      e_c = V * E1d;
      dz = E1d - Emd;
      double hd[3] = {1.0, 1.0, 1.0};
      if constexpr (SPH) {
        hd[0] = hd[1] = (double)geo.hr[i + NG];
        hd[2] = hd[0] * (double)geo.hs[j + NG];
      }
      double F2 = 0.0;
      for (int cc = 0; cc < a.ndim; ++cc) {
        const double fk = F1s[cc] / hd[cc];
        F2 += fk * fk;
      }
      const double cE = c * E1d;
      if (E1d > 0.0) mf2 = F2 / (cE * cE);
      const double u = (sizeof(S) == 8) ? 0x1p-53 : 0x1p-24;
      const double lim = cE * (1.0 + 8.0 * u);
      nun = (F2 > lim * lim) ? 1 : 0;
      nnp = (E1d > 0.0) ? 0 : 1;
    }
  }
  if (!a.p_energy && !a.dEm) return;
  __shared__ double sh_a[BLOCK];
  __shared__ double sh_b[BLOCK];
  __shared__ int sh_u[BLOCK];
  __shared__ int sh_p[BLOCK];
  const int t = threadIdx.x;
  // dE_matter: -sum over the zone's groups, in group order
  if (a.dEm) {
    sh_a[t] = dz;
    __syncthreads();
    if (act && grp == 0) {
      double s = 0.0;
      for (int g2 = 0; g2 < G; ++g2) s += sh_a[t + g2];
      a.dEm[z] = -s;
    }
    __syncthreads();
  }
  if (!a.p_energy) return;
  sh_a[t] = e_c;
  sh_b[t] = mf2;
  sh_u[t] = nun;
  sh_p[t] = nnp;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh_a[t] += sh_a[t + s];
      sh_b[t] = fmax(sh_b[t], sh_b[t + s]);
      sh_u[t] += sh_u[t + s];
      sh_p[t] += sh_p[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    a.p_energy[blockIdx.x] = sh_a[0];
    a.p_maxf2[blockIdx.x] = sh_b[0];
    a.p_nun[blockIdx.x] = sh_u[0];
    a.p_nnp[blockIdx.x] = sh_p[0];
  }
}

// second stage of the diagnostics reduction: fixed order, one block
__global__ void __launch_bounds__(BLOCK) k_finalize(const double* p_energy, const double* p_maxf2, const int* p_nun,
                                                     const int* p_nnp, int nb, double* energy, double* maxf,
                                                     int* nun, int* nnp) {
  __shared__ double sa[BLOCK], sb[BLOCK];
  __shared__ int su[BLOCK], sp[BLOCK];
  const int t = threadIdx.x;
  double ea = 0.0, mb = 0.0;
  int ua = 0, pa = 0;
  for (int b = t; b < nb; b += BLOCK) {
    ea += p_energy[b];
    mb = fmax(mb, p_maxf2[b]);
    ua += p_nun[b];
    pa += p_nnp[b];
  }
  sa[t] = ea;
  sb[t] = mb;
  su[t] = ua;
  sp[t] = pa;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) {
      sa[t] += sa[t + s];
      sb[t] = fmax(sb[t], sb[t + s]);
      su[t] += su[t + s];
      sp[t] += sp[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (energy) *energy = sa[0];
    if (maxf) *maxf = sqrt(sb[0]);
    if (nun) *nun = su[0];
    if (nnp) *nnp = sp[0];
  }
}

// ------------------------------------------------------------------------------------------
// Face fluxes only: one thread per face-group along direction d.
// ------------------------------------------------------------------------------------------
template <typename S, typename R, bool SPH>
__global__ void __launch_bounds__(BLOCK) k_flux(StepArgs<S> a, Geo<R> geo, int d, S* out) {
  int m[3] = {a.n[0], a.n[1], a.n[2]};
  m[d] += 1;
  const int64_t nfg = (int64_t)m[0] * m[1] * m[2] * a.G;
  const int64_t id = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (id >= nfg) return;
  const int grp = (int)(id % a.G);
  const int64_t f = id / a.G;
  int idx[3] = {(int)(f % m[0]), (int)((f / m[0]) % m[1]), (int)(f / ((int64_t)m[0] * m[1]))};
  const int fi = idx[d];
  // zones of the row: use an in-range index for the d position (fetch replaces it)
  int base[3] = {idx[0], idx[1], idx[2]};
  base[d] = 0;
  R q[4][4], ksL, ksR;
  for (int o = -2; o <= 1; ++o)
    fetch<S, R, SPH>(a, geo, d, fi + o, base[0], base[1], base[2], grp, q[o + 2],
                     o == -1 ? &ksL : (o == 0 ? &ksR : nullptr));
  R fl[4];
  face_flux<S, R, SPH>(a, geo, d, fi, base[0], base[1], reinterpret_cast<const R(*)[4]>(&q[0][0]), ksL, ksR, fl);
  const int nc = 1 + a.ndim;
  for (int c = 0; c < nc; ++c) out[id * nc + c] = (S)fl[c];
}

// ------------------------------------------------------------------------------------------
// Implicit interaction update alone (in place), double arithmetic.
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(BLOCK) k_source(StepArgs<S> a) {
  const int G = a.G;
  const int lz = threadIdx.x / G, grp = threadIdx.x - lz * G;
  const int64_t z = (int64_t)blockIdx.x * a.zones_per_block + lz;
  const bool act = (lz < a.zones_per_block) && (z < a.nzones);
  double dz = 0.0;
  if (act) {
    const int64_t zg = z * G + grp;
    const double kd = (double)a.kap[zg], sd = (double)a.sig[zg], Bd = (double)a.B[zg];
    const double c = a.c, dt = a.dt;
    const double Em = (double)a.E[zg];
    const double E1 = (Em + dt * (c * kd * Bd)) / (1.0 + (c * dt) * kd);
    const double fden = 1.0 + (c * dt) * (kd + sd);
    const S E1s = (S)E1;
    a.Eo[zg] = E1s;
    for (int cc = 0; cc < a.ndim; ++cc) a.Fo[cc][zg] = (S)((double)a.F[cc][zg] / fden);
    dz = (double)E1s - Em;
  }
  if (!a.dEm) return;
  __shared__ double sh[BLOCK];
  sh[threadIdx.x] = dz;
  __syncthreads();
  if (act && grp == 0) {
    double s = 0.0;
    for (int g2 = 0; g2 < G; ++g2) s += sh[threadIdx.x + g2];
    a.dEm[z] = -s;
  }
}

__global__ void __launch_bounds__(BLOCK) k_copy(float4* __restrict__ dst, const float4* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) dst[i] = src[i];
}

}  // namespace fm1

using namespace fm1;

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
namespace {

template <typename S>
void fill_args(const fornax_m1_ctx* ctx, StepArgs<S>& a, const fornax_m1_coeffs* cf, const double* inflow,
               double dt) {
  const fornax_m1_desc& D = ctx->desc;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = D.n[d];
    a.bc_lo[d] = D.bc_lo[d];
    a.bc_hi[d] = D.bc_hi[d];
  }
  a.G = D.ngroups;
  a.ndim = D.ndim;
  a.limiter = D.limiter;
  a.closure = D.closure;
  a.zones_per_block = BLOCK / D.ngroups;
  a.nzones = (int64_t)D.n[0] * D.n[1] * D.n[2];
  a.c = D.c;
  a.dt = dt;
  a.f2_fp64 = D.f_fp64 * D.f_fp64;
  a.inflow = inflow;
  a.kap = (const S*)cf->kappa;
  a.sig = (const S*)cf->sigma;
  a.B = (const S*)cf->B;
  a.E = nullptr;
  a.Eo = nullptr;
  for (int k = 0; k < 3; ++k) {
    a.F[k] = nullptr;
    a.Fo[k] = nullptr;
  }
  a.dEm = nullptr;
  a.p_energy = nullptr;
  a.p_maxf2 = nullptr;
  a.p_nun = nullptr;
  a.p_nnp = nullptr;
}

template <typename S, typename R>
int launch_step_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, fornax_m1_state* out,
                  const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_diag* diag,
                  hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, inflow, dt);
  a.E = (const S*)in->E;
  a.Eo = (S*)out->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) {
    a.F[k] = (const S*)in->F[k];
    a.Fo[k] = (S*)out->F[k];
  }
  bool want = diag && (diag->energy_total || diag->max_f || diag->n_unrealizable || diag->n_nonpositive);
  if (diag) a.dEm = diag->dE_matter;
  if (want) {
    a.p_energy = ctx->p_energy;
    a.p_maxf2 = ctx->p_maxf2;
    a.p_nun = ctx->p_nun;
    a.p_nnp = ctx->p_nnp;
  }
  const int nb = ctx->nblocks_step;
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  const int D = ctx->desc.ndim;
  dim3 grid(nb), block(BLOCK);
  if (sph) {
    if (D == 1) hipLaunchKernelGGL((k_step<S, R, 1, true>), grid, block, 0, st, a, geo);
    else if (D == 2) hipLaunchKernelGGL((k_step<S, R, 2, true>), grid, block, 0, st, a, geo);
    else hipLaunchKernelGGL((k_step<S, R, 3, true>), grid, block, 0, st, a, geo);
  } else {
    if (D == 1) hipLaunchKernelGGL((k_step<S, R, 1, false>), grid, block, 0, st, a, geo);
    else if (D == 2) hipLaunchKernelGGL((k_step<S, R, 2, false>), grid, block, 0, st, a, geo);
    else hipLaunchKernelGGL((k_step<S, R, 3, false>), grid, block, 0, st, a, geo);
  }
  if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  if (want) {
    hipLaunchKernelGGL(k_finalize, dim3(1), block, 0, st, ctx->p_energy, ctx->p_maxf2, ctx->p_nun, ctx->p_nnp, nb,
                       diag->energy_total, diag->max_f, diag->n_unrealizable, diag->n_nonpositive);
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  return FORNAX_OK;
}

template <typename S, typename R>
int launch_flux_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, const fornax_m1_coeffs* cf,
                  const double* inflow, void* face_flux[3], hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, inflow, 0.0);
  a.E = (const S*)in->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) a.F[k] = (const S*)in->F[k];
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  for (int d = 0; d < ctx->desc.ndim; ++d) {
    int64_t m[3] = {a.n[0], a.n[1], a.n[2]};
    m[d] += 1;
    int64_t nfg = m[0] * m[1] * m[2] * a.G;
    dim3 grid((unsigned)((nfg + BLOCK - 1) / BLOCK));
    if (sph) hipLaunchKernelGGL((k_flux<S, R, true>), grid, dim3(BLOCK), 0, st, a, geo, d, (S*)face_flux[d]);
    else hipLaunchKernelGGL((k_flux<S, R, false>), grid, dim3(BLOCK), 0, st, a, geo, d, (S*)face_flux[d]);
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  return FORNAX_OK;
}

template <typename S>
int launch_source_t(fornax_m1_ctx* ctx, fornax_m1_state* io, const fornax_m1_coeffs* cf, double dt, double* dEm,
                    hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, nullptr, dt);
  a.E = (const S*)io->E;
  a.Eo = (S*)io->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) {
    a.F[k] = (const S*)io->F[k];
    a.Fo[k] = (S*)io->F[k];
  }
  a.dEm = dEm;
  hipLaunchKernelGGL(k_source<S>, dim3(ctx->nblocks_step), dim3(BLOCK), 0, st, a);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

}  // namespace

int fm1_launch_step(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out, const fornax_m1_coeffs* cf,
                    const double* inflow, double dt, const fornax_m1_diag* diag, hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_step_t<double, double>(ctx, ctx->geo_d, in, out, cf, inflow, dt, diag, stream);
  return launch_step_t<float, float>(ctx, ctx->geo_f, in, out, cf, inflow, dt, diag, stream);
}

int fm1_launch_flux(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_coeffs* cf, const double* inflow,
                    void* face_flux[3], hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_flux_t<double, double>(ctx, ctx->geo_d, in, cf, inflow, face_flux, stream);
  return launch_flux_t<float, float>(ctx, ctx->geo_f, in, cf, inflow, face_flux, stream);
}

int fm1_launch_source(fornax_m1_ctx* ctx, fornax_m1_state* inout, const fornax_m1_coeffs* cf, double dt, double* dEm,
                      hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64) return launch_source_t<double>(ctx, inout, cf, dt, dEm, stream);
  return launch_source_t<float>(ctx, inout, cf, dt, dEm, stream);
}

int fm1_launch_adjoint(fornax_m1_ctx*, const fornax_m1_state*, const fornax_m1_coeffs*, const double*, double,
                       const fornax_m1_state*, fornax_m1_state*, void*, hipStream_t) {
  return FORNAX_EUNSUPPORTED;
}

int fm1_launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t stream) {
  int64_t n = nbytes / 16;
  if (n == 0) return FORNAX_OK;
  int64_t blocks = (n + BLOCK - 1) / BLOCK;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(BLOCK), 0, stream, (float4*)dst, (const float4*)src, n);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}
