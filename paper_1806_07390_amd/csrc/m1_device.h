// m1_device.h -- device functions of the M1 step shared by the kernels of libfornax_m1:
// ghost-zone rules, linear reconstruction with the realizability fallback, the M1 closure,
// the HLL flux with the diffusion correction, the geometric source terms and the implicit
// interaction update.  ND (1..3) is the number of active directions and flux components;
// components beyond ND are identically zero and never computed.
//
// Method (Skinner et al. 2019, FORNAX): eq:finite_vol, eq:recon_constraints (n = 1, minmod
// limited), the M1 closure, eq:hll / eq:epsilon, the covariant geometric sources with the
// overrides eq:angmom / eq:grad2P, eq:be_update.  Readings of details the paper leaves open:
// wavespeeds +-c (physical), i.e. +-c/h_d in x^d; tau_cell = mean (kappa + sigma) of the two
// zones times their mean proper width; epsilon on the energy flux only; a zone whose face
// state in direction d is not realizable (E <= 0 or |F^| > cE) is piecewise constant in d;
// emissivity j = c kappa B; f^2 clamped to 1, Eddington value for E <= 0.
#pragma once

#include <hip/hip_runtime.h>

#include "m1_internal.h"

namespace fm1 {

// minmod(a, b): 0 when a and b differ in sign, else the one of smaller magnitude; this is the
// median of a, b and 0 (which differs from the product test a b <= 0 only when the product
// underflows, below any slope that can change a face state).
__device__ __forceinline__ double minmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }

// 1/x: the hardware estimate (about 25 correct bits) refined by one Newton-Raphson step
// (double; within about 10 ulp for the normal, finite, non-zero arguments used here), or
// the 1-ulp float estimate.
__device__ __forceinline__ double rcp_(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }

// sqrt(x) for normal positive arguments: reciprocal square-root estimate, one coupled
// Newton step for (sqrt x, 1/(2 sqrt x)) and a final residual correction (double), or the
// hardware float square root.
__device__ __forceinline__ double sqrt_(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }

// A read of a geometry table.  The tables are written once, when the context is created, and
// never by a kernel: reads go through the constant address space, which lets the compiler use
// scalar loads where the index is uniform over the wave and keep the values across the
// kernel's own stores.
template <typename R>
__device__ __forceinline__ R gld(const R* p, int i) {
  return ((const __attribute__((address_space(4))) R*)p)[i];
}

// cell-centred scale factors sqrt(<g_kk>) at extended indices (ei, ej)
template <typename R, bool SPH>
__device__ __forceinline__ void cell_h(const Geo<R>& geo, int ei, int ej, R h[3]) {
  if constexpr (SPH) {
    R r = gld(geo.hr, ei);
    h[0] = r;
    h[1] = r;
    h[2] = r * gld(geo.hs, ej);
  } else {
    h[0] = h[1] = h[2] = R(1);
  }
}

// scale factors at the centre of a d-face with extended face index ef, zone row (ei, ej)
template <typename R, bool SPH>
__device__ __forceinline__ void face_h(const Geo<R>& geo, int d, int ei, int ej, int ef, R h[3]) {
  if constexpr (SPH) {
    R r = (d == 0) ? gld(geo.rf, ef) : gld(geo.rc, ei);
    R s = (d == 1) ? gld(geo.sf, ef) : gld(geo.sc, ej);
    h[0] = r;
    h[1] = r;
    h[2] = r * s;
  } else {
    h[0] = h[1] = h[2] = R(1);
  }
}

// inverse cell-centred scale factors 1/h (spherical tables of 1/sqrt(<r^2>), 1/sqrt(<sin^2>))
template <typename R, bool SPH>
__device__ __forceinline__ void cell_ih(const Geo<R>& geo, int ei, int ej, R ih[3]) {
  if constexpr (SPH) {
    const R ir = gld(geo.ihr, ei);
    ih[0] = ir;
    ih[1] = ir;
    ih[2] = ir * gld(geo.ihs, ej);
  } else {
    ih[0] = ih[1] = ih[2] = R(1);
  }
}

// inverse scale factors at the centre of a d-face (tables of 1/r and 1/|sin theta|; 0 on a
// polar-axis face, which is closed and never used)
template <typename R, bool SPH>
__device__ __forceinline__ void face_ih(const Geo<R>& geo, int d, int ei, int ej, int ef, R ih[3]) {
  if constexpr (SPH) {
    const R ir = (d == 0) ? gld(geo.irf, ef) : gld(geo.irc, ei);
    const R is = (d == 1) ? gld(geo.isf, ef) : gld(geo.isc, ej);
    ih[0] = ir;
    ih[1] = ir;
    ih[2] = ir * is;
  } else {
    ih[0] = ih[1] = ih[2] = R(1);
  }
}

// Proper width h_d Delta x^d of the zone with extended indices (ei, ej) along d.
template <typename R, bool SPH>
__device__ __forceinline__ R proper_width(const Geo<R>& geo, int d, int ei, int ej) {
  if constexpr (SPH) {
    R r = gld(geo.hr, ei);
    return (d == 2) ? r * gld(geo.hs, ej) * geo.dx[2] : r * geo.dx[d];
  } else {
    return geo.dx[d];
  }
}

// State of the zone whose index along d is m (possibly a ghost) in the row of (i, j, k), and
// optionally its total opacity.  Ghost rules: periodic wrap, outflow copy, reflection with
// the normal flux flipped, prescribed inflow (E, physical F) with the ghost's own scale
// factors, and the polar-axis copy (mirror in theta, shift n2/2 in phi, flip F_theta, F_phi).
// Zone-group indices fit in 32 bits (checked when the context is created).
template <typename S, typename R, bool SPH, int ND>
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
      mm[d] = low ? m + nd : m - nd;
      if (mm[d] < 0 || mm[d] >= nd) mm[d] = ((m % nd) + nd) % nd;
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
  const int zg = ((mm[2] * a.n[1] + mm[1]) * a.n[0] + mm[0]) * a.G + grp;
  if (ks) *ks = R(a.kap[zg]) + R(a.sig[zg]);
  if (infl) {
    const double* in = a.inflow + grp * (1 + ND);
    R h[3];
    cell_h<R, SPH>(geo, (d == 0 ? m : i) + NG, (d == 1 ? m : j) + NG, h);
    q[0] = R(in[0]);
    for (int c = 0; c < ND; ++c) q[1 + c] = h[c] * R(in[1 + c]);
  } else {
    q[0] = R(a.E[zg]);
    for (int c = 0; c < ND; ++c) q[1 + c] = sg[c] * R(a.F[c][zg]);
  }
  for (int c = ND; c < 3; ++c) q[1 + c] = R(0);
}

// E > 0 and |F^| <= cE with F^_k = F_k / h_k (ih = 1/h)
template <typename R, bool SPH, int ND>
__device__ __forceinline__ bool realizable(const R q[4], const R ih[3], R c) {
  R F2 = R(0);
  for (int k = 0; k < ND; ++k) {
    R fk = SPH ? q[1 + k] * ih[k] : q[1 + k];
    F2 += fk * fk;
  }
  R cE = c * q[0];
  return (q[0] > R(0)) && (F2 <= cE * cE);
}

// Linear reconstruction of one zone along d (extended index e), or parabolic with the PPM
// option: face states at its lower and upper faces, with the piecewise-constant fallback when
// either is not realizable.
// LIM: the limiter when known at compile time (a FORNAX_LIMITER_* value), -1 to read it from
// the arguments.  vs (spherical grids, nullable): the zone's idm, idp, dlo, dhi, idc of the
// tables, when the caller already holds them.
template <typename R, bool SPH, int ND, int LIM = -1>
__device__ __forceinline__ void reconstruct(const StepArgsBase& a, const Geo<R>& geo, int d, int e, const R qm[4],
                                            const R q0[4], const R qp[4], const R ihlo[3], const R ihhi[3],
                                            bool lo_open, bool hi_open, R lo[4], R hi[4], const R* vs = nullptr) {
  const R c = R(a.c);
  const int limiter = (LIM >= 0) ? LIM : a.limiter;
  R s[4];
  R dl = R(-0.5), dh = R(0.5);
  if constexpr (SPH) {
    if (limiter == FORNAX_LIMITER_PPM) {
      // parabolic, from the zone's weights in u = (x - x_i)/dx (volume-weighted moments); the
      // same decisions as the uniform Cartesian closed forms below
      const R* T = geo.ppm[d] + (size_t)PPM_TAB * e;
      for (int cp = 0; cp <= ND; ++cp) {
        const R pm = qm[cp], p0 = q0[cp], pp = qp[cp];
        R vl = p0, vh = p0;
        if ((p0 - pm) * (pp - p0) > R(0)) {
          vl = T[0] * pm + T[1] * p0 + T[2] * pp;
          vh = T[3] * pm + T[4] * p0 + T[5] * pp;
          const R c1 = T[6] * pm + T[7] * p0 + T[8] * pp, c2 = T[9] * pm + T[10] * p0 + T[11] * pp;
          if (fabs(c1) < R(2) * fabs(c2)) {
            if (c1 * c2 > R(0)) vl = pm + R(0.25) * (p0 - pm);
            else vh = pp + R(0.25) * (p0 - pp);
          }
          const R d1 = T[12] * vl + T[13] * p0 + T[14] * vh, d2 = T[15] * vl + T[16] * p0 + T[17] * vh;
          if (fabs(d1) < fabs(d2)) {
            if (d1 * d2 > R(0)) vl = T[18] * p0 + T[19] * vh;
            else vh = T[20] * vl + T[21] * p0;
          }
        }
        lo[cp] = vl;
        hi[cp] = vh;
      }
    }
    // slopes between volume centroids, face offsets from the centroid
    const R idm = vs ? vs[0] : gld(geo.idm[d], e), idp = vs ? vs[1] : gld(geo.idp[d], e);
    dl = vs ? vs[2] : gld(geo.dlo[d], e);
    dh = vs ? vs[3] : gld(geo.dhi[d], e);
    for (int cp = 0; cp <= ND; ++cp) {
      const R sa = (q0[cp] - qm[cp]) * idm, sb = (qp[cp] - q0[cp]) * idp;
      if (limiter == FORNAX_LIMITER_MINMOD) {
        s[cp] = minmod(sa, sb);
      } else if (limiter == FORNAX_LIMITER_MC) {
        s[cp] = minmod(R(2) * sa, minmod(R(2) * sb, (qp[cp] - qm[cp]) * (vs ? vs[4] : gld(geo.idc[d], e))));
      } else {
        s[cp] = R(0);
      }
    }
  } else if (limiter == FORNAX_LIMITER_PPM) {
    // uniform Cartesian zones, parabolic: in u = (x - x_i)/dx the parabola with the three
    // averages is p0 - c2/12 + c1 u + c2 u^2, c1 = (qp - qm)/2, c2 = (qm - 2 q0 + qp)/2
    (void)geo;
    (void)d;
    (void)e;
    for (int cp = 0; cp <= ND; ++cp) {
      const R pm = qm[cp], p0 = q0[cp], pp = qp[cp];
      R vl = p0, vh = p0;
      if ((p0 - pm) * (pp - p0) > R(0)) {
        vl = (R(2) * pm + R(5) * p0 - pp) * R(1.0 / 6.0);
        vh = (R(5) * p0 + R(2) * pp - pm) * R(1.0 / 6.0);
        // turning point -c1/(2 c2) between the centres of zones i-1 and i (c1 c2 > 0) or of
        // zones i and i+1 (c1 c2 < 0): that face from the parabola with zero slope at the
        // neighbour's centre through both averages, i.e. q_n + (q_i - q_n)/4
        const R c1 = R(0.5) * (pp - pm), c2 = R(0.5) * (pm - R(2) * p0 + pp);
        if (fabs(c1) < R(2) * fabs(c2)) {
          if (c1 * c2 > R(0)) vl = pm + R(0.25) * (p0 - pm);
          else vh = pp + R(0.25) * (p0 - pp);
        }
        // the parabola through vl, the average and vh: turning point -d1/(2 d2) inside the
        // zone (|d1| < |d2|) resets the nearer face so that the slope vanishes there
        const R d1 = vh - vl, d2 = R(3) * (vl + vh - R(2) * p0);
        if (fabs(d1) < fabs(d2)) {
          if (d1 * d2 > R(0)) vl = R(1.5) * p0 - R(0.5) * vh;
          else vh = R(1.5) * p0 - R(0.5) * vl;
        }
      }
      lo[cp] = vl;
      hi[cp] = vh;
    }
  } else {
    // uniform Cartesian zones: centroid = centre, faces at -+ dx/2 (slope times dx)
    (void)geo;
    (void)d;
    (void)e;
    for (int cp = 0; cp <= ND; ++cp) {
      const R dm = q0[cp] - qm[cp], dp = qp[cp] - q0[cp];
      if (limiter == FORNAX_LIMITER_MINMOD) {
        s[cp] = minmod(dm, dp);
      } else if (limiter == FORNAX_LIMITER_MC) {
        s[cp] = minmod(R(2) * dm, minmod(R(2) * dp, R(0.5) * (dm + dp)));
      } else {
        s[cp] = R(0);
      }
    }
  }
  if (limiter != FORNAX_LIMITER_PPM) {
    for (int cp = 0; cp <= ND; ++cp) {
      lo[cp] = q0[cp] + s[cp] * dl;
      hi[cp] = q0[cp] + s[cp] * dh;
    }
  }
  const bool ok =
      (!lo_open || realizable<R, SPH, ND>(lo, ihlo, c)) && (!hi_open || realizable<R, SPH, ND>(hi, ihhi, c));
  // the fallback is rare: the selects only run in a wave where some lane needs it
  if (__builtin_amdgcn_ballot_w64(!ok)) {
    for (int cp = 0; cp <= ND; ++cp) {
      lo[cp] = ok ? lo[cp] : q0[cp];
      hi[cp] = ok ? hi[cp] : q0[cp];
    }
  }
  for (int cp = ND + 1; cp < 4; ++cp) lo[cp] = hi[cp] = R(0);
}

// M1 closure: P^ = E [ (1 - f^2)/(1 + s) I + 3/(2 + s) f f ], s = sqrt(4 - 3 f^2), f = F^/(cE)
// (algebraically the Levermore form chi = (3 + 4 f^2)/(5 + 2 s), written without
// cancellation as f -> 1).  Physical components.  Full tensor (row-major 3x3) for the
// geometric sources.
template <typename R, bool SPH, int ND>
__device__ __forceinline__ void closure_full(const R q[4], const R ih[3], R c, int eddington, R P[9]) {
  const R E = q[0];
  for (int t = 0; t < 9; ++t) P[t] = R(0);
  if (eddington || !(E > R(0))) {
    P[0] = P[4] = P[8] = E * R(1.0 / 3.0);
    return;
  }
  R f[3] = {R(0), R(0), R(0)};
  const R icE = rcp_(c * E);
  R f2 = R(0);
  for (int k = 0; k < ND; ++k) {
    f[k] = (SPH ? q[1 + k] * ih[k] : q[1 + k]) * icE;
    f2 += f[k] * f[k];
  }
  if (f2 > R(1)) {
    const R sc = rcp_(sqrt_(f2));
    for (int k = 0; k < ND; ++k) f[k] *= sc;
    f2 = R(1);
  }
  const R s = sqrt_(R(4) - R(3) * f2);
  const R r = rcp_((R(1) + s) * (R(2) + s));
  const R iso = E * (R(1) - f2) * (R(2) + s) * r;
  const R ani = E * R(3) * (R(1) + s) * r;
  for (int p = 0; p < 3; ++p)
    for (int q2 = 0; q2 < 3; ++q2) P[3 * p + q2] = ani * f[p] * f[q2];
  P[0] += iso;
  P[4] += iso;
  P[8] += iso;
}

// Row d of the closure, P^^{dk} for k < ND.  In double, from E and F directly (one square
// root, one reciprocal); in the MIXED path (R = float) from f = F/(cE), in double where
// f^2 >= f2_fp64.
template <typename R, bool SPH, int ND>
__device__ __forceinline__ void closure_row(const R q[4], const R ih[3], int d, R c, int eddington, double f2_fp64,
                                            R P[3]) {
  const R E = q[0];
  for (int k = 0; k < 3; ++k) P[k] = R(0);
  if (eddington || !(E > R(0))) {
    P[d] = E * R(1.0 / 3.0);
    return;
  }
  if constexpr (sizeof(R) == 8) {
    // double: from E and F directly, with S = cE s = sqrt(4 (cE)^2 - 3 |F|^2),
    //   P = (S - cE)/(3c) delta + 3 F F / (c (2 cE + S)),
    // one square root and one reciprocal.  The tensor is homogeneous of degree one in
    // (E, F): a state with cE below 2^-450, whose squares could underflow, is evaluated
    // scaled by 2^600 (exact) and the row scaled back (only in waves that hold one).
    R Fh[3] = {R(0), R(0), R(0)};
    for (int k = 0; k < ND; ++k) Fh[k] = SPH ? q[1 + k] * ih[k] : q[1 + k];
    const R cE = c * E;
    R F2 = R(0);
    for (int k = 0; k < ND; ++k) F2 += Fh[k] * Fh[k];
    const R A = cE * cE;
    {
      const R S = sqrt_(R(4) * A - R(3) * F2);
      const R iso = (S - cE) * rcp_(R(3) * c);   // c is uniform: hoisted
      const R af = R(3) * rcp_(c * (R(2) * cE + S)) * Fh[d];
      for (int k = 0; k < ND; ++k) P[k] = af * Fh[k] + (k == d ? iso : R(0));
    }
    // the rare states are evaluated again, in a branch taken only by waves that hold one (the
    // empty asm keeps the compiler from computing it in every wave): |f| > 1 with the direction
    // of F at |f| = 1, and states with cE below 2^-450, whose squares could underflow, scaled
    // by 2^600 (exact) and the row scaled back
    const bool rare = cE < R(0x1p-450) || F2 > A;
    if (__builtin_amdgcn_ballot_w64(rare)) {
      __asm__ volatile("");
      if (rare) {
        const bool scl = cE < R(0x1p-450);
        const R sc0 = scl ? R(0x1p600) : R(1);
        const R cEs = cE * sc0;
        R F2s = R(0);
        for (int k = 0; k < ND; ++k) {
          Fh[k] *= sc0;
          F2s += Fh[k] * Fh[k];
        }
        const R As = cEs * cEs;
        if (F2s > As) {
          const R sc = cEs * rcp_(sqrt_(F2s));
          for (int k = 0; k < ND; ++k) Fh[k] *= sc;
          F2s = As;
        }
        const R S = sqrt_(R(4) * As - R(3) * F2s);
        const R iso = (S - cEs) * rcp_(R(3) * c);
        const R af = R(3) * rcp_(c * (R(2) * cEs + S)) * Fh[d];
        const R sb = scl ? R(0x1p-600) : R(1);
        for (int k = 0; k < ND; ++k) P[k] = (af * Fh[k] + (k == d ? iso : R(0))) * sb;
      }
    }
    return;
  }
  R f[3] = {R(0), R(0), R(0)};
  const R icE = rcp_(c * E);
  R f2 = R(0);
  for (int k = 0; k < ND; ++k) {
    f[k] = (SPH ? q[1 + k] * ih[k] : q[1 + k]) * icE;
    f2 += f[k] * f[k];
  }
  if constexpr (sizeof(R) == 4) {
    if ((double)f2 >= f2_fp64) {
      double fd[3] = {0.0, 0.0, 0.0}, f2d = 0.0;
      const double icEd = rcp_((double)c * (double)E);
      for (int k = 0; k < ND; ++k) {
        fd[k] = (SPH ? (double)q[1 + k] * (double)ih[k] : (double)q[1 + k]) * icEd;
        f2d += fd[k] * fd[k];
      }
      if (f2d > 1.0) {
        const double sc = rcp_(sqrt_(f2d));
        for (int k = 0; k < ND; ++k) fd[k] *= sc;
        f2d = 1.0;
      }
      // the cancellation-free form (1 - f^2)/(1 + s) in double near free streaming
      const double s = sqrt_(4.0 - 3.0 * f2d);
      const double r = rcp_((1.0 + s) * (2.0 + s));
      const double iso = (double)E * (1.0 - f2d) * (2.0 + s) * r;
      const double ani = (double)E * 3.0 * (1.0 + s) * r;
      for (int k = 0; k < ND; ++k) P[k] = (R)(ani * fd[d] * fd[k] + (k == d ? iso : 0.0));
      return;
    }
  }
  if (f2 > R(1)) {
    const R sc = rcp_(sqrt_(f2));
    for (int k = 0; k < ND; ++k) f[k] *= sc;
    f2 = R(1);
  }
  // (1 - f^2)/(1 + s) = (s - 1)/3 since s^2 = 4 - 3 f^2: one reciprocal, of 2 + s.  Near
  // f -> 1 the isotropic part loses relative accuracy, but only by a few ulp of E, while
  // the f f part carries the tensor there.
  const R s = sqrt_(R(4) - R(3) * f2);
  const R iso = E * (s - R(1)) * R(1.0 / 3.0);
  const R ani = R(3) * E * rcp_(R(2) + s);
  const R af = ani * f[d];
  for (int k = 0; k < ND; ++k) P[k] = af * f[k] + (k == d ? iso : R(0));
}

// Characteristic speeds (physical) of the one-dimensional M1 system at a face state with
// energy E and normal physical flux Fn: the eigenvalues of its flux Jacobian, which for the
// Levermore factor reduce to l-+ = c (f (1 + s) -+ 2 sqrt(3) (1 - f^2)) / (s (1 + s)),
// f = Fn / (cE) clamped to [-1, 1], s = sqrt(4 - 3 f^2) -- free of cancellation as |f| -> 1.
// Eddington closure: -+c/sqrt(3); E <= 0: -+c.
template <typename R>
__device__ __forceinline__ void m1_speeds(R E, R Fn, R c, int closure, R& lo, R& hi) {
  if (!(E > R(0))) {
    lo = -c;
    hi = c;
    return;
  }
  if (closure == FORNAX_CLOSURE_EDDINGTON) {
    hi = c * R(0.57735026918962576451);
    lo = -hi;
    return;
  }
  R f = Fn * rcp_(c * E);
  f = f > R(1) ? R(1) : (f < R(-1) ? R(-1) : f);
  const R g = R(1) - f * f;
  const R s = sqrt_(R(4) - R(3) * f * f);
  const R r = c * rcp_(s * (R(1) + s));
  const R u = f * (R(1) + s), v = R(3.46410161513775458705) * g;
  lo = (u - v) * r;
  hi = (u + v) * r;
}

// HLL flux (coordinate components) across a d-face with face scale factors h and their
// inverses ih, left/right states qL, qR and the correction factor eps of the energy flux.
// S_R = -S_L = c; with WS, a launch whose wavespeed option asks for them takes the HLLE bounds
// from the M1 characteristic speeds of both states instead.
template <typename R, bool SPH, int ND, bool WS = false>
__device__ __forceinline__ void hll(const StepArgsBase& a, int d, const R qL[4], const R qR[4], const R h[3],
                                    const R ih[3], R eps, R flux[4]) {
  const R c = R(a.c);
  R PL[3], PR[3];
  closure_row<R, SPH, ND>(qL, ih, d, c, a.closure, a.f2_fp64, PL);
  closure_row<R, SPH, ND>(qR, ih, d, c, a.closure, a.f2_fp64, PR);
  R ihd = R(1), S = c;
  if constexpr (SPH) {
    ihd = ih[d];
    S = c * ihd;
  }
  if constexpr (WS) {
    if (a.wavespeed == FORNAX_WAVESPEED_M1) {
      R lL, hL, lR, hR;
      m1_speeds<R>(qL[0], SPH ? qL[1 + d] * ihd : qL[1 + d], c, a.closure, lL, hL);
      m1_speeds<R>(qR[0], SPH ? qR[1 + d] * ihd : qR[1 + d], c, a.closure, lR, hR);
      const R SL = fmin(R(0), fmin(lL, lR)) * ihd, SR = fmax(R(0), fmax(hL, hR)) * ihd;
      const R SLR = SR * SL, id = rcp_(SR - SL);
      flux[0] = (SR * (qL[1 + d] * (ihd * ihd)) - SL * (qR[1 + d] * (ihd * ihd)) + eps * SLR * (qR[0] - qL[0])) * id;
      for (int k = 0; k < ND; ++k) {
        const R hk = SPH ? h[k] * ihd : R(1);
        flux[1 + k] = (SR * (c * c * PL[k] * hk) - SL * (c * c * PR[k] * hk) + SLR * (qR[1 + k] - qL[1 + k])) * id;
      }
      for (int k = ND; k < 3; ++k) flux[1 + k] = R(0);
      return;
    }
  }
  const R half = R(0.5);
  // energy: F^d = F_d / h_d^2; S_R = -S_L = S
  flux[0] = half * ((qL[1 + d] + qR[1 + d]) * (ihd * ihd)) - half * eps * S * (qR[0] - qL[0]);
  // covariant flux components: c^2 P^d_k = c^2 P^^{dk} h_k / h_d
  for (int k = 0; k < ND; ++k) {
    const R hk = SPH ? h[k] * ihd : R(1);
    flux[1 + k] = half * c * c * (PL[k] + PR[k]) * hk - half * S * (qR[1 + k] - qL[1 + k]);
  }
  for (int k = ND; k < 3; ++k) flux[1 + k] = R(0);
}

template <typename R>
__device__ __forceinline__ R epsilon_of(R ksL, R ksR, R dlL, R dlR) {
  const R tau = R(0.5) * (ksL + ksR) * (R(0.5) * (dlL + dlR));
  // the reciprocal only in a wave where some face is optically thick
  R eps = R(1);
  if (__builtin_amdgcn_ballot_w64(tau > R(1))) eps = (tau > R(1)) ? rcp_(tau) : R(1);
  return eps;
}

// Flux through the d-face with index f (face f-1/2 of zone f along d) of the row (i, j), from
// q[] holding zones f-2 .. f+1 and the opacities of zones f-1, f.
template <typename S, typename R, bool SPH, int ND>
__device__ __forceinline__ void face_flux(const StepArgs<S>& a, const Geo<R>& geo, int d, int f, int i, int j,
                                          const R q[4][4], R ksL, R ksR, R flux[4]) {
  const int ef = f + NG;
  for (int c = 0; c < 4; ++c) flux[c] = R(0);
  if (SPH && gld(geo.wf[d], ef) == R(0)) return;
  const int ei = i + NG, ej = j + NG;
  R ih0[3], h1[3], ih1[3], ih2[3];
  face_ih<R, SPH>(geo, d, ei, ej, ef - 1, ih0);
  face_h<R, SPH>(geo, d, ei, ej, ef, h1);
  face_ih<R, SPH>(geo, d, ei, ej, ef, ih1);
  face_ih<R, SPH>(geo, d, ei, ej, ef + 1, ih2);
  const bool o0 = !SPH || gld(geo.wf[d], ef - 1) != R(0), o2 = !SPH || gld(geo.wf[d], ef + 1) != R(0);
  R Llo[4], Lhi[4], Rlo[4], Rhi[4];
  reconstruct<R, SPH, ND>(a, geo, d, ef - 1, q[0], q[1], q[2], ih0, ih1, o0, true, Llo, Lhi);
  reconstruct<R, SPH, ND>(a, geo, d, ef, q[1], q[2], q[3], ih1, ih2, true, o2, Rlo, Rhi);
  const int eL = ef - 1;
  const R dlL = proper_width<R, SPH>(geo, d, d == 0 ? eL : ei, d == 1 ? eL : ej);
  const R dlR = proper_width<R, SPH>(geo, d, d == 0 ? ef : ei, d == 1 ? ef : ej);
  const R eps = epsilon_of(ksL, ksR, dlL, dlR);
  hll<R, SPH, ND, true>(a, d, Lhi, Rlo, h1, ih1, eps, flux);
}

// geometric source c^2 sum_{l,m} <Gamma^l_{km}> P^m_l for the covariant flux components of a
// spherical (ln r, theta, phi) zone, P^m_l = P^^{ml} h_l / h_m with cell-centred h
template <typename R>
__device__ __forceinline__ void geometric_source(const R P[9], const R h[3], const R ih[3], const R* gam, R c,
                                                 R Sg[3]) {
  const R G323 = gld(gam, 0), G133 = gld(gam, 1), G233 = gld(gam, 2), G222 = gld(gam, 3);
  const R c2 = c * c;
  // F_1: Gamma^1_11 = Gamma^2_12 = Gamma^3_13 = 1
  Sg[0] = c2 * (P[0] + P[4] + P[8]);
  // F_2: Gamma^1_22 = -1, Gamma^2_21 = 1, <Gamma^2_22>, <Gamma^3_23>
  const R ih0 = ih[0], ih1 = ih[1], ih2 = ih[2];
  Sg[1] = c2 * (-P[3] * (h[0] * ih1) + P[1] * (h[1] * ih0) + G222 * P[4] + G323 * P[8]);
  // F_3: <Gamma^1_33>, <Gamma^2_33>, Gamma^3_31 = 1, <Gamma^3_32>
  Sg[2] = c2 * (G133 * P[6] * (h[0] * ih2) + G233 * P[7] * (h[1] * ih2) + P[2] * (h[2] * ih0) +
                G323 * P[5] * (h[2] * ih1));
}

// Implicit interaction update of one zone-group in double (eq:be_update with j = c kappa B and
// F^{n+1} = F^- / (1 + c dt (kappa + sigma))), store, and the zone-group's diagnostics
// contributions: V E^{n+1}, f^2 = (|F^|/cE)^2, realizability and positivity counts.  Returns
// E^{n+1} - E^- (energy handed to matter, with the sign reversed).
struct ZoneDiag {
  double energy = 0.0;
  double fnum = 0.0, fden = 1.0;   // the largest f^2 seen, kept as the ratio fnum / fden
  int nun = 0, nnp = 0;
  __device__ double maxf2() const { return fnum / fden; }
};

// The coefficients enter as cdtk = c dt kappa, cdtks = c dt (kappa + sigma) and the emission
// term jB = c dt kappa B, all in double.  Returns E^{n+1} - E^- and the new state in the
// storage type (E1, F1); the caller stores it.  (i, j) are the zone's x and y indices.
template <typename S, typename R, bool SPH, int ND>
__device__ __forceinline__ double source_zone(const StepArgsBase& a, const Geo<R>& geo, int i, int j, const R Um[4],
                                              double cdtk, double cdtks, double jB, bool want_diag, double V,
                                              ZoneDiag& zd, S& E1o, S F1o[3]) {
  const double c = a.c;
  const double Emd = (double)Um[0];
  // one reciprocal for both denominators: 1/(1+x) = (1+y) / ((1+x)(1+y))
  const double dE = 1.0 + cdtk, dF = 1.0 + cdtks;
  const double rr = rcp_(dE * dF);
  const double E1 = (Emd + jB) * (dF * rr);
  const double ifden = dE * rr;
  const S E1s = (S)E1;
  E1o = E1s;
  double F1s[3] = {0.0, 0.0, 0.0};
  for (int cc = 0; cc < ND; ++cc) {
    const S v = (S)((double)Um[1 + cc] * ifden);
    F1o[cc] = v;
    F1s[cc] = (double)v;
  }
  const double E1d = (double)E1s;
  if (want_diag) {
    zd.energy += V * E1d;
    double hd[3] = {1.0, 1.0, 1.0};
    if constexpr (SPH) {
      hd[0] = hd[1] = (double)gld(geo.hr, i + NG);
      hd[2] = hd[0] * (double)gld(geo.hs, j + NG);
    }
    // |E| below 2^-400: the squares below could underflow; f and the counts are those of the
    // state scaled by 2^600 (exact), in waves that hold such a zone only
    double Es = E1d, sc = 1.0;
    if (__builtin_amdgcn_ballot_w64(fabs(E1d) < 0x1p-400) && fabs(E1d) < 0x1p-400) {
      sc = 0x1p600;
      Es = E1d * sc;
    }
    double F2 = 0.0;
    for (int cc = 0; cc < ND; ++cc) {
      const double fk = (SPH ? F1s[cc] * rcp_(hd[cc]) : F1s[cc]) * sc;
      F2 += fk * fk;
    }
    const double cE = c * Es;
    // f^2 = F2 / (cE)^2 compared by cross-multiplication (one division per thread at the end)
    const double cE2 = cE * cE;
    const bool up = Es > 0.0 && F2 * zd.fden > zd.fnum * cE2;
    zd.fnum = up ? F2 : zd.fnum;
    zd.fden = up ? cE2 : zd.fden;
    const double u = (sizeof(S) == 8) ? 0x1p-53 : 0x1p-24;
    const double lim = cE * (1.0 + 8.0 * u);
    // |F^| > lim: every state with E < 0 (lim < 0) counts, else compare the squares
    zd.nun += (lim < 0.0 || F2 > lim * lim) ? 1 : 0;
    zd.nnp += (E1d > 0.0) ? 0 : 1;
  }
  return E1d - Emd;
}

}  // namespace fm1
