// m1_adjoint_device.h -- vector-Jacobian products of the pieces of one M1 step (uniform
// Cartesian zones), used by the adjoint kernel.  Each function recomputes the forward
// quantities it needs and takes the derivative of the branch the forward step takes
// (minmod choice, realizability fallback, epsilon kink, clamp of f).
#pragma once

#include <hip/hip_runtime.h>

#include "m1_device.h"
#include "m1_internal.h"

namespace fm1 {

// Linear reconstruction of one zone (uniform Cartesian; see reconstruct()) with the branch
// decisions kept for its VJP: per component the slope selector sel (0: zero, 1: d-, 2: d+,
// 3: centred MC slope) and its factor (2 for the doubled MC slopes), and the fallback flag.
template <typename R, int ND>
struct ReconRec {
  R lo[4], hi[4];
  signed char sel[4];
  R fac[4];
  bool ok;
};

template <typename R>
__device__ __forceinline__ void minmod_sel(R a, R b, R& s, signed char& which) {
  // selects, not branches: the choice differs from lane to lane
  const bool same = a * b > R(0);
  const bool first = fabs(a) <= fabs(b);
  s = same ? (first ? a : b) : R(0);
  which = same ? (first ? 1 : 2) : 0;
}

// LIM: the limiter when known at compile time (a FORNAX_LIMITER_* value), -1 to read it from
// the arguments.
template <typename R, int ND, int LIM = -1>
__device__ __forceinline__ void reconstruct_rec(const StepArgsBase& a, const R qm[4], const R q0[4], const R qp[4],
                                                bool lo_open, bool hi_open, ReconRec<R, ND>& rr) {
  const R c = R(a.c);
  const int limiter = (LIM >= 0) ? LIM : a.limiter;
  const R one[3] = {R(1), R(1), R(1)};
  R s[4];
  for (int cp = 0; cp <= ND; ++cp) {
    const R dm = q0[cp] - qm[cp], dp = qp[cp] - q0[cp];
    rr.fac[cp] = R(1);
    if (limiter == FORNAX_LIMITER_MINMOD) {
      signed char w;
      minmod_sel(dm, dp, s[cp], w);
      rr.sel[cp] = w;
    } else if (limiter == FORNAX_LIMITER_MC) {
      // minmod(2 dm, minmod(2 dp, (dm + dp)/2))
      R inner;
      signed char wi, wo;
      minmod_sel(R(2) * dp, R(0.5) * (dm + dp), inner, wi);
      minmod_sel(R(2) * dm, inner, s[cp], wo);
      if (wo == 0) rr.sel[cp] = 0;
      else if (wo == 1) {
        rr.sel[cp] = 1;
        rr.fac[cp] = R(2);
      } else if (wi == 1) {
        rr.sel[cp] = 2;
        rr.fac[cp] = R(2);
      } else if (wi == 2) {
        rr.sel[cp] = 3;
      } else {
        rr.sel[cp] = 0;
      }
    } else {
      s[cp] = R(0);
      rr.sel[cp] = 0;
    }
  }
  for (int cp = 0; cp <= ND; ++cp) {
    rr.lo[cp] = q0[cp] - R(0.5) * s[cp];
    rr.hi[cp] = q0[cp] + R(0.5) * s[cp];
  }
  rr.ok = (!lo_open || realizable<R, false, ND>(rr.lo, one, c)) && (!hi_open || realizable<R, false, ND>(rr.hi, one, c));
  for (int cp = 0; cp <= ND; ++cp) {
    if (!rr.ok) rr.lo[cp] = rr.hi[cp] = q0[cp];
  }
  for (int cp = ND + 1; cp < 4; ++cp) rr.lo[cp] = rr.hi[cp] = R(0);
}

// VJP of the reconstruction: adjoints glo, ghi of the face states -> adds to gm, g0, gp
// (the adjoints of the zone and its two neighbours).
template <typename R, int ND>
__device__ __forceinline__ void reconstruct_vjp(const ReconRec<R, ND>& rr, const R glo[4], const R ghi[4], R gm[4],
                                                R g0[4], R gp[4]) {
  // with selects, not branches (the selector differs from lane to lane):
  //   sel 1: s = fac (q0 - qm);  sel 2: s = fac (qp - q0);  sel 3: s = (qp - qm)/2
  for (int cp = 0; cp <= ND; ++cp) {
    const R gs = rr.ok ? R(0.5) * (ghi[cp] - glo[cp]) : R(0);   // lo = q0 - s/2, hi = q0 + s/2
    const R gf = gs * rr.fac[cp];
    const int sel = rr.sel[cp];
    const R hm = (sel == 1) ? -gf : ((sel == 3) ? R(-0.5) * gs : R(0));
    const R h0 = (sel == 1) ? gf : ((sel == 2) ? -gf : R(0));
    const R hp = (sel == 2) ? gf : ((sel == 3) ? R(0.5) * gs : R(0));
    g0[cp] += (glo[cp] + ghi[cp]) + h0;
    gm[cp] += hm;
    gp[cp] += hp;
  }
}

// VJP of row d of the M1 closure (Cartesian scale factors): given weights w_k on P^{dk}
// (k < ND), add d(sum_k w_k P^{dk})/d(E, F_j) to g.
// With f = F/(cE), s = sqrt(4 - 3 f^2), a = (1 - f^2)/(1 + s), b = 3/(2 + s):
//   Q = E (a w_d + b f_d (w.f)),
//   dQ/df_j = E [2 f_j (a' w_d + b' f_d (w.f)) + b (delta_dj (w.f) + f_d w_j)],
//   dQ/dE   = a w_d - b f_d (w.f) - 2 f^2 (a' w_d + b' f_d (w.f)),   dQ/dF_j = dQ/df_j / (cE),
// a' = da/d(f^2) = -1/(1 + s) + (1 - f^2) (3/(2s)) / (1 + s)^2, b' = (9/(2s)) / (2 + s)^2.
// Clamped states (|F| > cE) use P = E n n with n = F/|F|.
template <typename R, int ND>
__device__ __forceinline__ void closure_row_vjp(const R q[4], int d, R c, int eddington, const R w[3], R g[4]) {
  const R E = q[0];
  if (eddington || !(E > R(0))) {
    g[0] += w[d] * R(1.0 / 3.0);
    return;
  }
  const R icE = rcp_(c * E);
  R f[3] = {R(0), R(0), R(0)};
  R f2 = R(0);
  for (int k = 0; k < ND; ++k) {
    f[k] = q[1 + k] * icE;
    f2 += f[k] * f[k];
  }
  if (f2 > R(1)) {
    R F2 = R(0);
    for (int k = 0; k < ND; ++k) F2 += q[1 + k] * q[1 + k];
    const R iF = rcp_(sqrt_(F2));
    R n[3] = {R(0), R(0), R(0)};
    R wn = R(0);
    for (int k = 0; k < ND; ++k) {
      n[k] = q[1 + k] * iF;
      wn += w[k] * n[k];
    }
    g[0] += n[d] * wn;
    for (int j = 0; j < ND; ++j)
      g[1 + j] += E * iF * ((j == d ? wn : R(0)) + n[d] * w[j] - R(2) * n[d] * n[j] * wn);
    return;
  }
  const R s = sqrt_(R(4) - R(3) * f2);
  // 1/s, 1/(1 + s), 1/(2 + s) from one reciprocal of s (1 + s)(2 + s)
  const R s1 = R(1) + s, s2 = R(2) + s;
  const R rall = rcp_(s * s1 * s2);
  const R i1s = s * s2 * rall, i2s = s * s1 * rall, is = s1 * s2 * rall;
  const R A = (R(1) - f2) * i1s;
  const R Bc = R(3) * i2s;
  const R Ap = -i1s + (R(1) - f2) * (R(1.5) * is) * (i1s * i1s);
  const R Bp = (R(4.5) * is) * (i2s * i2s);
  R wf = R(0);
  for (int k = 0; k < ND; ++k) wf += w[k] * f[k];
  const R T = Ap * w[d] + Bp * f[d] * wf;
  g[0] += A * w[d] - Bc * f[d] * wf - R(2) * f2 * T;
  for (int j = 0; j < ND; ++j) {
    const R dQdf = E * (R(2) * f[j] * T + Bc * ((j == d ? wf : R(0)) + f[d] * w[j]));
    g[1 + j] += dQdf * icE;
  }
}

// Forward flux and VJP of one face (uniform Cartesian): stencil zones q[0..3] = f-2 .. f+1,
// total opacities of zones f-1, f, face adjoint nu (the adjoint of the face flux).  Outputs
// the forward flux, the contributions C[p] to the adjoints of the four stencil zones and the
// adjoint contributions to kappa of zones f-1 (dkL) and f (dkR) through epsilon.
template <typename R, int ND, int LIM = -1>
__device__ __forceinline__ void face_vjp_cart(const StepArgsBase& a, int d, R dx, const R q[4][4], R ksL, R ksR,
                                              const R nu[4], R flux[4], R C[4][4], R& dkL, R& dkR) {
  const R c = R(a.c);
  ReconRec<R, ND> rl, rr;
  reconstruct_rec<R, ND, LIM>(a, q[0], q[1], q[2], true, true, rl);
  reconstruct_rec<R, ND, LIM>(a, q[1], q[2], q[3], true, true, rr);
  const R* qL = rl.hi;
  const R* qR = rr.lo;
  // epsilon
  const R tau = R(0.5) * (ksL + ksR) * dx;
  const bool thick = tau > R(1);
  const R itau = thick ? rcp_(tau) : R(1);
  const R eps = itau;
  // forward flux
  const R one[3] = {R(1), R(1), R(1)};
  hll<R, false, ND>(a, d, qL, qR, one, one, eps, flux);
  // adjoint of the HLL flux
  R gL[4] = {R(0), R(0), R(0), R(0)}, gR[4] = {R(0), R(0), R(0), R(0)};
  const R half = R(0.5);
  gL[0] += half * eps * c * nu[0];
  gR[0] -= half * eps * c * nu[0];
  gL[1 + d] += half * nu[0];
  gR[1 + d] += half * nu[0];
  R w[3] = {R(0), R(0), R(0)};
  for (int k = 0; k < ND; ++k) {
    gL[1 + k] += half * c * nu[1 + k];
    gR[1 + k] -= half * c * nu[1 + k];
    w[k] = half * c * c * nu[1 + k];
  }
  closure_row_vjp<R, ND>(qL, d, c, a.closure, w, gL);
  closure_row_vjp<R, ND>(qR, d, c, a.closure, w, gR);
  // epsilon: d flux_E / d eps = -c (E_R - E_L) / 2; eps = 1/tau for tau > 1,
  // tau = (ks_L + ks_R) dx / 2
  const R geps = -half * c * (qR[0] - qL[0]) * nu[0];
  const R gks = thick ? -geps * itau * itau * half * dx : R(0);
  dkL = gks;
  dkR = gks;
  // adjoint of the reconstructions
  for (int p = 0; p < 4; ++p)
    for (int cp = 0; cp < 4; ++cp) C[p][cp] = R(0);
  const R zero[4] = {R(0), R(0), R(0), R(0)};
  reconstruct_vjp<R, ND>(rl, zero, gL, C[0], C[1], C[2]);
  reconstruct_vjp<R, ND>(rr, gR, zero, C[1], C[2], C[3]);
}

}  // namespace fm1
