// m1_adjoint.hip -- adjoint (vector-Jacobian product) of one M1 step for gfx950.
//
//   lam_n = (dU^{n+1}/dU^n)^T lam_{n+1},   dkappa += (dU^{n+1}/dkappa)^T lam_{n+1}
//
// The step is U^{n+1} = S(U^-), U^- = U^n + dt L(U^n) with the implicit interaction update S
// (zone-local) and the flux divergence L.  With mu = (dS/dU^-)^T lam_{n+1}, the adjoint of
// the flux at face f between zones L and R is nu_f = dt (mu_R - mu_L) / dx, and
//   lam_n(z) = mu(z) + sum over the four faces whose stencil holds z of (d flux_f / d U_z)^T nu_f.
//
// Kernel layout mirrors the forward step: lanes = (zone column, group); a block owns TXB zone
// columns in x and marches along y (2-D).  The thread of column cx recomputes the face
// x0 - 1 + cx (forward flux and its VJP) and exchanges through LDS; along the march a
// register ring carries the contributions of the last four faces.  Each tile finalises
// TXB - 3 columns.  A direction periodic at both ends (and at least four zones long) has no
// ghost zones here: its zone indices wrap and its face 0 is face n, so the tiles cover the
// domain only.  Along any other direction the tiles also cover the two ghost layers on each
// side: contributions to a ghost zone go to a per-direction ghost buffer that k_adj_fold maps
// back through the boundary rule (outflow copy, reflection with the normal flux flipped;
// inflow ghosts are constant, so only their opacity dependence folds).  No atomics: every
// sum is taken in a fixed order, so the result is deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "m1_adjoint_device.h"
#include "m1_device.h"
#include "m1_internal.h"

namespace fm1 {

template <typename S>
struct AdjArgs : StepArgs<S> {
  const S* lam[3 + 1];    // lambda^{n+1}: E, F_1..F_ND
  S* lamo[3 + 1];         // lambda^n
  S* dk;                  // dkappa accumulator
  const S* U1[3 + 1];     // U^{n+1} of the step (E, F_1..F_ND)
  double* gbuf[3];        // ghost adjoints per direction: [side][layer][plane][G][NC+1]
  int gplane[3];          // zones of the plane normal to direction d
  int wrap[3];            // 1: direction d is periodic at both ends and wraps (no ghosts)
};

// whether direction d of the grid wraps in the adjoint (periodic at both ends, n >= 4)
static inline bool adj_wraps(const fornax_m1_desc& D, int d) {
  return d < D.ndim && D.bc_lo[d] == FORNAX_BC_PERIODIC && D.bc_hi[d] == FORNAX_BC_PERIODIC && D.n[d] >= 4;
}

struct AdjTile {
  int TXB, W;             // thread columns, finalised columns per tile (TXB - 3)
  int TM;                 // planes per tile along the march (2-D)
  int ntx, ntm, nblocks;
  int xq, xr;
  int nthreads;
};

// mu = (dS/dU^-)^T lam for an in-domain zone-group, in double: the interaction update divides
// E by 1 + c dt kappa and F by 1 + c dt (kappa + sigma)
template <typename S, int ND>
__device__ __forceinline__ void source_adjoint(const AdjArgs<S>& a, int zg, const double lam[4], double mu[4]) {
  const double kd = (double)a.kap[zg], sd = (double)a.sig[zg];
  const double cdt = a.c * a.dt;
  // one reciprocal for both denominators
  const double dE = 1.0 + cdt * kd, dF = 1.0 + cdt * (kd + sd);
  const double rr = rcp_(dE * dF);
  mu[0] = lam[0] * (dF * rr);
  for (int k = 0; k < ND; ++k) mu[1 + k] = lam[1 + k] * (dE * rr);
}

template <typename S, typename R, int DIM>
__device__ __forceinline__ void load_mu(const AdjArgs<S>& a, int zg, R mu[4]) {
  double lam[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0};
  lam[0] = (double)a.lam[0][zg];
  for (int k = 0; k < DIM; ++k) lam[1 + k] = (double)a.lam[1 + k][zg];
  source_adjoint<S, DIM>(a, zg, lam, m);
  for (int k = 0; k < 4; ++k) mu[k] = (R)m[k];
}

// Three waves per SIMD (at most 168 VGPRs): measured faster on gfx950 than the unconstrained
// allocation (two waves) despite a few spilled registers.  LIM: the limiter when known at
// compile time, -1 to read it from the arguments.  PER: every direction wraps (a periodic
// grid), so no index can leave the domain; with it fixed at compile time the kernel fits the
// register budget without spills.
template <typename S, typename R, int DIM, int LIM, bool PER>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3)))
k_adjoint(AdjArgs<S> a, Geo<R> geo, AdjTile tl) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NC = 1 + DIM;
  constexpr int NV = 2 * NC + 1;     // state, total opacity, mu
  constexpr int MD = DIM - 1;
  const int G = a.G;
  const int t = threadIdx.x;
  const int grp = t % G;
  const int cx = t / G;
  const int TXB = tl.TXB, W = tl.W;
  const int COLS = TXB + 3;
  R* PV = reinterpret_cast<R*>(smem);                  // [NV][COLS][G]
  R* CX = PV + (size_t)NV * COLS * G;                  // [4][NC][TXB][G]
  R* DKX = CX + (size_t)4 * NC * TXB * G;              // [2][TXB][G]
  auto pv = [&](int v, int colL) -> R& { return PV[((size_t)v * COLS + colL) * G + grp]; };
  auto cxr = [&](int p, int v, int col) -> R& { return CX[(((size_t)p * NC + v) * TXB + col) * G + grp]; };

  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int Lb = xcd * tl.xq + min(xcd, tl.xr) + slot;
  const int tx = Lb % tl.ntx;
  const int tm = Lb / tl.ntx;
  const int n0 = a.n[0];
  const int nM = (DIM >= 2) ? a.n[MD] : 1;
  const bool wx = PER || a.wrap[0] != 0;
  const bool wy = (DIM >= 2) && (PER || a.wrap[MD] != 0);
  const int x0 = (wx ? 0 : -2) + tx * W;
  const int mbeg = (DIM >= 2) ? (wy ? 0 : -2) + tm * tl.TM : 0;
  const int mend = (DIM >= 2) ? min(mbeg + tl.TM, wy ? nM : nM + 2) : 1;
  const int gx = x0 + cx;
  // a wrapping direction's zone index taken into [0, n): columns once (they stay fixed), planes
  // with one step (a block reads planes -3 .. nM + 2, and nM >= 4)
  auto wrapi = [](int i, int n) { return ((i % n) + n) % n; };
  auto wrapm = [&](int m) { return wy ? (m < 0 ? m + nM : (m >= nM ? m - nM : m)) : m; };
  const int gxl = wx ? wrapi(gx, n0) : gx;          // the column's zone (x index)
  const int hxl = wx ? wrapi(x0 - 3 + cx, n0) : x0 - 3 + cx;   // halo column of threads cx < 3
  const bool colin = gxl >= 0 && gxl < n0;          // column inside the domain
  // this thread finalises (gx, m)
  const bool fin = cx < W && (wx ? gx < n0 : (gx >= -2 && gx < n0 + 2));
  const R dx0 = geo.dx[0];
  const R nux = R(a.dt) * rcp_(dx0);

  // zone-group index of (x, m), both inside the domain
  auto zgi = [&](int x, int m) -> int { return (DIM >= 2) ? (m * n0 + x) * G + grp : x * G + grp; };
  // state and total opacity of zone (x, m) with at most one index outside the domain
  auto state = [&](int x, int m, R q[4], R& ks) {
    for (int v = 0; v < 4; ++v) q[v] = R(0);
    ks = R(0);
    if (!PER && (x < -2 || x > n0 + 1 || m < -2 || m > nM + 1)) return;
    const bool xin = PER || (x >= 0 && x < n0), min_ = PER || (m >= 0 && m < nM);
    if (!xin && !min_) return;
    if (!xin) fetch<S, R, false, DIM>(a, geo, 0, x, x, (DIM >= 2 ? m : 0), 0, grp, q, &ks);
    else fetch<S, R, false, DIM>(a, geo, MD < 0 ? 0 : MD, (DIM >= 2 ? m : x), x, (DIM >= 2 ? m : 0), 0, grp, q, &ks);
  };

  // ---------------- march-direction state (DIM 2) ----------------
  R wq[4][4], wks[4], wmu[4][4];           // planes m .. m+3 of this column
  R racc[4][4];                            // adjoint contributions to zones m .. m+3
  R rdk[4];                                // dkappa contributions to zones m .. m+3
  for (int i = 0; i < 4; ++i) {
    wks[i] = rdk[i] = R(0);
    for (int v = 0; v < 4; ++v) wq[i][v] = wmu[i][v] = racc[i][v] = R(0);
  }
  const R nuy = (DIM >= 2) ? R(a.dt) * rcp_(geo.dx[MD]) : R(0);
  auto load_plane_w = [&](int p, R q[4], R& ks, R mu[4]) {
    p = wrapm(p);
    state(gxl, p, q, ks);
    for (int v = 0; v < 4; ++v) mu[v] = R(0);
    if (p >= 0 && p < nM) load_mu<S, R, DIM>(a, zgi(gxl, p), mu);
  };
  // march face f (between planes f-1 and f) from window planes f-2 .. f+1 (q0 .. q3), the total
  // opacities and mu of planes f-1, f
  auto march_face_r = [&](int f, const R q0[4], const R q1[4], const R q2[4], const R q3[4], R ks1, R ks2,
                          const R mu1[4], const R mu2[4], R fl[4], R C[4][4], R& dkL, R& dkR) {
    for (int v = 0; v < 4; ++v) fl[v] = R(0);
    for (int p = 0; p < 4; ++p)
      for (int v = 0; v < 4; ++v) C[p][v] = R(0);
    dkL = dkR = R(0);
    if (!wy && (f < 0 || f > nM)) return;
    R nu[4] = {R(0), R(0), R(0), R(0)};
    for (int v = 0; v < NC; ++v) nu[v] = nuy * (mu2[v] - mu1[v]);
    R qq[4][4];
    for (int v = 0; v < 4; ++v) {
      qq[0][v] = q0[v];
      qq[1][v] = q1[v];
      qq[2][v] = q2[v];
      qq[3][v] = q3[v];
    }
    face_vjp_cart<R, DIM, LIM>(a, MD < 0 ? 0 : MD, geo.dx[MD < 0 ? 0 : MD], qq, ks1, ks2, nu, fl, C, dkL, dkR);
  };
  // (the window rows in ring order)
  auto march_face = [&](int f, R fl[4], R C[4][4], R& dkL, R& dkR) {
    march_face_r(f, wq[0], wq[1], wq[2], wq[3], wks[1], wks[2], wmu[1], wmu[2], fl, C, dkL, dkR);
  };
  if constexpr (DIM >= 2) {
    if (colin) {
      // faces mbeg-1, mbeg, mbeg+1 fill the rings; window planes start at mbeg-3
      for (int i = 0; i < 4; ++i) load_plane_w(mbeg - 3 + i, wq[i], wks[i], wmu[i]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int f = mbeg - 1 + i;
        if (i > 0) {
          for (int i2 = 0; i2 < 3; ++i2) {
            for (int v = 0; v < 4; ++v) {
              wq[i2][v] = wq[i2 + 1][v];
              wmu[i2][v] = wmu[i2 + 1][v];
            }
            wks[i2] = wks[i2 + 1];
          }
          load_plane_w(f + 1, wq[3], wks[3], wmu[3]);
        }
        R fl[4], C[4][4], dkL, dkR;
        march_face(f, fl, C, dkL, dkR);
        // face f contributes to zones f-2+p, i.e. ring slot i-3+p
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int r = i - 3 + p;
          if (r >= 0)
            for (int v = 0; v < NC; ++v) racc[r][v] += C[p][v];
        }
        if (i == 1) rdk[0] += dkR;
        if (i == 2) {
          rdk[0] += dkL;
          rdk[1] += dkR;
        }
      }
      // window now holds planes mbeg-1 .. mbeg+2; shift so that it holds mbeg .. mbeg+2
      for (int i = 0; i < 3; ++i) {
        for (int v = 0; v < 4; ++v) {
          wq[i][v] = wq[i + 1][v];
          wmu[i][v] = wmu[i + 1][v];
        }
        wks[i] = wks[i + 1];
      }
    }
  }

  // One plane of the march.  The rings are not shifted: ring slot i of the plane is array entry
  // (i + RT) & 3, RT the plane's offset from the tile's first plane modulo 4 (a compile-time
  // constant: the loop below is unrolled by four), so no values move between registers.
  auto plane_step = [&](auto rt_c, const int m) {
    constexpr int RT = decltype(rt_c)::value;
    auto sl = [](int i) { return (i + RT) & 3; };
    const bool rowin = (DIM < 2) || (m >= 0 && m < nM);
    // ---- march: load plane m+3, face m+2 ----
    if constexpr (DIM >= 2) {
      if (colin) {
        load_plane_w(m + 3, wq[sl(3)], wks[sl(3)], wmu[sl(3)]);
        R fl[4], C[4][4], dkL, dkR;
        march_face_r(m + 2, wq[sl(0)], wq[sl(1)], wq[sl(2)], wq[sl(3)], wks[sl(1)], wks[sl(2)], wmu[sl(1)],
                     wmu[sl(2)], fl, C, dkL, dkR);
        for (int p = 0; p < 4; ++p)
          for (int v = 0; v < NC; ++v) racc[sl(p)][v] += C[p][v];
        rdk[sl(1)] += dkL;
        rdk[sl(2)] += dkR;
      }
    }
    // ---- stage plane m: own column (LDS col cx + 3) and halo columns 0..2 ----
    if (rowin) {
      R q[4], ks, mu[4] = {R(0), R(0), R(0), R(0)};
      if ((DIM >= 2) && colin) {
        for (int v = 0; v < 4; ++v) {
          q[v] = wq[sl(0)][v];
          mu[v] = wmu[sl(0)][v];
        }
        ks = wks[sl(0)];
      } else {
        state(gxl, m, q, ks);
        if (colin) load_mu<S, R, DIM>(a, zgi(gxl, m), mu);
      }
      for (int v = 0; v < NC; ++v) {
        pv(v, cx + 3) = q[v];
        pv(NC + 1 + v, cx + 3) = mu[v];
      }
      pv(NC, cx + 3) = ks;
      if (cx < 3) {
        R hq[4], hks, hmu[4] = {R(0), R(0), R(0), R(0)};
        state(hxl, m, hq, hks);
        if (hxl >= 0 && hxl < n0) load_mu<S, R, DIM>(a, zgi(hxl, m), hmu);
        for (int v = 0; v < NC; ++v) {
          pv(v, cx) = hq[v];
          pv(NC + 1 + v, cx) = hmu[v];
        }
        pv(NC, cx) = hks;
      }
    }
    __syncthreads();
    // ---- x face x0 - 1 + cx ----
    {
      const int f = x0 - 1 + cx;
      R fl[4] = {R(0), R(0), R(0), R(0)}, C[4][4], dkL = R(0), dkR = R(0);
      for (int p = 0; p < 4; ++p)
        for (int v = 0; v < 4; ++v) C[p][v] = R(0);
      if (rowin && (wx || (f >= 0 && f <= n0))) {
        R q[4][4];
        for (int o = 0; o < 4; ++o) {
          for (int v = 0; v < NC; ++v) q[o][v] = pv(v, cx + o);
          for (int v = NC; v < 4; ++v) q[o][v] = R(0);
        }
        R nu[4] = {R(0), R(0), R(0), R(0)};
        for (int v = 0; v < NC; ++v) nu[v] = nux * (pv(NC + 1 + v, cx + 2) - pv(NC + 1 + v, cx + 1));
        face_vjp_cart<R, DIM, LIM>(a, 0, dx0, q, pv(NC, cx + 1), pv(NC, cx + 2), nu, fl, C, dkL, dkR);
      }
      for (int p = 0; p < 4; ++p)
        for (int v = 0; v < NC; ++v) cxr(p, v, cx) = C[p][v];
      DKX[((size_t)0 * TXB + cx) * G + grp] = dkL;
      DKX[((size_t)1 * TXB + cx) * G + grp] = dkR;
    }
    __syncthreads();
    // ---- finalise zone (gx, m) ----
    if (fin) {
      R gsum[4] = {R(0), R(0), R(0), R(0)};
      R dks = R(0);
      if (rowin) {
        for (int p = 0; p < 4; ++p)
          for (int v = 0; v < NC; ++v) gsum[v] += cxr(p, v, cx + 3 - p);
        dks += DKX[((size_t)1 * TXB + cx + 1) * G + grp] + DKX[((size_t)0 * TXB + cx + 2) * G + grp];
      }
      if constexpr (DIM >= 2) {
        if (colin) {
          for (int v = 0; v < NC; ++v) gsum[v] += racc[sl(0)][v];
          dks += rdk[sl(0)];
        }
      }
      if (colin && rowin) {
        // mu of this zone (staged in LDS) and U^{n+1} for the source derivative:
        //   dkappa_src = c dt [mu_E (B - E^{n+1}) - sum_k mu_Fk F_k^{n+1}]
        // (mu_E = lam_E / (1 + c dt kappa), mu_F = lam_F / (1 + c dt (kappa + sigma)))
        const int zg = zgi(gx, m);
        double mu[4] = {0, 0, 0, 0};
        for (int v = 0; v < NC; ++v) mu[v] = (double)pv(NC + 1 + v, cx + 3);
        double sdk = mu[0] * ((double)a.B[zg] - (double)a.U1[0][zg]);
        for (int k = 0; k < DIM; ++k) sdk -= mu[1 + k] * (double)a.U1[1 + k][zg];
        const double dk_src = (a.c * a.dt) * sdk;
        for (int v = 0; v < NC; ++v) a.lamo[v][zg] = (S)(mu[v] + (double)gsum[v]);
        a.dk[zg] = (S)((double)a.dk[zg] + dk_src + (double)dks);
      } else if (colin != rowin) {
        // ghost zone (exactly one index outside the domain)
        const int d = colin ? MD : 0;
        const int gi = colin ? m : gx;
        const int nd = colin ? nM : n0;
        const int side = gi < 0 ? 0 : 1;
        const int layer = gi < 0 ? -1 - gi : gi - nd;
        const int pidx = colin ? gx : ((DIM >= 2) ? m : 0);
        double* gb = a.gbuf[d] + ((((size_t)side * 2 + layer) * a.gplane[d] + pidx) * G + grp) * (NC + 1);
        for (int v = 0; v < NC; ++v) gb[v] = (double)gsum[v];
        gb[NC] = (double)dks;
      }
    }
    // ---- the finalised zone's ring slot starts the plane four ahead ----
    if constexpr (DIM >= 2) {
      for (int v = 0; v < 4; ++v) racc[sl(0)][v] = R(0);
      rdk[sl(0)] = R(0);
    }
    __syncthreads();
  };
  if constexpr (DIM >= 2) {
    for (int m = mbeg; m < mend; m += 4) {
      plane_step(std::integral_constant<int, 0>{}, m);
      if (m + 1 >= mend) break;
      plane_step(std::integral_constant<int, 1>{}, m + 1);
      if (m + 2 >= mend) break;
      plane_step(std::integral_constant<int, 2>{}, m + 2);
      if (m + 3 >= mend) break;
      plane_step(std::integral_constant<int, 3>{}, m + 3);
    }
  } else {
    for (int m = mbeg; m < mend; ++m) plane_step(std::integral_constant<int, 0>{}, m);
  }
}


// Ghost-zone adjoints of direction d that fold into zone dst along d (plane index pidx in the
// plane normal to d): the four ghost entries visited in a fixed order through the boundary
// rule.  Returns whether any ghost copies dst.
template <typename S, int ND>
__device__ bool fold_sum(const AdjArgs<S>& a, int d, int dst, int pidx, int grp, double acc[4], double& dka) {
  constexpr int NC = 1 + ND;
  const int G = a.G;
  const int np = a.gplane[d];
  const int nd = a.n[d];
  for (int v = 0; v < 4; ++v) acc[v] = 0.0;
  dka = 0.0;
  bool any = false;
  for (int side = 0; side < 2; ++side) {
    const int bc = side ? a.bc_hi[d] : a.bc_lo[d];
    for (int layer = 0; layer < 2; ++layer) {
      const int gi = side ? nd + layer : -1 - layer;
      int src;
      double sgn_d = 1.0;
      bool state_dep = true;
      if (bc == FORNAX_BC_PERIODIC) {
        src = ((gi % nd) + nd) % nd;
      } else if (bc == FORNAX_BC_REFLECT) {
        src = side ? 2 * nd - 1 - gi : -1 - gi;
        sgn_d = -1.0;
      } else if (bc == FORNAX_BC_INFLOW) {
        src = side ? nd - 1 : 0;
        state_dep = false;
      } else {  // outflow
        src = side ? nd - 1 : 0;
      }
      if (src != dst) continue;
      const double* gb = a.gbuf[d] + ((((size_t)side * 2 + layer) * np + pidx) * G + grp) * (NC + 1);
      if (state_dep)
        for (int v = 0; v < NC; ++v) acc[v] += (v == 1 + d ? sgn_d : 1.0) * gb[v];
      dka += gb[NC];
      any = true;
    }
  }
  return any;
}

// k-th distinct zone index within two of either end of an axis of n zones (k < 4), or -1
__device__ __forceinline__ int edge_zone(int k, int n) {
  const int cands[4] = {0, 1, n - 2, n - 1};
  const int z = cands[k];
  if (z < 0 || z >= n) return -1;
  for (int k2 = 0; k2 < k; ++k2)
    if (cands[k2] == z) return -1;
  return z;
}

__device__ __forceinline__ bool near_edge(int z, int n) { return z < 2 || z >= n - 2; }

// Fold the ghost-zone adjoints into the zones they copy, both directions in one launch (a
// wrapping direction has none).  One thread per (edge zone along d, plane, group): threads of
// direction 0 take the zones away from the y edges; a thread of direction 1 whose zone is also
// near an x edge applies the x fold first, then its own, so that every zone sees the same
// additions, in the same order, as with one launch per direction.
template <typename S, int ND>
__global__ void __launch_bounds__(256) k_adj_fold(AdjArgs<S> a) {
  constexpr int NC = 1 + ND;
  const int G = a.G;
  const int n0 = a.n[0];
  const int n1 = (ND >= 2) ? a.n[1] : 1;
  const int nx = a.wrap[0] ? 0 : 4 * a.gplane[0] * G;
  int id = blockIdx.x * 256 + threadIdx.x;
  int d = 0;
  if (id >= nx) {
    if (ND < 2 || a.wrap[1]) return;
    id -= nx;
    d = 1;
    if (id >= 4 * a.gplane[1] * G) return;
  }
  const int np = a.gplane[d];
  const int grp = id % G;
  const int pidx = (id / G) % np;
  const int dst = edge_zone(id / (G * np), a.n[d]);
  if (dst < 0) return;
  // zone (x, y) of this thread
  const int x = (d == 0) ? dst : pidx;
  const int y = (ND < 2) ? 0 : ((d == 0) ? pidx : dst);
  // folded by the direction-1 thread
  if (ND >= 2 && d == 0 && !a.wrap[1] && near_edge(y, n1)) return;
  const int zg = (y * n0 + x) * G + grp;
  double acc[4], dka;
  if (ND >= 2 && d == 1 && !a.wrap[0] && near_edge(x, n0) && fold_sum<S, ND>(a, 0, x, y, grp, acc, dka)) {
    for (int v = 0; v < NC; ++v) a.lamo[v][zg] = (S)((double)a.lamo[v][zg] + acc[v]);
    a.dk[zg] = (S)((double)a.dk[zg] + dka);
  }
  if (!fold_sum<S, ND>(a, d, dst, pidx, grp, acc, dka)) return;
  for (int v = 0; v < NC; ++v) a.lamo[v][zg] = (S)((double)a.lamo[v][zg] + acc[v]);
  a.dk[zg] = (S)((double)a.dk[zg] + dka);
}

// ------------------------------------------------------------------------------------------
static AdjTile make_adj_tile(const fornax_m1_desc& D, int TM, int TXB);

// Planes per block: a block walks TM + 3 faces along y (three to fill its rings) one after the
// other, each waiting on loads it has just issued, so the kernel's time is about the number of
// rounds of block slots times TM + 3.  Take the TM with the least such cost (three blocks of
// at most four waves per CU: three waves per SIMD), e.g. 7 planes on the periodic 256^2 grid
// (740 blocks, one round on 256 CUs); with ghost layers, 7 planes measured 8 % faster than 8
// (660 blocks) and 12 % faster than 4.
static int choose_adj_planes(const fornax_m1_desc& D, int TXB, int cus) {
  if (D.ndim < 2) return 1;
  const int G = D.ngroups;
  const int txb = TXB > 0 ? TXB : std::max(4, 256 / G);
  const int waves = (std::min(txb * G, 512) + 63) / 64;
  const int per_cu = std::max(1, 12 / waves);
  const long slots = (long)per_cu * (cus > 0 ? cus : 256);
  int best = 8;
  double best_cost = 1e30;
  for (int TM = 4; TM <= 32; ++TM) {
    const AdjTile t = make_adj_tile(D, TM, TXB);
    const long rounds = (t.nblocks + slots - 1) / slots;
    const double cost = (double)rounds * (TM + 3);
    if (cost < best_cost) {
      best_cost = cost;
      best = TM;
    }
  }
  return best;
}

static AdjTile make_adj_tile(const fornax_m1_desc& D, int TM, int TXB) {
  AdjTile tl;
  const int G = D.ngroups;
  tl.TXB = TXB > 0 ? TXB : std::max(4, 256 / G);
  if (tl.TXB * G > 512) tl.TXB = 512 / G;
  if (tl.TXB < 4) tl.TXB = 4;
  tl.W = tl.TXB - 3;
  tl.TM = TM;
  // a wrapping direction's tiles cover its zones, any other's the two ghost layers too
  tl.ntx = (D.n[0] + (adj_wraps(D, 0) ? 0 : 4) + tl.W - 1) / tl.W;
  const int nM = (D.ndim >= 2) ? D.n[D.ndim - 1] : 1;
  tl.ntm = (D.ndim >= 2) ? (nM + (adj_wraps(D, D.ndim - 1) ? 0 : 4) + TM - 1) / TM : 1;
  tl.nblocks = tl.ntx * tl.ntm;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  tl.nthreads = tl.TXB * G;
  return tl;
}

static size_t adj_lds_bytes(const AdjTile& tl, int dim, int G, size_t rsize) {
  const int NC = 1 + dim, NV = 2 * NC + 1;
  size_t n = (size_t)NV * (tl.TXB + 3) * G + (size_t)4 * NC * tl.TXB * G + (size_t)2 * tl.TXB * G;
  return n * rsize;
}

template <typename S, typename R>
static int launch_adjoint_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* Un,
                            const fornax_m1_state* Unp1, const fornax_m1_coeffs* cf, const double* inflow,
                            double dt, const fornax_m1_state* lam_np1, fornax_m1_state* lam_n, void* dkappa,
                            hipStream_t st) {
  const fornax_m1_desc& D = ctx->desc;
  // U^{n+1} of the step, from the caller (required)
  const fornax_m1_state u1 = *Unp1;
  AdjArgs<S> a;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = D.n[d];
    a.bc_lo[d] = D.bc_lo[d];
    a.bc_hi[d] = D.bc_hi[d];
  }
  fill_ghost_table(a);
  a.G = D.ngroups;
  a.ndim = D.ndim;
  a.limiter = D.limiter;
  a.closure = D.closure;
  a.wavespeed = D.wavespeed;
  a.zones_per_block = 0;
  a.nzones = (int64_t)D.n[0] * D.n[1] * D.n[2];
  a.c = D.c;
  a.dt = dt;
  a.f2_fp64 = D.f_fp64 * D.f_fp64;
  a.inflow = inflow;
  a.E = (const S*)Un->E;
  a.Eo = nullptr;
  for (int k = 0; k < 3; ++k) {
    a.F[k] = (k < D.ndim) ? (const S*)Un->F[k] : nullptr;
    a.Fo[k] = nullptr;
  }
  a.kap = (const S*)cf->kappa;
  a.sig = (const S*)cf->sigma;
  a.B = (const S*)cf->B;
  a.dEm = nullptr;
  a.p_energy = a.p_maxf2 = nullptr;
  a.p_nun = a.p_nnp = nullptr;
  a.lam[0] = (const S*)lam_np1->E;
  a.lamo[0] = (S*)lam_n->E;
  for (int k = 0; k < 3; ++k) {
    a.lam[1 + k] = (k < D.ndim) ? (const S*)lam_np1->F[k] : nullptr;
    a.lamo[1 + k] = (k < D.ndim) ? (S*)lam_n->F[k] : nullptr;
  }
  a.dk = (S*)dkappa;
  a.U1[0] = (const S*)u1.E;
  for (int k = 0; k < 3; ++k) a.U1[1 + k] = (const S*)u1.F[k];
  for (int d = 0; d < 3; ++d) {
    a.gbuf[d] = ctx->adj_gbuf[d];
    a.gplane[d] = ctx->adj_gplane[d];
    a.wrap[d] = adj_wraps(D, d) ? 1 : 0;
  }
  // tiling: the override read at create, else 256 threads and planes from the CU count
  const int txb = ctx->adj_txb;
  int tm = ctx->adj_tm;
  if (tm <= 0) tm = choose_adj_planes(D, txb, ctx->cus);
  AdjTile tl = make_adj_tile(D, tm, txb);
  if (tl.TXB * D.ngroups > 512) return FORNAX_EUNSUPPORTED;
  const size_t lds = adj_lds_bytes(tl, D.ndim, D.ngroups, sizeof(R));
  if (lds > 65536) return FORNAX_EUNSUPPORTED;
  // the method's default limiter is a compile-time constant of its own instantiation
  const bool mm = D.limiter == FORNAX_LIMITER_MINMOD;
  // every direction wrapping (a periodic grid) is an instantiation of its own for 2-D minmod
  const bool per = a.wrap[0] && a.wrap[1];
  constexpr int MM = FORNAX_LIMITER_MINMOD;
  const dim3 gr(tl.nblocks), bl(tl.nthreads);
  if (D.ndim == 1 && mm)
    hipLaunchKernelGGL((k_adjoint<S, R, 1, MM, false>), gr, bl, lds, st, a, geo, tl);
  else if (D.ndim == 1)
    hipLaunchKernelGGL((k_adjoint<S, R, 1, -1, false>), gr, bl, lds, st, a, geo, tl);
  else if (mm && per)
    hipLaunchKernelGGL((k_adjoint<S, R, 2, MM, true>), gr, bl, lds, st, a, geo, tl);
  else if (mm)
    hipLaunchKernelGGL((k_adjoint<S, R, 2, MM, false>), gr, bl, lds, st, a, geo, tl);
  else
    hipLaunchKernelGGL((k_adjoint<S, R, 2, -1, false>), gr, bl, lds, st, a, geo, tl);
  if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  // the ghost adjoints of the directions that do not wrap
  int nt = a.wrap[0] ? 0 : 4 * a.gplane[0] * a.G;
  if (D.ndim >= 2 && !a.wrap[1]) nt += 4 * a.gplane[1] * a.G;
  if (nt > 0) {
    if (D.ndim == 1)
      hipLaunchKernelGGL((k_adj_fold<S, 1>), dim3((nt + 255) / 256), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_adj_fold<S, 2>), dim3((nt + 255) / 256), dim3(256), 0, st, a);
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  return FORNAX_OK;
}

}  // namespace fm1

using namespace fm1;

int fm1_launch_adjoint(fornax_m1_ctx* ctx, const fornax_m1_state* Un, const fornax_m1_state* Unp1,
                       const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_state* lam_np1,
                       fornax_m1_state* lam_n, void* dkappa, hipStream_t stream) {
  const fornax_m1_desc& D = ctx->desc;
  if (D.coord != FORNAX_CARTESIAN || D.ndim > 2 || D.ngroups > 128) return FORNAX_EUNSUPPORTED;
  if (D.integrator != FORNAX_EULER) return FORNAX_EUNSUPPORTED;   // the adjoint is of the Euler push
  if (D.wavespeed != FORNAX_WAVESPEED_LIGHT || D.limiter == FORNAX_LIMITER_PPM) return FORNAX_EUNSUPPORTED;
  if (!ctx->adj_gbuf[0]) return FORNAX_ENOMEM;
  if (D.precision == FORNAX_FP64)
    return launch_adjoint_t<double, double>(ctx, ctx->geo_d, Un, Unp1, cf, inflow, dt, lam_np1, lam_n, dkappa,
                                            stream);
  return launch_adjoint_t<float, float>(ctx, ctx->geo_f, Un, Unp1, cf, inflow, dt, lam_np1, lam_n, dkappa, stream);
}
