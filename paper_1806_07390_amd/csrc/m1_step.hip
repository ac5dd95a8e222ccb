// m1_step.hip -- the fused step kernel of libfornax_m1 for gfx950.
//
// One launch advances every zone-group by one step: ghost rules, linear reconstruction,
// closure, HLL fluxes, conservative divergence (eq:finite_vol) plus geometric sources,
// backward-Euler interaction update, store, and block partials of the diagnostics.
//
// Work decomposition
//   * lanes = (zone column, group), group innermost: a wave reads and writes contiguous
//     runs of each component array (structure of arrays, group index innermost);
//   * a block owns a tile of TXB (x) by TYB (y, 3-D only) zone columns and marches along
//     the slowest active direction over TM planes.  In the march direction every face is
//     computed once from a five-plane register window and reused by the next plane;
//   * in-plane neighbours are exchanged through LDS.  Each thread computes the face on the
//     lower side of its column in every in-plane direction; the last column (row) of the
//     tile only supplies that face, so tiles overlap by one zone and update TXB-1 (TYB-1);
//   * blocks are renumbered so that each of the 8 XCDs processes a contiguous range of
//     tiles, keeping the halos that neighbouring tiles share in the same L2.
// Two block barriers per plane: after the plane is staged in LDS, and after the in-plane
// fluxes are.

#include <hip/hip_runtime.h>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

template <typename S, typename R, int DIM, bool SPH>
__global__ void __launch_bounds__(512) k_step_tiled(StepArgs<S> a, Geo<R> geo, Tile tl) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NC = 1 + DIM;   // E, F_1..F_DIM
  constexpr int NV = NC + 1;    // + total opacity
  constexpr int MD = DIM - 1;   // march direction (DIM >= 2)
  const int G = a.G;
  const int t = threadIdx.x;
  const int grp = t % G;
  const int col = t / G;
  const int TXB = tl.TXB, TYB = tl.TYB;
  const int cx = col % TXB, cy = col / TXB;
  const int COLS = TXB + 3;
  const int ROWS = (DIM == 3) ? TYB + 3 : 1;

  // LDS: plane values PV[v][row][col][g] (col = cx + 2, row = cy + 2), fluxes FX/FY[c][cy][cx][g]
  R* PV = reinterpret_cast<R*>(smem);
  R* FX = PV + (size_t)NV * ROWS * COLS * G;
  R* FY = FX + (size_t)NC * TYB * TXB * G;
  size_t dz_off = ((size_t)NV * ROWS * COLS * G + (size_t)NC * TYB * TXB * G * (DIM == 3 ? 2 : 1)) * sizeof(R);
  dz_off = (dz_off + 15) & ~(size_t)15;
  double* DZ = reinterpret_cast<double*>(smem + dz_off);
  auto pv = [&](int v, int rowL, int colL, int g) -> R& {
    return PV[(((size_t)v * ROWS + rowL) * COLS + colL) * G + g];
  };

  // logical tile of this block (XCD-aware renumbering)
  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int L = xcd * tl.xq + min(xcd, tl.xr) + slot;
  const int tx = L % tl.ntx;
  const int rest = L / tl.ntx;
  const int ty = (DIM == 3) ? rest % tl.nty : 0;
  const int tm = (DIM == 3) ? rest / tl.nty : (DIM == 2 ? rest : 0);
  const int x0 = tx * (TXB - 1);
  const int y0 = (DIM == 3) ? ty * (TYB - 1) : 0;
  const int nM = (DIM >= 2) ? a.n[MD] : 1;
  const int mbeg = tm * tl.TM;
  const int mend = min(mbeg + tl.TM, nM);

  const int n0 = a.n[0], n1 = a.n[1];
  const int gx = x0 + cx;
  const int gy = (DIM == 3) ? y0 + cy : 0;
  const bool inx = gx < n0;
  const bool iny = (DIM < 3) || gy < n1;
  const bool thread_ok = col < TXB * TYB;
  // this column's zone is updated
  const bool upd = thread_ok && inx && iny && cx < TXB - 1 && (DIM < 3 || cy < TYB - 1);
  // this column's own zone is staged in LDS (at most one index outside the domain)
  const bool own = thread_ok && gx <= n0 + 1 && (DIM < 3 || gy <= n1 + 1) && (inx || iny);
  // faces computed by this thread: x-face gx - 1/2 of row gy; y-face gy - 1/2 of column gx
  const bool do_xf = thread_ok && gx <= n0 && iny && (DIM < 3 || cy < TYB - 1);
  const bool do_yf = (DIM == 3) && thread_ok && gy <= n1 && inx && cx < TXB - 1;

  const bool want_diag = a.p_energy != nullptr;
  ZoneDiag zd;
  const R c = R(a.c);
  const R dtR = R(a.dt);

  // ---- halo slots of this thread (at most two; fixed for the whole march) ----
  // x halo: columns -2, -1, TXB of rows 0..TYB-1; y halo (3-D): rows -2, -1, TYB of columns
  // 0..TXB-1.  A slot is (group, LDS column, LDS row, direction of its ghost index).
  const int nhx = 3 * TYB;
  const int nslots = (nhx + ((DIM == 3) ? 3 * TXB : 0)) * G;
  int hsl_g[2], hsl_c[2], hsl_r[2], hsl_d[2];
  bool hsl_on[2];
  for (int k2 = 0; k2 < 2; ++k2) {
    const int sidx = t + k2 * (int)blockDim.x;
    hsl_on[k2] = false;
    hsl_g[k2] = hsl_c[k2] = hsl_r[k2] = hsl_d[k2] = 0;
    if (sidx < nslots) {
      const int hg = sidx % G, hs = sidx / G;
      int hc, hr, d;
      if (hs < nhx) {
        const int which = hs % 3;
        hr = hs / 3;
        hc = (which == 0) ? -2 : (which == 1 ? -1 : TXB);
        d = 0;
      } else {
        const int hs2 = hs - nhx;
        const int which = hs2 % 3;
        hc = hs2 / 3;
        hr = (which == 0) ? -2 : (which == 1 ? -1 : TYB);
        d = 1;
      }
      const int hx = x0 + hc;
      const int hy = (DIM == 3) ? y0 + hr : 0;
      const bool hinx = hx >= 0 && hx < n0, hiny = (DIM < 3) || (hy >= 0 && hy < n1);
      // needed: x-halo zones of rows inside the domain up to x = n0 + 1; y-halo zones of
      // columns inside the domain up to y = n1 + 1
      const bool need = (d == 0) ? (hiny && hx <= n0 + 1) : (hinx && hy <= n1 + 1);
      hsl_on[k2] = need;
      hsl_g[k2] = hg;
      hsl_c[k2] = hc;
      hsl_r[k2] = hr;
      hsl_d[k2] = d;
    }
  }
  // load plane-m values of this thread's non-window LDS entries: its own zone (when it is not
  // a marching column) and its halo slots
  auto load_plane = [&](int m, R own_q[4], R& own_ks, R hq[2][4], R hks[2]) {
    const int zj = (DIM == 2) ? m : gy;
    const int zk = (DIM == 3) ? m : 0;
    for (int cc = 0; cc < 4; ++cc) own_q[cc] = R(0);
    own_ks = R(0);
    if (own && !(DIM >= 2 && upd)) {
      if (!iny) fetch<S, R, SPH, DIM>(a, geo, 1, zj, gx, zj, zk, grp, own_q, &own_ks);
      else fetch<S, R, SPH, DIM>(a, geo, 0, gx, gx, zj, zk, grp, own_q, &own_ks);
    }
    for (int k2 = 0; k2 < 2; ++k2) {
      for (int cc = 0; cc < 4; ++cc) hq[k2][cc] = R(0);
      hks[k2] = R(0);
      if (hsl_on[k2]) {
        const int hx = x0 + hsl_c[k2];
        const int hy = (DIM == 3) ? y0 + hsl_r[k2] : zj;
        if (hsl_d[k2] == 0) fetch<S, R, SPH, DIM>(a, geo, 0, hx, hx, hy, zk, hsl_g[k2], hq[k2], &hks[k2]);
        else fetch<S, R, SPH, DIM>(a, geo, 1, hy, hx, hy, zk, hsl_g[k2], hq[k2], &hks[k2]);
      }
    }
  };

  // ---- march-direction window (DIM >= 2): q(m-2..m+2) + prefetched m+3, face state, flux ----
  R w[6][4];
  R ks0 = R(0), ks1 = R(0), ks2 = R(0), ks3 = R(0);   // total opacity of planes m .. m+3
  R sHi[4];                      // upper face state of plane m (reconstructed along MD)
  R fPrev[4];                    // march-direction flux at face m - 1/2
  for (int cc = 0; cc < 4; ++cc) {
    sHi[cc] = fPrev[cc] = R(0);
    for (int o = 0; o < 6; ++o) w[o][cc] = R(0);
  }
  const int ei = gx + NG;
  const int jj = (DIM == 3) ? gy : 0;
  if constexpr (DIM >= 2) {
    if (upd) {
      R ksb = R(0);
      for (int o = -2; o <= 2; ++o) {
        R ks = R(0);
        fetch<S, R, SPH, DIM>(a, geo, MD, mbeg + o, gx, jj, 0, grp, w[o + 2], o >= -1 ? &ks : nullptr);
        if (o == -1) ksb = ks;      // plane mbeg - 1
        if (o == 0) ks0 = ks;       // plane mbeg
        if (o == 1) ks1 = ks;       // plane mbeg + 1
        if (o == 2) ks2 = ks;       // plane mbeg + 2
      }
      // face mbeg - 1/2 from planes mbeg-1 (left) and mbeg (right)
      const int ej = (DIM == 3 ? gy : mbeg) + NG;
      const int ef = mbeg + NG;
      R h0[3], h1[3], h2[3];
      face_h<R, SPH>(geo, MD, ei, ej, ef - 1, h0);
      face_h<R, SPH>(geo, MD, ei, ej, ef, h1);
      face_h<R, SPH>(geo, MD, ei, ej, ef + 1, h2);
      const bool o0 = geo.wf[MD][ef - 1] != R(0), o1 = geo.wf[MD][ef] != R(0), o2 = geo.wf[MD][ef + 1] != R(0);
      R Llo[4], Lhi[4], Rlo[4];
      reconstruct<R, SPH, DIM>(a, geo, MD, ef - 1, w[0], w[1], w[2], h0, h1, o0, o1, Llo, Lhi);
      reconstruct<R, SPH, DIM>(a, geo, MD, ef, w[1], w[2], w[3], h1, h2, o1, o2, Rlo, sHi);
      if (o1) {
        const R dlL = proper_width<R, SPH>(geo, MD, ei, (DIM == 3) ? ej : ef - 1);
        const R dlR = proper_width<R, SPH>(geo, MD, ei, (DIM == 3) ? ej : ef);
        hll<R, SPH, DIM>(a, MD, Lhi, Rlo, h1, epsilon_of(ksb, ks0, dlL, dlR), fPrev);
      }
    }
  }
  R own_q[4], own_ks, hq[2][4], hks[2];

  int64_t dz_zone = -1;
  for (int m = mbeg; m < mend; ++m) {
    // zone indices of this column in plane m
    const int zi = gx;
    const int zj = (DIM == 2) ? m : gy;
    const int zk = (DIM == 3) ? m : 0;
    // ---- loads: window plane m + 3 (used by the next plane), own and halo values of plane m
    // (used after the march-direction face below) ----
    // (vector-memory loads retire in issue order: the plane-m loads go first so that staging
    // them does not wait for the prefetch)
    const bool more = m + 1 < mend;
    load_plane(m, own_q, own_ks, hq, hks);
    if constexpr (DIM >= 2) {
      if (upd && more) fetch<S, R, SPH, DIM>(a, geo, MD, m + 3, gx, jj, 0, grp, w[5], &ks3);
    }
    // ---- march direction: reconstruct plane m+1, flux at m + 1/2 ----
    R fNext[4] = {R(0), R(0), R(0), R(0)};
    R nHi[4] = {R(0), R(0), R(0), R(0)};
    if constexpr (DIM >= 2) {
      if (upd) {
        const int ej = (DIM == 3 ? gy : m) + NG;
        const int ef = m + 1 + NG;   // face m + 1/2
        R h1[3], h2[3];
        face_h<R, SPH>(geo, MD, ei, ej, ef, h1);
        face_h<R, SPH>(geo, MD, ei, ej, ef + 1, h2);
        const bool o1 = geo.wf[MD][ef] != R(0), o2 = geo.wf[MD][ef + 1] != R(0);
        R nLo[4];
        reconstruct<R, SPH, DIM>(a, geo, MD, ef, w[2], w[3], w[4], h1, h2, o1, o2, nLo, nHi);
        if (o1) {
          const R dlL = proper_width<R, SPH>(geo, MD, ei, (DIM == 3) ? ej : ef - 1);
          const R dlR = proper_width<R, SPH>(geo, MD, ei, (DIM == 3) ? ej : ef);
          hll<R, SPH, DIM>(a, MD, sHi, nLo, h1, epsilon_of(ks0, ks1, dlL, dlR), fNext);
        }
      }
    }
    // ---- (a) stage plane m in LDS ----
    if (thread_ok) {
      const int rowL = (DIM == 3) ? cy + 2 : 0;
      const bool win = (DIM >= 2) && upd;
      for (int v = 0; v < NC; ++v) pv(v, rowL, cx + 2, grp) = win ? w[2][v] : own_q[v];
      pv(NC, rowL, cx + 2, grp) = win ? ks0 : own_ks;
    }
    for (int k2 = 0; k2 < 2; ++k2) {
      if ((int)(t + k2 * (int)blockDim.x) < nslots) {
        const int rowL = (DIM == 3) ? hsl_r[k2] + 2 : 0;
        for (int v = 0; v < NC; ++v) pv(v, rowL, hsl_c[k2] + 2, hsl_g[k2]) = hq[k2][v];
        pv(NC, rowL, hsl_c[k2] + 2, hsl_g[k2]) = hks[k2];
      }
    }
    __syncthreads();
    // ---- (c) in-plane faces from LDS ----
    {
      const int rowL = (DIM == 3) ? cy + 2 : 0;
      if (do_xf) {
        R q[4][4];
        for (int o = 0; o < 4; ++o) {
          for (int v = 0; v < NC; ++v) q[o][v] = pv(v, rowL, cx + o, grp);
          for (int v = NC; v < 4; ++v) q[o][v] = R(0);
        }
        const R ksL = pv(NC, rowL, cx + 1, grp), ksR = pv(NC, rowL, cx + 2, grp);
        R fl[4];
        face_flux<S, R, SPH, DIM>(a, geo, 0, gx, gx, zj, q, ksL, ksR, fl);
        for (int v = 0; v < NC; ++v) FX[(((size_t)v * TYB + cy) * TXB + cx) * G + grp] = fl[v];
      }
      if constexpr (DIM == 3) {
        if (do_yf) {
          R q[4][4];
          for (int o = 0; o < 4; ++o) {
            for (int v = 0; v < NC; ++v) q[o][v] = pv(v, cy + o, cx + 2, grp);
            for (int v = NC; v < 4; ++v) q[o][v] = R(0);
          }
          const R ksL = pv(NC, cy + 1, cx + 2, grp), ksR = pv(NC, cy + 2, cx + 2, grp);
          R fl[4];
          face_flux<S, R, SPH, DIM>(a, geo, 1, gy, gx, gy, q, ksL, ksR, fl);
          for (int v = 0; v < NC; ++v) FY[(((size_t)v * TYB + cy) * TXB + cx) * G + grp] = fl[v];
        }
      }
    }
    // deferred dE_matter of the previous plane (DZ written before the last barrier)
    if (a.dEm && dz_zone >= 0 && grp == 0) {
      double sdz = 0.0;
      for (int g2 = 0; g2 < G; ++g2) sdz += DZ[(size_t)col * G + g2];
      a.dEm[dz_zone] = -sdz;
    }
    __syncthreads();
    // ---- (f) update ----
    dz_zone = -1;
    if (upd) {
      R q0[4];
      if constexpr (DIM >= 2) {
        for (int cc = 0; cc < 4; ++cc) q0[cc] = w[2][cc];
      } else {
        for (int cc = 0; cc < 4; ++cc) q0[cc] = own_q[cc];
      }
      R acc[4] = {R(0), R(0), R(0), R(0)};
      {
        const int e = gx + NG;
        R wlo = R(1), whi = R(1), iW = R(1) / geo.dx[0];
        if constexpr (SPH) {
          wlo = geo.wf[0][e];
          whi = geo.wf[0][e + 1];
          iW = geo.iW[0][e];
        }
        for (int v = 0; v < NC; ++v) {
          const R flo = FX[(((size_t)v * TYB + cy) * TXB + cx) * G + grp];
          const R fhi = FX[(((size_t)v * TYB + cy) * TXB + cx + 1) * G + grp];
          acc[v] += (whi * fhi - wlo * flo) * iW;
        }
      }
      if constexpr (DIM == 3) {
        const int e = gy + NG;
        R wlo = R(1), whi = R(1), iW = R(1) / geo.dx[1];
        if constexpr (SPH) {
          wlo = geo.wf[1][e];
          whi = geo.wf[1][e + 1];
          iW = geo.iW[1][e];
        }
        for (int v = 0; v < NC; ++v) {
          const R flo = FY[(((size_t)v * TYB + cy) * TXB + cx) * G + grp];
          const R fhi = FY[(((size_t)v * TYB + cy + 1) * TXB + cx) * G + grp];
          acc[v] += (whi * fhi - wlo * flo) * iW;
        }
      }
      if constexpr (DIM >= 2) {
        const int e = m + NG;
        R wlo = R(1), whi = R(1), iW = R(1) / geo.dx[MD];
        if constexpr (SPH) {
          wlo = geo.wf[MD][e];
          whi = geo.wf[MD][e + 1];
          iW = geo.iW[MD][e];
        }
        for (int v = 0; v < NC; ++v) acc[v] += (whi * fNext[v] - wlo * fPrev[v]) * iW;
      }
      R Um[4];
      for (int cc = 0; cc < 4; ++cc) Um[cc] = (cc < NC) ? q0[cc] - dtR * acc[cc] : R(0);
      if constexpr (SPH) {
        R h[3], P[9], Sg[3];
        cell_h<R, SPH>(geo, zi + NG, zj + NG, h);
        closure_full<R, SPH, DIM>(q0, h, c, a.closure, P);
        geometric_source<R>(P, h, geo.gam + 4 * zj, c, Sg);
        for (int cc = 0; cc < DIM; ++cc) Um[1 + cc] += dtR * Sg[cc];
      }
      const int64_t zone = ((int64_t)zk * n1 + zj) * n0 + zi;
      const double dz = finish_zone<S, R, SPH, DIM>(a, geo, (int)(zone * G + grp), zi, zj, zk, Um, want_diag, zd);
      if (a.dEm) {
        DZ[(size_t)col * G + grp] = dz;
        dz_zone = zone;
      }
    }
    // ---- advance the march window and the prefetched plane values ----
    if constexpr (DIM >= 2) {
      for (int o = 0; o < 5; ++o)
        for (int cc = 0; cc < 4; ++cc) w[o][cc] = w[o + 1][cc];
      for (int cc = 0; cc < 4; ++cc) {
        sHi[cc] = nHi[cc];
        fPrev[cc] = fNext[cc];
      }
      ks0 = ks1;
      ks1 = ks2;
      ks2 = ks3;
    }
  }
  if (a.dEm) {
    __syncthreads();
    if (dz_zone >= 0 && grp == 0) {
      double s = 0.0;
      for (int g2 = 0; g2 < G; ++g2) s += DZ[(size_t)col * G + g2];
      a.dEm[dz_zone] = -s;
    }
  }
  if (!want_diag) return;
  // ---- block partials of the diagnostics: wave reduction, then across waves ----
  double e = zd.energy, mf = zd.maxf2;
  int u = zd.nun, p = zd.nnp;
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off);
    mf = fmax(mf, __shfl_xor(mf, off));
    u += __shfl_xor(u, off);
    p += __shfl_xor(p, off);
  }
  __shared__ double we[16], wm[16];
  __shared__ int wu[16], wp[16];
  const int wave = t >> 6, lane = t & 63;
  __syncthreads();
  if (lane == 0) {
    we[wave] = e;
    wm[wave] = mf;
    wu[wave] = u;
    wp[wave] = p;
  }
  __syncthreads();
  if (t == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double se = 0.0, sm = 0.0;
    int su = 0, sp = 0;
    for (int k2 = 0; k2 < nw; ++k2) {
      se += we[k2];
      sm = fmax(sm, wm[k2]);
      su += wu[k2];
      sp += wp[k2];
    }
    a.p_energy[blockIdx.x] = se;
    a.p_maxf2[blockIdx.x] = sm;
    a.p_nun[blockIdx.x] = su;
    a.p_nnp[blockIdx.x] = sp;
  }
}

// ------------------------------------------------------------------------------------------
size_t tile_lds_bytes(const Tile& tl, int dim, int G, size_t rsize, bool dz) {
  const int NC = 1 + dim, NV = NC + 1;
  const int ROWS = (dim == 3) ? tl.TYB + 3 : 1;
  size_t b = (size_t)NV * ROWS * (tl.TXB + 3) * G * rsize;
  b += (size_t)NC * tl.TYB * tl.TXB * G * rsize * (dim == 3 ? 2 : 1);
  b = (b + 15) & ~(size_t)15;
  if (dz) b += (size_t)tl.TXB * tl.TYB * G * sizeof(double);
  return b;
}

// every thread stages at most two halo zone-groups per plane
bool halo_slots_fit(const Tile& tl, int dim) {
  const int nh = 3 * tl.TYB + (dim == 3 ? 3 * tl.TXB : 0);
  return nh <= 2 * tl.TXB * tl.TYB;
}

Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM) {
  Tile tl;
  tl.TXB = TXB;
  tl.TYB = (D.ndim == 3) ? TYB : 1;
  tl.TM = (D.ndim >= 2) ? TM : 1;
  tl.ntx = (D.n[0] + (tl.TXB - 1) - 1) / (tl.TXB - 1);
  tl.nty = (D.ndim == 3) ? (D.n[1] + (tl.TYB - 1) - 1) / (tl.TYB - 1) : 1;
  const int nM = (D.ndim >= 2) ? D.n[D.ndim - 1] : 1;
  tl.ntm = (nM + tl.TM - 1) / tl.TM;
  tl.nblocks = tl.ntx * tl.nty * tl.ntm;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  tl.nthreads = tl.TXB * tl.TYB * D.ngroups;
  return tl;
}

// Default tile: as many zone columns as fit in the thread and LDS budgets.
Tile choose_tile(const fornax_m1_desc& D, size_t rsize) {
  const int G = D.ngroups;
  int TM = 8;
  if (D.ndim < 3) {
    int TXB = 256 / G;
    if (TXB < 2) TXB = 2;
    return make_tile(D, TXB, 1, TM);
  }
  // 3-D: near-square tiles of up to 512 threads within 64 KiB of LDS
  for (int cols = 512 / G; cols >= 4; --cols) {
    int TXB = 2;
    while ((TXB + 1) * (TXB + 1) <= cols) ++TXB;
    int TYB = cols / TXB;
    if (TYB < 2) continue;
    Tile tl = make_tile(D, TXB, TYB, TM);
    if (tile_lds_bytes(tl, 3, G, rsize, true) <= 65536 && halo_slots_fit(tl, 3)) return tl;
  }
  return make_tile(D, 2, 2, TM);
}

template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, const Tile& tl, hipStream_t st) {
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  const int D = ctx->desc.ndim;
  const size_t lds = tile_lds_bytes(tl, D, a.G, sizeof(R), a.dEm != nullptr);
  dim3 grid(tl.nblocks), block(tl.nthreads);
#define FM1_LAUNCH(DIMV, SPHV) \
  hipLaunchKernelGGL((k_step_tiled<S, R, DIMV, SPHV>), grid, block, lds, st, a, geo, tl)
  if (sph) {
    if (D == 1) FM1_LAUNCH(1, true);
    else if (D == 2) FM1_LAUNCH(2, true);
    else FM1_LAUNCH(3, true);
  } else {
    if (D == 1) FM1_LAUNCH(1, false);
    else if (D == 2) FM1_LAUNCH(2, false);
    else FM1_LAUNCH(3, false);
  }
#undef FM1_LAUNCH
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template int launch_tiled<double, double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&, const Tile&,
                                          hipStream_t);
template int launch_tiled<float, float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, const Tile&,
                                        hipStream_t);

}  // namespace fm1
