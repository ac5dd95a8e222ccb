// m1_step.hip -- the fused step kernel of libfornax_m1 for gfx950.
//
// One launch advances every zone-group by one step: ghost rules, linear reconstruction,
// closure, HLL fluxes, conservative divergence (eq:finite_vol) plus geometric sources,
// backward-Euler interaction update, store, and block partials of the diagnostics.
//
// Work decomposition
//   * lanes = (zone column, group), group innermost: a wave reads and writes contiguous
//     runs of each component array (structure of arrays, group index innermost).  A block
//     holds GB groups (all G, or a divisor of G when the zone tile would otherwise be tiny);
//   * a block owns a tile of TXB (x) by TYB (y, 3-D only) zone columns and marches along the
//     slowest active direction over TM planes.  Tiles overlap by two columns (rows): the
//     edge columns only supply face states, the interior TXB-2 (TYB-2) columns are updated;
//   * march direction: every zone is reconstructed once and every face computed once from a
//     register window of planes m .. m+3 (m+3 prefetched one plane ahead);
//   * in-plane directions: each zone is reconstructed once per plane from its neighbours in
//     LDS; its lower face state goes to LDS, and the thread of the zone below the face
//     computes the flux there and passes it up through LDS;
//   * ghost zones are never stored: the source zone and the sign / inflow rules of every
//     in-plane index are resolved once per thread, the march index once per load;
//   * blocks are renumbered so that each of the 8 XCDs processes a contiguous range of
//     tiles (neighbouring tiles share halos in the same L2).
// Three block barriers per plane: after the plane is staged, after the lower face states
// are, and after the in-plane fluxes are.

#include <hip/hip_runtime.h>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

// Source of a zone index e (possibly a ghost, |e - clamp(e)| <= 2) along one axis of n zones.
// flags: bit 0 flips the flux component normal to this axis (reflect, polar axis), bit 1 takes
// the prescribed inflow state, bit 2 marks the polar-axis copy (shift n[2]/2 in phi, flip F_phi).
struct AxisSrc {
  int src;
  int flags;
};

__device__ __forceinline__ AxisSrc axis_src(int e, int n, int bclo, int bchi) {
  AxisSrc r{e, 0};
  if (e < 0 || e >= n) {
    const bool low = e < 0;
    const int bc = low ? bclo : bchi;
    if (bc == FORNAX_BC_PERIODIC) {
      int s = low ? e + n : e - n;
      if (s < 0) s += n;
      if (s >= n) s -= n;
      r.src = s;
    } else if (bc == FORNAX_BC_OUTFLOW || bc == FORNAX_BC_INFLOW) {
      r.src = low ? 0 : n - 1;
      r.flags = (bc == FORNAX_BC_INFLOW) ? 2 : 0;
    } else {  // reflect or polar axis: mirror
      r.src = low ? -1 - e : 2 * n - 1 - e;
      r.flags = (bc == FORNAX_BC_AXIS) ? 5 : 1;
    }
  }
  return r;
}

// Values of one zone-group from its per-axis sources; (ex, ey) are the zone's own extended
// x and y indices (for the scale factors of an inflow ghost).  q, kap and sig may be null.
template <typename S, typename R, bool SPH, int ND>
__device__ __forceinline__ void load_zone(const StepArgs<S>& a, const Geo<R>& geo, AxisSrc sx, AxisSrc sy, AxisSrc sz,
                                          int ex, int ey, int grp, R q[4], R* kap, R* sig) {
  const int fl = sx.flags | sy.flags | sz.flags;
  int iz = sz.src;
  if (fl & 4) {
    iz += a.n[2] >> 1;
    if (iz >= a.n[2]) iz -= a.n[2];
  }
  const int zg = ((iz * a.n[1] + sy.src) * a.n[0] + sx.src) * a.G + grp;
  if (kap) *kap = R(a.kap[zg]);
  if (sig) *sig = R(a.sig[zg]);
  if (!q) return;
  if (fl & 2) {
    const double* in = a.inflow + grp * (1 + ND);
    R h[3];
    cell_h<R, SPH>(geo, ex, ey, h);
    q[0] = R(in[0]);
    for (int c = 0; c < ND; ++c) q[1 + c] = h[c] * R(in[1 + c]);
  } else {
    q[0] = R(a.E[zg]);
    const bool fz = (sz.flags & 1) || (fl & 4);
    const bool flip[3] = {(sx.flags & 1) != 0, (sy.flags & 1) != 0, fz};
    for (int c = 0; c < ND; ++c) {
      const R v = R(a.F[c][zg]);
      q[1 + c] = flip[c] ? -v : v;
    }
  }
  for (int c = ND; c < 3; ++c) q[1 + c] = R(0);
}

template <typename S, typename R, int DIM, bool SPH>
__global__ void __launch_bounds__(512) k_step_tiled(StepArgs<S> a, Geo<R> geo, Tile tl) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NC = 1 + DIM;   // E, F_1..F_DIM
  constexpr int MD = DIM - 1;   // march direction (DIM >= 2)
  const int GB = tl.GB, TXB = tl.TXB, TYB = tl.TYB;
  const int t = threadIdx.x;
  const int gs = t % GB;
  const int col = t / GB;
  const int cx = col % TXB, cy = col / TXB;
  const int NCOL = TXB * TYB;
  const int PCOLS = TXB + 2;
  const int PROWS = (DIM == 3) ? TYB + 2 : 1;

  // LDS: plane values PV[v][prow][pcol][gs] (v = E, F.., kappa + sigma), lower face states
  // LX/LY[c][col][gs], in-plane fluxes FX/FY[c][col][gs] (face above the column), dE_matter
  // of the last plane DZ[col][gs]
  R* PV = reinterpret_cast<R*>(smem);
  R* LX = PV + (size_t)(NC + 1) * PROWS * PCOLS * GB;
  R* LY = LX + (size_t)NC * NCOL * GB;
  R* FX = LY + ((DIM == 3) ? (size_t)NC * NCOL * GB : 0);
  R* FY = FX + (size_t)NC * NCOL * GB;
  size_t dz_off = (size_t)((NC + 1) * PROWS * PCOLS + NC * NCOL * ((DIM == 3) ? 4 : 2)) * GB * sizeof(R);
  dz_off = (dz_off + 15) & ~(size_t)15;
  double* DZ = reinterpret_cast<double*>(smem + dz_off);
  auto pv = [&](int v, int prow, int pcol, int g) -> R& {
    return PV[(((size_t)v * PROWS + prow) * PCOLS + pcol) * GB + g];
  };
  auto cidx = [&](int c, int cl) -> size_t { return ((size_t)c * NCOL + cl) * GB + gs; };

  // logical tile of this block (XCD-aware renumbering; group blocks of a tile adjacent)
  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int L = xcd * tl.xq + min(xcd, tl.xr) + slot;
  const int gb = L % tl.ngb;
  int rest = L / tl.ngb;
  const int tx = rest % tl.ntx;
  rest /= tl.ntx;
  const int ty = (DIM == 3) ? rest % tl.nty : 0;
  const int tm = (DIM == 3) ? rest / tl.nty : rest;
  const int grp = gb * GB + gs;

  const int n0 = a.n[0], n1 = a.n[1];
  const int x0 = tx * (TXB - 2) - 1;                          // zone of column 0
  const int y0 = (DIM == 3) ? ty * (TYB - 2) - 1 : 0;         // zone of row 0 (3-D)
  const int gx = x0 + cx;
  const int gy = (DIM == 3) ? y0 + cy : 0;
  const int nM = (DIM >= 2) ? a.n[MD] : 1;
  const int mbeg = (DIM >= 2) ? tm * tl.TM : 0;
  const int mend = (DIM >= 2) ? min(mbeg + tl.TM, nM) : 1;

  // staged: the column's zone lies within two ghost layers; recon: within one (its face
  // states are used); upd: interior column of the tile inside the domain
  const bool staged = gx <= n0 + 1 && (DIM < 3 || gy <= n1 + 1);
  const bool recon = gx <= n0 && (DIM < 3 || gy <= n1);
  const bool upd = cx >= 1 && cx <= TXB - 2 && gx < n0 && (DIM < 3 || (cy >= 1 && cy <= TYB - 2 && gy < n1));
  const bool do_xf = recon && cx <= TXB - 2 && gx + 1 <= n0 && (DIM < 3 || (cy >= 1 && cy <= TYB - 2 && gy < n1));
  const bool do_yf = (DIM == 3) && recon && cy <= TYB - 2 && gy + 1 <= n1 && cx >= 1 && cx <= TXB - 2 && gx < n0;

  const bool want_diag = a.p_energy != nullptr;
  ZoneDiag zd;
  const R c = R(a.c);
  const R dtR = R(a.dt);
  const int ex = gx + NG;
  const int eyc = (DIM == 3) ? gy + NG : NG;   // extended y of the column (3-D) / unused row (1-D)

  // fixed sources of the in-plane indices of this column
  const AxisSrc sx = axis_src(gx, n0, a.bc_lo[0], a.bc_hi[0]);
  const AxisSrc sy = (DIM == 3) ? axis_src(gy, n1, a.bc_lo[1], a.bc_hi[1]) : AxisSrc{0, 0};
  const AxisSrc s0{0, 0};

  // ---- halo slot of this thread (at most one): x halo columns -1, TXB of every row, and
  // (3-D) y halo rows -1, TYB of every column ----
  const int nsx = 2 * TYB * GB;
  const int nslots = nsx + ((DIM == 3) ? 2 * TXB * GB : 0);
  bool hs_on = false;
  int hs_pcol = 0, hs_prow = 0, hs_g = 0, hs_ex = 0, hs_ey = NG;
  AxisSrc hsx{0, 0}, hsy{0, 0};
  if (t < nslots) {
    hs_g = t % GB;
    int hxz, hyz;
    if (t < nsx) {
      const int r = t / GB;
      const int side = r & 1, row = r >> 1;
      hs_pcol = side ? TXB + 1 : 0;
      hs_prow = (DIM == 3) ? row + 1 : 0;
      hxz = side ? x0 + TXB : x0 - 1;
      hyz = (DIM == 3) ? y0 + row : 0;
    } else {
      const int r = (t - nsx) / GB;
      const int side = r & 1, cl = r >> 1;
      hs_pcol = cl + 1;
      hs_prow = side ? TYB + 1 : 0;
      hxz = x0 + cl;
      hyz = side ? y0 + TYB : y0 - 1;
    }
    hs_on = hxz <= n0 + 1 && (DIM < 3 || hyz <= n1 + 1);
    hsx = axis_src(hxz, n0, a.bc_lo[0], a.bc_hi[0]);
    if constexpr (DIM == 3) hsy = axis_src(hyz, n1, a.bc_lo[1], a.bc_hi[1]);
    hs_ex = hxz + NG;
    hs_ey = (DIM == 3) ? hyz + NG : NG;
  }
  const int hs_grp = gb * GB + hs_g;
  R hq[4] = {R(0), R(0), R(0), R(0)}, hks = R(0);
  auto load_slot = [&](int m) {
    if (hs_on) {
      R k, s;
      if constexpr (DIM == 1) {
        load_zone<S, R, SPH, DIM>(a, geo, hsx, s0, s0, hs_ex, hs_ey, hs_grp, hq, &k, &s);
      } else if constexpr (DIM == 2) {
        const AxisSrc sm = axis_src(m, nM, a.bc_lo[MD], a.bc_hi[MD]);
        load_zone<S, R, SPH, DIM>(a, geo, hsx, sm, s0, hs_ex, m + NG, hs_grp, hq, &k, &s);
      } else {
        const AxisSrc sm = axis_src(m, nM, a.bc_lo[MD], a.bc_hi[MD]);
        load_zone<S, R, SPH, DIM>(a, geo, hsx, hsy, sm, hs_ex, hs_ey, hs_grp, hq, &k, &s);
      }
      hks = k + s;
    }
  };
  // zone of this column in plane m (window loads); kap/sig may be null
  auto load_own = [&](int m, R q[4], R* k, R* s) {
    if constexpr (DIM == 1) {
      load_zone<S, R, SPH, DIM>(a, geo, sx, s0, s0, ex, eyc, grp, q, k, s);
    } else if constexpr (DIM == 2) {
      const AxisSrc sm = axis_src(m, nM, a.bc_lo[MD], a.bc_hi[MD]);
      load_zone<S, R, SPH, DIM>(a, geo, sx, sm, s0, ex, m + NG, grp, q, k, s);
    } else {
      const AxisSrc sm = axis_src(m, nM, a.bc_lo[MD], a.bc_hi[MD]);
      load_zone<S, R, SPH, DIM>(a, geo, sx, sy, sm, ex, eyc, grp, q, k, s);
    }
  };
  // extended y index of the zone row in plane m (spherical tables; theta is y)
  auto ey_of = [&](int m) -> int { return (DIM == 2) ? m + NG : eyc; };

  // ---- register window along the march direction: q(m .. m+3), kappa/sigma(m .. m+2), B ----
  R q0[4], q1[4], q2[4], q3[4];
  R hiM[4], fPrev[4];
  for (int k = 0; k < 4; ++k) q0[k] = q1[k] = q2[k] = q3[k] = hiM[k] = fPrev[k] = R(0);
  R k0 = R(0), s0v = R(0), k1 = R(0), s1v = R(0), k2 = R(0), s2v = R(0), B0 = R(0), B1 = R(0);
  const int zgB = grp;   // B offset added to the zone index below
  auto loadB = [&](int m) -> R {
    // B of this column's zone in plane m (only updated columns use it; in-domain there)
    const int zi = gx, zj = (DIM == 2) ? m : gy, zk = (DIM == 3) ? m : 0;
    return R(a.B[((zk * n1 + zj) * n0 + zi) * a.G + zgB]);
  };
  if (staged) {
    if constexpr (DIM >= 2) {
      R qa[4], qb[4], ka, sa;
      load_own(mbeg - 2, qa, nullptr, nullptr);
      load_own(mbeg - 1, qb, &ka, &sa);
      load_own(mbeg, q0, &k0, &s0v);
      load_own(mbeg + 1, q1, &k1, &s1v);
      load_own(mbeg + 2, q2, nullptr, nullptr);
      if (upd) B0 = loadB(mbeg);
      // face mbeg - 1/2 from zones mbeg - 1 (upper state) and mbeg (lower state)
      const int ef = mbeg + NG;   // lower face of zone mbeg
      const int eyf = (DIM == 3) ? eyc : ef;
      R h0[3], h1[3], h2[3];
      face_h<R, SPH>(geo, MD, ex, eyf, ef - 1, h0);
      face_h<R, SPH>(geo, MD, ex, eyf, ef, h1);
      face_h<R, SPH>(geo, MD, ex, eyf, ef + 1, h2);
      const bool o0 = !SPH || geo.wf[MD][ef - 1] != R(0);
      const bool o1 = !SPH || geo.wf[MD][ef] != R(0);
      const bool o2 = !SPH || geo.wf[MD][ef + 1] != R(0);
      R lo[4], hiP[4];
      reconstruct<R, SPH, DIM>(a, geo, MD, ef - 1, qa, qb, q0, h0, h1, o0, o1, lo, hiP);
      reconstruct<R, SPH, DIM>(a, geo, MD, ef, qb, q0, q1, h1, h2, o1, o2, lo, hiM);
      if (o1) {
        const R dlL = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef - 1);
        const R dlR = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef);
        hll<R, SPH, DIM>(a, MD, hiP, lo, h1, epsilon_of(ka + sa, k0 + s0v, dlL, dlR), fPrev);
      }
    } else {
      load_own(0, q0, &k0, &s0v);
      if (upd) B0 = loadB(0);
    }
  }
  load_slot(mbeg);

  const int prow_own = (DIM == 3) ? cy + 1 : 0;
  const R idx0 = R(1) / geo.dx[0], idx1 = R(1) / geo.dx[1], idxM = R(1) / geo.dx[(DIM >= 2) ? MD : 0];
  int dz_zone = -1;
  for (int m = mbeg; m < mend; ++m) {
    const bool more = m + 1 < mend;
    // ---- (a) stage plane m: own zone, halo slot ----
    pv(NC, prow_own, cx + 1, gs) = k0 + s0v;
    for (int v = 0; v < NC; ++v) pv(v, prow_own, cx + 1, gs) = q0[v];
    if (t < nslots) {
      for (int v = 0; v < NC; ++v) pv(v, hs_prow, hs_pcol, hs_g) = hq[v];
      pv(NC, hs_prow, hs_pcol, hs_g) = hks;
    }
    // ---- prefetch for later planes: window q(m+3), kappa/sigma(m+2), B(m+1), slot m+1 ----
    if constexpr (DIM >= 2) {
      if (more) {
        if (staged) {
          load_own(m + 3, q3, nullptr, nullptr);
          load_own(m + 2, nullptr, &k2, &s2v);
          if (upd) B1 = loadB(m + 1);
        }
        load_slot(m + 1);
      }
    }
    __syncthreads();
    // ---- (b) deferred dE_matter of the previous plane ----
    if (a.dEm && dz_zone >= 0 && gs == 0) {
      double sdz = 0.0;
      for (int g2 = 0; g2 < GB; ++g2) sdz += DZ[(size_t)col * GB + g2];
      a.dEm[dz_zone] = -sdz;
    }
    // ---- (c) in-plane reconstruction (lower states to LDS), march face m + 1/2 ----
    const int eym = ey_of(m);
    R hiX[4] = {R(0), R(0), R(0), R(0)}, hiY[4] = {R(0), R(0), R(0), R(0)};
    if (recon) {
      R qm[4], qp[4], lo[4];
      for (int v = 0; v < 4; ++v) {
        qm[v] = (v < NC) ? pv(v, prow_own, cx, gs) : R(0);
        qp[v] = (v < NC) ? pv(v, prow_own, cx + 2, gs) : R(0);
      }
      R hlo[3], hhi[3];
      face_h<R, SPH>(geo, 0, ex, eym, ex, hlo);
      face_h<R, SPH>(geo, 0, ex, eym, ex + 1, hhi);
      const bool olo = !SPH || geo.wf[0][ex] != R(0), ohi = !SPH || geo.wf[0][ex + 1] != R(0);
      reconstruct<R, SPH, DIM>(a, geo, 0, ex, qm, q0, qp, hlo, hhi, olo, ohi, lo, hiX);
      for (int v = 0; v < NC; ++v) LX[cidx(v, col)] = lo[v];
      if constexpr (DIM == 3) {
        for (int v = 0; v < 4; ++v) {
          qm[v] = (v < NC) ? pv(v, prow_own - 1, cx + 1, gs) : R(0);
          qp[v] = (v < NC) ? pv(v, prow_own + 1, cx + 1, gs) : R(0);
        }
        face_h<R, SPH>(geo, 1, ex, eyc, eyc, hlo);
        face_h<R, SPH>(geo, 1, ex, eyc, eyc + 1, hhi);
        const bool ylo = !SPH || geo.wf[1][eyc] != R(0), yhi = !SPH || geo.wf[1][eyc + 1] != R(0);
        reconstruct<R, SPH, DIM>(a, geo, 1, eyc, qm, q0, qp, hlo, hhi, ylo, yhi, lo, hiY);
        for (int v = 0; v < NC; ++v) LY[cidx(v, col)] = lo[v];
      }
    }
    R fNext[4] = {R(0), R(0), R(0), R(0)};
    R nHi[4] = {R(0), R(0), R(0), R(0)};
    if constexpr (DIM >= 2) {
      if (upd) {
        // reconstruct zone m + 1 along the march direction; flux at m + 1/2
        const int ef = m + 1 + NG;   // lower face of zone m + 1
        const int eyf = (DIM == 3) ? eyc : ef;
        R h1[3], h2[3];
        face_h<R, SPH>(geo, MD, ex, eyf, ef, h1);
        face_h<R, SPH>(geo, MD, ex, eyf, ef + 1, h2);
        const bool o1 = !SPH || geo.wf[MD][ef] != R(0), o2 = !SPH || geo.wf[MD][ef + 1] != R(0);
        R nLo[4];
        reconstruct<R, SPH, DIM>(a, geo, MD, ef, q0, q1, q2, h1, h2, o1, o2, nLo, nHi);
        if (o1) {
          const R dlL = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef - 1);
          const R dlR = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef);
          hll<R, SPH, DIM>(a, MD, hiM, nLo, h1, epsilon_of(k0 + s0v, k1 + s1v, dlL, dlR), fNext);
        }
      }
    }
    __syncthreads();
    // ---- (d) in-plane faces above this column ----
    R fxR[4] = {R(0), R(0), R(0), R(0)}, fyR[4] = {R(0), R(0), R(0), R(0)};
    if (do_xf) {
      R qR[4] = {R(0), R(0), R(0), R(0)};
      for (int v = 0; v < NC; ++v) qR[v] = LX[cidx(v, col + 1)];
      const R ksR = pv(NC, prow_own, cx + 2, gs);
      const bool open = !SPH || geo.wf[0][ex + 1] != R(0);
      if (open) {
        R hf[3];
        face_h<R, SPH>(geo, 0, ex, eym, ex + 1, hf);
        const R dlL = proper_width<R, SPH>(geo, 0, ex, eym);
        const R dlR = proper_width<R, SPH>(geo, 0, ex + 1, eym);
        hll<R, SPH, DIM>(a, 0, hiX, qR, hf, epsilon_of(k0 + s0v, ksR, dlL, dlR), fxR);
      }
      for (int v = 0; v < NC; ++v) FX[cidx(v, col)] = fxR[v];
    }
    if constexpr (DIM == 3) {
      if (do_yf) {
        R qR[4] = {R(0), R(0), R(0), R(0)};
        for (int v = 0; v < NC; ++v) qR[v] = LY[cidx(v, col + TXB)];
        const R ksR = pv(NC, prow_own + 1, cx + 1, gs);
        const bool open = !SPH || geo.wf[1][eyc + 1] != R(0);
        if (open) {
          R hf[3];
          face_h<R, SPH>(geo, 1, ex, eyc, eyc + 1, hf);
          const R dlL = proper_width<R, SPH>(geo, 1, ex, eyc);
          const R dlR = proper_width<R, SPH>(geo, 1, ex, eyc + 1);
          hll<R, SPH, DIM>(a, 1, hiY, qR, hf, epsilon_of(k0 + s0v, ksR, dlL, dlR), fyR);
        }
        for (int v = 0; v < NC; ++v) FY[cidx(v, col)] = fyR[v];
      }
    }
    __syncthreads();
    // ---- (e) update ----
    dz_zone = -1;
    if (upd) {
      R acc[4] = {R(0), R(0), R(0), R(0)};
      {
        R wlo = R(1), whi = R(1), iW = idx0;
        if constexpr (SPH) {
          wlo = geo.wf[0][ex];
          whi = geo.wf[0][ex + 1];
          iW = geo.iW[0][ex];
        }
        for (int v = 0; v < NC; ++v) acc[v] += (whi * fxR[v] - wlo * FX[cidx(v, col - 1)]) * iW;
      }
      if constexpr (DIM == 3) {
        R wlo = R(1), whi = R(1), iW = idx1;
        if constexpr (SPH) {
          wlo = geo.wf[1][eyc];
          whi = geo.wf[1][eyc + 1];
          iW = geo.iW[1][eyc];
        }
        for (int v = 0; v < NC; ++v) acc[v] += (whi * fyR[v] - wlo * FY[cidx(v, col - TXB)]) * iW;
      }
      if constexpr (DIM >= 2) {
        const int e = m + NG;
        R wlo = R(1), whi = R(1), iW = idxM;
        if constexpr (SPH) {
          wlo = geo.wf[MD][e];
          whi = geo.wf[MD][e + 1];
          iW = geo.iW[MD][e];
        }
        for (int v = 0; v < NC; ++v) acc[v] += (whi * fNext[v] - wlo * fPrev[v]) * iW;
      }
      R Um[4];
      for (int cc = 0; cc < 4; ++cc) Um[cc] = (cc < NC) ? q0[cc] - dtR * acc[cc] : R(0);
      const int zi = gx, zj = (DIM == 2) ? m : gy, zk = (DIM == 3) ? m : 0;
      if constexpr (SPH) {
        R h[3], P[9], Sg[3];
        cell_h<R, SPH>(geo, ex, zj + NG, h);
        closure_full<R, SPH, DIM>(q0, h, c, a.closure, P);
        geometric_source<R>(P, h, geo.gam + 4 * zj, c, Sg);
        for (int cc = 0; cc < DIM; ++cc) Um[1 + cc] += dtR * Sg[cc];
      }
      const int zone = (zk * n1 + zj) * n0 + zi;
      const double dz = finish_zone_c<S, R, SPH, DIM>(a, geo, zone * a.G + grp, zi, zj, zk, Um, (double)k0,
                                                      (double)s0v, (double)B0, want_diag, zd);
      if (a.dEm) {
        DZ[(size_t)col * GB + gs] = dz;
        dz_zone = zone;
      }
    }
    // ---- advance the window ----
    if constexpr (DIM >= 2) {
      for (int cc = 0; cc < 4; ++cc) {
        q0[cc] = q1[cc];
        q1[cc] = q2[cc];
        q2[cc] = q3[cc];
        hiM[cc] = nHi[cc];
        fPrev[cc] = fNext[cc];
      }
      k0 = k1;
      s0v = s1v;
      k1 = k2;
      s1v = s2v;
      B0 = B1;
    }
  }
  if (a.dEm) {
    __syncthreads();
    if (dz_zone >= 0 && gs == 0) {
      double s = 0.0;
      for (int g2 = 0; g2 < GB; ++g2) s += DZ[(size_t)col * GB + g2];
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
    for (int k2i = 0; k2i < nw; ++k2i) {
      se += we[k2i];
      sm = fmax(sm, wm[k2i]);
      su += wu[k2i];
      sp += wp[k2i];
    }
    a.p_energy[blockIdx.x] = se;
    a.p_maxf2[blockIdx.x] = sm;
    a.p_nun[blockIdx.x] = su;
    a.p_nnp[blockIdx.x] = sp;
  }
}

// ------------------------------------------------------------------------------------------
// Dynamic LDS a block of the step kernel may use: the device's per-block limit (opt-in) less
// room for the kernel's static LDS, once the kernels have been allowed to use it; 64 KiB
// less that room before (or if raising the limit fails).
static size_t g_max_lds = 64 * 1024 - 1024;

static size_t lds_bytes(const Tile& tl, int dim, size_t rsize) {
  const int NC = 1 + dim;
  const int PROWS = (dim == 3) ? tl.TYB + 2 : 1;
  const size_t ncol = (size_t)tl.TXB * tl.TYB;
  size_t b = ((size_t)(NC + 1) * PROWS * (tl.TXB + 2) + (size_t)NC * ncol * (dim == 3 ? 4 : 2)) * tl.GB * rsize;
  b = (b + 15) & ~(size_t)15;
  b += ncol * tl.GB * sizeof(double);
  return b;
}

Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM, int GB) {
  Tile tl{};
  const size_t rsize = (D.precision == FORNAX_FP64) ? sizeof(double) : sizeof(float);
  tl.TXB = TXB;
  tl.TYB = (D.ndim == 3) ? TYB : 1;
  tl.TM = (D.ndim >= 2) ? TM : 1;
  tl.GB = GB;
  tl.nblocks = 0;
  if (TXB < 3 || (D.ndim == 3 && TYB < 4) || TM < 1 || GB < 1 || D.ngroups % GB != 0) return tl;
  if (D.ndim == 3 && TXB < 4) return tl;
  tl.nthreads = tl.TXB * tl.TYB * GB;
  if (tl.nthreads > 512) return tl;
  // every thread stages at most one halo zone-group per plane
  const int nslots = 2 * tl.TYB * GB + (D.ndim == 3 ? 2 * tl.TXB * GB : 0);
  if (nslots > tl.nthreads) return tl;
  tl.lds = lds_bytes(tl, D.ndim, rsize);
  if (tl.lds > g_max_lds) return tl;
  tl.ngb = D.ngroups / GB;
  tl.ntx = (D.n[0] + (tl.TXB - 2) - 1) / (tl.TXB - 2);
  tl.nty = (D.ndim == 3) ? (D.n[1] + (tl.TYB - 2) - 1) / (tl.TYB - 2) : 1;
  const int nM = (D.ndim >= 2) ? D.n[D.ndim - 1] : 1;
  tl.ntm = (nM + tl.TM - 1) / tl.TM;
  tl.nblocks = tl.ngb * tl.ntx * tl.nty * tl.ntm;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  return tl;
}

// Default tile.  1-D and 2-D: all groups, up to 16 (or 512/G) zone columns.  3-D: a
// near-square tile of 256-512 threads; with many groups per zone, groups are split across
// blocks so that the zone tile stays large enough to amortise its halo, unless all groups
// are needed in one block.
Tile choose_tile(const fornax_m1_desc& D, bool all_groups) {
  const int G = D.ngroups;
  if (D.ndim < 3) {
    int GB = G;
    if (3 * G > 512) {
      if (all_groups) return Tile{};
      GB = 32;
      while (G % GB != 0) --GB;
    }
    int TXB = std::max(3, std::min(16, 512 / GB));
    if (D.ndim == 1) TXB = std::max(3, std::min(512 / GB, D.n[0] + 2));
    return make_tile(D, TXB, 1, 16, GB);
  }
  Tile best{};
  double best_cost = 1e30;
  for (int GB = G; GB >= 1; --GB) {
    if (G % GB != 0) continue;
    if (all_groups && GB != G) break;
    for (int TXB = 4; TXB <= 32; ++TXB)
      for (int TYB = 4; TYB <= 32; ++TYB) {
        Tile t = make_tile(D, TXB, TYB, 8, GB);
        if (t.nblocks == 0 || t.nthreads < 128) continue;
        // loaded columns per updated column, and a mild preference for big blocks and
        // for keeping groups together (contiguous runs)
        const double upd = (double)(TXB - 2) * (TYB - 2);
        const double cost = ((double)(TXB + 2) * (TYB + 2) / upd) * (1.0 + 0.5 / GB) *
                            (t.lds > 80 * 1024 ? 1.5 : 1.0);
        if (cost < best_cost) {
          best_cost = cost;
          best = t;
        }
      }
  }
  return best;
}

template <typename S, typename R, int DIM, bool SPH>
static hipError_t raise_lds_limit(int bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step_tiled<S, R, DIM, SPH>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

int prepare_step_kernels() {
  static bool done = false;
  if (done) return FORNAX_OK;
  int dev = 0, optin = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FORNAX_EDEVICE;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || optin <= 0)
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) optin = 0;
  const int want = optin - 1024;
  done = true;
  if (want <= (int)g_max_lds) return FORNAX_OK;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (r != hipSuccess) e = r;
  };
  chk(raise_lds_limit<double, double, 1, false>(want));
  chk(raise_lds_limit<double, double, 2, false>(want));
  chk(raise_lds_limit<double, double, 3, false>(want));
  chk(raise_lds_limit<double, double, 1, true>(want));
  chk(raise_lds_limit<double, double, 2, true>(want));
  chk(raise_lds_limit<double, double, 3, true>(want));
  chk(raise_lds_limit<float, float, 1, false>(want));
  chk(raise_lds_limit<float, float, 2, false>(want));
  chk(raise_lds_limit<float, float, 3, false>(want));
  chk(raise_lds_limit<float, float, 1, true>(want));
  chk(raise_lds_limit<float, float, 2, true>(want));
  chk(raise_lds_limit<float, float, 3, true>(want));
  if (e == hipSuccess) g_max_lds = (size_t)want;
  (void)hipGetLastError();   // a refused attribute is not an error of later calls
  return FORNAX_OK;
}

template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, const Tile& tl, hipStream_t st) {
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  const int D = ctx->desc.ndim;
  // dE_matter sums over the groups of a zone inside one block
  if (tl.nblocks <= 0 || (a.dEm && tl.GB != a.G)) return FORNAX_EUNSUPPORTED;
  dim3 grid(tl.nblocks), block(tl.nthreads);
#define FM1_LAUNCH(DIMV, SPHV) \
  hipLaunchKernelGGL((k_step_tiled<S, R, DIMV, SPHV>), grid, block, tl.lds, st, a, geo, tl)
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
