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

// Source of a zone index e (possibly a ghost, -2 <= e <= n + 1) along axis d: the zone that
// supplies the values and flags (bit 0 flips the flux component normal to the axis, bit 1
// takes the prescribed inflow state, bit 2 marks the polar-axis copy: shift n[2]/2 in phi,
// flip F_phi), from the ghost table of the launch.
struct AxisSrc {
  int src;
  int flags;
};

__device__ __forceinline__ AxisSrc axis_src(const StepArgsBase& a, int d, int e) {
  const int n = a.n[d];
  AxisSrc r{e, 0};
  if (e < 0) {
    r.src = a.gsrc[d][e + 2];
    r.flags = a.gfl[d][e + 2];
  } else if (e >= n) {
    r.src = a.gsrc[d][e - n + 2];
    r.flags = a.gfl[d][e - n + 2];
  }
  return r;
}

// In-plane part of a zone column's source: element offset of the source column within a
// plane (including the group), the flux components it flips (bit c: F_c; reflect, and the
// polar-axis copy across theta, in-plane y in 3-D), whether it is an inflow ghost (inflow is
// prescribed on x only) and whether it is a polar-axis copy (its phi plane is shifted by
// n[2]/2).
struct ColSrc {
  int cb;
  int lm;
  bool infl;
  bool ax;
};

template <int DIM>
__device__ __forceinline__ ColSrc col_src(const StepArgsBase& a, int gx, int gy, int grp) {
  const AxisSrc sx = axis_src(a, 0, gx);
  ColSrc c;
  c.infl = (sx.flags & 2) != 0;
  c.ax = false;
  if constexpr (DIM == 3) {
    const AxisSrc sy = axis_src(a, 1, gy);
    c.cb = (sy.src * a.n[0] + sx.src) * a.G + grp;
    c.lm = (sx.flags & 1) | ((sy.flags & 1) << 1) | ((sy.flags & 4) ? 4 : 0);
    c.ax = (sy.flags & 4) != 0;
  } else {
    (void)gy;
    c.cb = sx.src * a.G + grp;
    c.lm = sx.flags & 1;
  }
  return c;
}

// Raw values (no sign or inflow rules) of one zone-group of the column cs in plane m (the
// march index, possibly a ghost; unused in 1-D), and the uniform flip mask of that plane.
// q, kap and sig may be null.  The rules are applied later (fix_zone), not right after the
// loads, so that the loads of one plane stay in flight while the previous plane is computed.
template <typename S, typename R, int DIM>
__device__ __forceinline__ int load_raw(const StepArgs<S>& a, ColSrc cs, int m, R q[4], R* kap, R* sig) {
  constexpr int MD = DIM - 1;
  int zg = cs.cb;
  int pm = 0;
  if constexpr (DIM >= 2) {
    // march index: uniform over the block
    const int nM = a.n[MD];
    const AxisSrc sm = axis_src(a, MD, m);
    int iz = sm.src;
    if (DIM == 3 && cs.ax) {
      iz += nM >> 1;
      if (iz >= nM) iz -= nM;
    }
    pm = (sm.flags & 1) ? (1 << MD) | ((sm.flags & 4) ? 4 : 0) : 0;
    const int P = (DIM == 3) ? a.n[0] * a.n[1] * a.G : a.n[0] * a.G;
    zg += iz * P;
  } else {
    (void)m;
  }
  if (kap) *kap = R(a.kap[zg]);
  if (sig) *sig = R(a.sig[zg]);
  if (q) {
    q[0] = R(a.E[zg]);
    for (int c = 0; c < DIM; ++c) q[1 + c] = R(a.F[c][zg]);
  }
  return pm;
}

// Element offset of plane m's source (the march index, possibly a ghost) for a column that is
// (ax) or is not a polar-axis copy, and the uniform flip mask of that plane.
template <int DIM>
__device__ __forceinline__ int plane_offset(const StepArgsBase& a, int m, bool ax, int& pm) {
  constexpr int MD = DIM - 1;
  pm = 0;
  if constexpr (DIM >= 2) {
    const int nM = a.n[MD];
    const AxisSrc sm = axis_src(a, MD, m);
    int iz = sm.src;
    if (DIM == 3 && ax) {
      iz += nM >> 1;
      if (iz >= nM) iz -= nM;
    }
    pm = (sm.flags & 1) ? (1 << MD) | ((sm.flags & 4) ? 4 : 0) : 0;
    const int P = (DIM == 3) ? a.n[0] * a.n[1] * a.G : a.n[0] * a.G;
    return iz * P;
  } else {
    (void)a;
    (void)m;
    (void)ax;
    return 0;
  }
}

// Apply the sign rules (flip F_c where bit c of lm ^ pm is set) and, on an inflow column,
// take the prescribed state instead (held in LDS: qin[c * stride], written once).
template <typename R, int DIM>
__device__ __forceinline__ void fix_zone(const R raw[4], ColSrc cs, int pm, const R* qin, int stride, R q[4]) {
  const int mask = cs.lm ^ pm;
  q[0] = raw[0];
  for (int c = 0; c < DIM; ++c) q[1 + c] = ((mask >> c) & 1) ? -raw[1 + c] : raw[1 + c];
  for (int c = DIM; c < 3; ++c) q[1 + c] = R(0);
  if (cs.infl)
    for (int c = 0; c <= DIM; ++c) q[c] = qin[c * stride];
}

// Prescribed inflow state of a column (x ghost): E and covariant F = h F^ with the ghost's own
// scale factors, for group grp.
template <typename R, bool SPH, int DIM>
__device__ __forceinline__ void inflow_state(const StepArgsBase& a, const Geo<R>& geo, int ex, int ey, int grp, R q[4]) {
  const double* in = a.inflow + grp * (1 + DIM);
  R h[3];
  cell_h<R, SPH>(geo, ex, ey, h);
  q[0] = R(in[0]);
  for (int c = 0; c < DIM; ++c) q[1 + c] = h[c] * R(in[1 + c]);
  for (int c = DIM; c < 3; ++c) q[1 + c] = R(0);
}

// Synchronisation of one tile unit: the whole block in 3-D; in 1-D and 2-D a unit is one
// wavefront, whose LDS operations execute in order, so only the compiler must be kept from
// moving LDS accesses across this point.
template <bool ROW>
__device__ __forceinline__ void unit_sync() {
  if constexpr (ROW) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS elements of one tile unit: plane values, lower face states, in-plane fluxes, and the
// prescribed inflow values of each thread (its column's state and up to 3 halo items)
__host__ __device__ inline size_t unit_lds_elems(int dim, int TXB, int TYB, int GB) {
  const int NC = 1 + dim;
  const int PROWS = (dim == 3) ? TYB + 2 : 1;
  return ((size_t)(NC + 1) * PROWS * (TXB + 2) + (size_t)NC * TXB * TYB * (dim == 3 ? 4 : 2) +
          (size_t)(NC + 3) * TXB * TYB) * GB;
}

template <typename S, typename R, int DIM, bool SPH, bool ROW, int GBC>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(GBC > 0 && !SPH ? 4 : 1)))
k_step_tiled(StepArgs<S> a, Geo<R> geo, Tile tl) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NC = 1 + DIM;   // E, F_1..F_DIM
  constexpr int MD = DIM - 1;   // march direction (DIM >= 2)
  // ROW (1-D / 2-D): a tile unit is one wavefront (one x-row of TXB = 64/GB zone columns);
  // the NW waves of a block march over the same tile with different groups.  Otherwise the
  // unit is the block (TXB x TYB columns of GB groups).
  // GBC > 0: wave rows of GBC groups known at compile time (constant LDS offsets); 0: runtime
  static_assert(!ROW || DIM < 3, "wave rows are for 1-D and 2-D");
  static_assert(GBC == 0 || (ROW && 64 % GBC == 0), "compile-time groups per wave row");
  const int GB = (GBC > 0) ? GBC : tl.GB;
  const int TXB = (GBC > 0) ? 64 / GBC : tl.TXB;
  const int TYB = (GBC > 0) ? 1 : tl.TYB;
  const int t = ROW ? (int)(threadIdx.x & 63) : (int)threadIdx.x;   // index in the unit
  const int wv = ROW ? (int)(threadIdx.x >> 6) : 0;                 // unit of the block
  const int gs = t % GB;
  const int col = t / GB;
  const int cx = col % TXB, cy = col / TXB;
  const int NCOL = TXB * TYB;
  const int PCOLS = TXB + 2;
  const int PROWS = (DIM == 3) ? TYB + 2 : 1;

  // LDS per unit: plane values PV[v][prow][pcol][gs] (v = E, F.., kappa + sigma), lower face
  // states LX/LY[c][col][gs], in-plane fluxes FX/FY[c][col][gs] (face above the column);
  // per block: dE_matter partials DZ
  const size_t unit_elems = unit_lds_elems(DIM, TXB, TYB, GB);
  R* PV = reinterpret_cast<R*>(smem) + (size_t)wv * unit_elems;
  R* LX = PV + (size_t)(NC + 1) * PROWS * PCOLS * GB;
  R* LY = LX + (size_t)NC * NCOL * GB;
  R* FX = LY + ((DIM == 3) ? (size_t)NC * NCOL * GB : 0);
  R* FY = FX + (size_t)NC * NCOL * GB;
  R* QI = FY + ((DIM == 3) ? (size_t)NC * NCOL * GB : 0);   // [NC + 3][NCOL * GB]
  const int qis = NCOL * GB;                                  // threads of the unit
  size_t dz_off = (ROW ? (size_t)tl.NW : (size_t)1) * unit_elems * sizeof(R);
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
  const int gbb = L % tl.ngb;
  const int gb = ROW ? gbb * tl.NW + wv : gbb;   // group subset of this unit
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

  // recon: the column's zone lies within one ghost layer (its face states are used); upd:
  // interior column of the tile inside the domain
  const bool recon = gx <= n0 && (DIM < 3 || gy <= n1);
  const bool upd = cx >= 1 && cx <= TXB - 2 && gx < n0 && (DIM < 3 || (cy >= 1 && cy <= TYB - 2 && gy < n1));
  const bool do_xf = recon && cx <= TXB - 2 && gx + 1 <= n0 && (DIM < 3 || (cy >= 1 && cy <= TYB - 2 && gy < n1));
  const bool do_yf = (DIM == 3) && recon && cy <= TYB - 2 && gy + 1 <= n1 && cx >= 1 && cx <= TXB - 2 && gx < n0;

  const bool want_diag = a.p_energy != nullptr;
  ZoneDiag zd;
  const R c = R(a.c);
  const R dtR = R(a.dt);
  // extended indices of the column for table lookups (clamped: columns beyond the second
  // ghost layer compute values that are never used)
  const int ex = min(gx, n0 + 1) + NG;
  const int eyc = (DIM == 3) ? min(gy, n1 + 1) + NG : NG;   // 3-D: the column's y; else unused

  // fixed in-plane source of this column (columns beyond the second ghost layer load the
  // last ghost's values, which are never used)
  const ColSrc csrc = col_src<DIM>(a, min(gx, n0 + 1), (DIM == 3) ? min(gy, n1 + 1) : 0, grp);

  // ---- halo items: the values of the unit's halo zone-groups (x halo columns -1 and TXB of
  // every row; 3-D also y halo rows -1 and TYB of every column), one value (E or F_c) per
  // item, spread over the unit's threads so that each plane's halo costs at most NITEM loads
  // per thread (the halo's opacities are never needed: only the faces between work columns
  // are computed) ----
  constexpr int NV = NC;
  constexpr int NITEM = ROW ? 1 : 3;
  const int nsx = 2 * TYB * GB;
  const int nitems = (nsx + ((DIM == 3) ? 2 * TXB * GB : 0)) * NV;
  const int nunit = ROW ? 64 : (int)blockDim.x;
  const S* hbase[NITEM];
  int hcb[NITEM], hinfo[NITEM], hlds[NITEM];   // hinfo: v | lm << 3 | inflow << 6 | axis << 7
  for (int k = 0; k < NITEM; ++k) {
    const int it = t + k * nunit;
    hbase[k] = a.E;   // a harmless in-range load for threads without an item
    hcb[k] = csrc.cb;
    hinfo[k] = 0;
    hlds[k] = -1;
    R hvin = R(0);
    if (it < nitems) {
      const int sl = it / NV, v = it % NV;
      const int g = sl % GB, r = sl / GB;
      int hxz, hyz, pcol, prow;
      if (sl < nsx) {
        const int side = r & 1, row = r >> 1;
        pcol = side ? TXB + 1 : 0;
        prow = (DIM == 3) ? row + 1 : 0;
        hxz = side ? x0 + TXB : x0 - 1;
        hyz = (DIM == 3) ? y0 + row : 0;
      } else {
        const int r2i = (sl - nsx) / GB;
        const int side = r2i & 1, cl = r2i >> 1;
        pcol = cl + 1;
        prow = side ? TYB + 1 : 0;
        hxz = x0 + cl;
        hyz = side ? y0 + TYB : y0 - 1;
      }
      const bool on = hxz <= n0 + 1 && (DIM < 3 || hyz <= n1 + 1);
      const int hg = gb * GB + g;
      const ColSrc cs = col_src<DIM>(a, min(hxz, n0 + 1), (DIM == 3) ? min(hyz, n1 + 1) : 0, hg);
      hbase[k] = (v == 0) ? a.E : a.F[v - 1];
      hcb[k] = cs.cb;
      hinfo[k] = v | (cs.lm << 3) | (cs.infl ? 64 : 0) | (cs.ax ? 128 : 0);
      if (on) hlds[k] = (int)((((size_t)v * PROWS + prow) * PCOLS + pcol) * GB + g);
      if (on && cs.infl) {
        R qi[4];
        inflow_state<R, SPH, DIM>(a, geo, min(hxz, n0 + 1) + NG, (DIM == 3) ? min(hyz, n1 + 1) + NG : NG, hg,
                                  qi);
        hvin = qi[v];
      }
    }
    QI[(NC + k) * qis + t] = hvin;
  }
  // Values in flight.  Every load of plane data targets one of the "pending" registers below
  // and is consumed, by arithmetic, at the start of the next plane, so that one plane of work
  // hides its latency (a register copy of a load still in flight would wait for it).
  R Pr[4], Pk = R(0), Ps = R(0), PB = R(0);   // own: raw q, kappa, sigma, B
  R Ph[NITEM];                                 // halo items
  int Ppm = 0;                                 // plane mask of the pending raw values
  {
    R qin[4] = {R(0), R(0), R(0), R(0)};
    if (csrc.infl) inflow_state<R, SPH, DIM>(a, geo, ex, eyc, grp, qin);
    for (int c = 0; c < NC; ++c) QI[c * qis + t] = qin[c];
  }
  const R* qinp = QI + t;
  for (int k = 0; k < 4; ++k) Pr[k] = R(0);
  for (int k = 0; k < NITEM; ++k) Ph[k] = R(0);
  auto load_halo = [&](int m) {
    for (int k = 0; k < NITEM; ++k) {
      int pmk;
      const int off = plane_offset<DIM>(a, m, (hinfo[k] & 128) != 0, pmk);
      Ph[k] = R(hbase[k][hcb[k] + off]);
    }
  };
  // halo values of plane m (loaded one plane ago) to LDS, with the sign and inflow rules
  auto stage_halo = [&](int m) {
    int pm;
    (void)plane_offset<DIM>(a, m, false, pm);
    for (int k = 0; k < NITEM; ++k) {
      if (hlds[k] >= 0) {
        const int v = hinfo[k] & 7;
        const int mask = (hinfo[k] >> 3 & 7) ^ pm;
        R val = Ph[k];
        if (v >= 1 && v <= DIM && ((mask >> (v - 1)) & 1)) val = -val;
        if (hinfo[k] & 64) val = QI[(NC + k) * qis + t];
        PV[hlds[k]] = val;
      }
    }
  };
  // raw values of this column's zone in plane m; returns the plane mask
  auto load_own = [&](int m, R* q, R* k, R* sg) -> int { return load_raw<S, R, DIM>(a, csrc, m, q, k, sg); };
  // extended y index of the zone row in plane m (spherical tables; theta is y)
  auto ey_of = [&](int m) -> int { return (DIM == 2) ? m + NG : eyc; };
  const int zgB = grp;   // B offset added to the zone index below
  auto loadB = [&](int m) -> R {
    // B of this column's zone in plane m (only updated columns use it; the index is clamped
    // into the domain so that every lane may load)
    const int zi = min(max(gx, 0), n0 - 1);
    const int zj = (DIM == 2) ? m : min(max(gy, 0), n1 - 1), zk = (DIM == 3) ? m : 0;
    return R(a.B[((zk * n1 + zj) * n0 + zi) * a.G + zgB]);
  };
  // zone volume factors for the energy diagnostic: the column's (fixed) and the plane's
  // (Cartesian zones all have the same volume; spherical: the plane's factor is fetched one
  // plane ahead with the other plane data)
  double Vcol = 0.0;   // Cartesian and 1-D: the whole volume; else 2-D: x, z factors; 3-D: x, y
  if (want_diag) {
    if constexpr (!SPH) Vcol = geo.Wd[0][NG] * geo.Wd[1][NG] * geo.Wd[2][NG];   // uniform zones
    if constexpr (DIM == 1 && SPH) Vcol = geo.Wd[0][ex] * geo.Wd[1][NG] * geo.Wd[2][NG];
    if constexpr (DIM == 2 && SPH) Vcol = geo.Wd[0][ex] * geo.Wd[2][NG];
    if constexpr (DIM == 3 && SPH) Vcol = geo.Wd[0][ex] * geo.Wd[1][eyc];
  }
  auto plane_vol = [&](int m) -> double {
    if constexpr (SPH && DIM >= 2) return want_diag ? geo.Wd[MD][min(m, nM - 1) + NG] : 0.0;
    return 1.0;
  };
  double Pvol = 0.0;

  // ---- register window along the march direction: q(m), q(m+1) with the ghost rules
  // applied; of planes m and m+1 the total opacity ks = kappa + sigma and, in double,
  // c dt kappa and c dt (kappa + sigma) ----
  const double cdt = a.c * a.dt;
  R q0[4], q1[4];
  R hiM[4], fPrev[4];
  for (int k = 0; k < 4; ++k) q0[k] = q1[k] = hiM[k] = fPrev[k] = R(0);
  R ks0 = R(0), ks1 = R(0);
  double ck0 = 0.0, cks0 = 0.0, ck1 = 0.0, cks1 = 0.0;
  {
    R raw[4], k0, s0;
    if constexpr (DIM >= 2) {
      R qa[4], qb[4], ka, sa;
      int pm = load_own(mbeg - 2, raw, nullptr, nullptr);
      fix_zone<R, DIM>(raw, csrc, pm, qinp, qis, qa);
      pm = load_own(mbeg - 1, raw, &ka, &sa);
      fix_zone<R, DIM>(raw, csrc, pm, qinp, qis, qb);
      pm = load_own(mbeg, raw, &k0, &s0);
      fix_zone<R, DIM>(raw, csrc, pm, qinp, qis, q0);
      pm = load_own(mbeg + 1, raw, nullptr, nullptr);
      fix_zone<R, DIM>(raw, csrc, pm, qinp, qis, q1);
      ks0 = k0 + s0;
      // in flight into the first plane: raw q(mbeg + 2), kappa/sigma(mbeg + 1), B(mbeg)
      Ppm = load_own(mbeg + 2, Pr, nullptr, nullptr);
      load_own(mbeg + 1, nullptr, &Pk, &Ps);
      PB = loadB(mbeg);
      Pvol = plane_vol(mbeg);
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
        hll<R, SPH, DIM>(a, MD, hiP, lo, h1, epsilon_of(ka + sa, ks0, dlL, dlR), fPrev);
      }
    } else {
      const int pm = load_own(0, raw, &k0, &s0);
      fix_zone<R, DIM>(raw, csrc, pm, qinp, qis, q0);
      ks0 = k0 + s0;
      PB = loadB(0);
      Pvol = plane_vol(0);
    }
    ck0 = cdt * (double)k0;
    cks0 = cdt * ((double)k0 + (double)s0);
  }
  load_halo(mbeg);

  const int prow_own = (DIM == 3) ? cy + 1 : 0;
  const R idx0 = geo.idx[0], idx1 = geo.idx[1], idxM = geo.idx[(DIM >= 2) ? MD : 0];
  int dz_zone = -1;
  for (int m = mbeg; m < mend; ++m) {
    // ---- consume the values loaded one plane ago ----
    R q2[4];
    fix_zone<R, DIM>(Pr, csrc, Ppm, qinp, qis, q2);   // plane m + 2
    ks1 = Pk + Ps;                              // plane m + 1
    ck1 = cdt * (double)Pk;
    cks1 = cdt * ((double)Pk + (double)Ps);
    const double jB = ck0 * (double)PB;         // c dt kappa B of plane m
    const double Vm = Vcol * Pvol;              // zone volume (diagnostics)
    stage_halo(m);
    // ---- (a) stage plane m: own zone ----
    for (int v = 0; v < NC; ++v) pv(v, prow_own, cx + 1, gs) = q0[v];
    pv(NC, prow_own, cx + 1, gs) = ks0;
    // ---- prefetch for the next plane: raw q(m+3), kappa/sigma(m+2), B(m+1), halo m+1.
    // Issued on every plane (indices clamped into the ghost range; the last plane's are
    // not used) so that the loads never sit in a branch ----
    if constexpr (DIM >= 2) {
      Ppm = load_own(min(m + 3, nM + 1), Pr, nullptr, nullptr);
      load_own(min(m + 2, nM + 1), nullptr, &Pk, &Ps);
      PB = loadB(min(m + 1, nM - 1));
      Pvol = plane_vol(m + 1);
      load_halo(m + 1);
    }
    unit_sync<ROW>();
    // ---- (b) deferred dE_matter of the previous plane (3-D: all groups in the block) ----
    if (!ROW && a.dEm && dz_zone >= 0 && gs == 0) {
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
          hll<R, SPH, DIM>(a, MD, hiM, nLo, h1, epsilon_of(ks0, ks1, dlL, dlR), fNext);
        }
      }
    }
    unit_sync<ROW>();
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
        hll<R, SPH, DIM>(a, 0, hiX, qR, hf, epsilon_of(ks0, ksR, dlL, dlR), fxR);
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
          hll<R, SPH, DIM>(a, 1, hiY, qR, hf, epsilon_of(ks0, ksR, dlL, dlR), fyR);
        }
        for (int v = 0; v < NC; ++v) FY[cidx(v, col)] = fyR[v];
      }
    }
    unit_sync<ROW>();
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
      const double V = Vm;
      const double dz = finish_zone_c<S, R, SPH, DIM>(a, geo, zone * a.G + grp, zi, zj, zk, Um, ck0, cks0, jB,
                                                      want_diag, V, zd);
      if (!ROW && a.dEm) {
        DZ[(size_t)col * GB + gs] = dz;
        dz_zone = zone;
      }
      if (ROW && a.dEm) {
        // sum over the GB groups of this column (consecutive lanes), one partial per wave
        double p = dz;
        for (int off = 1; off < GB; off <<= 1) p += __shfl_xor(p, off);
        if (gs == 0) DZ[((size_t)(m - mbeg) * tl.NW + wv) * TXB + cx] = p;
      }
    }
    // ---- advance the window ----
    if constexpr (DIM >= 2) {
      for (int cc = 0; cc < 4; ++cc) {
        q0[cc] = q1[cc];
        q1[cc] = q2[cc];
        hiM[cc] = nHi[cc];
        fPrev[cc] = fNext[cc];
      }
      ks0 = ks1;
      ck0 = ck1;
      cks0 = cks1;
    }
  }
  if (a.dEm) {
    __syncthreads();
    if constexpr (ROW) {
      // dE_matter of every updated zone of the tile: sum of the wave partials, in order
      const int nzt = (mend - mbeg) * TXB;
      for (int i = threadIdx.x; i < nzt; i += blockDim.x) {
        const int mm = mbeg + i / TXB, ccx = i % TXB;
        const int zx = x0 + ccx;
        if (ccx >= 1 && ccx <= TXB - 2 && zx < n0) {
          double sdz = 0.0;
          for (int w2 = 0; w2 < tl.NW; ++w2) sdz += DZ[((size_t)(mm - mbeg) * tl.NW + w2) * TXB + ccx];
          a.dEm[(size_t)((DIM == 2) ? mm : 0) * n0 + zx] = -sdz;
        }
      }
    } else {
      if (dz_zone >= 0 && gs == 0) {
        double s = 0.0;
        for (int g2 = 0; g2 < GB; ++g2) s += DZ[(size_t)col * GB + g2];
        a.dEm[dz_zone] = -s;
      }
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
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
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
  size_t b = unit_lds_elems(dim, tl.TXB, tl.TYB, tl.GB) * rsize * (tl.row ? tl.NW : 1);
  b = (b + 15) & ~(size_t)15;
  // dE_matter partials: wave rows per plane, wave and column; block units per column and group
  if (tl.row) b += (size_t)tl.TM * tl.NW * tl.TXB * sizeof(double);
  else b += (size_t)tl.TXB * tl.TYB * tl.GB * sizeof(double);
  return b;
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM, int GB, int NW) {
  Tile tl{};
  const size_t rsize = (D.precision == FORNAX_FP64) ? sizeof(double) : sizeof(float);
  // 1-D/2-D with NW >= 1: wave rows; NW = 0 (and always in 3-D): one unit per block
  const bool row = D.ndim < 3 && NW >= 1;
  tl.nblocks = 0;
  if (GB < 1 || TM < 1 || D.ngroups % GB != 0) return tl;
  if (row) {
    // one x-row of 64/GB zone columns per wave, NW waves (group subsets) per block
    if (!pow2(GB) || GB > 16 || NW > 8 || (D.ngroups / GB) % NW != 0) return tl;
    TXB = 64 / GB;
    TYB = 1;
  } else {
    NW = 1;
    if (D.ndim < 3) TYB = 1;
    if (TXB < 4 || (D.ndim == 3 && TYB < 4)) return tl;
  }
  tl.row = row;
  tl.TXB = TXB;
  tl.TYB = TYB;
  tl.TM = (D.ndim >= 2) ? TM : 1;
  tl.GB = GB;
  tl.NW = NW;
  tl.nthreads = row ? 64 * NW : TXB * TYB * GB;
  if (tl.nthreads > 512) return tl;
  // halo items (one value of one halo zone-group each): at most 1 per thread of a wave unit,
  // 3 per thread of a block unit
  const int nunit = row ? 64 : tl.nthreads;
  const int nitems = (2 * TYB * GB + (D.ndim == 3 ? 2 * TXB * GB : 0)) * (D.ndim + 1);
  if (nitems > (row ? 1 : 3) * nunit) return tl;
  tl.lds = lds_bytes(tl, D.ndim, rsize);
  if (tl.lds > g_max_lds) return tl;
  tl.ngb = D.ngroups / (GB * NW);
  tl.ntx = (D.n[0] + (TXB - 2) - 1) / (TXB - 2);
  tl.nty = (D.ndim == 3) ? (D.n[1] + (TYB - 2) - 1) / (TYB - 2) : 1;
  const int nM = (D.ndim >= 2) ? D.n[D.ndim - 1] : 1;
  tl.ntm = (nM + tl.TM - 1) / tl.TM;
  tl.nblocks = tl.ngb * tl.ntx * tl.nty * tl.ntm;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  return tl;
}

// Default tile.
//  * 1-D / 2-D: GB = the largest power of two up to 4 dividing G (16 zone columns per wave,
//    runs of 4 groups), all G / GB group subsets of a tile in one block when they fit in 8
//    waves; planes per block halved from 32 until the grid has at least 1024 (FP64) or 2048
//    (MIXED) blocks, TM >= 4.
//    With all_groups, GB grows until the block holds every group.
//  * 3-D: a near-square tile of 128-512 threads; with many groups per zone, groups are split
//    across blocks so that the zone tile stays large enough to amortise its halo, unless all
//    groups are needed in one block.
Tile choose_tile(const fornax_m1_desc& D, bool all_groups) {
  const int G = D.ngroups;
  if (D.ndim < 3) {
    int GB = 1;
    while (GB < 4 && G % (2 * GB) == 0) GB *= 2;
    if (all_groups)
      while (G / GB > 8 && GB < 16 && G % (2 * GB) == 0) GB *= 2;
    int NW = std::min(8, G / GB);
    while ((G / GB) % NW != 0) --NW;
    if (all_groups && NW * GB != G) return Tile{};
    // FP64 waves hold more registers (fewer of them per SIMD): longer marches amortise the
    // first face of each march better there
    const int want = (D.precision == FORNAX_FP64) ? 1024 : 2048;
    Tile t{};
    for (int TM = 32; TM >= 4; TM /= 2) {
      t = make_tile(D, 0, 1, TM, GB, NW);
      if (t.nblocks >= want || D.ndim == 1) break;
    }
    return t;
  }
  Tile best{};
  double best_cost = 1e30;
  for (int GB = G; GB >= 1; --GB) {
    if (G % GB != 0) continue;
    if (all_groups && GB != G) break;
    for (int TXB = 4; TXB <= 32; ++TXB)
      for (int TYB = 4; TYB <= 32; ++TYB) {
        Tile t = make_tile(D, TXB, TYB, 8, GB, 1);
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

template <typename S, typename R, int DIM, bool SPH, bool ROW, int GBC = 0>
static hipError_t raise_lds_limit(int bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step_tiled<S, R, DIM, SPH, ROW, GBC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename S, typename R>
static hipError_t raise_all(int bytes) {
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (r != hipSuccess) e = r;
  };
  chk(raise_lds_limit<S, R, 1, false, true>(bytes));
  chk(raise_lds_limit<S, R, 2, false, true>(bytes));
  chk(raise_lds_limit<S, R, 1, true, true>(bytes));
  chk(raise_lds_limit<S, R, 2, true, true>(bytes));
  chk(raise_lds_limit<S, R, 2, false, true, 4>(bytes));
  chk(raise_lds_limit<S, R, 2, true, true, 4>(bytes));
  chk(raise_lds_limit<S, R, 1, false, false>(bytes));
  chk(raise_lds_limit<S, R, 2, false, false>(bytes));
  chk(raise_lds_limit<S, R, 3, false, false>(bytes));
  chk(raise_lds_limit<S, R, 1, true, false>(bytes));
  chk(raise_lds_limit<S, R, 2, true, false>(bytes));
  chk(raise_lds_limit<S, R, 3, true, false>(bytes));
  return e;
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
  hipError_t e = raise_all<double, double>(want);
  const hipError_t e2 = raise_all<float, float>(want);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) g_max_lds = (size_t)want;
  (void)hipGetLastError();   // a refused attribute is not an error of later calls
  return FORNAX_OK;
}

template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, const Tile& tl, hipStream_t st) {
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  const int D = ctx->desc.ndim;
  // dE_matter sums over the groups of a zone inside one block
  if (tl.nblocks <= 0 || (a.dEm && tl.GB * tl.NW != a.G)) return FORNAX_EUNSUPPORTED;
  dim3 grid(tl.nblocks), block(tl.nthreads);
#define FM1_LAUNCH(DIMV, SPHV, ROWV, GBV) \
  hipLaunchKernelGGL((k_step_tiled<S, R, DIMV, SPHV, ROWV, GBV>), grid, block, tl.lds, st, a, geo, tl)
  if (sph) {
    if (D == 1) {
      if (tl.row) FM1_LAUNCH(1, true, true, 0);
      else FM1_LAUNCH(1, true, false, 0);
    } else if (D == 2) {
      if (tl.row && tl.GB == 4) FM1_LAUNCH(2, true, true, 4);
      else if (tl.row) FM1_LAUNCH(2, true, true, 0);
      else FM1_LAUNCH(2, true, false, 0);
    } else {
      FM1_LAUNCH(3, true, false, 0);
    }
  } else {
    if (D == 1) {
      if (tl.row) FM1_LAUNCH(1, false, true, 0);
      else FM1_LAUNCH(1, false, false, 0);
    } else if (D == 2) {
      if (tl.row && tl.GB == 4) FM1_LAUNCH(2, false, true, 4);
      else if (tl.row) FM1_LAUNCH(2, false, true, 0);
      else FM1_LAUNCH(2, false, false, 0);
    } else {
      FM1_LAUNCH(3, false, false, 0);
    }
  }
#undef FM1_LAUNCH
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template int launch_tiled<double, double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&, const Tile&,
                                          hipStream_t);
template int launch_tiled<float, float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, const Tile&,
                                        hipStream_t);

}  // namespace fm1
