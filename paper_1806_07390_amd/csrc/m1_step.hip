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

#include <type_traits>

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

// V consecutive values of array p from element zg (zg a multiple of V): one vector load.
template <typename S, typename R, int V>
__device__ __forceinline__ void ldv(const S* p, int zg, R out[V]) {
  if constexpr (V == 1) {
    out[0] = R(p[zg]);
  } else {
    static_assert(V == 2, "one or two values per lane");
    using T2 = typename std::conditional<sizeof(S) == 8, double2, float2>::type;
    const T2 v = *reinterpret_cast<const T2*>(p + zg);
    out[0] = R(v.x);
    out[1] = R(v.y);
  }
}

template <typename S, int V>
__device__ __forceinline__ void stv(S* p, int zg, const S in[V]) {
  if constexpr (V == 1) {
    p[zg] = in[0];
  } else {
    using T2 = typename std::conditional<sizeof(S) == 8, double2, float2>::type;
    T2 v;
    v.x = in[0];
    v.y = in[1];
    *reinterpret_cast<T2*>(p + zg) = v;
  }
}

// Raw values (no sign or inflow rules) of the V zone-groups of the column cs in plane m (the
// march index, possibly a ghost; unused in 1-D), and the uniform flip mask of that plane.
// q, kap and sig may be null.  The rules are applied later (fix_zone), not right after the
// loads, so that the loads of one plane stay in flight while the previous plane is computed.
template <typename S, typename R, int DIM, int V>
__device__ __forceinline__ int load_raw(const StepArgs<S>& a, ColSrc cs, int m, R (*q)[4], R* kap, R* sig) {
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
  if (kap) ldv<S, R, V>(a.kap, zg, kap);
  if (sig) ldv<S, R, V>(a.sig, zg, sig);
  if (q) {
    R t[V];
    ldv<S, R, V>(a.E, zg, t);
    for (int u = 0; u < V; ++u) q[u][0] = t[u];
    for (int c = 0; c < DIM; ++c) {
      ldv<S, R, V>(a.F[c], zg, t);
      for (int u = 0; u < V; ++u) q[u][1 + c] = t[u];
    }
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

// Waves per SIMD for the compile-time wave-row kernels (measured on gfx950): 3 in double
// (at most 168 VGPRs, no spills), 5 in float (at most 96 VGPRs).  LIM: the limiter when
// known at compile time, -1 to read it from the arguments (that instantiation also takes the
// wavespeed option from the arguments; the others use S = -+c).
// The spherical 3-D step in double needs more than the 256 registers of a wave that shares its
// SIMD: its blocks are limited to 256 threads (one wave per SIMD) and the empty asm statement
// at its start, which names an accumulation register, keeps that bank available to the
// register allocator, which then holds there what it would otherwise spill to scratch memory.
template <typename S, typename R, int DIM, bool SPH, bool ROW, int GBC, int V, int LIM>
__global__ void __launch_bounds__((DIM == 3 && SPH && sizeof(R) == 8) ? 256 : 512) __attribute__((amdgpu_waves_per_eu(GBC > 0 && !SPH && V == 1 ? (sizeof(R) == 8 ? 3 : 5) : 1)))
k_step_tiled(StepArgs<S> a, Geo<R> geo, Tile tl) {
  if constexpr (DIM == 3 && SPH && sizeof(R) == 8) asm volatile("" ::: "a0");
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NC = 1 + DIM;   // E, F_1..F_DIM
  constexpr int MD = DIM - 1;   // march direction (DIM >= 2)
  // ROW (1-D / 2-D): a tile unit is one wavefront (one x-row of TXB zone columns); the NW
  // waves of a block march over the same tile with different groups.  Otherwise the unit is
  // the block (TXB x TYB columns of GB groups).  Each lane handles V consecutive groups of
  // one column (V = 2: 16-byte loads).  GBC > 0: groups per wave row known at compile time.
  static_assert(!ROW || DIM < 3, "wave rows are for 1-D and 2-D");
  static_assert(GBC == 0 || (ROW && (64 * V) % GBC == 0), "compile-time groups per wave row");
  const int GB = (GBC > 0) ? GBC : tl.GB;
  const int LPC = GB / V;                                            // lanes per zone column
  const int TXB = (GBC > 0) ? 64 * V / GBC : tl.TXB;
  const int TYB = (GBC > 0) ? 1 : tl.TYB;
  const int t = ROW ? (int)(threadIdx.x & 63) : (int)threadIdx.x;   // index in the unit
  const int wv = ROW ? (int)(threadIdx.x >> 6) : 0;                 // unit of the block
  const int gl = t % LPC;                                            // group pair (V = 2) of the lane
  const int col = t / LPC;
  const int cx = col % TXB, cy = col / TXB;
  const int NCOL = TXB * TYB;
  const int PCOLS = TXB + 2;
  const int PROWS = (DIM == 3) ? TYB + 2 : 1;
  const int nunit = NCOL * LPC;                                      // threads of the unit

  // LDS per unit: plane values PV[v][prow][pcol][g] (v = E, F.., kappa + sigma), lower face
  // states LX/LY[c][col][g], in-plane fluxes FX/FY[c][col][g] (face above the column), the
  // prescribed inflow values QI; per block: dE_matter partials DZ
  const size_t unit_elems = unit_lds_elems(DIM, TXB, TYB, GB);
  R* PV = reinterpret_cast<R*>(smem) + (size_t)wv * unit_elems;
  R* LX = PV + (size_t)(NC + 1) * PROWS * PCOLS * GB;
  R* LY = LX + (size_t)NC * NCOL * GB;
  R* FX = LY + ((DIM == 3) ? (size_t)NC * NCOL * GB : 0);
  R* FY = FX + (size_t)NC * NCOL * GB;
  R* QI = FY + ((DIM == 3) ? (size_t)NC * NCOL * GB : 0);   // [NC + 3][nunit][V]
  size_t dz_off = (ROW ? (size_t)tl.NW : (size_t)1) * unit_elems * sizeof(R);
  dz_off = (dz_off + 15) & ~(size_t)15;
  double* DZ = reinterpret_cast<double*>(smem + dz_off);
  // element index of (v, prow, pcol) for this lane's first group
  auto pvi = [&](int v, int prow, int pcol) -> int { return ((v * PROWS + prow) * PCOLS + pcol) * GB + gl * V; };
  auto cidx = [&](int c, int cl) -> int { return (c * NCOL + cl) * GB + gl * V; };
  auto qii = [&](int c) -> int { return (c * nunit + t) * V; };

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
  const int grp0 = gb * GB + gl * V;              // first group of the lane
  // dE_matter of a zone from the groups of this block: the value itself when the block holds
  // every group of the zone, else the block's partial (the group blocks are summed after
  // the launch)
  auto put_dem = [&](int64_t zone, double s) {
    if (tl.ngb == 1) a.dEm[zone] = -s;
    else a.dzp[(int64_t)gbb * a.nzones + zone] = s;
  };

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
  const ColSrc csrc = col_src<DIM>(a, min(gx, n0 + 1), (DIM == 3) ? min(gy, n1 + 1) : 0, grp0);

  // ---- halo items: the values of the unit's halo zone-groups (x halo columns -1 and TXB of
  // every row; 3-D also y halo rows -1 and TYB of every column), one value (E or F_c) of V
  // groups per item, spread over the unit's threads so that each plane's halo costs at most
  // NITEM loads per thread (the halo's opacities are never needed: only the faces between
  // work columns are computed) ----
  constexpr int NITEM = ROW ? 1 : 3;
  const int nsx = 2 * TYB * LPC;
  const int nitems = (nsx + ((DIM == 3) ? 2 * TXB * LPC : 0)) * NC;
  const S* hbase[NITEM];
  int hcb[NITEM], hinfo[NITEM], hlds[NITEM];   // hinfo: v | lm << 3 | inflow << 6 | axis << 7
  for (int k = 0; k < NITEM; ++k) {
    const int it = t + k * nunit;
    hbase[k] = a.E;   // a harmless in-range load for threads without an item
    hcb[k] = csrc.cb;
    hinfo[k] = 0;
    hlds[k] = -1;
    R hvin[V];
    for (int u = 0; u < V; ++u) hvin[u] = R(0);
    if (it < nitems) {
      const int sl = it / NC, v = it % NC;
      const int g = sl % LPC, r = sl / LPC;
      int hxz, hyz, pcol, prow;
      if (sl < nsx) {
        const int side = r & 1, row = r >> 1;
        pcol = side ? TXB + 1 : 0;
        prow = (DIM == 3) ? row + 1 : 0;
        hxz = side ? x0 + TXB : x0 - 1;
        hyz = (DIM == 3) ? y0 + row : 0;
      } else {
        const int r2i = (sl - nsx) / LPC;
        const int side = r2i & 1, cl = r2i >> 1;
        pcol = cl + 1;
        prow = side ? TYB + 1 : 0;
        hxz = x0 + cl;
        hyz = side ? y0 + TYB : y0 - 1;
      }
      const bool on = hxz <= n0 + 1 && (DIM < 3 || hyz <= n1 + 1);
      const int hg = gb * GB + g * V;
      const ColSrc cs = col_src<DIM>(a, min(hxz, n0 + 1), (DIM == 3) ? min(hyz, n1 + 1) : 0, hg);
      hbase[k] = (v == 0) ? a.E : a.F[v - 1];
      hcb[k] = cs.cb;
      hinfo[k] = v | (cs.lm << 3) | (cs.infl ? 64 : 0) | (cs.ax ? 128 : 0);
      if (on) hlds[k] = ((v * PROWS + prow) * PCOLS + pcol) * GB + g * V;
      if (on && cs.infl) {
        for (int u = 0; u < V; ++u) {
          R qi[4];
          inflow_state<R, SPH, DIM>(a, geo, min(hxz, n0 + 1) + NG, (DIM == 3) ? min(hyz, n1 + 1) + NG : NG,
                                    hg + u, qi);
          hvin[u] = qi[v];
        }
      }
    }
    for (int u = 0; u < V; ++u) QI[qii(NC + k) + u] = hvin[u];
  }
  // Values in flight.  Every load of plane data targets one of the "pending" registers below
  // and is consumed, by arithmetic, at the start of the next plane, so that one plane of work
  // hides its latency (a register copy of a load still in flight would wait for it).
  R Pr[V][4], Pk[V], Ps[V], PB[V];   // own: raw q, kappa, sigma, B
  R Ph[NITEM][V];                    // halo items
  int Ppm = 0;                       // plane mask of the pending raw values
  for (int u = 0; u < V; ++u) {
    R qin[4] = {R(0), R(0), R(0), R(0)};
    if (csrc.infl) inflow_state<R, SPH, DIM>(a, geo, ex, eyc, grp0 + u, qin);
    for (int cc = 0; cc < NC; ++cc) QI[qii(cc) + u] = qin[cc];
    for (int k = 0; k < 4; ++k) Pr[u][k] = R(0);
    Pk[u] = Ps[u] = PB[u] = R(0);
    for (int k = 0; k < NITEM; ++k) Ph[k][u] = R(0);
  }
  // the sign and inflow rules for the V groups of this column
  auto fix_all = [&](R (*raw)[4], int pm, R (*q)[4]) {
    for (int u = 0; u < V; ++u) fix_zone<R, DIM>(raw[u], csrc, pm, QI + qii(0) + u, nunit * V, q[u]);
  };
  auto load_halo = [&](int m) {
    for (int k = 0; k < NITEM; ++k) {
      int pmk;
      const int off = plane_offset<DIM>(a, m, (hinfo[k] & 128) != 0, pmk);
      ldv<S, R, V>(hbase[k], hcb[k] + off, Ph[k]);
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
        for (int u = 0; u < V; ++u) {
          R val = Ph[k][u];
          if (v >= 1 && v <= DIM && ((mask >> (v - 1)) & 1)) val = -val;
          if (hinfo[k] & 64) val = QI[qii(NC + k) + u];
          PV[hlds[k] + u] = val;
        }
      }
    }
  };
  // raw values of this column's zones in plane m; returns the plane mask
  auto load_own = [&](int m, R (*q)[4], R* k, R* sg) -> int { return load_raw<S, R, DIM, V>(a, csrc, m, q, k, sg); };
  // extended y index of the zone row in plane m (spherical tables; theta is y)
  auto ey_of = [&](int m) -> int { return (DIM == 2) ? m + NG : eyc; };
  // B of this column's zones in plane m (only updated columns use it; the index is clamped
  // into the domain so that every lane may load)
  const int zib = min(max(gx, 0), n0 - 1);
  const int zjb = (DIM == 3) ? min(max(gy, 0), n1 - 1) : 0;
  auto loadB = [&](int m, R out[V]) {
    const int zj = (DIM == 2) ? m : zjb, zk = (DIM == 3) ? m : 0;
    ldv<S, R, V>(a.B, ((zk * n1 + zj) * n0 + zib) * a.G + grp0, out);
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
  R q0[V][4], q1[V][4];
  R hiM[V][4], fPrev[V][4];
  R ks0[V], ks1[V];
  double ck0[V], cks0[V], ck1[V], cks1[V];
  for (int u = 0; u < V; ++u) {
    for (int k = 0; k < 4; ++k) q0[u][k] = q1[u][k] = hiM[u][k] = fPrev[u][k] = R(0);
    ks0[u] = ks1[u] = R(0);
    ck0[u] = cks0[u] = ck1[u] = cks1[u] = 0.0;
  }
  {
    R raw[V][4], k0[V], s0[V];
    if constexpr (DIM >= 2) {
      R qa[V][4], qb[V][4], ka[V], sa[V];
      int pm = load_own(mbeg - 2, raw, nullptr, nullptr);
      fix_all(raw, pm, qa);
      pm = load_own(mbeg - 1, raw, ka, sa);
      fix_all(raw, pm, qb);
      pm = load_own(mbeg, raw, k0, s0);
      fix_all(raw, pm, q0);
      pm = load_own(mbeg + 1, raw, nullptr, nullptr);
      fix_all(raw, pm, q1);
      for (int u = 0; u < V; ++u) ks0[u] = k0[u] + s0[u];
      // in flight into the first plane: raw q(mbeg + 2), kappa/sigma(mbeg + 1), B(mbeg)
      Ppm = load_own(mbeg + 2, Pr, nullptr, nullptr);
      load_own(mbeg + 1, nullptr, Pk, Ps);
      loadB(mbeg, PB);
      Pvol = plane_vol(mbeg);
      // face mbeg - 1/2 from zones mbeg - 1 (upper state) and mbeg (lower state)
      const int ef = mbeg + NG;   // lower face of zone mbeg
      const int eyf = (DIM == 3) ? eyc : ef;
      R ih0[3], h1[3], ih1[3], ih2[3];
      face_ih<R, SPH>(geo, MD, ex, eyf, ef - 1, ih0);
      face_h<R, SPH>(geo, MD, ex, eyf, ef, h1);
      face_ih<R, SPH>(geo, MD, ex, eyf, ef, ih1);
      face_ih<R, SPH>(geo, MD, ex, eyf, ef + 1, ih2);
      const bool o0 = !SPH || geo.wf[MD][ef - 1] != R(0);
      const bool o1 = !SPH || geo.wf[MD][ef] != R(0);
      const bool o2 = !SPH || geo.wf[MD][ef + 1] != R(0);
      const R dlL = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef - 1);
      const R dlR = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef);
      for (int u = 0; u < V; ++u) {
        R lo[4], hiP[4];
        reconstruct<R, SPH, DIM, LIM>(a, geo, MD, ef - 1, qa[u], qb[u], q0[u], ih0, ih1, o0, o1, lo, hiP);
        reconstruct<R, SPH, DIM, LIM>(a, geo, MD, ef, qb[u], q0[u], q1[u], ih1, ih2, o1, o2, lo, hiM[u]);
        if (o1) hll<R, SPH, DIM, (LIM < 0)>(a, MD, hiP, lo, h1, ih1, epsilon_of(ka[u] + sa[u], ks0[u], dlL, dlR), fPrev[u]);
      }
    } else {
      const int pm = load_own(0, raw, k0, s0);
      fix_all(raw, pm, q0);
      for (int u = 0; u < V; ++u) ks0[u] = k0[u] + s0[u];
      loadB(0, PB);
      Pvol = plane_vol(0);
    }
    for (int u = 0; u < V; ++u) {
      ck0[u] = cdt * (double)k0[u];
      cks0[u] = cdt * ((double)k0[u] + (double)s0[u]);
    }
  }
  load_halo(mbeg);

  const int prow_own = (DIM == 3) ? cy + 1 : 0;
  const R idx0 = geo.idx[0], idx1 = geo.idx[1], idxM = geo.idx[(DIM >= 2) ? MD : 0];
  int dz_zone = -1;
  for (int m = mbeg; m < mend; ++m) {
    // ---- consume the values loaded one plane ago ----
    R q2[V][4];
    fix_all(Pr, Ppm, q2);   // plane m + 2
    double jB[V];
    for (int u = 0; u < V; ++u) {
      ks1[u] = Pk[u] + Ps[u];   // plane m + 1
      ck1[u] = cdt * (double)Pk[u];
      cks1[u] = cdt * ((double)Pk[u] + (double)Ps[u]);
      jB[u] = ck0[u] * (double)PB[u];   // c dt kappa B of plane m
    }
    const double Vm = Vcol * Pvol;   // zone volume (diagnostics)
    stage_halo(m);
    // ---- (a) stage plane m: own zones ----
    for (int u = 0; u < V; ++u) {
      for (int v = 0; v < NC; ++v) PV[pvi(v, prow_own, cx + 1) + u] = q0[u][v];
      PV[pvi(NC, prow_own, cx + 1) + u] = ks0[u];
    }
    // ---- prefetch for the next plane: raw q(m+3), kappa/sigma(m+2), B(m+1), halo m+1.
    // Issued on every plane (indices clamped into the ghost range; the last plane's are
    // not used) so that the loads never sit in a branch ----
    if constexpr (DIM >= 2) {
      Ppm = load_own(min(m + 3, nM + 1), Pr, nullptr, nullptr);
      load_own(min(m + 2, nM + 1), nullptr, Pk, Ps);
      loadB(min(m + 1, nM - 1), PB);
      Pvol = plane_vol(m + 1);
      load_halo(m + 1);
    }
    unit_sync<ROW>();
    // ---- (b) deferred dE_matter of the previous plane (block units: all groups in the block) ----
    if (!ROW && a.dEm && dz_zone >= 0 && gl == 0) {
      double sdz = 0.0;
      for (int g2 = 0; g2 < GB; ++g2) sdz += DZ[(size_t)col * GB + g2];
      put_dem(dz_zone, sdz);
    }
    // ---- (c) in-plane reconstruction (lower states to LDS), march face m + 1/2 ----
    const int eym = ey_of(m);
    R hiX[V][4], hiY[V][4];
    for (int u = 0; u < V; ++u)
      for (int k = 0; k < 4; ++k) hiX[u][k] = hiY[u][k] = R(0);
    if (recon) {
      R hlo[3], hhi[3];
      face_ih<R, SPH>(geo, 0, ex, eym, ex, hlo);
      face_ih<R, SPH>(geo, 0, ex, eym, ex + 1, hhi);
      const bool olo = !SPH || geo.wf[0][ex] != R(0), ohi = !SPH || geo.wf[0][ex + 1] != R(0);
      for (int u = 0; u < V; ++u) {
        R qm[4], qp[4], lo[4];
        for (int v = 0; v < 4; ++v) {
          qm[v] = (v < NC) ? PV[pvi(v, prow_own, cx) + u] : R(0);
          qp[v] = (v < NC) ? PV[pvi(v, prow_own, cx + 2) + u] : R(0);
        }
        reconstruct<R, SPH, DIM, LIM>(a, geo, 0, ex, qm, q0[u], qp, hlo, hhi, olo, ohi, lo, hiX[u]);
        for (int v = 0; v < NC; ++v) LX[cidx(v, col) + u] = lo[v];
      }
      if constexpr (DIM == 3) {
        face_ih<R, SPH>(geo, 1, ex, eyc, eyc, hlo);
        face_ih<R, SPH>(geo, 1, ex, eyc, eyc + 1, hhi);
        const bool ylo = !SPH || geo.wf[1][eyc] != R(0), yhi = !SPH || geo.wf[1][eyc + 1] != R(0);
        for (int u = 0; u < V; ++u) {
          R qm[4], qp[4], lo[4];
          for (int v = 0; v < 4; ++v) {
            qm[v] = (v < NC) ? PV[pvi(v, prow_own - 1, cx + 1) + u] : R(0);
            qp[v] = (v < NC) ? PV[pvi(v, prow_own + 1, cx + 1) + u] : R(0);
          }
          reconstruct<R, SPH, DIM, LIM>(a, geo, 1, eyc, qm, q0[u], qp, hlo, hhi, ylo, yhi, lo, hiY[u]);
          for (int v = 0; v < NC; ++v) LY[cidx(v, col) + u] = lo[v];
        }
      }
    }
    R fNext[V][4], nHi[V][4];
    for (int u = 0; u < V; ++u)
      for (int k = 0; k < 4; ++k) fNext[u][k] = nHi[u][k] = R(0);
    if constexpr (DIM >= 2) {
      if (upd) {
        // reconstruct zone m + 1 along the march direction; flux at m + 1/2
        const int ef = m + 1 + NG;   // lower face of zone m + 1
        const int eyf = (DIM == 3) ? eyc : ef;
        R h1[3], ih1[3], ih2[3];
        face_h<R, SPH>(geo, MD, ex, eyf, ef, h1);
        face_ih<R, SPH>(geo, MD, ex, eyf, ef, ih1);
        face_ih<R, SPH>(geo, MD, ex, eyf, ef + 1, ih2);
        const bool o1 = !SPH || geo.wf[MD][ef] != R(0), o2 = !SPH || geo.wf[MD][ef + 1] != R(0);
        const R dlL = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef - 1);
        const R dlR = proper_width<R, SPH>(geo, MD, ex, (DIM == 3) ? eyc : ef);
        for (int u = 0; u < V; ++u) {
          R nLo[4];
          reconstruct<R, SPH, DIM, LIM>(a, geo, MD, ef, q0[u], q1[u], q2[u], ih1, ih2, o1, o2, nLo, nHi[u]);
          if (o1) hll<R, SPH, DIM, (LIM < 0)>(a, MD, hiM[u], nLo, h1, ih1, epsilon_of(ks0[u], ks1[u], dlL, dlR), fNext[u]);
        }
      }
    }
    unit_sync<ROW>();
    // ---- (d) in-plane faces above this column ----
    R fxR[V][4], fyR[V][4];
    for (int u = 0; u < V; ++u)
      for (int k = 0; k < 4; ++k) fxR[u][k] = fyR[u][k] = R(0);
    if (do_xf) {
      const bool open = !SPH || geo.wf[0][ex + 1] != R(0);
      R hf[3], ihf[3];
      face_h<R, SPH>(geo, 0, ex, eym, ex + 1, hf);
      face_ih<R, SPH>(geo, 0, ex, eym, ex + 1, ihf);
      const R dlL = proper_width<R, SPH>(geo, 0, ex, eym);
      const R dlR = proper_width<R, SPH>(geo, 0, ex + 1, eym);
      for (int u = 0; u < V; ++u) {
        R qR[4] = {R(0), R(0), R(0), R(0)};
        for (int v = 0; v < NC; ++v) qR[v] = LX[cidx(v, col + 1) + u];
        const R ksR = PV[pvi(NC, prow_own, cx + 2) + u];
        if (open) hll<R, SPH, DIM, (LIM < 0)>(a, 0, hiX[u], qR, hf, ihf, epsilon_of(ks0[u], ksR, dlL, dlR), fxR[u]);
        for (int v = 0; v < NC; ++v) FX[cidx(v, col) + u] = fxR[u][v];
      }
    }
    if constexpr (DIM == 3) {
      if (do_yf) {
        const bool open = !SPH || geo.wf[1][eyc + 1] != R(0);
        R hf[3], ihf[3];
        face_h<R, SPH>(geo, 1, ex, eyc, eyc + 1, hf);
        face_ih<R, SPH>(geo, 1, ex, eyc, eyc + 1, ihf);
        const R dlL = proper_width<R, SPH>(geo, 1, ex, eyc);
        const R dlR = proper_width<R, SPH>(geo, 1, ex, eyc + 1);
        for (int u = 0; u < V; ++u) {
          R qR[4] = {R(0), R(0), R(0), R(0)};
          for (int v = 0; v < NC; ++v) qR[v] = LY[cidx(v, col + TXB) + u];
          const R ksR = PV[pvi(NC, prow_own + 1, cx + 1) + u];
          if (open) hll<R, SPH, DIM, (LIM < 0)>(a, 1, hiY[u], qR, hf, ihf, epsilon_of(ks0[u], ksR, dlL, dlR), fyR[u]);
          for (int v = 0; v < NC; ++v) FY[cidx(v, col) + u] = fyR[u][v];
        }
      }
    }
    unit_sync<ROW>();
    // ---- (e) update ----
    dz_zone = -1;
    if (upd) {
      R wxl = R(1), wxh = R(1), iWx = idx0;
      if constexpr (SPH) {
        wxl = geo.wf[0][ex];
        wxh = geo.wf[0][ex + 1];
        iWx = geo.iW[0][ex];
      }
      R wyl = R(1), wyh = R(1), iWy = idx1;
      if constexpr (SPH && DIM == 3) {
        wyl = geo.wf[1][eyc];
        wyh = geo.wf[1][eyc + 1];
        iWy = geo.iW[1][eyc];
      }
      R wml = R(1), wmh = R(1), iWm = idxM;
      if constexpr (SPH && DIM >= 2) {
        wml = geo.wf[MD][m + NG];
        wmh = geo.wf[MD][m + NG + 1];
        iWm = geo.iW[MD][m + NG];
      }
      const int zi = gx, zj = (DIM == 2) ? m : gy, zk = (DIM == 3) ? m : 0;
      const int zone = (zk * n1 + zj) * n0 + zi;
      S Eo[V], Fo[3][V];
      double dzs = 0.0;
      for (int u = 0; u < V; ++u) {
        R acc[4] = {R(0), R(0), R(0), R(0)};
        for (int v = 0; v < NC; ++v) acc[v] += (wxh * fxR[u][v] - wxl * FX[cidx(v, col - 1) + u]) * iWx;
        if constexpr (DIM == 3)
          for (int v = 0; v < NC; ++v) acc[v] += (wyh * fyR[u][v] - wyl * FY[cidx(v, col - TXB) + u]) * iWy;
        if constexpr (DIM >= 2)
          for (int v = 0; v < NC; ++v) acc[v] += (wmh * fNext[u][v] - wml * fPrev[u][v]) * iWm;
        R Um[4];
        for (int cc = 0; cc < 4; ++cc) Um[cc] = (cc < NC) ? q0[u][cc] - dtR * acc[cc] : R(0);
        if constexpr (SPH) {
          R h[3], ih[3], P[9], Sg[3];
          cell_h<R, SPH>(geo, ex, zj + NG, h);
          cell_ih<R, SPH>(geo, ex, zj + NG, ih);
          closure_full<R, SPH, DIM>(q0[u], ih, c, a.closure, P);
          geometric_source<R>(P, h, ih, geo.gam + 4 * zj, c, Sg);
          for (int cc = 0; cc < DIM; ++cc) Um[1 + cc] += dtR * Sg[cc];
        }
        if (a.Ea) {
          // second Runge-Kutta stage: the average with U^n
          const int zgu = zone * a.G + grp0 + u;
          Um[0] = R(0.5) * (R(a.Ea[zgu]) + Um[0]);
          for (int cc = 0; cc < DIM; ++cc) Um[1 + cc] = R(0.5) * (R(a.Fa[cc][zgu]) + Um[1 + cc]);
        }
        S F1[3];
        double dz = 0.0;
        if (a.src) {
          dz = source_zone<S, R, SPH, DIM>(a, geo, zi, zj, Um, ck0[u], cks0[u], jB[u], want_diag, Vm, zd, Eo[u], F1);
        } else {
          Eo[u] = S(Um[0]);
          for (int cc = 0; cc < DIM; ++cc) F1[cc] = S(Um[1 + cc]);
        }
        for (int cc = 0; cc < DIM; ++cc) Fo[cc][u] = F1[cc];
        dzs += dz;
        if (!ROW && a.dEm) DZ[(size_t)col * GB + gl * V + u] = dz;
      }
      const int zg = zone * a.G + grp0;
      stv<S, V>(a.Eo, zg, Eo);
      for (int cc = 0; cc < DIM; ++cc) stv<S, V>(a.Fo[cc], zg, Fo[cc]);
      if (!ROW && a.dEm) dz_zone = zone;
      if (ROW && a.dEm) {
        // sum over the groups of this column (consecutive lanes), one partial per wave
        double p = dzs;
        for (int off = 1; off < LPC; off <<= 1) p += __shfl_xor(p, off);
        if (gl == 0) DZ[((size_t)(m - mbeg) * tl.NW + wv) * TXB + cx] = p;
      }
    }
    // ---- advance the window ----
    if constexpr (DIM >= 2) {
      for (int u = 0; u < V; ++u) {
        for (int cc = 0; cc < 4; ++cc) {
          q0[u][cc] = q1[u][cc];
          q1[u][cc] = q2[u][cc];
          hiM[u][cc] = nHi[u][cc];
          fPrev[u][cc] = fNext[u][cc];
        }
        ks0[u] = ks1[u];
        ck0[u] = ck1[u];
        cks0[u] = cks1[u];
      }
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
          put_dem((int64_t)((DIM == 2) ? mm : 0) * n0 + zx, sdz);
        }
      }
    } else {
      if (dz_zone >= 0 && gl == 0) {
        double s2 = 0.0;
        for (int g2 = 0; g2 < GB; ++g2) s2 += DZ[(size_t)col * GB + g2];
        put_dem(dz_zone, s2);
      }
    }
  }
  if (!want_diag) return;
  // ---- block partials of the diagnostics: wave reduction, then across waves ----
  double e = zd.energy, mf = zd.maxf2();
  int un = zd.nun, p = zd.nnp;
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off);
    mf = fmax(mf, __shfl_xor(mf, off));
    un += __shfl_xor(un, off);
    p += __shfl_xor(p, off);
  }
  __shared__ double we[16], wm[16];
  __shared__ int wu[16], wp[16];
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  __syncthreads();
  if (lane == 0) {
    we[wave] = e;
    wm[wave] = mf;
    wu[wave] = un;
    wp[wave] = p;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
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

Tile make_tile(const fornax_m1_desc& D, int TXB, int TYB, int TM, int GB, int NW, int V) {
  Tile tl{};
  const size_t rsize = (D.precision == FORNAX_FP64) ? sizeof(double) : sizeof(float);
  // 1-D/2-D with NW >= 1: wave rows; NW = 0 (and always in 3-D): one unit per block
  const bool row = D.ndim < 3 && NW >= 1;
  tl.nblocks = 0;
  if (GB < 1 || TM < 1 || D.ngroups % GB != 0) return tl;
  // V = 2: pairs of groups per lane (16-byte FP64 / 8-byte FP32 accesses)
  if (V != 1 && V != 2) return tl;
  if (V == 2 && (GB % 2 != 0 || D.ngroups % 2 != 0)) return tl;
  if (D.ndim == 1 && (!row || V != 1)) return tl;
  if (D.ndim == 2 && !row && V != 1) return tl;
  const int LPC = GB / V;
  if (row) {
    // one x-row of 64/LPC zone columns per wave, NW waves (group subsets) per block
    if (!pow2(LPC) || LPC > 16 || NW > 8 || (D.ngroups / GB) % NW != 0) return tl;
    TXB = 64 / LPC;
    TYB = 1;
  } else {
    NW = 1;
    if (D.ndim < 3) TYB = 1;
    if (TXB < 4 || (D.ndim == 3 && TYB < 4)) return tl;
  }
  tl.row = row;
  tl.V = V;
  tl.TXB = TXB;
  tl.TYB = TYB;
  tl.TM = (D.ndim >= 2) ? TM : 1;
  tl.GB = GB;
  tl.NW = NW;
  tl.nthreads = row ? 64 * NW : TXB * TYB * LPC;
  if (tl.nthreads > 512) return tl;
  // the spherical 3-D double kernel takes at most 256 threads per block
  if (D.ndim == 3 && D.coord == FORNAX_SPHERICAL_LOGR && D.precision == FORNAX_FP64 && tl.nthreads > 256) return tl;
  // halo items (one value of V groups of one halo column each): at most 1 per thread of a
  // wave unit, 3 per thread of a block unit
  const int nunit = row ? 64 : tl.nthreads;
  const int nitems = (2 * TYB * LPC + (D.ndim == 3 ? 2 * TXB * LPC : 0)) * (D.ndim + 1);
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
//  * 1-D / 2-D wave rows: with V = 2 (G even) each lane takes a pair of groups and GB = the
//    largest power of two up to 8 dividing G, so that a wave row of 16 columns reads runs of
//    8 groups; with V = 1, GB up to 4.  All G / GB group subsets of a tile share a block when
//    they fit in 8 waves.  Planes per block are halved from 32 until the grid has at least
//    1024 (FP64) or 2048 (MIXED) blocks, TM >= 4.
//  * 3-D: a near-square tile of 128-512 threads; with many groups per zone, groups are split
//    across blocks so that the zone tile stays large enough to amortise its halo.
Tile choose_tile(const fornax_m1_desc& D, int V) {
  const int G = D.ngroups;
  if (V == 2 && G % 2 != 0) return Tile{};
  if (D.ndim < 3) {
    int GB = V;
    while (GB < 4 * V && G % (2 * GB) == 0) GB *= 2;
    int NW = std::min(8, G / GB);
    while ((G / GB) % NW != 0) --NW;
    const int want = (D.precision == FORNAX_FP64) ? 1024 : 2048;
    Tile t{};
    for (int TM = 32; TM >= 4; TM /= 2) {
      t = make_tile(D, 0, 1, TM, GB, NW, V);
      if (t.nblocks >= want || D.ndim == 1) break;
    }
    return t;
  }
  // measured on gfx950 (192^3 x 12 and 256 x 64 x 128 x 20): Cartesian FP64 8 x 8 columns of
  // up to 4 groups, 16 planes; Cartesian FP32 pairs of groups per lane, 16 x 16 columns of 2
  // groups, 8 planes; spherical FP64 16 x 8 columns of 2 groups, 16 planes; spherical FP32
  // 16 x 8 columns of up to 4 groups, 16 planes (in 512-thread blocks: at 256 threads with the
  // accumulation registers, as in double, it takes 1.8x longer)
  {
    Tile t{};
    const bool sph = D.coord == FORNAX_SPHERICAL_LOGR;
    if (D.precision == FORNAX_FP64) {
      int GB = sph ? 2 : 4;
      while (G % GB != 0) --GB;
      t = sph ? make_tile(D, 16, 8, 16, GB, 1, 1) : make_tile(D, 8, 8, 16, GB, 1, 1);
    } else if (V == 2) {
      t = make_tile(D, 16, 16, 8, 2, 1, 2);
    } else if (sph) {
      int GB = 4;
      while (G % GB != 0) --GB;
      t = make_tile(D, 16, 8, 16, GB, 1, 1);
    }
    if (t.nblocks > 0) return t;
  }
  Tile best{};
  double best_cost = 1e30;
  for (int GB = G; GB >= 1; --GB) {
    if (G % GB != 0) continue;
    for (int TXB = 4; TXB <= 32; ++TXB)
      for (int TYB = 4; TYB <= 32; ++TYB) {
        Tile t = make_tile(D, TXB, TYB, 8, GB, 1, V);
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

template <typename S, typename R, int DIM, bool SPH, bool ROW, int GBC, int V>
static hipError_t raise_lds_limit(int bytes) {
  const hipError_t e1 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&k_step_tiled<S, R, DIM, SPH, ROW, GBC, V, FORNAX_LIMITER_MINMOD>),
      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  const hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step_tiled<S, R, DIM, SPH, ROW, GBC, V, -1>),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e1 != hipSuccess ? e1 : e2;
}

// Every instantiation that launch_tiled can pick.
template <typename S, typename R, bool SPH>
static hipError_t raise_coord(int bytes) {
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (r != hipSuccess) e = r;
  };
  chk(raise_lds_limit<S, R, 1, SPH, true, 0, 1>(bytes));
  chk(raise_lds_limit<S, R, 2, SPH, true, 0, 1>(bytes));
  chk(raise_lds_limit<S, R, 2, SPH, true, 4, 1>(bytes));
  chk(raise_lds_limit<S, R, 2, SPH, true, 8, 2>(bytes));
  chk(raise_lds_limit<S, R, 2, SPH, true, 16, 2>(bytes));
  chk(raise_lds_limit<S, R, 2, SPH, true, 0, 2>(bytes));
  chk(raise_lds_limit<S, R, 2, SPH, false, 0, 1>(bytes));
  chk(raise_lds_limit<S, R, 3, SPH, false, 0, 1>(bytes));
  chk(raise_lds_limit<S, R, 3, SPH, false, 0, 2>(bytes));
  return e;
}

template <typename S, typename R>
static hipError_t raise_all(int bytes) {
  const hipError_t e1 = raise_coord<S, R, false>(bytes);
  const hipError_t e2 = raise_coord<S, R, true>(bytes);
  return e1 != hipSuccess ? e1 : e2;
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

template <typename S, typename R, bool SPH>
static int launch_coord(const Geo<R>& geo, const StepArgs<S>& a, const Tile& tl, int D, hipStream_t st) {
  dim3 grid(tl.nblocks), block(tl.nthreads);
  // the method's default limiter (with the -+c wavespeed bounds) is a compile-time constant of
  // its own instantiation; the instantiation that reads the limiter at run time also takes the
  // M1-speed bounds
  const bool mm = a.limiter == FORNAX_LIMITER_MINMOD && a.wavespeed == FORNAX_WAVESPEED_LIGHT;
#define FM1_LAUNCH(DIMV, ROWV, GBV, VV)                                                                          \
  do {                                                                                                          \
    if (mm)                                                                                                     \
      hipLaunchKernelGGL((k_step_tiled<S, R, DIMV, SPH, ROWV, GBV, VV, FORNAX_LIMITER_MINMOD>), grid, block,     \
                         tl.lds, st, a, geo, tl);                                                                \
    else                                                                                                        \
      hipLaunchKernelGGL((k_step_tiled<S, R, DIMV, SPH, ROWV, GBV, VV, -1>), grid, block, tl.lds, st, a, geo, tl); \
  } while (0)
  if (D == 1) {
    if (!tl.row || tl.V != 1) return FORNAX_EUNSUPPORTED;
    FM1_LAUNCH(1, true, 0, 1);
  } else if (D == 2) {
    if (tl.row && tl.V == 1 && tl.GB == 4) FM1_LAUNCH(2, true, 4, 1);
    else if (tl.row && tl.V == 1) FM1_LAUNCH(2, true, 0, 1);
    else if (tl.row && tl.V == 2 && tl.GB == 8) FM1_LAUNCH(2, true, 8, 2);
    else if (tl.row && tl.V == 2 && tl.GB == 16) FM1_LAUNCH(2, true, 16, 2);
    else if (tl.row && tl.V == 2) FM1_LAUNCH(2, true, 0, 2);
    else if (!tl.row && tl.V == 1) FM1_LAUNCH(2, false, 0, 1);
    else return FORNAX_EUNSUPPORTED;
  } else {
    if (tl.V == 1) FM1_LAUNCH(3, false, 0, 1);
    else FM1_LAUNCH(3, false, 0, 2);
  }
#undef FM1_LAUNCH
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

static bool aligned_to(const void* p, size_t n) { return p == nullptr || ((uintptr_t)p % n) == 0; }

template <typename S, typename R>
int launch_tiled(fornax_m1_ctx* ctx, const Geo<R>& geo, const StepArgs<S>& a, hipStream_t st) {
  // the whole-zone kernel does the Euler push; Runge-Kutta stages run on the tiled kernel
  if constexpr (std::is_same<S, R>::value) {
    if (ctx->rows.nblocks > 0 && a.src && !a.Ea) return launch_rows<S>(ctx, geo, a, st);
    // the 3-D Cartesian kernel takes every stage of its grids
    if (ctx->c3.nblocks > 0) return launch_c3<S>(ctx, geo, a, st);
  }
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  const int D = ctx->desc.ndim;
  // pairs of groups per lane need arrays aligned to two elements
  const Tile* tl = &ctx->tile;
  bool al = true;
  const void* ptrs[] = {a.E,   a.F[0], a.F[1], a.F[2],  a.Eo,    a.Fo[0], a.Fo[1],
                        a.Fo[2], a.kap, a.sig,  a.B,    a.Ea,    a.Fa[0], a.Fa[1], a.Fa[2]};
  for (const void* q : ptrs) al = al && aligned_to(q, 2 * sizeof(S));
  if (tl->V == 2 && !al) tl = &ctx->tile_v1;
  if (tl->nblocks <= 0) return FORNAX_EUNSUPPORTED;
  if (a.dEm && tl->ngb > 1 && !a.dzp) return FORNAX_EUNSUPPORTED;
  *ctx->last_tile = *tl;
  return sph ? launch_coord<S, R, true>(geo, a, *tl, D, st) : launch_coord<S, R, false>(geo, a, *tl, D, st);
}

template int launch_tiled<double, double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&, hipStream_t);
template int launch_tiled<float, float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, hipStream_t);

}  // namespace fm1
