// m1_step_rows.hip -- the fused M1 step for 2-D Cartesian grids with 16 groups, the layout of
// the 512 x 512 x 16 workload: whole zones moved between HBM and LDS.
//
// Same method and arithmetic as k_step_tiled (eq:finite_vol with minmod reconstruction
// eq:recon_constraints, the M1 closure, the HLL flux eq:hll with the correction eq:epsilon,
// the backward-Euler interaction update eq:be_update); what differs is the data movement:
//   * a block of 4 NWX waves owns TXB = 16 NWX zone columns (TXB - 2 updated) and marches
//     along y; lane = (column, group), 4 groups per wave row, the 4 wave rows of a column
//     hold its 16 groups;
//   * every plane of 5 input arrays (E, F_x, F_y, kappa, sigma) is copied into LDS as
//     whole 128-byte zones by direct-to-LDS loads (global_load_lds_dwordx4), three planes
//     ahead of use in a ring of three slots (a slot per static LDS array, so that the compiler
//     orders each LDS read after the loads of its own slot only); B, needed for the own zone
//     only, is loaded into a register one plane ahead;
//   * lower face states and in-plane fluxes are exchanged between the waves through LDS, so no
//     wave recomputes a neighbour's column;
//   * the outputs of a plane are staged in LDS and stored as whole zones by raw buffer stores
//     (a fixed number per wave; chunks outside the domain fall beyond the buffer and are
//     dropped), so that the wait for the next plane's loads can count the stores exactly.
// Four block barriers per plane: loads of the next plane arrived, lower states written,
// fluxes written, outputs staged.  The Euler push only (Runge-Kutta stages use k_step_tiled).

#include <hip/hip_runtime.h>

#include <type_traits>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

constexpr int RG = 16;       // groups (the kernel's fixed layout)
constexpr int RNA = 5;       // arrays of a plane in LDS: E, F_x, F_y, kappa, sigma
constexpr int RNC = 3;       // state components in 2-D

// LDS sizes of the instantiation (elements of S)
template <typename S, int NWX>
struct RowsLds {
  static constexpr int TXB = 16 * NWX;
  static constexpr int NCOL = TXB + 2;                 // zone columns of a slot (one halo each side)
  static constexpr int EPC = 16 / (int)sizeof(S);      // elements per 16-byte chunk
  static constexpr int CPZ = RG / EPC;                 // chunks per zone
  static constexpr int SLOT = RNA * NCOL * RG;         // elements per slot
  static constexpr int ROT = 4 / EPC > 0 ? 4 / EPC : 1; // chunks of a zone that one wave row reads
  static constexpr int GS = RG + 4;                    // padded group stride of the exchange arrays
  static constexpr int XCH = RNC * TXB * GS;           // elements per exchange array
};

// Ghost rule of an x index (-2 <= e <= n0 + 1): source column and flags (bit 0 flips F_x,
// bit 1 takes the prescribed inflow state)
__device__ __forceinline__ void x_rule(const StepArgsBase& a, int e, int& src, int& fl) {
  src = e;
  fl = 0;
  if (e < 0) {
    src = a.gsrc[0][e + 2];
    fl = a.gfl[0][e + 2];
  } else if (e >= a.n[0]) {
    src = a.gsrc[0][e - a.n[0] + 2];
    fl = a.gfl[0][e - a.n[0] + 2];
  }
}

__device__ __forceinline__ void y_rule(const StepArgsBase& a, int e, int& src, int& fl) {
  src = e;
  fl = 0;
  if (e < 0) {
    src = a.gsrc[1][e + 2];
    fl = a.gfl[1][e + 2];
  } else if (e >= a.n[1]) {
    src = a.gsrc[1][e - a.n[1] + 2];
    fl = a.gfl[1][e - a.n[1] + 2];
  }
}

#define FM1_LDSP(p) ((__attribute__((address_space(3))) void*)(p))

template <typename S, int LIM, int NWX>
__global__ void __launch_bounds__(64 * 4 * NWX) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 3 : 4)))
k_step_rows(StepArgs<S> a, Geo<S> geo, RowsTile tl) {
  using R = S;
  using L = RowsLds<S, NWX>;
  constexpr int TXB = L::TXB, NCOL = L::NCOL, EPC = L::EPC, CPZ = L::CPZ, GS = L::GS, ROT = L::ROT;
  constexpr int NW = 4 * NWX;                      // waves
  constexpr int NT = 64 * NW;                      // threads
  constexpr int NI = (NCOL * CPZ + 63) / 64;      // wave loads of 64 16-byte chunks per array
  constexpr int NDMA = (RNA * NI + NW - 1) / NW;   // direct-to-LDS loads per wave and plane
  constexpr int NOUT = RNC * TXB * CPZ;            // output chunks of a plane
  constexpr int NST = (NOUT + NT - 1) / NT;        // stores per thread and plane
  static_assert((TXB * CPZ) % 64 == 0, "the output chunks of an array fill whole waves");
  __shared__ __align__(16) S ring0[L::SLOT];
  __shared__ __align__(16) S ring1[L::SLOT];
  __shared__ __align__(16) S ring2[L::SLOT];
  __shared__ __align__(16) R LX[L::XCH];           // lower x-face states; then the staged outputs
  __shared__ __align__(16) R FX[L::XCH];           // x fluxes at the upper face of each column
  __shared__ double DZ[4][TXB];                    // dE_matter partials of the wave rows
  __shared__ double we[NW], wm[NW];
  __shared__ int wu[NW], wp[NW];

  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // wave index (uniform)
  const int wx = w % NWX, wg = w / NWX;
  const int c = wx * 16 + (lane >> 2);             // lane column (LDS column c + 1)
  const int g = wg * 4 + (lane & 3);               // group

  // tile of the block (XCD-aware renumbering)
  const int b = blockIdx.x;
  const int xcd = b & 7, sl = b >> 3;
  const int Lb = xcd * tl.xq + min(xcd, tl.xr) + sl;
  const int tx = Lb % tl.ntx, tm = Lb / tl.ntx;
  const int n0 = a.n[0], n1 = a.n[1];
  const int x0 = tx * (TXB - 2) - 1;               // zone of lane column 0 (LDS column j: zone x0 - 1 + j)
  const int gx = x0 + c;
  const int mbeg = tm * tl.TM, mend = min(mbeg + tl.TM, n1);
  const bool recon = gx <= n0;
  const bool upd = c >= 1 && c <= TXB - 2 && gx < n0;
  const bool do_xf = c <= TXB - 2 && gx + 1 <= n0;
  const bool want_diag = a.p_energy != nullptr;
  ZoneDiag zd;
  const R cR = R(a.c);
  const R dtR = R(a.dt);
  const double cdt = a.c * a.dt;
  const R idx0 = geo.idx[0], idx1 = geo.idx[1];
  const R dx0 = geo.dx[0], dx1 = geo.dx[1];
  const R hone[3] = {R(1), R(1), R(1)};
  const double Vz = want_diag ? geo.Wd[0][NG] * geo.Wd[1][NG] * geo.Wd[2][NG] : 0.0;   // uniform zones

  // ghost rules of the lane's three columns (left neighbour, own, right neighbour)
  int xs_m, xf_m, xs_o, xf_o, xs_p, xf_p;
  x_rule(a, min(gx - 1, n0 + 1), xs_m, xf_m);
  x_rule(a, min(gx, n0 + 1), xs_o, xf_o);
  x_rule(a, min(gx + 1, n0 + 1), xs_p, xf_p);
  (void)xs_m;
  (void)xs_p;
  R qin[3] = {R(0), R(0), R(0)};   // prescribed inflow state of this group (inflow is on x only)
  if ((xf_m | xf_o | xf_p) & 2)
    for (int k = 0; k < 3; ++k) qin[k] = R(a.inflow[g * 3 + k]);

  // element of (array, LDS column, group) in a slot: each zone's chunks are rotated by ROT
  // per pair of columns, so that the chunks a wave row reads from 8 consecutive columns fall
  // on distinct banks of gfx950's 64 (measured: a third of the conflicts of a rotation per
  // column)
  auto ridx = [&](int arr, int jc, int gg) -> int {
    return ((arr * NCOL + jc) * CPZ + ((gg / EPC + ROT * (jc >> 1)) % CPZ)) * EPC + gg % EPC;
  };
  auto slot_ptr = [&](int s) -> S* { return s == 0 ? ring0 : (s == 1 ? ring1 : ring2); };
  auto arr_ptr = [&](int arr) -> const S* {
    return arr == 0 ? a.E : arr == 1 ? a.F[0] : arr == 2 ? a.F[1] : arr == 3 ? a.kap : a.sig;
  };
  // B of the own zone in plane m (updated columns only use it; the index is clamped into the
  // domain so that every lane may load)
  const int zib = min(max(gx, 0), n0 - 1);
  auto loadB = [&](int m) -> S { return a.B[((size_t)min(m, n1 - 1) * n0 + zib) * RG + g]; };

  // direct-to-LDS loads of plane p (any index; ghost planes by the y rule, planes beyond the
  // second ghost layer clamped: their values are never used) into slot s.  Each array's
  // NCOL * CPZ chunks take NI wave loads of 64 chunks; load J = NI * array + i goes to wave
  // J mod NW, so that the array of a load is uniform over its wave.  The in-plane source of
  // every chunk (x rule included) is fixed per thread: element offsets xo, computed once.
  int xo[NDMA];
  bool xv[NDMA];
#pragma unroll
  for (int k = 0; k < NDMA; ++k) {
    const int J = k * NW + w;
    const int i = J % NI;
    const int r = i * 64 + lane;                        // chunk within the array's region
    xv[k] = J < RNA * NI && r < NCOL * CPZ;
    const int rr = xv[k] ? r : 0;
    const int jc = rr / CPZ;
    const int part = (rr - jc * CPZ + CPZ * ROT * NCOL - ROT * (jc >> 1)) % CPZ;   // inverse of the rotation
    int xsrc, xfl;
    x_rule(a, min(x0 - 1 + jc, n0 + 1), xsrc, xfl);
    (void)xfl;
    xo[k] = xsrc * RG + part * EPC;
  }
  auto issue = [&](int p, auto slot_tag) {
    constexpr int s = decltype(slot_tag)::value;
    S* base = slot_ptr(s);
    int ysrc, yfl;
    y_rule(a, min(max(p, -2), n1 + 1), ysrc, yfl);
    (void)yfl;
    const size_t yoff = (size_t)ysrc * n0 * RG;
#pragma unroll
    for (int k = 0; k < NDMA; ++k) {
      const int J = k * NW + w;
      if (J < RNA * NI) {
        const int arr = J / NI, i = J - arr * NI;
        if (xv[k]) {
          const S* src = arr_ptr(arr) + yoff + xo[k];
          __builtin_amdgcn_global_load_lds((const void*)src, FM1_LDSP(base + ((size_t)arr * NCOL * CPZ + i * 64) * EPC),
                                           16, 0, 0);
        }
      }
    }
  };
  // state of LDS column jc of the plane in slot s, with the x rule of that column and the
  // y flip of the plane
  auto read_state = [&](const S* base, int jc, int xfl, int yflip, R q[4]) {
    q[0] = R(base[ridx(0, jc, g)]);
    q[1] = R(base[ridx(1, jc, g)]);
    q[2] = R(base[ridx(2, jc, g)]);
    q[3] = R(0);
    if (xfl & 1) q[1] = -q[1];
    if (yflip) q[2] = -q[2];
    if (xfl & 2) {
      q[0] = qin[0];
      q[1] = qin[1];
      q[2] = qin[2];
    }
  };
  auto yflip_of = [&](int p) -> int {
    int ys, yf;
    y_rule(a, min(max(p, -2), n1 + 1), ys, yf);
    return yf & 1;
  };
  // own zone of plane p (-2 <= p < n1) loaded directly (the two planes below the tile)
  auto load_direct = [&](int p, R q[4], R& ks) {
    int ys, yf;
    y_rule(a, p, ys, yf);
    const int zg = ((int)ys * n0 + xs_o) * RG + g;
    q[0] = R(a.E[zg]);
    q[1] = R(a.F[0][zg]);
    q[2] = R(a.F[1][zg]);
    q[3] = R(0);
    ks = R(a.kap[zg]) + R(a.sig[zg]);
    if (xf_o & 1) q[1] = -q[1];
    if (yf & 1) q[2] = -q[2];
    if (xf_o & 2) {
      q[0] = qin[0];
      q[1] = qin[1];
      q[2] = qin[2];
    }
  };
  // raw buffer stores of the staged outputs of plane m (whole zones; chunks of columns that
  // are not updated get an offset beyond the buffer and are dropped)
  const uint32_t nbytes = (uint32_t)((size_t)n0 * n1 * RG * sizeof(S));
  __amdgpu_buffer_rsrc_t rsE = __builtin_amdgcn_make_buffer_rsrc(a.Eo, 0, (int)nbytes, 0x00020000);
  __amdgpu_buffer_rsrc_t rsF0 = __builtin_amdgcn_make_buffer_rsrc(a.Fo[0], 0, (int)nbytes, 0x00020000);
  __amdgpu_buffer_rsrc_t rsF1 = __builtin_amdgcn_make_buffer_rsrc(a.Fo[1], 0, (int)nbytes, 0x00020000);
  typedef int v4i __attribute__((ext_vector_type(4)));
  auto store_plane = [&](int m) {
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      // a wave's 64 chunks lie in one array (TXB * CPZ is a multiple of 64): uniform descriptor
      const int q = k * NT + t;
      const int qw = k * NT + w * 64;
      const int arr = qw < NOUT ? qw / (TXB * CPZ) : 0;
      const int qq = q < NOUT ? q : arr * (TXB * CPZ);
      const int r = qq - arr * (TXB * CPZ);
      const int cc = r / CPZ, part = r - cc * CPZ;
      const int zx = x0 + cc;
      const bool ok = q < NOUT && cc >= 1 && cc <= TXB - 2 && zx < n0;
      const v4i v = *reinterpret_cast<const v4i*>(&LX[(arr * TXB + cc) * GS + part * EPC]);
      const uint32_t off = ok ? (uint32_t)((((size_t)m * n0 + zx) * RG + part * EPC) * sizeof(S)) : 0x7ffffff0u;
      const __amdgpu_buffer_rsrc_t rs = arr == 0 ? rsE : (arr == 1 ? rsF0 : rsF1);
      __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, 0);
    }
  };
  // dE_matter of the updated zones of plane m from the wave-row partials
  auto dem_store = [&](int m) {
    if (t < TXB) {
      const int zx = x0 + t;
      if (t >= 1 && t <= TXB - 2 && zx < n0) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += DZ[k][t];
        a.dEm[(size_t)m * n0 + zx] = -s;
      }
    }
  };
  // Block barrier for LDS data (no wait for the loads into the ring, which the counted
  // waits cover).  The empty asm statements keep the compiler from moving memory accesses
  // across it, so that the loads and stores of a plane stay in the order the counts assume.
  auto barrier = [&] {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  // ---- prologue: planes mbeg, mbeg + 1, mbeg + 2 into the ring; planes mbeg - 2, mbeg - 1
  // of the own column loaded directly; the register window ----
  issue(mbeg, std::integral_constant<int, 0>{});
  issue(mbeg + 1, std::integral_constant<int, 1>{});
  issue(mbeg + 2, std::integral_constant<int, 2>{});
  R qa[4], qb[4], ksa, ksb;
  load_direct(mbeg - 2, qa, ksa);
  load_direct(mbeg - 1, qb, ksb);
  S Bm = loadB(mbeg);   // B of the current plane (the next plane's is loaded one plane ahead)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
  barrier();
  R q0[4], q1[4], hiM[4], fPrev[4];
  read_state(ring0, c + 1, xf_o, 0, q0);
  read_state(ring1, c + 1, xf_o, yflip_of(mbeg + 1), q1);
  const S k0s = ring0[ridx(3, c + 1, g)], s0s = ring0[ridx(4, c + 1, g)];
  R ks0 = R(k0s) + R(s0s);
  double ck0 = cdt * (double)k0s, cks0 = cdt * ((double)k0s + (double)s0s);
  for (int k = 0; k < 4; ++k) hiM[k] = fPrev[k] = R(0);
  {
    R lo[4], hiP[4];
    reconstruct<R, false, 2, LIM>(a, geo, 1, mbeg - 1 + NG, qa, qb, q0, hone, hone, true, true, lo, hiP);
    reconstruct<R, false, 2, LIM>(a, geo, 1, mbeg + NG, qb, q0, q1, hone, hone, true, true, lo, hiM);
    hll<R, false, 2>(a, 1, hiP, lo, hone, hone, epsilon_of(ksb, ks0, dx1, dx1), fPrev);
  }

  // ---- one plane; SP = slot of plane m (the slots of m + 1, m + 2 follow cyclically) ----
  auto plane = [&](int m, auto sp_tag) {
    constexpr int s0 = decltype(sp_tag)::value, s1 = (s0 + 1) % 3, s2 = (s0 + 2) % 3;
    const S* P0 = slot_ptr(s0);
    const S* P1 = slot_ptr(s1);
    const S* P2 = slot_ptr(s2);
    if (m > mbeg) {
      // the loads of plane m + 2 (issued one plane ago, before that plane's NST stores)
      asm volatile("" ::: "memory");
      if constexpr (NST == 1) __builtin_amdgcn_s_waitcnt(0x0f70 | 1);
      else if constexpr (NST == 2) __builtin_amdgcn_s_waitcnt(0x0f70 | 2);
      else __builtin_amdgcn_s_waitcnt(0x0f70);
      barrier();
      if (a.dEm) dem_store(m - 1);
    }
    // own values: q(m + 2), kappa and sigma of m + 1, B of m
    R q2[4];
    read_state(P2, c + 1, xf_o, yflip_of(m + 2), q2);
    const S k1s = P1[ridx(3, c + 1, g)], s1s = P1[ridx(4, c + 1, g)];
    const R ks1 = R(k1s) + R(s1s);
    const double ck1 = cdt * (double)k1s, cks1 = cdt * ((double)k1s + (double)s1s);
    const double jB = ck0 * (double)Bm;
    // B of the next plane, issued before this plane's loads into the ring (so that the counted
    // wait at the top of the next plane covers it)
    const S Bn = loadB(m + 1);
    // x reconstruction of the own column (lower state to LDS)
    R hiX[4] = {R(0), R(0), R(0), R(0)};
    if (recon) {
      R qm[4], qp[4], lo[4];
      read_state(P0, c, xf_m, 0, qm);
      read_state(P0, c + 2, xf_p, 0, qp);
      reconstruct<R, false, 2, LIM>(a, geo, 0, gx + NG, qm, q0, qp, hone, hone, true, true, lo, hiX);
      for (int v = 0; v < RNC; ++v) LX[(v * TXB + c) * GS + g] = lo[v];
    }
    // march: zone m + 1 along y, flux at m + 1/2
    R fNext[4] = {R(0), R(0), R(0), R(0)}, nHi[4] = {R(0), R(0), R(0), R(0)};
    if (upd) {
      R nLo[4];
      reconstruct<R, false, 2, LIM>(a, geo, 1, m + 1 + NG, q0, q1, q2, hone, hone, true, true, nLo, nHi);
      hll<R, false, 2>(a, 1, hiM, nLo, hone, hone, epsilon_of(ks0, ks1, dx1, dx1), fNext);
    }
    barrier();
    // x face above the own column
    R fx[4] = {R(0), R(0), R(0), R(0)};
    if (do_xf) {
      R qR[4] = {R(0), R(0), R(0), R(0)};
      for (int v = 0; v < RNC; ++v) qR[v] = LX[(v * TXB + c + 1) * GS + g];
      const R ksR = R(P0[ridx(3, c + 2, g)]) + R(P0[ridx(4, c + 2, g)]);
      hll<R, false, 2>(a, 0, hiX, qR, hone, hone, epsilon_of(ks0, ksR, dx0, dx0), fx);
      for (int v = 0; v < RNC; ++v) FX[(v * TXB + c) * GS + g] = fx[v];
    }
    barrier();
    // slot s0 is free: plane m + 3 (needed one plane from now)
    if (m + 3 <= mend + 1) issue(m + 3, sp_tag);
    // update of the own zone, outputs staged in LDS (LX is free)
    if (upd) {
      R acc[4] = {R(0), R(0), R(0), R(0)};
      for (int v = 0; v < RNC; ++v) acc[v] += (fx[v] - FX[(v * TXB + c - 1) * GS + g]) * idx0;
      for (int v = 0; v < RNC; ++v) acc[v] += (fNext[v] - fPrev[v]) * idx1;
      R Um[4];
      for (int k = 0; k < 4; ++k) Um[k] = (k < RNC) ? q0[k] - dtR * acc[k] : R(0);
      S Eo, F1[3];
      const double dz = source_zone<S, R, false, 2>(a, geo, gx, m, Um, ck0, cks0, jB, want_diag, Vz, zd, Eo, F1);
      LX[(0 * TXB + c) * GS + g] = Eo;
      LX[(1 * TXB + c) * GS + g] = F1[0];
      LX[(2 * TXB + c) * GS + g] = F1[1];
      if (a.dEm) {
        double p = dz;
        p += __shfl_xor(p, 1);
        p += __shfl_xor(p, 2);
        if ((lane & 3) == 0) DZ[wg][c] = p;
      }
    }
    // advance the window
    for (int k = 0; k < 4; ++k) {
      q0[k] = q1[k];
      q1[k] = q2[k];
      hiM[k] = nHi[k];
      fPrev[k] = fNext[k];
    }
    ks0 = ks1;
    ck0 = ck1;
    cks0 = cks1;
    Bm = Bn;
    barrier();
    store_plane(m);
  };
  (void)cR;
  for (int m = mbeg; m < mend; m += 3) {
    plane(m, std::integral_constant<int, 0>{});
    if (m + 1 < mend) plane(m + 1, std::integral_constant<int, 1>{});
    if (m + 2 < mend) plane(m + 2, std::integral_constant<int, 2>{});
  }
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): no load into LDS outlives the block
  barrier();
  if (a.dEm) dem_store(mend - 1);

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
    we[w] = e;
    wm[w] = mf;
    wu[w] = un;
    wp[w] = pnp;
  }
  __syncthreads();
  if (t == 0) {
    double se = 0.0, sm = 0.0;
    int su = 0, sp = 0;
    for (int k = 0; k < NW; ++k) {
      se += we[k];
      sm = fmax(sm, wm[k]);
      su += wu[k];
      sp += wp[k];
    }
    a.p_energy[blockIdx.x] = se;
    a.p_maxf2[blockIdx.x] = sm;
    a.p_nun[blockIdx.x] = su;
    a.p_nnp[blockIdx.x] = sp;
  }
}

#undef FM1_LDSP

// ------------------------------------------------------------------------------------------
size_t rows_lds_bytes(const fornax_m1_desc& D, int NWX) {
  const size_t s = (D.precision == FORNAX_FP64) ? 8 : 4;
  const size_t txb = 16 * (size_t)NWX;
  const size_t slot = RNA * (txb + 2) * RG * s;
  const size_t xch = RNC * txb * (RG + 4) * s;
  return 3 * slot + 2 * xch + 4 * txb * 8 + 16 * 24;
}

RowsTile make_rows_tile(const fornax_m1_desc& D, int NWX, int TM) {
  RowsTile tl{};
  tl.nblocks = 0;
  if (D.ndim != 2 || D.coord != FORNAX_CARTESIAN || D.ngroups != RG) return tl;
  if (NWX != 1 && NWX != 2) return tl;
  if (TM < 3 || TM % 3 != 0) return tl;
  const size_t s = (D.precision == FORNAX_FP64) ? 8 : 4;
  if ((size_t)D.n[0] * D.n[1] * RG * s >= ((size_t)1 << 31)) return tl;   // 32-bit buffer offsets
  tl.NWX = NWX;
  tl.TXB = 16 * NWX;
  tl.TM = TM;
  tl.ntx = (D.n[0] + tl.TXB - 3) / (tl.TXB - 2);
  tl.ntm = (D.n[1] + TM - 1) / TM;
  tl.nblocks = tl.ntx * tl.ntm;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  tl.nthreads = 256 * NWX;
  tl.lds = rows_lds_bytes(D, NWX);
  return tl;
}

RowsTile choose_rows_tile(const fornax_m1_desc& D) {
  // measured on gfx950 (512 x 512 x 16): in double one wave row per block and 9 planes beat
  // the tiled kernel; in float (half the bytes per zone) the tiled kernel is faster
  if (D.precision != FORNAX_FP64) return RowsTile{};
  return make_rows_tile(D, 1, 9);
}

template <typename S>
int launch_rows(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, hipStream_t st) {
  const RowsTile& tl = ctx->rows;
  if (tl.nblocks <= 0) return FORNAX_EUNSUPPORTED;
  const bool mm = a.limiter == FORNAX_LIMITER_MINMOD;
  dim3 grid(tl.nblocks), block(tl.nthreads);
  if (tl.NWX == 2) {
    if (mm)
      hipLaunchKernelGGL((k_step_rows<S, FORNAX_LIMITER_MINMOD, 2>), grid, block, 0, st, a, geo, tl);
    else
      hipLaunchKernelGGL((k_step_rows<S, -1, 2>), grid, block, 0, st, a, geo, tl);
  } else {
    if (mm)
      hipLaunchKernelGGL((k_step_rows<S, FORNAX_LIMITER_MINMOD, 1>), grid, block, 0, st, a, geo, tl);
    else
      hipLaunchKernelGGL((k_step_rows<S, -1, 1>), grid, block, 0, st, a, geo, tl);
  }
  // the reduction bookkeeping of the step (one diagnostics partial per block; every block
  // holds all groups of its zones)
  Tile lt{};
  lt.nblocks = tl.nblocks;
  lt.ngb = 1;
  *ctx->last_tile = lt;
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template int launch_rows<double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&, hipStream_t);
template int launch_rows<float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, hipStream_t);

}  // namespace fm1
