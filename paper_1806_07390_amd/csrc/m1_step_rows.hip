// m1_step_rows.hip -- the fused M1 step for 2-D Cartesian grids with 16 groups, the layout of
// the 512 x 512 x 16 workload: whole zones moved from HBM into LDS.
//
// Same method and arithmetic as k_step_tiled (eq:finite_vol with minmod reconstruction
// eq:recon_constraints, the M1 closure, the HLL flux eq:hll with the correction eq:epsilon,
// the backward-Euler interaction update eq:be_update); what differs is the data movement:
//   * a block of 4 waves owns 16 zone columns (14 updated) and marches along y; lane =
//     (column, group), 4 groups per wave: a wave holds 16 columns of 4 groups, the 4 waves of
//     the block hold a column's 16 groups;
//   * every plane of the 6 input arrays (E, F_x, F_y on 18 columns, kappa, sigma, B on the 16
//     own columns) is copied into LDS as whole 128-byte zones by direct-to-LDS loads
//     (global_load_lds_dwordx4) into a ring of four slots, three planes ahead: the loads of
//     plane m + 3 go out at the top of plane m, into the slot plane m - 1 has just left, and
//     are waited for at the top of plane m + 1;
//   * the ring is read with LDS reads that complete within their own statement: the compiler,
//     which cannot tell the slots of the loads in flight apart, would otherwise wait for all
//     of them before every read;
//   * the neighbouring columns of a lane are 4 lanes away in the same wave: lower face states
//     and x fluxes move between columns by lane permutes (ds_bpermute);
//   * each lane stores its zone-group's outputs with raw buffer stores at the top of the next
//     plane, behind that plane's loads (lanes of columns that are not updated store beyond the
//     buffer: dropped).
// One block barrier per plane.  The Euler push only (Runge-Kutta stages use k_step_tiled).

#include <hip/hip_runtime.h>

#include <type_traits>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

constexpr int RG = 16;       // groups (the kernel's fixed layout)
constexpr int RNA = 6;       // arrays of a plane in LDS: E, F_x, F_y, kappa, sigma, B
constexpr int RNS = 3;       // of which the state (on the halo columns as well)
constexpr int RNC = 3;       // state components in 2-D
constexpr int RTX = 16;      // zone columns of a block (RTX - 2 updated)
constexpr int RNW = 4;       // waves of a block
constexpr int RRING = 4;     // slots of the LDS ring

// LDS layout of a slot, in 16-byte chunks: E, F_x, F_y on LDS columns 0 .. RTX + 1 (zones
// x0 - 1 .. x0 + RTX), then kappa, sigma, B on LDS columns 1 .. RTX (the block's own columns),
// each array's zones contiguous.  A wave load copies 64 consecutive chunks: a state array's
// last load runs into the next array, whose first chunks it copies again (the same bytes to
// the same place), so that every lane of every load has a chunk.
template <typename S>
struct RowsLds {
  static constexpr int EPC = 16 / (int)sizeof(S);      // elements per 16-byte chunk
  static constexpr int CPZ = RG / EPC;                 // chunks per zone
  static constexpr int SCH = (RTX + 2) * CPZ;          // chunks of a state array
  static constexpr int CCH = RTX * CPZ;                // chunks of a coefficient array
  static constexpr int SLOTCH = RNS * SCH + (RNA - RNS) * CCH;
  static constexpr int SLOT = SLOTCH * EPC;            // elements per slot
  static constexpr int SLOTB = SLOTCH * 16;            // bytes per slot
  static constexpr int ROT = 4 / EPC > 0 ? 4 / EPC : 1; // chunks of a zone that one wave reads
  static constexpr int NIS = (SCH + 63) / 64, NIC = CCH / 64;   // wave loads per array
  static constexpr int NLOAD = RNS * NIS + (RNA - RNS) * NIC;
  static_assert(CCH % 64 == 0 && NIS * 64 - SCH <= CCH, "slot layout");
  __host__ __device__ static constexpr int start(int arr) { return arr < RNS ? arr * SCH : RNS * SCH + (arr - RNS) * CCH; }
  __host__ __device__ static constexpr int col0(int arr) { return arr < RNS ? 0 : 1; }
  // first chunk of wave load J
  __host__ __device__ static constexpr int load_start(int J) {
    return J < RNS * NIS ? start(J / NIS) + (J % NIS) * 64 : start(RNS + (J - RNS * NIS) / NIC) + ((J - RNS * NIS) % NIC) * 64;
  }
  // array of chunk q
  __host__ __device__ static constexpr int array_of(int q) {
    int arr = 0;
    for (int k = 1; k < RNA; ++k)
      if (q >= start(k)) arr = k;
    return arr;
  }
  // bytes from the address of (E, column jc) to that of (arr, column jc), in a slot
  __host__ __device__ static constexpr int arr_bytes(int arr) { return (start(arr) - col0(arr) * CPZ) * 16; }
};

// Ghost rule of a y index (-2 <= e <= n1 + 1; uniform over the block): source row and flags
// (bit 0 flips F_y)
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

// the value v of the lane whose byte address (4 x lane) is addr
__device__ __forceinline__ double lane_fetch(int addr, double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
__device__ __forceinline__ float lane_fetch(int addr, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}

// Three LDS reads at byte addresses b_i + O_i, completed before the statement ends (its own
// wait for them).  The ring slots are read this way inside the plane loop: the counted wait and
// the block barrier at the top of the plane already order the reads after the loads of their
// slot.
template <int O0, int O1, int O2>
__device__ __forceinline__ void lds_read3(unsigned b0, unsigned b1, unsigned b2, double x[3]) {
  asm volatile(
      "ds_read_b64 %0, %3 offset:%6\n\tds_read_b64 %1, %4 offset:%7\n\tds_read_b64 %2, %5 offset:%8\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2])
      : "v"(b0), "v"(b1), "v"(b2), "i"(O0), "i"(O1), "i"(O2));
}
template <int O0, int O1, int O2>
__device__ __forceinline__ void lds_read3(unsigned b0, unsigned b1, unsigned b2, float x[3]) {
  asm volatile(
      "ds_read_b32 %0, %3 offset:%6\n\tds_read_b32 %1, %4 offset:%7\n\tds_read_b32 %2, %5 offset:%8\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2])
      : "v"(b0), "v"(b1), "v"(b2), "i"(O0), "i"(O1), "i"(O2));
}
// eight reads: three at b0 + O0..O2, three at b1 + O3..O5, two at b2 + O6, O7
template <int O0, int O1, int O2, int O3, int O4, int O5, int O6, int O7>
__device__ __forceinline__ void lds_read8(unsigned b0, unsigned b1, unsigned b2, double x[8]) {
  asm volatile(
      "ds_read_b64 %0, %8 offset:%11\n\tds_read_b64 %1, %8 offset:%12\n\tds_read_b64 %2, %8 offset:%13\n\t"
      "ds_read_b64 %3, %9 offset:%14\n\tds_read_b64 %4, %9 offset:%15\n\tds_read_b64 %5, %9 offset:%16\n\t"
      "ds_read_b64 %6, %10 offset:%17\n\tds_read_b64 %7, %10 offset:%18\n\ts_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]), "=&v"(x[7])
      : "v"(b0), "v"(b1), "v"(b2), "i"(O0), "i"(O1), "i"(O2), "i"(O3), "i"(O4), "i"(O5), "i"(O6), "i"(O7));
}
template <int O0, int O1, int O2, int O3, int O4, int O5, int O6, int O7>
__device__ __forceinline__ void lds_read8(unsigned b0, unsigned b1, unsigned b2, float x[8]) {
  asm volatile(
      "ds_read_b32 %0, %8 offset:%11\n\tds_read_b32 %1, %8 offset:%12\n\tds_read_b32 %2, %8 offset:%13\n\t"
      "ds_read_b32 %3, %9 offset:%14\n\tds_read_b32 %4, %9 offset:%15\n\tds_read_b32 %5, %9 offset:%16\n\t"
      "ds_read_b32 %6, %10 offset:%17\n\tds_read_b32 %7, %10 offset:%18\n\ts_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]), "=&v"(x[7])
      : "v"(b0), "v"(b1), "v"(b2), "i"(O0), "i"(O1), "i"(O2), "i"(O3), "i"(O4), "i"(O5), "i"(O6), "i"(O7));
}

// a value that is the same in every lane, made opaque to the compiler (kernel-argument values
// selected per lane would otherwise be indexed out of a private copy of the arguments)
__device__ __forceinline__ int uniform_(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ const T* uniform_(const T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = (unsigned)uniform_((int)(unsigned)v), hi = (unsigned)uniform_((int)(unsigned)(v >> 32));
  return (const T*)(((unsigned long long)hi << 32) | lo);
}

#define FM1_LDSP(p) ((__attribute__((address_space(3))) void*)(p))

template <typename S, int LIM>
__global__ void __launch_bounds__(64 * RNW) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 3 : 4)))
k_step_rows(StepArgs<S> a, Geo<S> geo, RowsTile tl) {
  using R = S;
  using L = RowsLds<S>;
  constexpr int RR = RRING;
  constexpr int EPC = L::EPC, CPZ = L::CPZ, ROT = L::ROT;
  constexpr int NW = RNW;                              // waves
  constexpr int NDMA = (L::NLOAD + NW - 1) / NW;       // direct-to-LDS loads per wave and plane
  static_assert(RR == 4, "the plane loop is written for a ring of four slots");
  static_assert(RR * L::SLOTB < 65536, "LDS read offsets");
  __shared__ __align__(16) S ring[RR * L::SLOT];
  __shared__ double DZ[2][4][RTX];                     // dE_matter partials of the waves, per plane parity
  __shared__ double we[NW], wm[NW];
  __shared__ int wu[NW], wp[NW];

  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // wave index (uniform)
  const int c = lane >> 2;                         // lane column (LDS column c + 1)
  const int g = w * 4 + (lane & 3);                // group
  const int up_addr = ((lane + 4) & 63) << 2;      // the lane of column c + 1 (same group)
  const int dn_addr = ((lane - 4) & 63) << 2;      // the lane of column c - 1

  // tile of the block (XCD-aware renumbering)
  const int b = blockIdx.x;
  const int xcd = b & 7, sl = b >> 3;
  const int Lb = xcd * tl.xq + min(xcd, tl.xr) + sl;
  const int tx = Lb % tl.ntx, tm = Lb / tl.ntx;
  const int n0 = a.n[0], n1 = a.n[1];
  const int x0 = tx * (RTX - 2) - 1;               // zone of lane column 0 (LDS column j: zone x0 - 1 + j)
  const int gx = x0 + c;
  const int mbeg = tm * tl.TM, mend = min(mbeg + tl.TM, n1);
  const bool recon = gx <= n0;
  const bool upd = c >= 1 && c <= RTX - 2 && gx < n0;
  const bool do_xf = c <= RTX - 2 && gx + 1 <= n0;
  const bool want_diag = a.p_energy != nullptr;
  ZoneDiag zd;
  const double cdt = a.c * a.dt;
  const R dtR = R(a.dt);
  const R idx0 = geo.idx[0], idx1 = geo.idx[1];
  const R dx0 = geo.dx[0], dx1 = geo.dx[1];
  const R hone[3] = {R(1), R(1), R(1)};
  const double Vz = want_diag ? geo.Wd[0][NG] * geo.Wd[1][NG] * geo.Wd[2][NG] : 0.0;   // uniform zones

  // ghost rule of an x index (-2 <= e <= n0 + 1, per lane): source column and flags (bit 0
  // flips F_x, bit 1 takes the prescribed inflow state)
  int xgs[4], xgf[4];
  for (int k = 0; k < 4; ++k) {
    xgs[k] = uniform_(a.gsrc[0][k]);
    xgf[k] = uniform_(a.gfl[0][k]);
  }
  // (only blocks at an x edge have columns outside the domain)
  const bool x_edge = x0 - 1 < 0 || x0 + RTX > n0 - 1;
  auto x_rule = [&](int e, int& src, int& fl) {
    src = e;
    fl = 0;
    if (x_edge) {
      const bool lo = e < 0, e2 = lo ? e == -2 : e == n0;
      if (lo || e >= n0) {
        src = lo ? (e2 ? xgs[0] : xgs[1]) : (e2 ? xgs[2] : xgs[3]);
        fl = lo ? (e2 ? xgf[0] : xgf[1]) : (e2 ? xgf[2] : xgf[3]);
      }
    }
  };
  // ghost rules of the lane's three columns (left neighbour, own, right neighbour)
  int xs_m, xf_m, xs_o, xf_o, xs_p, xf_p;
  x_rule(min(gx - 1, n0 + 1), xs_m, xf_m);
  x_rule(min(gx, n0 + 1), xs_o, xf_o);
  x_rule(min(gx + 1, n0 + 1), xs_p, xf_p);
  (void)xs_m;
  (void)xs_p;
  R qin[3] = {R(0), R(0), R(0)};   // prescribed inflow state of this group (inflow is on x only)
  if ((xf_m | xf_o | xf_p) & 2)
    for (int k = 0; k < 3; ++k) qin[k] = R(a.inflow[g * 3 + k]);

  // element of (array, LDS column, group) in slot 0: each zone's chunks are rotated by ROT
  // per pair of columns, so that the chunks a wave reads from 8 consecutive columns fall on
  // distinct banks of gfx950's 64 (measured: a third of the conflicts of a rotation per
  // column)
  auto ridx = [&](int arr, int jc, int gg) -> int {
    return (L::start(arr) + (jc - L::col0(arr)) * CPZ + (gg / EPC + ROT * (jc >> 1)) % CPZ) * EPC + gg % EPC;
  };
  const S* const pE = uniform_(a.E);
  const S* const pF0 = uniform_(a.F[0]);
  const S* const pF1 = uniform_(a.F[1]);
  const S* const pK = uniform_(a.kap);
  const S* const pS = uniform_(a.sig);
  const S* const pB = uniform_(a.B);
  auto arr_ptr = [&](int arr) -> const S* {
    return arr == 0 ? pE : arr == 1 ? pF0 : arr == 2 ? pF1 : arr == 3 ? pK : arr == 4 ? pS : pB;
  };

  // direct-to-LDS loads of plane p (any index; ghost planes by the y rule, planes beyond the
  // second ghost layer clamped: their values are never used) into slot s.  Load J copies the
  // 64 chunks from L::load_start(J) on and goes to wave J mod NW; every wave issues NDMA
  // loads (a wave short of one repeats load 0: same bytes to the same place), so that the
  // waits are the same for all waves.  The source of every chunk (array, column with its x
  // rule, part of the zone) is fixed per thread: the array per load (uniform, or two arrays
  // split at a lane where a load runs into the next array) and the element offset xo within
  // the array's row, computed once.
  int xo[NDMA], ksplit[NDMA], kch[NDMA];
  const S* ka[NDMA];
  const S* kb2[NDMA];
#pragma unroll
  for (int k = 0; k < NDMA; ++k) {
    const int J0 = k * NW + w;
    const int J = J0 < L::NLOAD ? J0 : 0;
    const int q0 = L::load_start(J), q = q0 + lane;
    const int arr = L::array_of(q), arr0 = L::array_of(q0);
    const int lc = q - L::start(arr);                  // chunk within the array
    const int jc = lc / CPZ + L::col0(arr);            // LDS column
    const int part = (lc % CPZ + CPZ * ROT * (RTX + 2) - ROT * (jc >> 1)) % CPZ;   // inverse of the rotation
    int xsrc, xfl;
    x_rule(min(x0 - 1 + jc, n0 + 1), xsrc, xfl);
    (void)xfl;
    xo[k] = xsrc * RG + part * EPC;
    kch[k] = q0;
    ksplit[k] = uniform_(arr0 + 1 < RNA ? L::start(arr0 + 1) - q0 : 64);
    ka[k] = uniform_(arr_ptr(arr0));
    kb2[k] = uniform_(arr_ptr(arr0 + 1 < RNA ? arr0 + 1 : arr0));
  }
  auto issue = [&](int p, auto slot_tag) {
    constexpr int s = decltype(slot_tag)::value;
    int ysrc, yfl;
    y_rule(a, min(max(p, -2), n1 + 1), ysrc, yfl);
    (void)yfl;
    const size_t yoff = (size_t)ysrc * n0 * RG;
#pragma unroll
    for (int k = 0; k < NDMA; ++k) {
      const S* src = lane < ksplit[k] ? ka[k] : kb2[k];
      __builtin_amdgcn_global_load_lds((const void*)(src + yoff + xo[k]),
                                       FM1_LDSP(ring + s * L::SLOT + (size_t)kch[k] * EPC), 16, 0, 0);
    }
  };
  // LDS byte addresses of E at the lane's columns c, c + 1, c + 2 and at column min(c + 2, RTX)
  // (the coefficients' last column) in slot 0; the other arrays and slots are constant offsets
  const unsigned lbase = (unsigned)(size_t)FM1_LDSP(ring);
  const unsigned bcm = lbase + ridx(0, c, g) * sizeof(S);
  const unsigned bco = lbase + ridx(0, c + 1, g) * sizeof(S);
  const unsigned bcp = lbase + ridx(0, c + 2, g) * sizeof(S);
  const unsigned bcr = lbase + ridx(0, min(c + 2, RTX), g) * sizeof(S);
  // x rule of a column (only blocks at an x edge have flags) and y flip of a plane (uniform)
  // applied to a state read from the ring
  auto fix_state = [&](R q[4], int xfl, int yflip) {
    if (x_edge) {
      if (xfl & 1) q[1] = -q[1];
      if (yflip) q[2] = -q[2];
      if (xfl & 2) {
        q[0] = qin[0];
        q[1] = qin[1];
        q[2] = qin[2];
      }
    } else if (yflip) {
      q[2] = -q[2];
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
    fix_state(q, xf_o, yf & 1);
  };
  // raw buffer stores of the lane's outputs (lanes of columns that are not updated store at
  // an offset beyond the buffer: dropped)
  const uint32_t nbytes = (uint32_t)((size_t)n0 * n1 * RG * sizeof(S));
  const __amdgpu_buffer_rsrc_t rsE = __builtin_amdgcn_make_buffer_rsrc(a.Eo, 0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rsF0 = __builtin_amdgcn_make_buffer_rsrc(a.Fo[0], 0, (int)nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rsF1 = __builtin_amdgcn_make_buffer_rsrc(a.Fo[1], 0, (int)nbytes, 0x00020000);
  auto store_out = [&](const __amdgpu_buffer_rsrc_t& rs, uint32_t off, S v) {
    if constexpr (sizeof(S) == 8) {
      typedef unsigned v2u __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), rs, (int)off, 0, 0);
    } else {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, (int)off, 0, 0);
    }
  };
  // dE_matter of the updated zones of plane m from the wave partials
  auto dem_store = [&](int m) {
    if (t < RTX) {
      const int zx = x0 + t;
      if (t >= 1 && t <= RTX - 2 && zx < n0) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += DZ[m & 1][k][t];
        a.dEm[(size_t)m * n0 + zx] = -s;
      }
    }
  };
  // Block barrier for LDS data.  The empty asm statements keep the compiler from moving memory
  // accesses across it.
  auto barrier = [&] {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  // ---- prologue: planes mbeg .. mbeg + 2 into the ring, planes mbeg - 2, mbeg - 1 of the
  // own column loaded directly; the register window ----
  issue(mbeg, std::integral_constant<int, 0>{});
  issue(mbeg + 1, std::integral_constant<int, 1>{});
  issue(mbeg + 2, std::integral_constant<int, 2>{});
  R qa[4], qb[4], ksa, ksb;
  load_direct(mbeg - 2, qa, ksa);
  load_direct(mbeg - 1, qb, ksb);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
  barrier();
  R q0[4], q1[4], hiM[4], fPrev[4];
  {
    S v[3];
    lds_read3<0, L::arr_bytes(1), L::arr_bytes(2)>(bco, bco, bco, v);
    q0[0] = R(v[0]);
    q0[1] = R(v[1]);
    q0[2] = R(v[2]);
    q0[3] = R(0);
    fix_state(q0, xf_o, 0);
    lds_read3<L::SLOTB, L::SLOTB + L::arr_bytes(1), L::SLOTB + L::arr_bytes(2)>(bco, bco, bco, v);
    q1[0] = R(v[0]);
    q1[1] = R(v[1]);
    q1[2] = R(v[2]);
    q1[3] = R(0);
    fix_state(q1, xf_o, yflip_of(mbeg + 1));
  }
  S k0v[3];
  lds_read3<L::arr_bytes(3), L::arr_bytes(4), L::arr_bytes(5)>(bco, bco, bco, k0v);
  R ks0 = R(k0v[0]) + R(k0v[1]);
  double ck0 = cdt * (double)k0v[0], cks0 = cdt * ((double)k0v[0] + (double)k0v[1]);
  for (int k = 0; k < 4; ++k) hiM[k] = fPrev[k] = R(0);
  {
    R lo[4], hiP[4];
    reconstruct<R, false, 2, LIM>(a, geo, 1, mbeg - 1 + NG, qa, qb, q0, hone, hone, true, true, lo, hiP);
    reconstruct<R, false, 2, LIM>(a, geo, 1, mbeg + NG, qb, q0, q1, hone, hone, true, true, lo, hiM);
    hll<R, false, 2>(a, 1, hiP, lo, hone, hone, epsilon_of(ksb, ks0, dx1, dx1), fPrev);
  }

  // outputs of the previous plane, stored at the top of the next one (behind the loads of
  // that plane's new slot)
  S Eo_o = S(0), F0_o = S(0), F1_o = S(0);
  uint32_t off_o = 0x7ffffff0u;

  // ---- one plane; s0 = slot of plane m (the slots of m + 1, m + 2, m + 3 follow cyclically) ----
  auto plane = [&](int m, auto sp_tag) {
    constexpr int s0 = decltype(sp_tag)::value, s1 = (s0 + 1) % RR, s2 = (s0 + 2) % RR, s3 = (s0 + 3) % RR;
    constexpr int B0 = s0 * L::SLOTB, B1 = s1 * L::SLOTB, B2 = s2 * L::SLOTB;
    if (m > mbeg) {
      // everything issued at the top of plane m - 1: the loads of plane m + 2 and the stores
      // of plane m - 2
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
      barrier();
    }
    // the slot plane m - 1 has left: plane m + 3, when it is used (up to mend + 1)
    if (m + 3 <= mend + 1) issue(m + 3, std::integral_constant<int, s3>{});
    // the outputs of plane m - 1
    if (m > mbeg) {
      store_out(rsE, off_o, Eo_o);
      store_out(rsF0, off_o, F0_o);
      store_out(rsF1, off_o, F1_o);
      if (a.dEm) dem_store(m - 1);
    }
    // kappa and sigma of m + 1, B of m
    S cf[3];
    lds_read3<B1 + L::arr_bytes(3), B1 + L::arr_bytes(4), B0 + L::arr_bytes(5)>(bco, bco, bco, cf);
    const R ks1 = R(cf[0]) + R(cf[1]);
    const double ck1 = cdt * (double)cf[0], cks1 = cdt * ((double)cf[0] + (double)cf[1]);
    const double jB = ck0 * (double)cf[2];
    // x: reconstruction of the own column, the lower state of column c + 1 and the flux below
    // the own column by lane permutes, the x part of the divergence
    R acc[4] = {R(0), R(0), R(0), R(0)};
    {
      // the neighbouring columns' states, and kappa, sigma of column c + 1 (LDS column RTX + 1
      // has no coefficients; its lane has no x face)
      S xv[8];
      lds_read8<B0, B0 + L::arr_bytes(1), B0 + L::arr_bytes(2), B0, B0 + L::arr_bytes(1), B0 + L::arr_bytes(2),
                B0 + L::arr_bytes(3), B0 + L::arr_bytes(4)>(bcm, bcp, bcr, xv);
      R hiX[4] = {R(0), R(0), R(0), R(0)}, lo[4] = {R(0), R(0), R(0), R(0)};
      if (recon) {
        R qm[4] = {R(xv[0]), R(xv[1]), R(xv[2]), R(0)}, qp[4] = {R(xv[3]), R(xv[4]), R(xv[5]), R(0)};
        fix_state(qm, xf_m, 0);
        fix_state(qp, xf_p, 0);
        reconstruct<R, false, 2, LIM>(a, geo, 0, gx + NG, qm, q0, qp, hone, hone, true, true, lo, hiX);
      }
      R qR[4] = {R(0), R(0), R(0), R(0)};
      for (int v = 0; v < RNC; ++v) qR[v] = lane_fetch(up_addr, lo[v]);
      R fx[4] = {R(0), R(0), R(0), R(0)};
      if (do_xf) {
        const R ksR = R(xv[6]) + R(xv[7]);
        hll<R, false, 2>(a, 0, hiX, qR, hone, hone, epsilon_of(ks0, ksR, dx0, dx0), fx);
      }
      for (int v = 0; v < RNC; ++v) acc[v] += (fx[v] - lane_fetch(dn_addr, fx[v])) * idx0;
    }
    // y: zone m + 1 from q(m + 2), flux at m + 1/2
    R q2[4];
    {
      S v[3];
      lds_read3<B2, B2 + L::arr_bytes(1), B2 + L::arr_bytes(2)>(bco, bco, bco, v);
      q2[0] = R(v[0]);
      q2[1] = R(v[1]);
      q2[2] = R(v[2]);
      q2[3] = R(0);
      fix_state(q2, xf_o, yflip_of(m + 2));
    }
    R fNext[4] = {R(0), R(0), R(0), R(0)}, nHi[4] = {R(0), R(0), R(0), R(0)};
    if (upd) {
      R nLo[4];
      reconstruct<R, false, 2, LIM>(a, geo, 1, m + 1 + NG, q0, q1, q2, hone, hone, true, true, nLo, nHi);
      hll<R, false, 2>(a, 1, hiM, nLo, hone, hone, epsilon_of(ks0, ks1, dx1, dx1), fNext);
    }
    // update of the own zone (stored at the top of the next plane)
    S Eo = S(0), F1[3] = {S(0), S(0), S(0)};
    if (upd) {
      for (int v = 0; v < RNC; ++v) acc[v] += (fNext[v] - fPrev[v]) * idx1;
      R Um[4];
      for (int k = 0; k < 4; ++k) Um[k] = (k < RNC) ? q0[k] - dtR * acc[k] : R(0);
      const double dz = source_zone<S, R, false, 2>(a, geo, gx, m, Um, ck0, cks0, jB, want_diag, Vz, zd, Eo, F1);
      if (a.dEm) {
        double p = dz;
        p += __shfl_xor(p, 1);
        p += __shfl_xor(p, 2);
        if ((lane & 3) == 0) DZ[m & 1][w][c] = p;
      }
    }
    off_o = upd ? (uint32_t)((((size_t)m * n0 + gx) * RG + g) * sizeof(S)) : 0x7ffffff0u;
    Eo_o = Eo;
    F0_o = F1[0];
    F1_o = F1[1];
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
  };
  for (int m = mbeg; m < mend; m += 4) {
    plane(m, std::integral_constant<int, 0>{});
    if (m + 1 < mend) plane(m + 1, std::integral_constant<int, 1>{});
    if (m + 2 < mend) plane(m + 2, std::integral_constant<int, 2>{});
    if (m + 3 < mend) plane(m + 3, std::integral_constant<int, 3>{});
  }
  store_out(rsE, off_o, Eo_o);
  store_out(rsF0, off_o, F0_o);
  store_out(rsF1, off_o, F1_o);
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
size_t rows_lds_bytes(const fornax_m1_desc& D) {
  const size_t s = (D.precision == FORNAX_FP64) ? 8 : 4;
  const size_t slot = (RNS * (RTX + 2) + (RNA - RNS) * RTX) * RG * s;
  return RRING * slot + 2 * 4 * RTX * 8 + RNW * 24;
}

RowsTile make_rows_tile(const fornax_m1_desc& D, int NWX, int TM) {
  RowsTile tl{};
  tl.nblocks = 0;
  if (D.ndim != 2 || D.coord != FORNAX_CARTESIAN || D.ngroups != RG) return tl;
  if (D.wavespeed != FORNAX_WAVESPEED_LIGHT) return tl;   // -+c bounds only
  if (NWX != 1) return tl;
  if (TM < 3) return tl;
  const size_t s = (D.precision == FORNAX_FP64) ? 8 : 4;
  // 32-bit buffer offsets, and the dropped stores' offset beyond every buffer
  if ((size_t)D.n[0] * D.n[1] * RG * s > (size_t)0x7fffff00) return tl;
  tl.NWX = NWX;
  tl.TXB = RTX;
  tl.TM = TM;
  tl.ntx = (D.n[0] + RTX - 3) / (RTX - 2);
  tl.ntm = (D.n[1] + TM - 1) / TM;
  tl.nblocks = tl.ntx * tl.ntm;
  tl.xq = tl.nblocks / 8;
  tl.xr = tl.nblocks % 8;
  tl.nthreads = 64 * RNW;
  tl.lds = rows_lds_bytes(D);
  return tl;
}

RowsTile choose_rows_tile(const fornax_m1_desc& D, int cus) {
  // in float (half the bytes per zone) the tiled kernel is faster (measured on gfx950); the
  // M1-speed bounds are in the tiled kernel only
  if (D.precision != FORNAX_FP64 || D.wavespeed != FORNAX_WAVESPEED_LIGHT) return RowsTile{};
  // planes per block: every block loads TM + 3 planes (two below, two above, one repeated) and
  // holds its CU's LDS share (three blocks per CU); take the TM whose blocks fill whole rounds
  // of the CUs' block slots (at least 90 %) at the least TM + 3 per round, measured best on
  // the 512 x 512 x 16 workload (26 planes: one round of 740 blocks on 256 CUs)
  const int slots = 3 * (cus > 0 ? cus : 256);
  int best = 9;
  double best_cost = 1e30;
  for (int TM = 6; TM <= 32; ++TM) {
    const RowsTile t = make_rows_tile(D, 1, TM);
    if (t.nblocks <= 0) return t;
    const int rounds = (t.nblocks + slots - 1) / slots;
    if ((double)t.nblocks < 0.9 * rounds * slots) continue;
    const double cost = (double)rounds * (TM + 3);
    if (cost < best_cost) {
      best_cost = cost;
      best = TM;
    }
  }
  return make_rows_tile(D, 1, best);
}

template <typename S>
int launch_rows(fornax_m1_ctx* ctx, const Geo<S>& geo, const StepArgs<S>& a, hipStream_t st) {
  const RowsTile& tl = ctx->rows;
  if (tl.nblocks <= 0) return FORNAX_EUNSUPPORTED;
  const bool mm = a.limiter == FORNAX_LIMITER_MINMOD;
  dim3 grid(tl.nblocks), block(tl.nthreads);
  if (mm)
    hipLaunchKernelGGL((k_step_rows<S, FORNAX_LIMITER_MINMOD>), grid, block, 0, st, a, geo, tl);
  else
    hipLaunchKernelGGL((k_step_rows<S, -1>), grid, block, 0, st, a, geo, tl);
  // the reduction bookkeeping of the step (one diagnostics partial per block, summed by the
  // second launch; every block holds all groups of its zones)
  Tile lt{};
  lt.nblocks = tl.nblocks;
  lt.ngb = 1;
  *ctx->last_tile = lt;
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template int launch_rows<double>(fornax_m1_ctx*, const Geo<double>&, const StepArgs<double>&, hipStream_t);
template int launch_rows<float>(fornax_m1_ctx*, const Geo<float>&, const StepArgs<float>&, hipStream_t);

}  // namespace fm1
