// m1_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, double-precision CPU implementation ("the oracle") of one explicit
// transport + implicit interaction step of the multigroup two-moment (M1) radiation
// equations in a static medium, following Skinner, Dolence, Burrows, Radice & Vartanyan,
// "FORNAX: a Flexible Code for Multiphysics Astrophysical Simulations" (ApJS 2019).
//
// Only the tests, the smoke check and the CPU-baseline leg of the benchmark may load this
// library.  It shares no code, header, table or helper with the GPU library, and the GPU
// library never calls it.
//
// Parity with the original FORNAX code is unpinned: no FORNAX code or output exists to
// compare with.  This oracle is pinned instead against closed forms, limits and invariants
// (tests/test_oracle_*.py).  Where the paper leaves a detail open, the reading taken is
// named in a comment starting with "Reading".
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so that every
// operation rounds once, in source order.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

// ------------------------------------------------------------------------------------
// Scalars: double, and a forward-mode dual number so that the same step code yields
// exact Jacobian-vector products (used to check the GPU adjoint).
// ------------------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
static inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
static inline double val(double a) { return a; }
static inline double val(const Dual& a) { return a.v; }
static inline double der(double) { return 0.0; }
static inline double der(const Dual& a) { return a.d; }

// ------------------------------------------------------------------------------------
// Problem description (the oracle's own; not shared with the GPU library)
// ------------------------------------------------------------------------------------
enum { OC_CART = 0, OC_SPH_LOGR = 1 };
enum { OB_OUTFLOW = 0, OB_PERIODIC = 1, OB_REFLECT = 2, OB_INFLOW = 3, OB_AXIS = 4 };
enum { OL_MINMOD = 0, OL_MC = 1, OL_CONST = 2, OL_PPM = 3 };

extern "C" {
struct OrcDesc {
  int32_t ndim;       // 1, 2 or 3 active directions
  int32_t n[3];       // zones per direction (1 for inactive directions)
  int32_t G;          // energy groups
  int32_t coord;      // OC_CART, or OC_SPH_LOGR: x1 = ln r, x2 = theta, x3 = phi
  double lo[3], hi[3];
  int32_t bc_lo[3], bc_hi[3];
  int32_t limiter;    // OL_MINMOD (default), OL_MC, OL_CONST (piecewise constant), OL_PPM (parabolic)
  int32_t closure;    // 0 = M1 (Levermore), 1 = Eddington (P = E/3 I)
  int32_t eps_mode;   // 0 = eq:epsilon as in the paper; 1 = epsilon forced to 1 (plain HLL)
  double c;           // (reduced) speed of light
  int32_t nthreads;   // OpenMP threads (0 = runtime default)
  int32_t integrator; // OI_EULER (default): one forward-Euler push; OI_SSPRK2: Shu-Osher RK2
  int32_t wavespeed;  // OW_LIGHT (default): S_L = -c, S_R = +c; OW_M1: HLLE with the M1 speeds
};
}
enum { OI_EULER = 0, OI_SSPRK2 = 1 };
enum { OW_LIGHT = 0, OW_M1 = 1 };

static const int NG = 2;  // ghost layers required by linear reconstruction

// Romberg integration of a smooth function on [a, b] (the paper precomputes the volume
// averages of the coordinates and connection coefficients this way; Appendix, general
// spherical metric).
static double romberg(const std::function<double(double)>& f, double a, double b) {
  if (a == b) return 0.0;
  const int KMAX = 16;
  double R[KMAX][KMAX];
  double h = b - a;
  R[0][0] = 0.5 * h * (f(a) + f(b));
  for (int k = 1; k < KMAX; ++k) {
    h *= 0.5;
    double s = 0.0;
    long m = 1L << (k - 1);
    for (long i = 1; i <= m; ++i) s += f(a + (2 * i - 1) * h);
    R[k][0] = 0.5 * R[k - 1][0] + h * s;
    double p = 1.0;
    for (int j = 1; j <= k; ++j) {
      p *= 4.0;
      R[k][j] = R[k][j - 1] + (R[k][j - 1] - R[k - 1][j - 1]) / (p - 1.0);
    }
    double diff = std::fabs(R[k][k] - R[k - 1][k - 1]);
    if (k >= 4 && diff <= 1e-15 * std::fabs(R[k][k])) return R[k][k];
  }
  return R[KMAX - 1][KMAX - 1];
}

// ------------------------------------------------------------------------------------
// Geometry (Numerical Discretization; Appendix: general spherical metric, connection
// coefficients).  Both coordinate systems have a separable volume element
// sqrt(g) = w_1(x1) w_2(x2) w_3(x3):
//   Cartesian:            w = 1, h = 1, all connection coefficients vanish;
//   spherical, x1 = ln r: r = e^{x1}, g_11 = g_22 = r^2, g_33 = r^2 sin^2(theta),
//                         sqrt(g) = r^3 sin(theta)   (w_1 = e^{3 x1}, w_2 = |sin x2|, w_3 = 1).
// Per-axis tables cover the extended zone range [-NG, n+NG) so that ghost zones have
// geometry too (uniform continuation of the coordinate grid; |sin| for zones mirrored
// across the polar axis).
// ------------------------------------------------------------------------------------
struct Geom {
  OrcDesc D;
  int n[3];
  std::vector<double> xf[3];   // face coordinate x_{i-1/2}, i in [-NG, n+NG]   (index i+NG)
  std::vector<double> xc[3];   // coordinate centre of zone i                   (index i+NG)
  std::vector<double> W[3];    // integral of w_d over the zone
  std::vector<double> X[3];    // volume centroid <x^d> of the zone
  std::vector<double> wf[3];   // w_d at face i-1/2 (exactly 0 on a polar-axis boundary face)
  // parabolic reconstruction: volume averages <u>, <u^2> of u = x - xc_i over zones i-1, i,
  // i+1 (index 3 (i+NG) + k, k = 0, 1, 2), for every zone with both neighbours in the table
  std::vector<double> pu1[3], pu2[3];
  std::vector<double> r2;      // <r^2> over the zone (axis 0), spherical only
  std::vector<double> s2;      // <sin^2 theta> over the zone (axis 1), spherical only
  // volume-averaged connection coefficients that depend on theta (axis 1):
  std::vector<double> G323;    // <Gamma^3_23> = <cot theta>
  std::vector<double> G133;    // <Gamma^1_33>  (after the angular-momentum override)
  std::vector<double> G233;    // <Gamma^2_33>  (after the angular-momentum override)
  std::vector<double> G222;    // <Gamma^2_22>  (after the d_2 P = 0 balance override)

  bool sph() const { return D.coord == OC_SPH_LOGR; }

  double w(int d, double x) const {
    if (!sph()) return 1.0;
    if (d == 0) return std::exp(3.0 * x);
    if (d == 1) return std::fabs(std::sin(x));
    return 1.0;
  }

  void build(const OrcDesc& desc) {
    D = desc;
    for (int d = 0; d < 3; ++d) n[d] = desc.n[d];
    for (int d = 0; d < 3; ++d) {
      int m = n[d] + 2 * NG;
      double dx = (D.hi[d] - D.lo[d]) / n[d];
      xf[d].assign(m + 1, 0.0);
      xc[d].assign(m, 0.0);
      W[d].assign(m, 0.0);
      X[d].assign(m, 0.0);
      wf[d].assign(m + 1, 0.0);
      for (int e = 0; e <= m; ++e) xf[d][e] = D.lo[d] + (e - NG) * dx;
      for (int e = 0; e < m; ++e) {
        double a = xf[d][e], b = xf[d][e + 1];
        xc[d][e] = 0.5 * (a + b);
        auto wd = [&](double x) { return w(d, x); };
        W[d][e] = romberg(wd, a, b);
        X[d][e] = romberg([&](double x) { return x * w(d, x); }, a, b) / W[d][e];
      }
      for (int e = 0; e <= m; ++e) wf[d][e] = w(d, xf[d][e]);
      pu1[d].assign(3 * m, 0.0);
      pu2[d].assign(3 * m, 0.0);
      if (D.limiter == OL_PPM) {
        for (int e = 1; e + 1 < m; ++e)
          for (int k = 0; k < 3; ++k) {
            const int z = e - 1 + k;
            const double a = xf[d][z], b = xf[d][z + 1], u0 = xc[d][e];
            pu1[d][3 * e + k] = romberg([&](double x) { return (x - u0) * w(d, x); }, a, b) / W[d][z];
            pu2[d][3 * e + k] = romberg([&](double x) { return (x - u0) * (x - u0) * w(d, x); }, a, b) / W[d][z];
          }
      }
      // Reading: a face on the polar axis has zero area (sin theta = 0 there); the
      // floating-point sin(pi) is not exactly 0, so the axis faces are set to 0 exactly.
      if (sph() && d == 1) {
        if (D.bc_lo[1] == OB_AXIS) wf[1][NG] = 0.0;
        if (D.bc_hi[1] == OB_AXIS) wf[1][NG + n[1]] = 0.0;
      }
    }
    if (sph()) {
      int m0 = n[0] + 2 * NG, m1 = n[1] + 2 * NG;
      r2.assign(m0, 0.0);
      for (int e = 0; e < m0; ++e)
        r2[e] = romberg([&](double x) { return std::exp(2.0 * x) * w(0, x); }, xf[0][e], xf[0][e + 1]) / W[0][e];
      s2.assign(m1, 0.0);
      G323.assign(m1, 0.0);
      G133.assign(m1, 0.0);
      G233.assign(m1, 0.0);
      G222.assign(m1, 0.0);
      for (int e = 0; e < m1; ++e) {
        double a = xf[1][e], b = xf[1][e + 1];
        double Wt = W[1][e];
        s2[e] = romberg([&](double x) { double s = std::sin(x); return s * s * w(1, x); }, a, b) / Wt;
        if (e < NG || e >= NG + n[1]) continue;  // connection coefficients: active zones only
        // <Gamma^3_23> = <d_2 ln h_3> = <cot theta>; integrand cot(theta) sin(theta), theta in [0, pi]
        G323[e] = romberg([&](double x) { return std::cos(x); }, a, b) / Wt;
        // Angular-momentum override (eq:angmom and the two settings that follow it):
        // <Gamma^1_33> = -<g33>/<g11> <Gamma^3_13>, <Gamma^2_33> = -<g33>/<g22> <Gamma^3_23>,
        // with <Gamma^3_13> = <d_1 ln h_3> = 1 and <g33>/<g11> = <g33>/<g22> = <sin^2 theta>.
        double G313 = 1.0;
        G133[e] = -s2[e] * G313;
        G233[e] = -s2[e] * G323[e];
        // Balance override (eq:grad2P): <Gamma^2_22> = Delta A_2 / Delta V - <Gamma^3_32>,
        // A_2 = int sqrt(g) dx1 dx3, so Delta A_2 / Delta V = Delta(w_2) / W_2.
        double wa = std::fabs(std::sin(a)), wb = std::fabs(std::sin(b));
        if (D.bc_lo[1] == OB_AXIS && e == NG) wa = 0.0;
        if (D.bc_hi[1] == OB_AXIS && e == NG + n[1] - 1) wb = 0.0;
        G222[e] = (wb - wa) / Wt - G323[e];
      }
    }
  }

  // scale factors h_k at a point (x1, x2)
  void h_point(double x1, double x2, double h[3]) const {
    if (!sph()) { h[0] = h[1] = h[2] = 1.0; return; }
    double r = std::exp(x1);
    h[0] = r;
    h[1] = r;
    h[2] = r * std::fabs(std::sin(x2));
  }
  // cell-centred scale factors h_k = sqrt(<g_kk>) of zone (i, j) (extended indices allowed)
  void h_cell(int i, int j, double h[3]) const {
    if (!sph()) { h[0] = h[1] = h[2] = 1.0; return; }
    double rr = std::sqrt(r2[i + NG]);
    h[0] = rr;
    h[1] = rr;
    h[2] = rr * std::sqrt(s2[j + NG]);
  }
  double volume(int i, int j, int k) const { return W[0][i + NG] * W[1][j + NG] * W[2][k + NG]; }
  // coordinate area int sqrt(g) d^2x of the d-face at index f along d (face f-1/2),
  // the other two indices being zone indices
  double area(int d, const int idx[3]) const {
    double a = 1.0;
    for (int e = 0; e < 3; ++e) a *= (e == d) ? wf[e][idx[e] + NG] : W[e][idx[e] + NG];
    return a;
  }
  // proper length of zone idx across direction d: h_d (cell-centred) * Delta x^d
  double dlen(int d, const int idx[3]) const {
    double h[3];
    h_cell(idx[0], idx[1], h);
    return h[d] * (xf[d][idx[d] + NG + 1] - xf[d][idx[d] + NG]);
  }
  // volume-averaged connection coefficients <Gamma^l_{k m}> of active zone (i, j),
  // indices 0-based (l, k, m in 0..2).  Spherical (x1 = ln r) values from eq:Gamma:
  //   Gamma^1_11 = d_1 ln h_1 = 1, Gamma^2_12 = d_1 ln h_2 = 1, Gamma^3_13 = d_1 ln h_3 = 1,
  //   Gamma^3_23 = d_2 ln h_3 = cot theta, Gamma^1_22 = -g_22,1/(2 g_11) = -1,
  //   Gamma^1_33 = -g_33,1/(2 g_11) = -sin^2 theta, Gamma^2_33 = -g_33,2/(2 g_22) = -sin cos,
  //   Gamma^2_22 = d_2 ln h_2 = 0; symmetric in the lower pair; the rest vanish.
  // theta-dependent ones come from the tables above (with the paper's overrides).
  void gamma(int i, int j, double Gm[3][3][3]) const {
    (void)i;
    std::memset(Gm, 0, sizeof(double) * 27);
    if (!sph()) return;
    int e = j + NG;
    Gm[0][0][0] = 1.0;                                  // Gamma^1_11
    Gm[1][0][1] = Gm[1][1][0] = 1.0;                    // Gamma^2_12
    Gm[2][0][2] = Gm[2][2][0] = 1.0;                    // Gamma^3_13
    Gm[2][1][2] = Gm[2][2][1] = G323[e];                // Gamma^3_23
    Gm[0][1][1] = -1.0;                                 // Gamma^1_22
    Gm[0][2][2] = G133[e];                              // Gamma^1_33
    Gm[1][2][2] = G233[e];                              // Gamma^2_33
    Gm[1][1][1] = G222[e];                              // Gamma^2_22
  }
};

// ------------------------------------------------------------------------------------
// One step
// ------------------------------------------------------------------------------------
template <class T>
struct Ctx {
  const OrcDesc* D;
  const Geom* geo;
  int n[3], G, ndim;
  double c, dt;
  const T* E;
  const T* F[3];
  const T* kap;
  const double* sig;
  const double* B;
  const double* inflow;  // [G][1+ndim]: E and physical flux components of the inflow ghosts
  // prescribed velocity (null for a static medium): vf[d], d < ndim, holds the coordinate
  // components v^0..v^{ndim-1} on the d-faces, [ndim][faces_d], faces_d over (k, j, i) with
  // the d index in 0..n_d, x fastest; nu_edge: the G + 1 group edges in frequency
  const double* vf[3] = {nullptr, nullptr, nullptr};
  const double* nu_edge = nullptr;
  size_t zone(const int m[3]) const { return ((size_t)m[2] * n[1] + m[1]) * n[0] + m[0]; }
};

// State (E, F_1, F_2, F_3) and total opacity of a zone, one index of which may lie in the
// ghost range along one direction.  Ghost rules: Boundary Conditions subsection (periodic
// map, polar-axis copy with a shift of N_phi/2 and sign flips of the theta and phi vector
// components, outflow, Dirichlet inflow).
// Reading: outflow copies the edge zone (zero gradient) for E and every F component;
// reflecting mirrors the zone and flips the normal flux; an inflow ghost holds the
// prescribed E and physical flux (covariant F_k = h_k F^_k with the ghost's own h), and its
// opacity is the edge zone's.
template <class T>
static void zone_state(const Ctx<T>& C, const int idx[3], int g, T q[4], T* ks) {
  int m[3] = {idx[0], idx[1], idx[2]};
  double sg[4] = {1.0, 1.0, 1.0, 1.0};
  int inflow_dir = -1;
  for (int d = 0; d < 3; ++d) {
    int nd = C.n[d];
    if (m[d] >= 0 && m[d] < nd) continue;
    bool low = m[d] < 0;
    int bc = low ? C.D->bc_lo[d] : C.D->bc_hi[d];
    switch (bc) {
      case OB_PERIODIC:
        m[d] = ((m[d] % nd) + nd) % nd;
        break;
      case OB_OUTFLOW:
        m[d] = low ? 0 : nd - 1;
        break;
      case OB_REFLECT:
        m[d] = low ? -1 - m[d] : 2 * nd - 1 - m[d];
        sg[1 + d] = -1.0;
        break;
      case OB_INFLOW:
        inflow_dir = d;
        m[d] = low ? 0 : nd - 1;
        break;
      case OB_AXIS:
        m[d] = low ? -1 - m[d] : 2 * nd - 1 - m[d];
        m[2] = (m[2] + C.n[2] / 2) % C.n[2];
        sg[2] = -1.0;
        sg[3] = -1.0;
        break;
    }
  }
  size_t z = C.zone(m);
  size_t zg = z * C.G + g;
  if (ks) *ks = C.kap[zg] + C.sig[zg];
  if (inflow_dir >= 0) {
    double h[3];
    C.geo->h_cell(idx[0], idx[1], h);
    const double* in = C.inflow + (size_t)g * (1 + C.ndim);
    q[0] = T(in[0]);
    for (int k = 0; k < 3; ++k) q[1 + k] = T(k < C.ndim ? h[k] * in[1 + k] : 0.0);
    return;
  }
  q[0] = C.E[zg];
  for (int k = 0; k < 3; ++k) q[1 + k] = (k < C.ndim) ? T(sg[1 + k]) * C.F[k][zg] : T(0.0);
}

// scale factors at the centre of the d-face at face index f (face f-1/2 along d) of the
// zone row given by idx (other indices = that zone's)
template <class T>
static void face_h(const Ctx<T>& C, int d, const int idx[3], int f, double h[3]) {
  const Geom& G = *C.geo;
  double x1 = (d == 0) ? G.xf[0][f + NG] : G.xc[0][idx[0] + NG];
  double x2 = (d == 1) ? G.xf[1][f + NG] : G.xc[1][idx[1] + NG];
  G.h_point(x1, x2, h);
}

// minmod: 0 unless a and b have the same strict sign, else the one of smaller magnitude (the
// sign test is written without the product a b, which underflows for tiny differences)
template <class T>
static T minmod2(T a, T b) {
  const bool same = (val(a) > 0.0 && val(b) > 0.0) || (val(a) < 0.0 && val(b) < 0.0);
  if (!same) return T(0.0);
  return (std::fabs(val(a)) <= std::fabs(val(b))) ? a : b;
}
template <class T>
static T minmod3(T a, T b, T cc) { return minmod2(a, minmod2(b, cc)); }

// Reading (the paper does not discuss non-realizable face states): a face state is
// realizable when E > 0 and |F^| <= c E, with physical components F^_k = F_k / h_k at the
// face centre.  Faces of zero area (the polar axis) carry no flux and are not checked.
template <class T>
static bool realizable(const Ctx<T>& C, const T q[4], const double h[3]) {
  if (!(val(q[0]) > 0.0)) return false;
  double f2 = 0.0;
  for (int k = 0; k < C.ndim; ++k) {
    double fk = val(q[1 + k]) / h[k];
    f2 += fk * fk;
  }
  double cE = C.c * val(q[0]);
  return f2 <= cE * cE;
}

// Solution of A c = r for a 3x3 matrix of geometry (Cramer's rule).
template <class T>
static void solve3(const double A[3][3], const T r[3], T c[3]) {
  auto det3 = [](const double M[3][3]) {
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  };
  const double det = det3(A);
  for (int j = 0; j < 3; ++j) {
    // column j replaced by r: expand along that column
    double cof[3];
    for (int i = 0; i < 3; ++i) {
      double M[2][2];
      int a = 0;
      for (int ii = 0; ii < 3; ++ii) {
        if (ii == i) continue;
        int b = 0;
        for (int jj = 0; jj < 3; ++jj) {
          if (jj == j) continue;
          M[a][b++] = A[ii][jj];
        }
        ++a;
      }
      cof[i] = (((i + j) & 1) ? -1.0 : 1.0) * (M[0][0] * M[1][1] - M[0][1] * M[1][0]);
    }
    c[j] = (r[0] * T(cof[0]) + r[1] * T(cof[1]) + r[2] * T(cof[2])) / T(det);
  }
}

// Parabolic reconstruction of one component along d (Reconstruction subsection, n = 2), in
// the local coordinate u = x - x_i (x_i the zone's coordinate centre, x_{i-+1/2} = x_i -+ dx/2):
//  1. where q_i is not between q_{i-1} and q_{i+1} the zone is piecewise constant;
//  2. else the parabola p(u) = c0 + c1 u + c2 u^2 with the three zones' volume averages
//     (eq:recon_system1, <u^j> over each zone with the volume element) gives the face states
//     p(u_{i-1/2}) and p(u_{i+1/2});
//  3. if p has its extremum between the centres of zones i-1 and i, the lower face state is
//     reset to make the profile monotone there with zero slope at the centre of zone i-1:
//     the parabola through (x_{i-1}, q_{i-1}) and (x_i, q_i) with zero slope at x_{i-1},
//     evaluated at the face; likewise the upper face state with zones i and i+1 and zero
//     slope at x_{i+1};
//  4. the parabola through the two face states and the zone's average (eq:recon_system2);
//     if its extremum lies inside the zone, the face state nearer to it (the upper one when
//     the extremum is at the centre) is reset so that the parabola through the other face
//     state and the average has zero slope at that face.
// Readings: the extremum test of step 1 is (q_i - q_{i-1})(q_{i+1} - q_i) <= 0; steps 3 and 4
// take the paper's "zero slope" conditions at the places it names, with the neighbours'
// averages as the values at their centres in step 3; "nearest" in step 4 is by position.
template <class T>
static void parabolic_faces(const Geom& G, int d, int e, T qm, T q0, T qp, T& vl, T& vh) {
  vl = vh = q0;
  if (!(val((q0 - qm) * (qp - q0)) > 0.0)) return;
  const double ulo = G.xf[d][e] - G.xc[d][e], uhi = G.xf[d][e + 1] - G.xc[d][e];
  const double um = G.xc[d][e - 1] - G.xc[d][e], up = G.xc[d][e + 1] - G.xc[d][e];
  const double* m1 = &G.pu1[d][3 * e];
  const double* m2 = &G.pu2[d][3 * e];
  // step 2 (eq:recon_system1)
  const double A1[3][3] = {{1.0, m1[0], m2[0]}, {1.0, m1[1], m2[1]}, {1.0, m1[2], m2[2]}};
  const T r1[3] = {qm, q0, qp};
  T c[3];
  solve3(A1, r1, c);
  vl = c[0] + c[1] * T(ulo) + c[2] * T(ulo * ulo);
  vh = c[0] + c[1] * T(uhi) + c[2] * T(uhi * uhi);
  // step 3
  if (val(c[2]) != 0.0) {
    const double us = -val(c[1]) / (2.0 * val(c[2]));
    if (us > um && us < 0.0) {
      const double t = (ulo - um) / (0.0 - um);
      vl = qm + (q0 - qm) * T(t * t);
    } else if (us > 0.0 && us < up) {
      const double t = (uhi - up) / (0.0 - up);
      vh = qp + (q0 - qp) * T(t * t);
    }
  }
  // step 4 (eq:recon_system2)
  const double A2[3][3] = {{1.0, ulo, ulo * ulo}, {1.0, m1[1], m2[1]}, {1.0, uhi, uhi * uhi}};
  const T r2[3] = {vl, q0, vh};
  solve3(A2, r2, c);
  if (val(c[2]) != 0.0) {
    const double us = -val(c[1]) / (2.0 * val(c[2]));
    if (us > ulo && us < uhi) {
      if (us - ulo < uhi - us) {
        // zero slope at the lower face, through the upper face state and the average
        const double A3[3][3] = {{0.0, 1.0, 2.0 * ulo}, {1.0, m1[1], m2[1]}, {1.0, uhi, uhi * uhi}};
        const T r3[3] = {T(0.0), q0, vh};
        solve3(A3, r3, c);
        vl = c[0] + c[1] * T(ulo) + c[2] * T(ulo * ulo);
      } else {
        const double A3[3][3] = {{1.0, ulo, ulo * ulo}, {1.0, m1[1], m2[1]}, {0.0, 1.0, 2.0 * uhi}};
        const T r3[3] = {vl, q0, T(0.0)};
        solve3(A3, r3, c);
        vh = c[0] + c[1] * T(uhi) + c[2] * T(uhi * uhi);
      }
    }
  }
}

// Linear reconstruction along d in the volume coordinate (Reconstruction subsection,
// eq:recon_constraints with n = 1; the paper reconstructs radiation with linear profiles):
// p(x) = q_i + s (x - <x>_i) has the zone's volume average, and the slope s is the minmod
// of the one-sided differences taken between volume centroids.  Face states are
// p(x_{i-1/2}) and p(x_{i+1/2}).
// Reading (non-realizable face states): if either face state of the zone fails the
// realizability test, the zone falls back to piecewise-constant in direction d.  With the
// parabolic option (OL_PPM) the face states come from parabolic_faces instead, with the same
// fallback.
template <class T>
static void reconstruct(const Ctx<T>& C, int d, const int idx[3], int g, T lo[4], T hi[4]) {
  const Geom& G = *C.geo;
  int im[3] = {idx[0], idx[1], idx[2]}, ip[3] = {idx[0], idx[1], idx[2]};
  im[d] -= 1;
  ip[d] += 1;
  T qm[4], q0[4], qp[4];
  zone_state(C, im, g, qm, (T*)nullptr);
  zone_state(C, idx, g, q0, (T*)nullptr);
  zone_state(C, ip, g, qp, (T*)nullptr);
  double Xm = G.X[d][im[d] + NG], X0 = G.X[d][idx[d] + NG], Xp = G.X[d][ip[d] + NG];
  double xlo = G.xf[d][idx[d] + NG], xhi = G.xf[d][idx[d] + NG + 1];
  for (int cpt = 0; cpt < 4; ++cpt) {
    if (C.D->limiter == OL_PPM) {
      if (cpt <= C.ndim) {
        parabolic_faces(G, d, idx[d] + NG, qm[cpt], q0[cpt], qp[cpt], lo[cpt], hi[cpt]);
      } else {
        lo[cpt] = hi[cpt] = q0[cpt];
      }
      continue;
    }
    T s = T(0.0);
    if (cpt <= C.ndim) {
      if (C.D->limiter == OL_MINMOD) {
        T a = (q0[cpt] - qm[cpt]) / T(X0 - Xm);
        T b = (qp[cpt] - q0[cpt]) / T(Xp - X0);
        s = minmod2(a, b);
      } else if (C.D->limiter == OL_MC) {
        T a = (q0[cpt] - qm[cpt]) / T(X0 - Xm);
        T b = (qp[cpt] - q0[cpt]) / T(Xp - X0);
        T ce = (qp[cpt] - qm[cpt]) / T(Xp - Xm);
        s = minmod3(T(2.0) * a, T(2.0) * b, ce);
      }
    }
    lo[cpt] = q0[cpt] + s * T(xlo - X0);
    hi[cpt] = q0[cpt] + s * T(xhi - X0);
  }
  double hlo[3], hhi[3];
  face_h(C, d, idx, idx[d], hlo);
  face_h(C, d, idx, idx[d] + 1, hhi);
  int flo[3] = {idx[0], idx[1], idx[2]}, fhi[3] = {idx[0], idx[1], idx[2]};
  fhi[d] += 1;
  bool ok_lo = (G.area(d, flo) == 0.0) || realizable(C, lo, hlo);
  bool ok_hi = (G.area(d, fhi) == 0.0) || realizable(C, hi, hhi);
  if (!(ok_lo && ok_hi)) {
    for (int cpt = 0; cpt < 4; ++cpt) lo[cpt] = hi[cpt] = q0[cpt];
  }
}

// M1 closure (Formulation: radiation; the paper uses the M1 tensor closure of Dubroca &
// Feugeas / Levermore).  With f = |F^|/(cE) and unit direction n,
//   P^ = E [ (1 - chi)/2 I + (3 chi - 1)/2 n n ],  chi(f) = (3 + 4 f^2) / (5 + 2 sqrt(4 - 3 f^2)),
// which tends to the Eddington closure P^ = E/3 I as f -> 0 (Interaction Terms subsection).
// Reading: f^2 is clamped to 1; for E <= 0 the Eddington value is used.
// Returns the full 3x3 physical-component tensor P^.
template <class T>
static void closure(const Ctx<T>& C, const T q[4], const double h[3], T P[3][3]) {
  T E = q[0];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) P[a][b] = T(0.0);
  if (C.D->closure == 1 || !(val(E) > 0.0)) {
    for (int a = 0; a < 3; ++a) P[a][a] = E / T(3.0);
    return;
  }
  // the reduced flux f = F^/(cE) is formed before any square, so that states with a tiny E
  // (whose squares would underflow) get the same tensor as any scaled copy of them
  T cE = T(C.c) * E;
  T f[3];
  for (int k = 0; k < 3; ++k) f[k] = q[1 + k] / T(h[k] != 0.0 ? h[k] : 1.0) / cE;
  const T fsq = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
  T f2 = fsq;
  if (val(f2) > 1.0) f2 = T(1.0);
  T chi = (T(3.0) + T(4.0) * f2) / (T(5.0) + T(2.0) * sqrt(T(4.0) - T(3.0) * f2));
  T iso = (T(1.0) - chi) / T(2.0);
  T ani = (T(3.0) * chi - T(1.0)) / T(2.0);
  for (int a = 0; a < 3; ++a) P[a][a] = E * iso;
  if (val(fsq) > 0.0) {
    T fm = sqrt(fsq);
    T nn[3] = {f[0] / fm, f[1] / fm, f[2] / fm};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) P[a][b] = P[a][b] + E * ani * nn[a] * nn[b];
  }
}

// Third moment (heat-flux tensor) Q^^{kji} of a state, physical components, in units of F.
// Reading: the paper uses Q^k_{ji} in the frequency-advection terms of the flux rows without
// giving its closure.  It is taken from the same interpolation as the M1 pressure tensor
// (P^ = 3(1 - chi)/2 P_thick + (3 chi - 1)/2 P_thin, P_thick = E/3 I, P_thin = E n n) between
//   Q_thick = (c E / 5) (f^k delta^{ji} + f^j delta^{ki} + f^i delta^{kj}), the third moment of
//             the intensity linear in the direction cosine (c E / 4 pi)(1 + 3 f . Omega), and
//   Q_thin  = c E f n n n, a beam along n (f = 1: c E n n n),
// with f = F^/(cE) (clamped to 1 in length, as in the closure), n = f/|f|:
//   Q^ = |F^_clamped| [ 3(1 - chi)/10 (n^k delta^{ji} + n^j delta^{ki} + n^i delta^{kj})
//                       + (3 chi - 1)/2 n^k n^j n^i ].
// Contracting two indices gives F^ for every chi (Q^{kjj} = |F^| n^k (3(1 - chi)/2 + (3 chi - 1)/2)),
// as it must for any intensity.  E <= 0 or F = 0 (and the Eddington closure's F = 0): Q = 0.
template <class T>
static void closure3(const Ctx<T>& C, const T q[4], const double h[3], T Q[3][3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int d = 0; d < 3; ++d) Q[a][b][d] = T(0.0);
  const T E = q[0];
  if (!(val(E) > 0.0)) return;
  const T cE = T(C.c) * E;
  T f[3];
  for (int k = 0; k < 3; ++k) f[k] = q[1 + k] / T(h[k] != 0.0 ? h[k] : 1.0) / cE;
  const T fsq = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
  if (!(val(fsq) > 0.0)) return;
  const T fm = sqrt(fsq);
  T f2 = fsq;
  if (val(f2) > 1.0) f2 = T(1.0);
  const T fa = (val(fsq) > 1.0) ? T(1.0) : fm;     // |f| after the clamp
  T chi = T(1.0) / T(3.0);
  if (C.D->closure != 1) chi = (T(3.0) + T(4.0) * f2) / (T(5.0) + T(2.0) * sqrt(T(4.0) - T(3.0) * f2));
  const T Fa = cE * fa;
  const T A = Fa * T(3.0) * (T(1.0) - chi) / T(10.0);
  const T B = Fa * (T(3.0) * chi - T(1.0)) / T(2.0);
  const T nn[3] = {f[0] / fm, f[1] / fm, f[2] / fm};
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        T v = B * nn[k] * nn[j] * nn[i];
        if (j == i) v = v + A * nn[k];
        if (k == i) v = v + A * nn[j];
        if (k == j) v = v + A * nn[i];
        Q[k][j][i] = v;
      }
}

// Characteristic speeds (physical units) of the M1 system along direction d at a face state,
// the reading of the HLLE speed bounds (eq:hll names the fastest left- and right-moving wave
// speeds without a formula for them): the eigenvalues of the flux Jacobian of the
// one-dimensional system U = (E, F), flux (F, c^2 chi(f) E), f = F / (c E), taken with the
// state's normal reduced flux f = F^_d / (c E):
//   dFlux/dU = [[0, 1], [c^2 (chi - f chi'), c chi']],
//   lambda = (c / 2) (chi' -+ sqrt(chi'^2 + 4 (chi - f chi'))).
// With the Levermore factor chi = (5 - 2 s) / 3, s = sqrt(4 - 3 f^2), chi' = 2 f / s, the
// discriminant is 16 (s - 1)^2 / (3 s^2), so
//   lambda = (c / s) (f -+ 2 (s - 1) / sqrt(3)),   s - 1 = 3 (1 - f^2) / (1 + s),
// which keeps full accuracy as |f| -> 1 (both speeds -> c f).  |f| is clamped to 1; the
// Eddington closure (chi = 1/3) and a state with E <= 0 give -+c/sqrt(3) and -+c.
template <class T>
static void m1_speeds(const Ctx<T>& C, const T q[4], const double h[3], int d, T& lmin, T& lmax) {
  const T E = q[0];
  const double c = C.c;
  if (!(val(E) > 0.0)) {
    lmin = T(-c);
    lmax = T(c);
    return;
  }
  if (C.D->closure == 1) {
    lmin = T(-c / std::sqrt(3.0));
    lmax = T(c / std::sqrt(3.0));
    return;
  }
  T f = q[1 + d] / T(h[d] != 0.0 ? h[d] : 1.0) / (T(c) * E);
  if (val(f) > 1.0) f = T(1.0);
  if (val(f) < -1.0) f = T(-1.0);
  const T s = sqrt(T(4.0) - T(3.0) * f * f);
  const T w = T(2.0 * std::sqrt(3.0)) * (T(1.0) - f * f) / (T(1.0) + s);   // 2 (s - 1) / sqrt(3)
  lmin = T(c) * (f - w) / s;
  lmax = T(c) * (f + w) / s;
}

template <class T>
static T tmin(T a, T b) { return val(b) < val(a) ? b : a; }
template <class T>
static T tmax(T a, T b) { return val(b) > val(a) ? b : a; }

// ------------------------------------------------------------------------------------
// Prescribed velocity (Riemann Solvers subsection, the advective fluxes and the
// volume-averaged velocity gradient).  The paper takes the face velocities from the
// hydrodynamics' HLLC solve; here they are an input.
// ------------------------------------------------------------------------------------
// Coordinate (contravariant) component v^comp of the velocity on the d-face with face index f
// of the zone row idx (the input holds coordinate components: on spherical grids
// v^1 = v^_r / r, v^2 = v^_theta / r, v^3 = v^_phi / (r sin theta), finite on the polar axis).
// Components along inactive directions are 0.
template <class T>
static double face_vc(const Ctx<T>& C, int d, const int idx[3], int f, int comp) {
  if (comp >= C.ndim) return 0.0;
  int m[3] = {C.n[0], C.n[1], C.n[2]};
  m[d] += 1;
  int fi[3] = {idx[0], idx[1], idx[2]};
  fi[d] = f;
  const size_t nf = (size_t)m[0] * m[1] * m[2];
  const size_t at = ((size_t)fi[2] * m[1] + fi[1]) * m[0] + fi[0];
  return C.vf[d][(size_t)comp * nf + at];
}

// Volume-averaged velocity gradient of active zone idx: the paper's approximation
//   <v^i_{;j}> = <v^i_{,j}> + <Gamma^i_{jk}> <v^k>,
// with each coordinate component linear in x^j across the zone, so that <v^i_{,j}> is the
// difference of v^i between the two j-faces over Delta x^j, and <v^k> the volume average of the
// linear profile of v^k between its two k-faces (its value at the zone's volume centroid
// <x^k>).  Reading: the connection coefficients are the volume averages used by the geometric
// source terms (with the paper's overrides), as the paper computes this term "as in" those.
// Vg[i][j] = <v^i_{;j}>, vbar[k] = <v^k>.
template <class T>
static void vel_grad(const Ctx<T>& C, const int idx[3], double Vg[3][3], double vbar[3]) {
  const Geom& G = *C.geo;
  double dv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int k = 0; k < 3; ++k) vbar[k] = 0.0;
  for (int j = 0; j < C.ndim; ++j) {
    const int e = idx[j] + NG;
    const double x0 = G.xf[j][e], x1 = G.xf[j][e + 1];
    for (int i = 0; i < C.ndim; ++i) {
      const double vlo = face_vc(C, j, idx, idx[j], i);
      const double vhi = face_vc(C, j, idx, idx[j] + 1, i);
      dv[i][j] = (vhi - vlo) / (x1 - x0);
      if (i == j) vbar[j] = vlo + (vhi - vlo) * (G.X[j][e] - x0) / (x1 - x0);
    }
  }
  double Gm[3][3][3];
  G.gamma(idx[0], idx[1], Gm);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = dv[i][j];
      for (int k = 0; k < 3; ++k) s += Gm[i][j][k] * vbar[k];
      Vg[i][j] = s;
    }
}

// Numerical flux across the d-face at face index f (between zones f-1 and f along d) of
// the row idx.  Riemann Solvers subsection: HLL fluxes for the radiation subsystem, the
// energy flux corrected as in eq:hll with epsilon = min(1, 1/tau_cell) (eq:epsilon).
// Written in coordinate components, as in the finite-volume form eq:finite_vol:
//   E   : flux F^d = F^_d / h_d,
//   F_k : flux c^2 P^d_k = c^2 P^^{dk} h_k / h_d      (mixed components of the pressure).
// Reading (wavespeeds, not given in the paper): S_R = +c, S_L = -c physical, i.e. +-c/h_d
// in the coordinate x^d; or, as an option, HLLE bounds from the M1 characteristic speeds of
// both face states, S_L = min(0, lambda_-(L), lambda_-(R)), S_R = max(0, lambda_+(L),
// lambda_+(R)) (m1_speeds), also divided by h_d.  Reading (tau_cell): arithmetic mean of (kappa + sigma) of the two
// zones times the mean proper zone width h_d Delta x^d of the two.  Reading: epsilon enters
// the energy flux only (the Riemann Solvers subsection applies it to the energy fluxes,
// eq:hll with eq:epsilon).
// A face of zero area returns a zero flux.

template <class T>
static void face_flux(const Ctx<T>& C, int d, const int row[3], int f, int g, T flux[4]) {
  const Geom& G = *C.geo;
  for (int k = 0; k < 4; ++k) flux[k] = T(0.0);
  int fi[3] = {row[0], row[1], row[2]};
  fi[d] = f;
  if (G.area(d, fi) == 0.0) return;
  int ia[3] = {row[0], row[1], row[2]}, ib[3] = {row[0], row[1], row[2]};
  ia[d] = f - 1;
  ib[d] = f;
  T alo[4], ahi[4], blo[4], bhi[4];
  reconstruct(C, d, ia, g, alo, ahi);
  reconstruct(C, d, ib, g, blo, bhi);
  const T* qL = ahi;  // left state: upper face of zone f-1
  const T* qR = blo;  // right state: lower face of zone f
  double h[3];
  face_h(C, d, fi, f, h);
  T PL[3][3], PR[3][3];
  closure(C, qL, h, PL);
  closure(C, qR, h, PR);
  // wavespeeds in the coordinate x^d
  T SR = T(C.c / h[d]), SL = T(-C.c / h[d]);
  if (C.D->wavespeed == OW_M1) {
    T aL, bL, aR, bR;
    m1_speeds(C, qL, h, d, aL, bL);
    m1_speeds(C, qR, h, d, aR, bR);
    SL = tmin(T(0.0), tmin(aL, aR)) / T(h[d]);
    SR = tmax(T(0.0), tmax(bL, bR)) / T(h[d]);
  }
  // epsilon (eq:epsilon)
  T ksa, ksb, tmp[4];
  zone_state(C, ia, g, tmp, &ksa);
  zone_state(C, ib, g, tmp, &ksb);
  double dl = 0.5 * (G.dlen(d, ia) + G.dlen(d, ib));
  T tau = T(0.5) * (ksa + ksb) * T(dl);
  T eps = T(1.0);
  if (C.D->eps_mode == 0 && val(tau) > 1.0) eps = T(1.0) / tau;
  // energy: F^d_{L,R} = F^_d / h_d = F_d / h_d^2 (coordinate contravariant component)
  T FdL = qL[1 + d] / T(h[d] * h[d]);
  T FdR = qR[1 + d] / T(h[d] * h[d]);
  flux[0] = (SR * FdL - SL * FdR + eps * (SR * SL) * (qR[0] - qL[0])) / (SR - SL);
  // flux components: conserved F_k, flux c^2 P^d_k, plain HLL
  for (int k = 0; k < C.ndim; ++k) {
    double hk = h[k] != 0.0 ? h[k] : 1.0;
    T PdkL = T(C.c * C.c) * PL[d][k] * T(hk / h[d]);
    T PdkR = T(C.c * C.c) * PR[d][k] * T(hk / h[d]);
    flux[1 + k] = (SR * PdkL - SL * PdkR + (SR * SL) * (qR[1 + k] - qL[1 + k])) / (SR - SL);
  }
  // advective fluxes (v E) and (v F_k) of the comoving-frame moments: the face's normal
  // velocity v^d times the reconstructed state on its upwind side, the left one for v^d >= 0
  if (C.vf[0]) {
    const double vd = face_vc(C, d, fi, f, d);
    const T* qu = (vd >= 0.0) ? qL : qR;
    flux[0] = flux[0] + T(vd) * qu[0];
    for (int k = 0; k < C.ndim; ++k) flux[1 + k] = flux[1 + k] + T(vd) * qu[1 + k];
  }
}

// Explicit update of one zone-group (Algorithmic Steps, step 1, radiation rows, v = 0):
// dU/dt = -(1/V) sum_d [A_d F^d]_{i-1/2}^{i+1/2} (eq:finite_vol) plus, for the covariant
// flux components, the volume-averaged geometric source c^2 <Gamma^l_{km}> P^m_l(<U>)
// (Numerical Discretization; covariant form of the momentum equation).  Forward Euler push.
template <class T>
static void explicit_update(const Ctx<T>& C, const int idx[3], int g, T Um[4]) {
  const Geom& G = *C.geo;
  T q[4];
  zone_state(C, idx, g, q, (T*)nullptr);
  double V = G.volume(idx[0], idx[1], idx[2]);
  T div[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int d = 0; d < C.ndim; ++d) {
    T flo[4], fhi[4];
    face_flux(C, d, idx, idx[d], g, flo);
    face_flux(C, d, idx, idx[d] + 1, g, fhi);
    int ilo[3] = {idx[0], idx[1], idx[2]}, ihi[3] = {idx[0], idx[1], idx[2]};
    ihi[d] += 1;
    double Alo = G.area(d, ilo), Ahi = G.area(d, ihi);
    for (int k = 0; k <= C.ndim; ++k) div[k] = div[k] + (T(Ahi) * fhi[k] - T(Alo) * flo[k]);
  }
  for (int k = 0; k <= C.ndim; ++k) Um[k] = q[k] - T(C.dt) * div[k] / T(V);
  for (int k = C.ndim + 1; k < 4; ++k) Um[k] = T(0.0);
  if (G.sph()) {
    // geometric source c^2 sum_{l,m} <Gamma^l_{km}> P^m_l, P^m_l = P^^{ml} h_l / h_m,
    // cell-centred h_k = sqrt(<g_kk>)
    double h[3], Gm[3][3][3];
    G.h_cell(idx[0], idx[1], h);
    G.gamma(idx[0], idx[1], Gm);
    T P[3][3];
    closure(C, q, h, P);
    for (int k = 0; k < C.ndim; ++k) {
      T s = T(0.0);
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m)
          if (Gm[l][k][m] != 0.0) s = s + T(Gm[l][k][m]) * P[m][l] * T(h[l] / h[m]);
      Um[1 + k] = Um[1 + k] + T(C.dt) * T(C.c * C.c) * s;
    }
  }
  if (C.vf[0]) {
    // velocity terms of the flux rows in Step 1: the connection part of the covariant
    // divergence (v^i F_k)_{;i}, i.e. + <Gamma^l_{ik}> <v^i> F_l, and - <v^i_{;k}> F_i
    // (eq:rad_mom2), with the zone's own state
    double Vg[3][3], vb[3], Gm[3][3][3];
    vel_grad(C, idx, Vg, vb);
    G.gamma(idx[0], idx[1], Gm);
    for (int k = 0; k < C.ndim; ++k) {
      T s = T(0.0);
      for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l)
          if (Gm[l][i][k] != 0.0) s = s + T(Gm[l][i][k] * vb[i]) * q[1 + l];
      for (int i = 0; i < 3; ++i) s = s - T(Vg[i][k]) * q[1 + i];
      Um[1 + k] = Um[1 + k] + T(C.dt) * s;
    }
  }
}

// Implicit interaction update (Interaction Terms subsection): backward Euler for each group,
// eq:be_update with a prescribed emissivity j = c kappa B (Reading: the emission is given as
// a group-integrated source function B, Kirchhoff's law, so that E -> B in the thick limit),
// and the flux update F^{n+1} = F^- / (1 + c dt (kappa + sigma)).
template <class T>
static void implicit_source(T E_m, const T F_m[3], T kap, double sig, double B, double c, double dt, int ndim,
                            T& E1, T F1[3]) {
  T j = T(c) * kap * T(B);
  E1 = (E_m + T(dt) * j) / (T(1.0) + T(c * dt) * kap);
  for (int k = 0; k < 3; ++k)
    F1[k] = (k < ndim) ? F_m[k] / (T(1.0) + T(c * dt) * (kap + T(sig))) : T(0.0);
}

// The interaction update of one zone-group from its explicitly updated state U^-.
template <class T>
static void source_of(const Ctx<T>& C, const int idx[3], int g, const T Um[4], T Un1[4]) {
  size_t zg = C.zone(idx) * C.G + g;
  T Fm[3] = {Um[1], Um[2], Um[3]}, F1[3];
  T E1;
  implicit_source(Um[0], Fm, C.kap[zg], C.sig[zg], C.B[zg], C.c, C.dt, C.ndim, E1, F1);
  Un1[0] = E1;
  for (int k = 0; k < 3; ++k) Un1[1 + k] = F1[k];
}

// One step of one zone-group with the forward-Euler push: U^- = U^n + dt L(U^n), then the
// interaction update.
template <class T>
static void zone_step(const Ctx<T>& C, const int idx[3], int g, T Un1[4], T* Em_out) {
  T Um[4];
  explicit_update(C, idx, g, Um);
  source_of(C, idx, g, Um, Un1);
  if (Em_out) *Em_out = Um[0];
}

// The explicit part with Shu & Osher's second-order TVD Runge-Kutta scheme (Numerical
// Discretization: the paper's explicit integrator; Algorithmic Steps: the Euler push is its
// first-order case), written as
//   U* = U^n + dt L(U^n),   U^- = (U^n + (U* + dt L(U*))) / 2,
// with the stiff interaction update applied once, to U^-, as in the Euler push.
// Stage 1 over every zone-group: U* into Es, Fs (boundary rules then apply to U* as to U^n).
template <class T>
static void rk2_stage1(const Ctx<T>& C, std::vector<T>& Es, std::vector<std::vector<T>>& Fs) {
  long nz = (long)C.n[0] * C.n[1] * C.n[2];
  Es.assign((size_t)nz * C.G, T(0.0));
  Fs.assign(3, std::vector<T>());
  for (int k = 0; k < C.ndim; ++k) Fs[k].assign((size_t)nz * C.G, T(0.0));
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    for (int g = 0; g < C.G; ++g) {
      T Us[4];
      explicit_update(C, idx, g, Us);
      size_t zg = (size_t)z * C.G + g;
      Es[zg] = Us[0];
      for (int k = 0; k < C.ndim; ++k) Fs[k][zg] = Us[1 + k];
    }
  }
}

// Stage 2 of one zone-group from the stage-1 context C1 (state U*): U^- as above, then the
// interaction update.  C holds U^n.
template <class T>
static void rk2_zone(const Ctx<T>& C, const Ctx<T>& C1, const int idx[3], int g, T Un1[4], T* Em_out) {
  T Uss[4], Um[4];
  explicit_update(C1, idx, g, Uss);
  size_t zg = C.zone(idx) * C.G + g;
  Um[0] = T(0.5) * (C.E[zg] + Uss[0]);
  for (int k = 0; k < 3; ++k) Um[1 + k] = (k < C.ndim) ? T(0.5) * (C.F[k][zg] + Uss[1 + k]) : T(0.0);
  source_of(C, idx, g, Um, Un1);
  if (Em_out) *Em_out = Um[0];
}

static void set_threads(const OrcDesc* D) {
#ifdef _OPENMP
  if (D->nthreads > 0) omp_set_num_threads(D->nthreads);
#else
  (void)D;
#endif
}

// diagnostics record (oracle's own layout)
extern "C" {
struct OrcDiag {
  double energy_total;     // sum_i V_i sum_g E_g^{n+1}
  double max_f;            // max |F^|/(cE) over zone-groups with E > 0 (cell-centred h)
  int64_t n_unrealizable;  // #(|F^| > cE (1 + 8u)), u = 2^-53
  int64_t n_nonpositive;   // #(E <= 0)
};
}

// One full step on every zone.  E, F[k], kappa, sigma, B: [n2][n1][n0][G] (G innermost).
template <class T>
static void full_step(const OrcDesc* D, const Geom& geo, const T* E, const T* const* F, const T* kap, const double* sig,
                      const double* B, const double* inflow, double dt, T* Eo, T* const* Fo, double* dEm,
                      OrcDiag* diag) {
  Ctx<T> C;
  C.D = D;
  C.geo = &geo;
  for (int d = 0; d < 3; ++d) C.n[d] = D->n[d];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = dt;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (k < D->ndim) ? F[k] : nullptr;
  C.kap = kap;
  C.sig = sig;
  C.B = B;
  C.inflow = inflow;
  long nz = (long)C.n[0] * C.n[1] * C.n[2];
  std::vector<double> Em_all(nz * C.G);
  set_threads(D);
  const bool rk2 = D->integrator == OI_SSPRK2;
  std::vector<T> Es;
  std::vector<std::vector<T>> Fs;
  Ctx<T> C1 = C;
  if (rk2) {
    rk2_stage1(C, Es, Fs);
    C1.E = Es.data();
    for (int k = 0; k < D->ndim; ++k) C1.F[k] = Fs[k].data();
  }
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    for (int g = 0; g < C.G; ++g) {
      T U1[4], Em;
      if (rk2)
        rk2_zone(C, C1, idx, g, U1, &Em);
      else
        zone_step(C, idx, g, U1, &Em);
      size_t zg = (size_t)z * C.G + g;
      Eo[zg] = U1[0];
      for (int k = 0; k < D->ndim; ++k) Fo[k][zg] = U1[1 + k];
      Em_all[zg] = val(Em);
    }
  }
  // diagnostics, summed serially in zone-major then group order
  if (diag || dEm) {
    double etot = 0.0, maxf = 0.0;
    int64_t nun = 0, nnp = 0;
    const double u = std::ldexp(1.0, -53);
    for (long z = 0; z < nz; ++z) {
      int i = (int)(z % C.n[0]), j = (int)((z / C.n[0]) % C.n[1]), k = (int)(z / ((long)C.n[0] * C.n[1]));
      double V = geo.volume(i, j, k);
      double h[3];
      geo.h_cell(i, j, h);
      double esum = 0.0, dsum = 0.0;
      for (int g = 0; g < C.G; ++g) {
        size_t zg = (size_t)z * C.G + g;
        double e = val(Eo[zg]);
        esum += e;
        dsum += e - Em_all[zg];
        // f = |F^|/(cE) from the reduced components (no squares of tiny values)
        if (e > 0.0) {
          double f2 = 0.0;
          for (int kk = 0; kk < D->ndim; ++kk) {
            double fk = val(Fo[kk][zg]) / h[kk] / (C.c * e);
            f2 += fk * fk;
          }
          double fm = std::sqrt(f2);
          maxf = std::max(maxf, fm);
          if (fm > 1.0 + 8.0 * u) nun++;
        } else {
          nnp++;
          bool fz = true;
          for (int kk = 0; kk < D->ndim; ++kk) fz = fz && val(Fo[kk][zg]) == 0.0;
          if (e < 0.0 || !fz) nun++;
        }
      }
      etot += V * esum;
      if (dEm) dEm[z] = -dsum;
    }
    if (diag) {
      diag->energy_total = etot;
      diag->max_f = maxf;
      diag->n_unrealizable = nun;
      diag->n_nonpositive = nnp;
    }
  }
}

// ------------------------------------------------------------------------------------
// Velocity-dependent terms (prescribed velocity)
// ------------------------------------------------------------------------------------
// Frequency advection of the groups of one zone (Algorithmic Steps, Step 2, eq:freq_adv_system
// with the upwind intergroup fluxes), applied to the zone's state U[g] after Step 1:
//   E_g   <- E_g   + dt ( Phi_{g+1/2} - Phi_{g-1/2} - <v^i_{;j}> P^j_{g i} ),
//   F_g,j <- F_g,j + dt ( Psi_{j,g+1/2} - Psi_{j,g-1/2} ),
//   Phi_{g-1/2}   = nu_{g-1/2} sum_{ij} <v^i_{;j}> <P^j_i>_{L or R},
//   Psi_{j,g-1/2} = nu_{g-1/2} sum_{ik} <v^i_{;k}> <Q^k_{ji}>_{L or R},
// the left (lower group) side where the velocity-gradient component is negative, the right
// side otherwise; <X>_g = X_g / dnu_g the group's spectral density.  Mixed components from the
// physical tensors of U[g] with cell-centred h: P^j_i = P^^{ji} h_i / h_j,
// Q^k_{ji} = Q^^{kji} h_j h_i / h_k (closure3).
// Readings:
//  - Since the side depends only on the zone's <v^i_{;j}>, each edge value is reconstructed for
//    the two parts of the contraction, over the components with <v^i_{;j}> < 0 (X-, Y-_j) and
//    the rest (X+, Y+_j): each linear in nu across the group with the minmod-limited slope of
//    the neighbouring groups' values over their centre distances (a TVD limiter, as the
//    paper's Doppler test describes for its frequency advection), zero
//    slope in the first and last group; in one Cartesian dimension these are <P^x_x> and
//    <Q^x_{xx}> themselves.  Phi_{g-1/2} = nu_{g-1/2} (X-_{g-1} at its upper edge + X+_g at its
//    lower edge), Psi likewise.
//  - The frequency range is closed: Phi = Psi = 0 at nu_{1/2} and nu_{G+1/2}, so the intergroup
//    fluxes only move energy and momentum between groups.
//  - The flux rows take the intergroup term of eq:rad_mom2 only; the local term
//    -<v^i_{;k}> Q^k_{ji} that the listing of Step 1 adds would count it twice (the group sum of
//    d_nu(nu Q) vanishes) and would break the free-streaming balance F = cE.
static void freq_advect(const Ctx<double>& C, const int idx[3], std::vector<double>& U) {
  const int G = C.G;
  const int nd = C.ndim;
  double Vg[3][3], vb[3], h[3];
  vel_grad(C, idx, Vg, vb);
  C.geo->h_cell(idx[0], idx[1], h);
  // parts: 0 = X-, 1 = X+, 2 + 2 j = Y-_j, 3 + 2 j = Y+_j
  const int np = 2 + 2 * nd;
  std::vector<std::vector<double>> X(np, std::vector<double>(G, 0.0));
  std::vector<double> vP(G), nuc(G), dnu(G);
  for (int g = 0; g < G; ++g) {
    nuc[g] = 0.5 * (C.nu_edge[g] + C.nu_edge[g + 1]);
    dnu[g] = C.nu_edge[g + 1] - C.nu_edge[g];
    const double* q = &U[(size_t)4 * g];
    double P[3][3], Q[3][3][3];
    closure(C, q, h, P);
    closure3(C, q, h, Q);
    double vp = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double t = Vg[i][j] * (P[j][i] * h[i] / h[j]);
        vp += t;
        X[Vg[i][j] < 0.0 ? 0 : 1][g] += t;
      }
    for (int j = 0; j < nd; ++j)
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
          const double t = Vg[i][k] * (Q[k][j][i] * h[j] * h[i] / h[k]);
          X[Vg[i][k] < 0.0 ? 2 + 2 * j : 3 + 2 * j][g] += t;
        }
    vP[g] = vp;
    for (int a = 0; a < np; ++a) X[a][g] /= dnu[g];
  }
  auto slope = [&](const std::vector<double>& Xa, int g) {
    if (g == 0 || g == G - 1) return 0.0;
    return minmod2((Xa[g + 1] - Xa[g]) / (nuc[g + 1] - nuc[g]), (Xa[g] - Xa[g - 1]) / (nuc[g] - nuc[g - 1]));
  };
  // edge fluxes of the energy (row 0) and of the flux components (rows 1 + j)
  std::vector<std::vector<double>> Phi(1 + nd, std::vector<double>(G + 1, 0.0));
  for (int r = 0; r <= nd; ++r) {
    const std::vector<double>& Xm = X[2 * r];
    const std::vector<double>& Xp = X[2 * r + 1];
    for (int g = 1; g < G; ++g) {
      const double xm_up = Xm[g - 1] + slope(Xm, g - 1) * (0.5 * dnu[g - 1]);
      const double xp_lo = Xp[g] - slope(Xp, g) * (0.5 * dnu[g]);
      Phi[r][g] = C.nu_edge[g] * (xm_up + xp_lo);
    }
  }
  for (int g = 0; g < G; ++g) {
    U[(size_t)4 * g] += C.dt * (Phi[0][g + 1] - Phi[0][g] - vP[g]);
    for (int j = 0; j < nd; ++j) U[(size_t)4 * g + 1 + j] += C.dt * (Phi[1 + j][g + 1] - Phi[1 + j][g]);
  }
}

// One full step with the velocity terms (Algorithmic Steps 1 to 4, Euler push, matter fixed):
// Step 1 with the advective fluxes and the flux-row velocity terms, Step 2 on its result,
// then the interaction update (Steps 3 and 4) of U^- = the state after Step 2.
static void full_step_v(const OrcDesc* D, const Geom& geo, const double* E, const double* const* F,
                        const double* kap, const double* sig, const double* B, const double* inflow,
                        const double* const* vf, const double* nu_edge, double dt, double* Eo, double* const* Fo,
                        double* dEm, OrcDiag* diag) {
  Ctx<double> C;
  C.D = D;
  C.geo = &geo;
  for (int d = 0; d < 3; ++d) C.n[d] = D->n[d];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = dt;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (k < D->ndim) ? F[k] : nullptr;
  C.kap = kap;
  C.sig = sig;
  C.B = B;
  C.inflow = inflow;
  for (int k = 0; k < 3; ++k) C.vf[k] = (k < D->ndim) ? vf[k] : nullptr;
  C.nu_edge = nu_edge;
  const long nz = (long)C.n[0] * C.n[1] * C.n[2];
  const int G = C.G;
  std::vector<double> Em_all((size_t)nz * G);
  set_threads(D);
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    std::vector<double> U((size_t)4 * G);
    for (int g = 0; g < G; ++g) explicit_update(C, idx, g, &U[(size_t)4 * g]);
    freq_advect(C, idx, U);
    for (int g = 0; g < G; ++g) {
      double U1[4];
      source_of(C, idx, g, &U[(size_t)4 * g], U1);
      const size_t zg = (size_t)z * G + g;
      Eo[zg] = U1[0];
      for (int k = 0; k < D->ndim; ++k) Fo[k][zg] = U1[1 + k];
      Em_all[zg] = U[(size_t)4 * g];
    }
  }
  if (diag || dEm) {
    double etot = 0.0, maxf = 0.0;
    int64_t nun = 0, nnp = 0;
    const double u = std::ldexp(1.0, -53);
    for (long z = 0; z < nz; ++z) {
      int i = (int)(z % C.n[0]), j = (int)((z / C.n[0]) % C.n[1]), k = (int)(z / ((long)C.n[0] * C.n[1]));
      double h[3];
      geo.h_cell(i, j, h);
      double esum = 0.0, dsum = 0.0;
      for (int g = 0; g < G; ++g) {
        const size_t zg = (size_t)z * G + g;
        const double e = Eo[zg];
        esum += e;
        dsum += e - Em_all[zg];
        if (e > 0.0) {
          double f2 = 0.0;
          for (int kk = 0; kk < D->ndim; ++kk) {
            double fk = Fo[kk][zg] / h[kk] / (C.c * e);
            f2 += fk * fk;
          }
          double fm = std::sqrt(f2);
          maxf = std::max(maxf, fm);
          if (fm > 1.0 + 8.0 * u) nun++;
        } else {
          nnp++;
          bool fz = true;
          for (int kk = 0; kk < D->ndim; ++kk) fz = fz && Fo[kk][zg] == 0.0;
          if (e < 0.0 || !fz) nun++;
        }
      }
      etot += geo.volume(i, j, k) * esum;
      if (dEm) dEm[z] = -dsum;
    }
    if (diag) {
      diag->energy_total = etot;
      diag->max_f = maxf;
      diag->n_unrealizable = nun;
      diag->n_nonpositive = nnp;
    }
  }
}

// ------------------------------------------------------------------------------------
// C API used by the tests (through ctypes)
// ------------------------------------------------------------------------------------
extern "C" {

// Largest stable time step for a given CFL number.
// Reading (the paper only says the light-crossing time of a zone sets the step):
//   dt = cfl / max_i sum_d c / (h_d Delta x^d)_i  over active zones.
double orc_max_dt(const OrcDesc* D, double cfl) {
  Geom geo;
  geo.build(*D);
  double worst = 0.0;
  for (int k = 0; k < D->n[2]; ++k)
    for (int j = 0; j < D->n[1]; ++j)
      for (int i = 0; i < D->n[0]; ++i) {
        int idx[3] = {i, j, k};
        double s = 0.0;
        for (int d = 0; d < D->ndim; ++d) s += D->c / geo.dlen(d, idx);
        worst = std::max(worst, s);
      }
  return cfl / worst;
}

// nsteps full steps.  F and Fo are arrays of ndim pointers.  dEm (per zone, nullable) and
// diag (nullable) describe the last step.
int orc_run(const OrcDesc* D, const double* E, const double* const* F, const double* kap, const double* sig,
            const double* B, const double* inflow, double dt, int nsteps, double* Eo, double* const* Fo, double* dEm,
            OrcDiag* diag) {
  Geom geo;
  geo.build(*D);
  size_t nzg = (size_t)D->n[0] * D->n[1] * D->n[2] * D->G;
  std::vector<double> Ea(E, E + nzg), Eb(nzg);
  std::vector<std::vector<double>> Fa(3), Fb(3);
  for (int k = 0; k < D->ndim; ++k) {
    Fa[k].assign(F[k], F[k] + nzg);
    Fb[k].assign(nzg, 0.0);
  }
  for (int s = 0; s < nsteps; ++s) {
    const double* Fin[3] = {nullptr, nullptr, nullptr};
    double* Fout[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < D->ndim; ++k) {
      Fin[k] = Fa[k].data();
      Fout[k] = Fb[k].data();
    }
    bool last = (s == nsteps - 1);
    full_step<double>(D, geo, Ea.data(), Fin, kap, sig, B, inflow, dt, Eb.data(), Fout, last ? dEm : nullptr,
                      last ? diag : nullptr);
    std::swap(Ea, Eb);
    for (int k = 0; k < D->ndim; ++k) std::swap(Fa[k], Fb[k]);
  }
  std::memcpy(Eo, Ea.data(), nzg * sizeof(double));
  for (int k = 0; k < D->ndim; ++k) std::memcpy(Fo[k], Fa[k].data(), nzg * sizeof(double));
  return 0;
}

// One step evaluated only at the listed zones (flat zone index z = (k n1 + j) n0 + i).
// Outputs U^{n+1} as [nsel][G] per component, and U^- (after the explicit update) likewise.
int orc_step_zones(const OrcDesc* D, const double* E, const double* const* F, const double* kap, const double* sig,
                   const double* B, const double* inflow, double dt, int nsel, const int64_t* zones, double* Eo,
                   double* const* Fo, double* Em_out) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  C.D = D;
  C.geo = &geo;
  for (int d = 0; d < 3; ++d) C.n[d] = D->n[d];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = dt;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (k < D->ndim) ? F[k] : nullptr;
  C.kap = kap;
  C.sig = sig;
  C.B = B;
  C.inflow = inflow;
  set_threads(D);
  // SSP-RK2: stage 1 everywhere (the stencil of a zone's stage 2 reaches two zones out)
  const bool rk2 = D->integrator == OI_SSPRK2;
  std::vector<double> Es;
  std::vector<std::vector<double>> Fs;
  Ctx<double> C1 = C;
  if (rk2) {
    rk2_stage1(C, Es, Fs);
    C1.E = Es.data();
    for (int k = 0; k < D->ndim; ++k) C1.F[k] = Fs[k].data();
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int s = 0; s < nsel; ++s) {
    long z = (long)zones[s];
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    for (int g = 0; g < C.G; ++g) {
      double U1[4], Em;
      if (rk2)
        rk2_zone(C, C1, idx, g, U1, &Em);
      else
        zone_step(C, idx, g, U1, &Em);
      Eo[(size_t)s * C.G + g] = U1[0];
      for (int k = 0; k < D->ndim; ++k) Fo[k][(size_t)s * C.G + g] = U1[1 + k];
      if (Em_out) Em_out[(size_t)s * C.G + g] = Em;
    }
  }
  return 0;
}

// Numerical face fluxes (coordinate flux densities, area not included) for direction d.
// out: [faces along d][G][1+ndim], faces enumerated with the d index running 0..n_d and the
// other two indices over the active zones, x fastest.
int orc_flux(const OrcDesc* D, const double* E, const double* const* F, const double* kap, const double* sig,
             const double* B, const double* inflow, int d, double* out) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  C.D = D;
  C.geo = &geo;
  for (int e = 0; e < 3; ++e) C.n[e] = D->n[e];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = 0.0;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (k < D->ndim) ? F[k] : nullptr;
  C.kap = kap;
  C.sig = sig;
  C.B = B;
  C.inflow = inflow;
  int m[3] = {D->n[0], D->n[1], D->n[2]};
  m[d] += 1;
  long nf = (long)m[0] * m[1] * m[2];
  int nc = 1 + D->ndim;
  set_threads(D);
#pragma omp parallel for schedule(static)
  for (long f = 0; f < nf; ++f) {
    int idx[3] = {(int)(f % m[0]), (int)((f / m[0]) % m[1]), (int)(f / ((long)m[0] * m[1]))};
    int row[3] = {idx[0], idx[1], idx[2]};
    for (int g = 0; g < D->G; ++g) {
      double fl[4];
      face_flux(C, d, row, idx[d], g, fl);
      for (int k = 0; k < nc; ++k) out[((size_t)f * D->G + g) * nc + k] = fl[k];
    }
  }
  return 0;
}

// Face states of every zone along d (the reconstruction step, with its realizability
// fallback): out[((zone * G + g) * 2 + side) * (1 + ndim) + k], side 0 = lower face.
int orc_faces(const OrcDesc* D, const double* E, const double* const* F, const double* inflow, int d, double* out) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  C.D = D;
  C.geo = &geo;
  for (int e = 0; e < 3; ++e) C.n[e] = D->n[e];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = 0.0;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (k < D->ndim) ? F[k] : nullptr;
  std::vector<double> zero((size_t)D->n[0] * D->n[1] * D->n[2] * D->G, 0.0);
  C.kap = zero.data();
  C.sig = zero.data();
  C.B = zero.data();
  C.inflow = inflow;
  const long nz = (long)D->n[0] * D->n[1] * D->n[2];
  const int nc = 1 + D->ndim;
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % D->n[0]), (int)((z / D->n[0]) % D->n[1]), (int)(z / ((long)D->n[0] * D->n[1]))};
    for (int g = 0; g < D->G; ++g) {
      double lo[4], hi[4];
      reconstruct(C, d, idx, g, lo, hi);
      for (int k = 0; k < nc; ++k) {
        out[((z * D->G + g) * 2 + 0) * nc + k] = lo[k];
        out[((z * D->G + g) * 2 + 1) * nc + k] = hi[k];
      }
    }
  }
  return 0;
}

// Implicit interaction update alone, in place.  dEm (nullable): -sum_g (E^{n+1} - E^-) per zone.
int orc_source(const OrcDesc* D, double* E, double* const* F, const double* kap, const double* sig, const double* B,
               double dt, double* dEm) {
  long nz = (long)D->n[0] * D->n[1] * D->n[2];
  for (long z = 0; z < nz; ++z) {
    double dsum = 0.0;
    for (int g = 0; g < D->G; ++g) {
      size_t zg = (size_t)z * D->G + g;
      double Fm[3] = {0, 0, 0}, F1[3], E1;
      for (int k = 0; k < D->ndim; ++k) Fm[k] = F[k][zg];
      implicit_source<double>(E[zg], Fm, kap[zg], sig[zg], B[zg], D->c, dt, D->ndim, E1, F1);
      dsum += E1 - E[zg];
      E[zg] = E1;
      for (int k = 0; k < D->ndim; ++k) F[k][zg] = F1[k];
    }
    if (dEm) dEm[z] = -dsum;
  }
  return 0;
}

// Forward-mode derivative of nsteps steps: U0 + t dU0 and kappa + t dkappa, returns U_N and
// dU_N/dt (exact, via dual numbers).
int orc_jvp(const OrcDesc* D, const double* E, const double* const* F, const double* dE, const double* const* dF,
            const double* kap, const double* dkap, const double* sig, const double* B, const double* inflow, double dt,
            int nsteps, double* Eo, double* const* Fo, double* dEo, double* const* dFo) {
  Geom geo;
  geo.build(*D);
  size_t nzg = (size_t)D->n[0] * D->n[1] * D->n[2] * D->G;
  std::vector<Dual> Ea(nzg), Eb(nzg), K(nzg);
  std::vector<std::vector<Dual>> Fa(3), Fb(3);
  for (size_t i = 0; i < nzg; ++i) {
    Ea[i] = Dual(E[i], dE ? dE[i] : 0.0);
    K[i] = Dual(kap[i], dkap ? dkap[i] : 0.0);
  }
  for (int k = 0; k < D->ndim; ++k) {
    Fa[k].resize(nzg);
    Fb[k].resize(nzg);
    for (size_t i = 0; i < nzg; ++i) Fa[k][i] = Dual(F[k][i], (dF && dF[k]) ? dF[k][i] : 0.0);
  }
  for (int s = 0; s < nsteps; ++s) {
    const Dual* Fin[3] = {nullptr, nullptr, nullptr};
    Dual* Fout[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < D->ndim; ++k) {
      Fin[k] = Fa[k].data();
      Fout[k] = Fb[k].data();
    }
    full_step<Dual>(D, geo, Ea.data(), Fin, K.data(), sig, B, inflow, dt, Eb.data(), Fout, nullptr, nullptr);
    std::swap(Ea, Eb);
    for (int k = 0; k < D->ndim; ++k) std::swap(Fa[k], Fb[k]);
  }
  for (size_t i = 0; i < nzg; ++i) {
    Eo[i] = Ea[i].v;
    dEo[i] = Ea[i].d;
  }
  for (int k = 0; k < D->ndim; ++k)
    for (size_t i = 0; i < nzg; ++i) {
      Fo[k][i] = Fa[k][i].v;
      dFo[k][i] = Fa[k][i].d;
    }
  return 0;
}

// Geometry tables for tests: per zone volume (active zones), per face coordinate areas for
// each direction, and for spherical grids the per-theta-zone connection coefficients
// [<Gamma^3_23>, <Gamma^1_33>, <Gamma^2_33>, <Gamma^2_22>] and per-zone cell-centred h.
int orc_geometry(const OrcDesc* D, double* vol, double* area0, double* area1, double* area2, double* gam_theta,
                 double* hcell, double* centroid0, double* centroid1) {
  Geom geo;
  geo.build(*D);
  int n0 = D->n[0], n1 = D->n[1], n2 = D->n[2];
  for (int k = 0; k < n2; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n0; ++i) {
        size_t z = ((size_t)k * n1 + j) * n0 + i;
        if (vol) vol[z] = geo.volume(i, j, k);
        if (hcell) geo.h_cell(i, j, hcell + 3 * z);
      }
  double* areas[3] = {area0, area1, area2};
  for (int d = 0; d < 3; ++d) {
    if (!areas[d]) continue;
    int m[3] = {n0, n1, n2};
    m[d] += 1;
    for (int k = 0; k < m[2]; ++k)
      for (int j = 0; j < m[1]; ++j)
        for (int i = 0; i < m[0]; ++i) {
          int idx[3] = {i, j, k};
          areas[d][((size_t)k * m[1] + j) * m[0] + i] = geo.area(d, idx);
        }
  }
  if (gam_theta && geo.sph())
    for (int j = 0; j < n1; ++j) {
      gam_theta[4 * j + 0] = geo.G323[j + NG];
      gam_theta[4 * j + 1] = geo.G133[j + NG];
      gam_theta[4 * j + 2] = geo.G233[j + NG];
      gam_theta[4 * j + 3] = geo.G222[j + NG];
    }
  if (centroid0)
    for (int i = 0; i < n0; ++i) centroid0[i] = geo.X[0][i + NG];
  if (centroid1)
    for (int j = 0; j < n1; ++j) centroid1[j] = geo.X[1][j + NG];
  return 0;
}

// Closure alone, for tests: physical-component P^ (3x3, row-major) of a state (E, F^ phys).
int orc_closure(const OrcDesc* D, double E, const double* Fphys, double* P) {
  Geom geo;  // unused, Cartesian scale factors
  Ctx<double> C;
  C.D = D;
  C.c = D->c;
  C.ndim = 3;
  double q[4] = {E, Fphys[0], Fphys[1], Fphys[2]}, h[3] = {1.0, 1.0, 1.0};
  double Pm[3][3];
  closure(C, q, h, Pm);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) P[3 * a + b] = Pm[a][b];
  (void)geo;
  return 0;
}

// The third moment of one state (Cartesian scale factors): Q [27] as [k][j][i].
int orc_closure3(const OrcDesc* D, double E, const double* Fphys, double* Q) {
  Ctx<double> C;
  C.D = D;
  C.c = D->c;
  C.ndim = 3;
  double q[4] = {E, Fphys[0], Fphys[1], Fphys[2]}, h[3] = {1.0, 1.0, 1.0};
  double Qm[3][3][3];
  closure3(C, q, h, Qm);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int d = 0; d < 3; ++d) Q[9 * a + 3 * b + d] = Qm[a][b][d];
  return 0;
}

// The M1 characteristic speeds of one state along x (Cartesian): F_x = Fn (physical).
int orc_m1_speeds(const OrcDesc* D, double E, double Fn, double* lmin, double* lmax) {
  Ctx<double> C;
  C.D = D;
  C.c = D->c;
  C.ndim = 3;
  double q[4] = {E, Fn, 0.0, 0.0}, h[3] = {1.0, 1.0, 1.0};
  m1_speeds(C, q, h, 0, *lmin, *lmax);
  return 0;
}

}  // extern "C"

// ------------------------------------------------------------------------------------
// Explicit transport alone (Algorithmic Steps, Step 1 for a static medium): U^- = U^n +
// dt L(U^n) for every zone-group, without the interaction update.
// ------------------------------------------------------------------------------------
extern "C" int orc_explicit(const OrcDesc* D, const double* E, const double* const* F, const double* kap,
                            const double* sig, const double* inflow, double dt, double* Eo, double* const* Fo) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  C.D = D;
  C.geo = &geo;
  for (int d = 0; d < 3; ++d) C.n[d] = D->n[d];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = dt;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (k < D->ndim) ? F[k] : nullptr;
  C.kap = kap;
  C.sig = sig;
  C.B = nullptr;
  C.inflow = inflow;
  set_threads(D);
  long nz = (long)C.n[0] * C.n[1] * C.n[2];
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    for (int g = 0; g < C.G; ++g) {
      double Um[4];
      explicit_update(C, idx, g, Um);
      size_t zg = (size_t)z * C.G + g;
      Eo[zg] = Um[0];
      for (int k = 0; k < D->ndim; ++k) Fo[k][zg] = Um[1 + k];
    }
  }
  return 0;
}

// ------------------------------------------------------------------------------------
// Velocity-dependent terms: C API
// ------------------------------------------------------------------------------------
static bool velocity_ok(const OrcDesc* D, const double* nu_edge) {
  if (D->integrator != OI_EULER) return false;
  if (!nu_edge) return true;
  for (int g = 0; g < D->G; ++g)
    if (!(nu_edge[g + 1] > nu_edge[g]) || !std::isfinite(nu_edge[g + 1]) || nu_edge[g] < 0.0) return false;
  return true;
}

// nsteps full steps with the velocity terms (forward-Euler push only; -1 otherwise or for bad
// group edges).  vf: ndim face-velocity arrays (see Ctx::vf); nu_edge: G + 1 finite edges.
extern "C" int orc_run_v(const OrcDesc* D, const double* E, const double* const* F, const double* kap,
                         const double* sig, const double* B, const double* inflow, const double* const* vf,
                         const double* nu_edge, double dt, int nsteps, double* Eo, double* const* Fo, double* dEm,
                         OrcDiag* diag) {
  if (!velocity_ok(D, nu_edge) || !nu_edge) return -1;
  Geom geo;
  geo.build(*D);
  size_t nzg = (size_t)D->n[0] * D->n[1] * D->n[2] * D->G;
  std::vector<double> Ea(E, E + nzg), Eb(nzg);
  std::vector<std::vector<double>> Fa(3), Fb(3);
  for (int k = 0; k < D->ndim; ++k) {
    Fa[k].assign(F[k], F[k] + nzg);
    Fb[k].assign(nzg, 0.0);
  }
  for (int s = 0; s < nsteps; ++s) {
    const double* Fin[3] = {nullptr, nullptr, nullptr};
    double* Fout[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < D->ndim; ++k) {
      Fin[k] = Fa[k].data();
      Fout[k] = Fb[k].data();
    }
    const bool last = (s == nsteps - 1);
    full_step_v(D, geo, Ea.data(), Fin, kap, sig, B, inflow, vf, nu_edge, dt, Eb.data(), Fout, last ? dEm : nullptr,
                last ? diag : nullptr);
    std::swap(Ea, Eb);
    for (int k = 0; k < D->ndim; ++k) std::swap(Fa[k], Fb[k]);
  }
  std::memcpy(Eo, Ea.data(), nzg * sizeof(double));
  for (int k = 0; k < D->ndim; ++k) std::memcpy(Fo[k], Fa[k].data(), nzg * sizeof(double));
  return 0;
}

static void velocity_ctx(Ctx<double>& C, const OrcDesc* D, const Geom& geo, const double* E, const double* const* F,
                         const double* kap, const double* sig, const double* inflow, const double* const* vf,
                         const double* nu_edge, double dt) {
  C.D = D;
  C.geo = &geo;
  for (int d = 0; d < 3; ++d) C.n[d] = D->n[d];
  C.G = D->G;
  C.ndim = D->ndim;
  C.c = D->c;
  C.dt = dt;
  C.E = E;
  for (int k = 0; k < 3; ++k) C.F[k] = (F && k < D->ndim) ? F[k] : nullptr;
  C.kap = kap;
  C.sig = sig;
  C.B = nullptr;
  C.inflow = inflow;
  for (int k = 0; k < 3; ++k) C.vf[k] = (k < D->ndim) ? vf[k] : nullptr;
  C.nu_edge = nu_edge;
}

// Step 1 alone with the velocity terms (advective fluxes, flux-row velocity terms).
extern "C" int orc_explicit_v(const OrcDesc* D, const double* E, const double* const* F, const double* kap,
                              const double* sig, const double* inflow, const double* const* vf, double dt, double* Eo,
                              double* const* Fo) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  velocity_ctx(C, D, geo, E, F, kap, sig, inflow, vf, nullptr, dt);
  set_threads(D);
  const long nz = (long)C.n[0] * C.n[1] * C.n[2];
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    for (int g = 0; g < C.G; ++g) {
      double Um[4];
      explicit_update(C, idx, g, Um);
      const size_t zg = (size_t)z * C.G + g;
      Eo[zg] = Um[0];
      for (int k = 0; k < D->ndim; ++k) Fo[k][zg] = Um[1 + k];
    }
  }
  return 0;
}

// Step 2 alone on the state (E, F): the energies and fluxes after the frequency advection.
extern "C" int orc_freq_adv(const OrcDesc* D, const double* E, const double* const* F, const double* const* vf,
                            const double* nu_edge, double dt, double* Eo, double* const* Fo) {
  if (!velocity_ok(D, nu_edge) || !nu_edge) return -1;
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  velocity_ctx(C, D, geo, E, F, nullptr, nullptr, nullptr, vf, nu_edge, dt);
  const long nz = (long)C.n[0] * C.n[1] * C.n[2];
  const int G = C.G;
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    std::vector<double> U((size_t)4 * G, 0.0);
    for (int g = 0; g < G; ++g) {
      const size_t zg = (size_t)z * G + g;
      U[(size_t)4 * g] = E[zg];
      for (int k = 0; k < D->ndim; ++k) U[(size_t)4 * g + 1 + k] = F[k][zg];
    }
    freq_advect(C, idx, U);
    for (int g = 0; g < G; ++g) {
      Eo[(size_t)z * G + g] = U[(size_t)4 * g];
      for (int k = 0; k < D->ndim; ++k) Fo[k][(size_t)z * G + g] = U[(size_t)4 * g + 1 + k];
    }
  }
  return 0;
}

// <v^i_{;j}> (row-major [i][j]) and <v^k> of every zone: Vg [nzones][9], vbar [nzones][3].
extern "C" int orc_vel_grad(const OrcDesc* D, const double* const* vf, double* Vg, double* vbar) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  velocity_ctx(C, D, geo, nullptr, nullptr, nullptr, nullptr, nullptr, vf, nullptr, 0.0);
  const long nz = (long)C.n[0] * C.n[1] * C.n[2];
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    double V[3][3], vb[3];
    vel_grad(C, idx, V, vb);
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) Vg[(size_t)z * 9 + 3 * i + j] = V[i][j];
      vbar[(size_t)z * 3 + i] = vb[i];
    }
  }
  return 0;
}

// Group-summed radiation energy and physical flux of every zone transformed to the laboratory
// frame to first order in v/c (the comoving-to-lab transformation used for the transparent
// shock test): with v^_k = h_k <v^k> (cell-centred h),
//   E_lab = sum_g (E_g + 2 v^ . F^_g / c^2),   F^_lab = sum_g (F^_g + v^ E_g + v^ . P^_g).
// Elab [nzones], Flab[k] [nzones] for k < ndim (physical components).
extern "C" int orc_lab_frame(const OrcDesc* D, const double* E, const double* const* F, const double* const* vf,
                             double* Elab, double* const* Flab) {
  Geom geo;
  geo.build(*D);
  Ctx<double> C;
  velocity_ctx(C, D, geo, E, F, nullptr, nullptr, nullptr, vf, nullptr, 0.0);
  const long nz = (long)C.n[0] * C.n[1] * C.n[2];
  const double c = D->c;
  for (long z = 0; z < nz; ++z) {
    int idx[3] = {(int)(z % C.n[0]), (int)((z / C.n[0]) % C.n[1]), (int)(z / ((long)C.n[0] * C.n[1]))};
    double V[3][3], vb[3], h[3];
    vel_grad(C, idx, V, vb);
    geo.h_cell(idx[0], idx[1], h);
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = h[k] * vb[k];
    double el = 0.0, fl[3] = {0.0, 0.0, 0.0};
    for (int g = 0; g < D->G; ++g) {
      const size_t zg = (size_t)z * D->G + g;
      double q[4] = {E[zg], 0.0, 0.0, 0.0};
      for (int k = 0; k < D->ndim; ++k) q[1 + k] = F[k][zg];
      double P[3][3];
      closure(C, q, h, P);
      double Fh[3];
      for (int k = 0; k < 3; ++k) Fh[k] = q[1 + k] / h[k];
      el += q[0] + 2.0 * (v[0] * Fh[0] + v[1] * Fh[1] + v[2] * Fh[2]) / (c * c);
      for (int k = 0; k < 3; ++k) fl[k] += Fh[k] + v[k] * q[0] + (v[0] * P[0][k] + v[1] * P[1][k] + v[2] * P[2][k]);
    }
    Elab[z] = el;
    for (int k = 0; k < D->ndim; ++k) Flab[k][z] = fl[k];
  }
  return 0;
}

// ------------------------------------------------------------------------------------
// Radiation-matter energy exchange with the matter temperature as unknown (Interaction
// Terms subsection, photon case: one outer equation; Algorithmic Steps, Steps 3 and 4).
//
// Matter model (Reading: the paper leaves the equation of state and the opacities to the
// application; this follows its multigroup pulse test):
//   internal energy density u = cv T (ideal gas, cv per zone);
//   absorption kappa_g(T) = kappa0 kg_g T^(-1/2) (1 - exp(-nu_g / T)) (the pulse test's
//     frequency- and temperature-dependent opacity at the group's frequency nu_g, with
//     kg_g holding the normalisation and the nu^-3 factor; units with h = k_B = 1);
//   emission j_g = c kappa_g B_g(T), B_g(T) = a_R T^4 (15/pi^4) int_{x_g}^{x_{g+1}}
//     x^3 / (e^x - 1) dx, x = nu / T, over the group's frequency edges (Kirchhoff's law
//     with the group-integrated Planck function; edges 0 and infinity allowed);
//   scattering sigma_g per zone-group, independent of T.
// ------------------------------------------------------------------------------------
static const double ORC_PI4_15 = 6.4939394022668291;   // pi^4 / 15 = int_0^inf x^3/(e^x-1) dx

// int_0^x t^3 / (e^t - 1) dt for 0 <= x < 2 pi: the series from t/(e^t - 1) = sum_k B_k t^k / k!
// (Bernoulli numbers), integrated term by term.
static double orc_planck_head_(double x) {
  // B_k / k! for k = 0 .. 24 (odd k > 1 vanish)
  static const double bk[25] = {1.0,
                                -0.5,
                                1.0 / 12.0,
                                0.0,
                                -1.0 / 720.0,
                                0.0,
                                1.0 / 30240.0,
                                0.0,
                                -1.0 / 1209600.0,
                                0.0,
                                1.0 / 47900160.0,
                                0.0,
                                -691.0 / 1307674368000.0,
                                0.0,
                                1.0 / 74724249600.0,
                                0.0,
                                -3617.0 / 10670622842880000.0,
                                0.0,
                                43867.0 / 5109094217170944000.0,
                                0.0,
                                -174611.0 / 802857662698291200000.0,
                                0.0,
                                77683.0 / 14101100039391805440000.0,
                                0.0,
                                -236364091.0 / 1693824136731743669452800000.0};
  double head = 0.0, p = x * x * x;
  for (int k = 0; k < 25; ++k) {
    head += bk[k] * p / (double)(k + 3);
    p *= x;
  }
  return head;
}

// int_x^inf t^3 / (e^t - 1) dt for x >= 1.5 (infinity gives 0): 1/(e^t - 1) = sum_n e^(-n t)
// and t^3 e^(-n t) integrated in closed form.
static double orc_planck_exp_tail_(double x) {
  if (!(x < INFINITY)) return 0.0;
  double s = 0.0;
  for (int n = 1; n <= 60; ++n) {
    double e = std::exp(-n * x);
    if (e < 1e-300) break;
    double dn = (double)n;
    s += e * (x * x * x / dn + 3.0 * x * x / (dn * dn) + 6.0 * x / (dn * dn * dn) + 6.0 / (dn * dn * dn * dn));
    if (e < 1e-18 * s) break;
  }
  return s;
}

static const double ORC_PLANCK_SPLIT = 1.5;   // the head series below, the exponential series above

// int_x^inf t^3 / (e^t - 1) dt for x >= 0
static double orc_planck_tail_(double x) {
  return x < ORC_PLANCK_SPLIT ? ORC_PI4_15 - orc_planck_head_(x) : orc_planck_exp_tail_(x);
}

// int_a^b t^3 / (e^t - 1) dt for 0 <= a <= b <= infinity, without subtracting two large
// integrals where the interval is small: heads below the split, tails above it
static double orc_planck_between_(double a, double b) {
  if (b <= ORC_PLANCK_SPLIT) return orc_planck_head_(b) - orc_planck_head_(a);
  if (a >= ORC_PLANCK_SPLIT) return orc_planck_exp_tail_(a) - orc_planck_exp_tail_(b);
  return (orc_planck_head_(ORC_PLANCK_SPLIT) - orc_planck_head_(a)) +
         (orc_planck_exp_tail_(ORC_PLANCK_SPLIT) - orc_planck_exp_tail_(b));
}

struct OrcMatterModel {
  int G;
  const double* nu_edge;   // [G + 1] group frequency edges (0 and infinity allowed)
  const double* nu_c;      // [G] frequency of the group's opacity
  const double* kg;        // [G] opacity factor of the group
  double a_rad;            // radiation constant
  double c;                // speed of light
  double tol;              // relative change of T that ends the Newton iteration
  int max_newton;          // Newton iterations before bisection takes over
};

static double orc_group_B(const OrcMatterModel& M, int g, double T) {
  const double part = orc_planck_between_(M.nu_edge[g] / T, M.nu_edge[g + 1] / T);
  return M.a_rad * T * T * T * T * part / ORC_PI4_15;
}

static double orc_group_kappa(const OrcMatterModel& M, int g, double kappa0, double T) {
  return kappa0 * M.kg[g] / std::sqrt(T) * (1.0 - std::exp(-M.nu_c[g] / T));
}

// Inner update of every group at temperature T (eq:be_update), and the outer residual
// r(T) = u(T) - u^- + sum_g (E_g(T) - E_g^-) (Interaction Terms: r_E with Delta E^k).
static double orc_residual(const OrcMatterModel& M, double dt, double cv, double kappa0, double Tm, const double* Em,
                           double T, double* Eout) {
  double dE = 0.0;
  for (int g = 0; g < M.G; ++g) {
    double kap = orc_group_kappa(M, g, kappa0, T);
    double j = M.c * kap * orc_group_B(M, g, T);
    double E = (Em[g] + dt * j) / (1.0 + M.c * dt * kap);
    if (Eout) Eout[g] = E;
    dE += E - Em[g];
  }
  return cv * (T - Tm) + dE;
}

// Outer update of one zone: Newton-Raphson on r(T) = 0 from T^- with a forward-difference
// derivative and a backtracking line search (halving the step until |r| decreases), ended
// when the relative change of T is below tol; bisection between 0 and the temperature that
// holds all the radiation's energy when Newton fails (r is increasing in T and negative at
// 0: the root is bracketed).  Reading: the paper gives the method (finite-difference
// Jacobian, backtracking, bisection fallback, tolerance on the relative change of T,
// typically 1e-6) but not its constants; those here are: derivative step 1e-7 T, at most 10
// halvings, bisection until the bracket is 1e-13 of its upper end.  Returns the number of
// Newton iterations, or -(bisection steps) when bisection decided T.
static int orc_solve_T(const OrcMatterModel& M, double dt, double cv, double kappa0, double Tm, const double* Em,
                       double* Tout) {
  double T = Tm;
  double r = orc_residual(M, dt, cv, kappa0, Tm, Em, T, nullptr);
  for (int it = 0; it < M.max_newton; ++it) {
    double h = 1e-7 * T;
    double J = (orc_residual(M, dt, cv, kappa0, Tm, Em, T + h, nullptr) - r) / h;
    if (!(J > 0.0)) break;
    double d = -r / J;
    if (std::fabs(d) <= M.tol * T) {
      *Tout = T + d;
      return it + 1;
    }
    double lam = 1.0, Tn = T, rn = r;
    bool ok = false;
    for (int ls = 0; ls <= 10; ++ls) {
      Tn = T + lam * d;
      if (Tn > 0.0) {
        rn = orc_residual(M, dt, cv, kappa0, Tm, Em, Tn, nullptr);
        if (std::fabs(rn) < std::fabs(r)) {
          ok = true;
          break;
        }
      }
      lam *= 0.5;
    }
    if (!ok) break;
    bool conv = std::fabs(Tn - T) <= M.tol * Tn;
    T = Tn;
    r = rn;
    if (conv) {
      *Tout = T;
      return it + 1;
    }
  }
  double esum = 0.0;
  for (int g = 0; g < M.G; ++g) esum += std::max(Em[g], 0.0);
  double lo = 0.0, hi = Tm + esum / cv;
  int steps = 0;
  while (hi - lo > 1e-13 * hi && steps < 400) {
    double mid = 0.5 * (lo + hi);
    if (orc_residual(M, dt, cv, kappa0, Tm, Em, mid, nullptr) > 0.0)
      hi = mid;
    else
      lo = mid;
    ++steps;
  }
  *Tout = 0.5 * (lo + hi);
  return -steps;
}

extern "C" {

double orc_planck_tail(double x) { return orc_planck_tail_(x); }

// kappa_g(T) and B_g(T) of every zone-group: kap, B [nz][G].
int orc_matter_coeffs(int G, const double* nu_edge, const double* nu_c, const double* kg, double a_rad, long nz,
                      const double* kappa0, const double* T, double* kap, double* B) {
  OrcMatterModel M{G, nu_edge, nu_c, kg, a_rad, 1.0, 0.0, 0};
  for (long z = 0; z < nz; ++z)
    for (int g = 0; g < G; ++g) {
      kap[z * G + g] = orc_group_kappa(M, g, kappa0[z], T[z]);
      B[z * G + g] = orc_group_B(M, g, T[z]);
    }
  return 0;
}

// The interaction update with the matter energy equation, in place on E, F[k] (ndim arrays)
// and T, per zone: the outer solve for T^{n+1}, the groups' inner update at T^{n+1}, then the
// flux update F^{n+1} = F^- / (1 + c dt (kappa_g(T^{n+1}) + sigma_g)).  dEm (nullable):
// u^{n+1} - u^- per zone; iters (nullable): the solve's return value per zone.
int orc_matter_source(int G, const double* nu_edge, const double* nu_c, const double* kg, double a_rad, double c,
                      double tol, int max_newton, int ndim, long nz, double* E, double* const* F, const double* sig,
                      const double* cv, const double* kappa0, double* T, double dt, double* dEm, int* iters) {
  OrcMatterModel M{G, nu_edge, nu_c, kg, a_rad, c, tol, max_newton};
#pragma omp parallel for schedule(dynamic, 64)
  for (long z = 0; z < nz; ++z) {
    double* Ez = E + z * G;
    std::vector<double> Em(Ez, Ez + G), E1(G);
    double T1 = T[z];
    int it = orc_solve_T(M, dt, cv[z], kappa0[z], T[z], Em.data(), &T1);
    orc_residual(M, dt, cv[z], kappa0[z], T[z], Em.data(), T1, E1.data());
    for (int g = 0; g < G; ++g) {
      Ez[g] = E1[g];
      double kap = orc_group_kappa(M, g, kappa0[z], T1);
      for (int k = 0; k < ndim; ++k) F[k][z * G + g] /= (1.0 + c * dt * (kap + sig[z * G + g]));
    }
    if (dEm) dEm[z] = cv[z] * (T1 - T[z]);
    if (iters) iters[z] = it;
    T[z] = T1;
  }
  return 0;
}

}  // extern "C"
