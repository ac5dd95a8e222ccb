// m1_host.cpp -- host side of libfornax_m1: argument checking, geometry tables, C interface.
//
// Geometry (Numerical Discretization and the Appendix of the paper): the volume element is
// separable, sqrt(g) = w_1(x1) w_2(x2) w_3(x3), with w = 1 on Cartesian grids and, for the
// spherical grid x1 = ln r, x2 = theta, x3 = phi, w_1 = e^{3 x1}, w_2 = |sin x2|, w_3 = 1
// (r^3 sin(theta) with dr = r dx1).  Zone volumes are products of the 1-D integrals W_d and
// face areas replace one factor by w_d at the face; volume-averaged quantities that a
// closed form gives stably come from it, the others from 24-point Gauss-Legendre quadrature
// of the zone (all integrands are smooth inside a zone).  The angular-momentum override
// (eq:angmom) and the d_2 P = 0 balance override (eq:grad2P) are applied to the
// connection coefficients.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <functional>
#include <new>
#include <vector>

#include "m1_internal.h"
#include "m1_step.h"

using namespace fm1;

namespace {

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n)
struct GaussLegendre {
  static constexpr int N = 24;
  double x[N], w[N];
  GaussLegendre() {
    for (int i = 0; i < N; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (N + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= N; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        double dp = N * (z * p1 - p0) / (z * z - 1.0);
        double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-17) break;
      }
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= N; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = N * (z * p1 - p0) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
  // integral of f over [a, b], f evaluated at offsets t = x - a (no cancellation near a)
  double offset_integral(const std::function<double(double)>& f, double a, double b) const {
    double h = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < N; ++i) s += w[i] * f(h * (x[i] + 1.0));
    (void)a;
    return h * s;
  }
};

const GaussLegendre& gl() {
  static GaussLegendre g;
  return g;
}

bool valid_bc(int bc) { return bc >= FORNAX_BC_OUTFLOW && bc <= FORNAX_BC_AXIS; }

int validate(const fornax_m1_desc* d) {
  if (!d) return FORNAX_EINVAL;
  if (d->ndim < 1 || d->ndim > 3) return FORNAX_EINVAL;
  if (d->ngroups < 1) return FORNAX_EINVAL;
  if (d->ngroups > BLOCK) return FORNAX_EUNSUPPORTED;
  if (d->coord != FORNAX_CARTESIAN && d->coord != FORNAX_SPHERICAL_LOGR) return FORNAX_EINVAL;
  if (d->precision != FORNAX_FP64 && d->precision != FORNAX_MIXED) return FORNAX_EINVAL;
  if (d->limiter < 0 || d->limiter > 3) return FORNAX_EINVAL;
  if (d->closure < 0 || d->closure > 1) return FORNAX_EINVAL;
  if (d->integrator != FORNAX_EULER && d->integrator != FORNAX_SSPRK2) return FORNAX_EINVAL;
  if (d->wavespeed != FORNAX_WAVESPEED_LIGHT && d->wavespeed != FORNAX_WAVESPEED_M1) return FORNAX_EINVAL;
  if (!(d->c > 0.0) || !std::isfinite(d->c)) return FORNAX_EINVAL;
  int64_t nz = 1;
  for (int k = 0; k < 3; ++k) {
    if (d->n[k] < 1) return FORNAX_EINVAL;
    if (k >= d->ndim && d->n[k] != 1) return FORNAX_EINVAL;
    if (!(d->hi[k] > d->lo[k]) || !std::isfinite(d->lo[k]) || !std::isfinite(d->hi[k])) return FORNAX_EINVAL;
    nz *= d->n[k];
    if (k < d->ndim) {
      if (!valid_bc(d->bc_lo[k]) || !valid_bc(d->bc_hi[k])) return FORNAX_EINVAL;
      if ((d->bc_lo[k] == FORNAX_BC_PERIODIC) != (d->bc_hi[k] == FORNAX_BC_PERIODIC)) return FORNAX_EINVAL;
      // mirrored ghosts (reflect, axis) read zones 0 and 1 of the edge: at least two zones
      for (int side = 0; side < 2; ++side) {
        int bc = side ? d->bc_hi[k] : d->bc_lo[k];
        if ((bc == FORNAX_BC_REFLECT || bc == FORNAX_BC_AXIS) && d->n[k] < 2) return FORNAX_EINVAL;
      }
      // prescribed inflow ghosts are supported on x (x1 = ln r: the inner radial boundary)
      if (k != 0 && (d->bc_lo[k] == FORNAX_BC_INFLOW || d->bc_hi[k] == FORNAX_BC_INFLOW)) return FORNAX_EUNSUPPORTED;
      bool axis = d->bc_lo[k] == FORNAX_BC_AXIS || d->bc_hi[k] == FORNAX_BC_AXIS;
      if (axis) {
        if (d->coord != FORNAX_SPHERICAL_LOGR || k != 1) return FORNAX_EINVAL;
        if (d->bc_lo[k] == FORNAX_BC_AXIS && std::fabs(d->lo[1]) > 1e-12) return FORNAX_EINVAL;
        if (d->bc_hi[k] == FORNAX_BC_AXIS && std::fabs(d->hi[1] - M_PI) > 1e-12) return FORNAX_EINVAL;
        if (d->n[2] != 1 && (d->n[2] % 2) != 0) return FORNAX_EINVAL;
      }
    }
  }
  if (d->coord == FORNAX_SPHERICAL_LOGR) {
    if (d->lo[1] < -1e-12 || d->hi[1] > M_PI + 1e-12) return FORNAX_EINVAL;
  }
  // zone-group and face-group indices are 32-bit in the kernels
  int64_t nf = 0;
  for (int k = 0; k < d->ndim; ++k) nf = std::max<int64_t>(nf, nz / d->n[k] * (d->n[k] + 1));
  if (std::max(nz, nf) * (int64_t)d->ngroups * (1 + d->ndim) >= ((int64_t)1 << 31)) return FORNAX_EUNSUPPORTED;
  if (d->precision == FORNAX_MIXED && !(d->f_fp64 >= 0.0)) return FORNAX_EINVAL;
  return FORNAX_OK;
}

// Inverse of a 3x3 matrix (cofactors), for the parabolic reconstruction's weights.
static void inv3(const double A[3][3], double B[3][3]) {
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      // cofactor of A[j][i]
      const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
      B[i][j] = (A[r0][c0] * A[r1][c1] - A[r0][c1] * A[r1][c0]) / det;
    }
}

// Parabolic reconstruction weights of one zone (spherical grids; the Reconstruction
// subsection's n = 2 case in the volume coordinate).  u = (x - x_i)/dx is the zone's own
// coordinate (its faces at -+1/2, the neighbours' centres at -+1), mu1[k], mu2[k] the volume
// averages of u and u^2 over zones i-1, i, i+1.  Layout as PPM_TAB describes.
static void ppm_weights(const double mu1[3], const double mu2[3], double* T) {
  const double ulo = -0.5, uhi = 0.5;
  const double A1[3][3] = {{1.0, mu1[0], mu2[0]}, {1.0, mu1[1], mu2[1]}, {1.0, mu1[2], mu2[2]}};
  double B1[3][3];
  inv3(A1, B1);
  for (int k = 0; k < 3; ++k) {
    T[k] = B1[0][k] + ulo * B1[1][k] + ulo * ulo * B1[2][k];
    T[3 + k] = B1[0][k] + uhi * B1[1][k] + uhi * uhi * B1[2][k];
    T[6 + k] = B1[1][k];
    T[9 + k] = B1[2][k];
  }
  const double A2[3][3] = {{1.0, ulo, ulo * ulo}, {1.0, mu1[1], mu2[1]}, {1.0, uhi, uhi * uhi}};
  double B2[3][3];
  inv3(A2, B2);
  for (int k = 0; k < 3; ++k) {
    T[12 + k] = B2[1][k];
    T[15 + k] = B2[2][k];
  }
  // zero slope at the lower face through (average, upper face state): rows p'(ulo) = 0,
  // <p> = q_i, p(uhi) = v_hi; the lower face state p(ulo) on (q_i, v_hi)
  const double A3[3][3] = {{0.0, 1.0, 2.0 * ulo}, {1.0, mu1[1], mu2[1]}, {1.0, uhi, uhi * uhi}};
  double B3[3][3];
  inv3(A3, B3);
  for (int k = 1; k < 3; ++k) T[18 + k - 1] = B3[0][k] + ulo * B3[1][k] + ulo * ulo * B3[2][k];
  const double A4[3][3] = {{1.0, ulo, ulo * ulo}, {1.0, mu1[1], mu2[1]}, {0.0, 1.0, 2.0 * uhi}};
  double B4[3][3];
  inv3(A4, B4);
  for (int k = 0; k < 2; ++k) T[20 + k] = B4[0][k] + uhi * B4[1][k] + uhi * uhi * B4[2][k];
}

void build_geometry(const fornax_m1_desc& D, HostGeo& H) {
  const bool sph = D.coord == FORNAX_SPHERICAL_LOGR;
  const auto& Q = gl();
  for (int d = 0; d < 3; ++d) {
    int n = D.n[d];
    H.n[d] = n;
    int m = n + 2 * NG;             // extended zones
    double dx = (D.hi[d] - D.lo[d]) / n;
    H.dx[d] = dx;
    // zone e covers [a_e, a_e + dx], a_e = lo + (e - NG) dx; one extra zone on each side for
    // the centroid differences at the ends of the extended range
    std::vector<double> X(m + 2), a(m + 3);
    for (int e = -1; e <= m + 1; ++e) a[e + 1] = D.lo[d] + (e - NG) * dx;
    std::vector<double> W(m + 2);
    for (int e = -1; e <= m; ++e) {
      double lo = a[e + 1], hi = lo + dx;
      double Wz, off;
      if (!sph || d == 2) {
        Wz = dx;
        off = 0.5 * dx;
      } else if (d == 0) {
        // w = e^{3x}: W = e^{3 lo} (e^{3 dx} - 1)/3; centroid offset by quadrature
        Wz = std::exp(3.0 * lo) * std::expm1(3.0 * dx) / 3.0;
        double num = Q.offset_integral([&](double t) { return t * std::exp(3.0 * t); }, lo, hi);
        double den = Q.offset_integral([&](double t) { return std::exp(3.0 * t); }, lo, hi);
        off = num / den;
      } else {
        // w = |sin x|: W = |cos lo - cos hi| = 2 |sin(mid) sin(dx/2)|
        Wz = std::fabs(2.0 * std::sin(lo + 0.5 * dx) * std::sin(0.5 * dx));
        double num = Q.offset_integral([&](double t) { return t * std::fabs(std::sin(lo + t)); }, lo, hi);
        double den = Q.offset_integral([&](double t) { return std::fabs(std::sin(lo + t)); }, lo, hi);
        off = num / den;
      }
      W[e + 1] = Wz;
      X[e + 1] = lo + off;
    }
    H.idm[d].resize(m);
    H.idp[d].resize(m);
    H.idc[d].resize(m);
    H.dlo[d].resize(m);
    H.dhi[d].resize(m);
    H.iW[d].resize(m);
    H.W[d].resize(m);
    H.wf[d].resize(m + 1);
    for (int e = 0; e < m; ++e) {
      double Xm = X[e], X0 = X[e + 1], Xp = X[e + 2];
      H.idm[d][e] = 1.0 / (X0 - Xm);
      H.idp[d][e] = 1.0 / (Xp - X0);
      H.idc[d][e] = 1.0 / (Xp - Xm);
      H.dlo[d][e] = a[e + 1] - X0;
      H.dhi[d][e] = (a[e + 1] + dx) - X0;
      H.W[d][e] = W[e + 1];
      H.iW[d][e] = 1.0 / W[e + 1];
    }
    // parabolic reconstruction on spherical grids: the moments of u = (x - x_e)/dx over zones
    // e - 1, e, e + 1 with the axis's volume element, by Gauss-Legendre quadrature
    H.ppm[d].clear();
    if (sph && D.limiter == FORNAX_LIMITER_PPM) {
      H.ppm[d].resize((size_t)PPM_TAB * m);
      for (int e = 0; e < m; ++e) {
        const double xc = a[e + 1] + 0.5 * dx;
        double mu1[3], mu2[3];
        for (int k = 0; k < 3; ++k) {
          const double lo = a[e + k];   // zone e - 1 + k
          auto wt = [&](double t) {
            if (d == 0) return std::exp(3.0 * (lo + t - xc));
            if (d == 1) return std::fabs(std::sin(lo + t));
            return 1.0;
          };
          const double den = Q.offset_integral(wt, lo, lo + dx);
          mu1[k] = Q.offset_integral([&](double t) { return (lo + t - xc) / dx * wt(t); }, lo, lo + dx) / den;
          mu2[k] = Q.offset_integral([&](double t) { const double u = (lo + t - xc) / dx; return u * u * wt(t); },
                                     lo, lo + dx) / den;
        }
        ppm_weights(mu1, mu2, &H.ppm[d][(size_t)PPM_TAB * e]);
      }
    }
    for (int e = 0; e <= m; ++e) {
      double xf = D.lo[d] + (e - NG) * dx;
      double w = 1.0;
      if (sph && d == 0) w = std::exp(3.0 * xf);
      if (sph && d == 1) w = std::fabs(std::sin(xf));
      H.wf[d][e] = w;
    }
    if (sph && d == 1) {
      if (D.bc_lo[1] == FORNAX_BC_AXIS) H.wf[1][NG] = 0.0;
      if (D.bc_hi[1] == FORNAX_BC_AXIS) H.wf[1][NG + n] = 0.0;
    }
  }
  int m0 = D.n[0] + 2 * NG, m1 = D.n[1] + 2 * NG;
  if (sph) {
    double dx0 = H.dx[0], dx1 = H.dx[1];
    H.rc.resize(m0);
    H.rf.resize(m0 + 1);
    H.hr.resize(m0);
    for (int e = 0; e < m0; ++e) {
      double lo = D.lo[0] + (e - NG) * dx0;
      H.rc[e] = std::exp(lo + 0.5 * dx0);
      // <r^2> with weight r^3 dx1: (3/5) e^{2 lo} (e^{5 dx} - 1) / (e^{3 dx} - 1)
      double r2 = 0.6 * std::exp(2.0 * lo) * std::expm1(5.0 * dx0) / std::expm1(3.0 * dx0);
      H.hr[e] = std::sqrt(r2);
    }
    for (int e = 0; e <= m0; ++e) H.rf[e] = std::exp(D.lo[0] + (e - NG) * dx0);
    H.sc.resize(m1);
    H.sf.resize(m1 + 1);
    H.hs.resize(m1);
    H.gam.assign(4 * (size_t)D.n[1], 0.0);
    for (int e = 0; e < m1; ++e) {
      double lo = D.lo[1] + (e - NG) * dx1, hi = lo + dx1;
      H.sc[e] = std::fabs(std::sin(lo + 0.5 * dx1));
      double num = Q.offset_integral([&](double t) { double s = std::fabs(std::sin(lo + t)); return s * s * s; },
                                     lo, hi);
      double den = Q.offset_integral([&](double t) { return std::fabs(std::sin(lo + t)); }, lo, hi);
      H.hs[e] = std::sqrt(num / den);             // sqrt(<sin^2 theta>)
    }
    for (int e = 0; e <= m1; ++e) H.sf[e] = std::fabs(std::sin(D.lo[1] + (e - NG) * dx1));
    for (int j = 0; j < D.n[1]; ++j) {
      int e = j + NG;
      double mid = D.lo[1] + (j + 0.5) * dx1;
      double cot = std::cos(mid) / std::sin(mid);     // <cot theta> = cot(theta_mid) exactly
      double s2 = H.hs[e] * H.hs[e];               // <sin^2 theta>
      H.gam[4 * j + 0] = cot;                        // <Gamma^3_23>
      H.gam[4 * j + 1] = -s2 * 1.0;                  // <Gamma^1_33> = -<g33>/<g11> <Gamma^3_13>
      H.gam[4 * j + 2] = -s2 * cot;                  // <Gamma^2_33> = -<g33>/<g22> <Gamma^3_23>
      H.gam[4 * j + 3] = (H.wf[1][e + 1] - H.wf[1][e]) * H.iW[1][e] - cot;   // eq:grad2P
    }
    auto inv = [](const std::vector<double>& v) {
      std::vector<double> r(v.size());
      for (size_t i = 0; i < v.size(); ++i) r[i] = v[i] != 0.0 ? 1.0 / v[i] : 0.0;
      return r;
    };
    H.irc = inv(H.rc);
    H.irf = inv(H.rf);
    H.isc = inv(H.sc);
    H.isf = inv(H.sf);
    H.ihr = inv(H.hr);
    H.ihs = inv(H.hs);
  }
}

template <typename R>
size_t table_bytes(const HostGeo& H, bool sph) {
  size_t n = 0;
  for (int d = 0; d < 3; ++d) n += 7 * H.idm[d].size() + H.wf[d].size() + H.ppm[d].size();
  if (sph)
    n += 2 * (H.rc.size() + H.rf.size() + H.hr.size() + H.sc.size() + H.sf.size() + H.hs.size()) + H.gam.size();
  size_t b = n * sizeof(R);
  for (int d = 0; d < 3; ++d) b += H.W[d].size() * sizeof(double);
  return b + 256 * 48;   // 256-byte alignment of each of the (at most 40) tables
}

struct Packer {
  char* host;
  char* dev;
  size_t off = 0;
  template <typename R>
  const R* put(const std::vector<double>& v) {
    off = (off + 255) & ~(size_t)255;
    R* h = reinterpret_cast<R*>(host + off);
    for (size_t i = 0; i < v.size(); ++i) h[i] = (R)v[i];
    const R* dptr = reinterpret_cast<const R*>(dev + off);
    off += v.size() * sizeof(R);
    return v.empty() ? nullptr : dptr;
  }
};

template <typename R>
void pack(const HostGeo& H, bool sph, Packer& P, Geo<R>& G) {
  for (int d = 0; d < 3; ++d) {
    G.idm[d] = P.put<R>(H.idm[d]);
    G.idp[d] = P.put<R>(H.idp[d]);
    G.idc[d] = P.put<R>(H.idc[d]);
    G.dlo[d] = P.put<R>(H.dlo[d]);
    G.dhi[d] = P.put<R>(H.dhi[d]);
    G.iW[d] = P.put<R>(H.iW[d]);
    G.wf[d] = P.put<R>(H.wf[d]);
    G.Wd[d] = P.put<double>(H.W[d]);
    G.ppm[d] = H.ppm[d].empty() ? nullptr : P.put<R>(H.ppm[d]);
    G.dx[d] = (R)H.dx[d];
    G.idx[d] = (R)(1.0 / H.dx[d]);
  }
  G.rc = G.rf = G.hr = G.sc = G.sf = G.hs = G.gam = nullptr;
  G.irc = G.irf = G.isc = G.isf = G.ihr = G.ihs = nullptr;
  if (sph) {
    G.irc = P.put<R>(H.irc);
    G.irf = P.put<R>(H.irf);
    G.isc = P.put<R>(H.isc);
    G.isf = P.put<R>(H.isf);
    G.ihr = P.put<R>(H.ihr);
    G.ihs = P.put<R>(H.ihs);
    G.rc = P.put<R>(H.rc);
    G.rf = P.put<R>(H.rf);
    G.hr = P.put<R>(H.hr);
    G.sc = P.put<R>(H.sc);
    G.sf = P.put<R>(H.sf);
    G.hs = P.put<R>(H.hs);
    G.gam = P.put<R>(H.gam);
  }
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

// ------------------------------------------------------------------------------------------
extern "C" {

const char* fornax_m1_strerror(int code) {
  switch (code) {
    case FORNAX_OK: return "ok";
    case FORNAX_EINVAL: return "invalid argument";
    case FORNAX_ECFL: return "time step above the CFL limit (or not positive)";
    case FORNAX_EDEVICE: return "HIP device error";
    case FORNAX_ENOMEM: return "device allocation failed";
    case FORNAX_EUNSUPPORTED: return "unsupported configuration";
    case FORNAX_ESCRATCH:
      return "the step's scratch does not fit the static array of fornax_m1_step_noalloc "
             "(FORNAX_M1_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown error";
  }
}

int fornax_m1_create(const fornax_m1_desc* desc, fornax_m1_ctx** out) {
  if (!out) return FORNAX_EINVAL;
  *out = nullptr;
  int rc = validate(desc);
  if (rc != FORNAX_OK) return rc;
  fornax_m1_ctx* ctx = new (std::nothrow) fornax_m1_ctx();
  if (!ctx) return FORNAX_ENOMEM;
  ctx->desc = *desc;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return FORNAX_EDEVICE;
  }
  // set-up of the static scratch of fornax_m1_step_noalloc on this device (once per device)
  if (fm1_static_scratch_setup(ctx->device) != FORNAX_OK) {
    delete ctx;
    return FORNAX_EDEVICE;
  }
  build_geometry(*desc, ctx->hgeo);
  const bool sph = desc->coord == FORNAX_SPHERICAL_LOGR;
  size_t bd = table_bytes<double>(ctx->hgeo, sph), bf = table_bytes<float>(ctx->hgeo, sph);
  ctx->geo_bytes = bd + bf;
  if (hipMalloc(&ctx->geo_mem, ctx->geo_bytes) != hipSuccess) {
    delete ctx;
    return FORNAX_ENOMEM;
  }
  std::vector<char> host(ctx->geo_bytes, 0);
  Packer P{host.data(), (char*)ctx->geo_mem};
  pack<double>(ctx->hgeo, sph, P, ctx->geo_d);
  pack<float>(ctx->hgeo, sph, P, ctx->geo_f);
  if (P.off > ctx->geo_bytes ||
      hipMemcpy(ctx->geo_mem, host.data(), ctx->geo_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(ctx->geo_mem);
    delete ctx;
    return FORNAX_EDEVICE;
  }
  // max_dt at cfl = 1
  double worst = 0.0;
  const HostGeo& H = ctx->hgeo;
  for (int j = 0; j < desc->n[1]; ++j)
    for (int i = 0; i < desc->n[0]; ++i) {
      double s = 0.0;
      for (int d = 0; d < desc->ndim; ++d) {
        double dl = H.dx[d];
        if (sph) {
          double hr = H.hr[i + NG], hs = H.hs[j + NG];
          dl = (d == 2) ? hr * hs * H.dx[2] : hr * H.dx[d];
        }
        s += desc->c / dl;
      }
      if (s > worst) worst = s;
    }
  ctx->max_dt1 = 1.0 / worst;
  // tiling of the step kernel (FORNAX_M1_TILE="TXB,TYB,TM[,GB]" overrides the default choice)
  if (prepare_step_kernels() != FORNAX_OK) {
    (void)hipFree(ctx->geo_mem);
    delete ctx;
    return FORNAX_EDEVICE;
  }
  {
    // pairs of groups per lane (FORNAX_M1_PAIRS=0 disables)
    const char* pe = std::getenv("FORNAX_M1_PAIRS");
    // (measured: in 1-D/2-D, in 3-D FP64 and on spherical grids the second group's registers
    // cost more waves, or spill, than the wider accesses gain; 3-D Cartesian MIXED gains)
    const int V = (desc->ndim == 3 && desc->precision == FORNAX_MIXED && desc->coord == FORNAX_CARTESIAN &&
                   desc->ngroups % 2 == 0 && !(pe && pe[0] == '0'))
                      ? 2
                      : 1;
    ctx->tile = choose_tile(*desc, V);
    if (ctx->tile.nblocks <= 0) ctx->tile = choose_tile(*desc, 1);
    ctx->tile_v1 = (ctx->tile.V == 1) ? ctx->tile : choose_tile(*desc, 1);
  }
  if (const char* env = std::getenv("FORNAX_M1_TILE")) {
    // "TXB,TYB,TM,GB[,NW[,V]]" (TXB, TYB ignored for 1-D/2-D wave rows, where TXB = 64 V/GB)
    int tx = 0, ty = 0, tm = 0, gbk = desc->ngroups, nw = 1, vv = 1;
    const int nread = std::sscanf(env, "%d,%d,%d,%d,%d,%d", &tx, &ty, &tm, &gbk, &nw, &vv);
    if (nread >= 4) {
      if (nread < 5 && desc->ndim < 3) {
        nw = std::min(8, desc->ngroups / std::max(gbk, 1));
        while (nw > 1 && (desc->ngroups / gbk) % nw != 0) --nw;
      }
      Tile t = make_tile(*desc, tx, ty, tm, gbk, nw, vv);
      if (t.nblocks > 0) ctx->tile = t;
      if (t.nblocks > 0 && t.V == 1) ctx->tile_v1 = t;
    }
  }
  // the whole-zone kernel where the grid qualifies (FORNAX_M1_ROWS="0" disables it,
  // "NWX,TM" picks its tiling)
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) cus = 0;
  ctx->cus = cus;
  ctx->rows = choose_rows_tile(*desc, cus);
  if (const char* env = std::getenv("FORNAX_M1_ROWS")) {
    int nwx = 0, tm = 0;
    if (env[0] == '0' && env[1] == 0) ctx->rows = fm1::RowsTile{};
    else if (std::sscanf(env, "%d,%d", &nwx, &tm) == 2) ctx->rows = make_rows_tile(*desc, nwx, tm);
  }
  // the 3-D Cartesian kernel where the grid qualifies (FORNAX_M1_C3="0" disables it, "NR,TM"
  // picks its tiling)
  ctx->c3 = choose_c3_tile(*desc, cus);
  ctx->c3v = choose_c3_vel_tile(*desc, cus);
  if (const char* env = std::getenv("FORNAX_M1_C3")) {
    int nr = 0, tm = 0;
    if (env[0] == '0' && env[1] == 0) ctx->c3 = fm1::C3Tile{};
    else if (std::sscanf(env, "%d,%d", &nr, &tm) == 2) ctx->c3 = make_c3_tile(*desc, nr, tm);
  }
  if (ctx->tile.nblocks <= 0) {
    (void)hipFree(ctx->geo_mem);
    delete ctx;
    return FORNAX_EUNSUPPORTED;
  }
  // reduction scratch: one partial per block of the step kernel, and per block of the
  // zone-block kernels (source)
  int zpb = BLOCK / desc->ngroups;
  int64_t nz = (int64_t)desc->n[0] * desc->n[1] * desc->n[2];
  ctx->nblocks_step = (int)((nz + zpb - 1) / zpb);
  size_t nb = (size_t)std::max(std::max(std::max(ctx->nblocks_step, ctx->rows.nblocks), ctx->c3.nblocks),
                               std::max(ctx->tile_v1.nblocks, ctx->tile.nblocks));
  // dE_matter partials when a tile splits the groups of a zone over several blocks
  const size_t ngbm = (size_t)std::max(std::max(ctx->tile.ngb, ctx->tile_v1.ngb), ctx->c3.ngb);
  const size_t dzp_bytes = ngbm > 1 ? ngbm * (size_t)nz * sizeof(double) : 0;
  const size_t red_bytes = (nb * (2 * sizeof(double) + 2 * sizeof(int)) + 256 + 1023) & ~(size_t)255;
  void* red = nullptr;
  if (hipMalloc(&red, red_bytes + dzp_bytes) != hipSuccess) {
    (void)hipFree(ctx->geo_mem);
    delete ctx;
    return FORNAX_ENOMEM;
  }
  ctx->nb_partials =
      (size_t)std::max(std::max(ctx->rows.nblocks, ctx->c3.nblocks), std::max(ctx->tile_v1.nblocks, ctx->tile.nblocks));
  ctx->p_energy = (double*)red;
  ctx->p_maxf2 = ctx->p_energy + nb;
  ctx->p_nun = (int*)(ctx->p_maxf2 + nb);
  ctx->p_nnp = ctx->p_nun + nb;
  ctx->dzp = dzp_bytes ? (double*)((char*)red + red_bytes) : nullptr;
  // SSP-RK2: storage of the first stage's state
  ctx->stage_mem = nullptr;
  if (desc->integrator == FORNAX_SSPRK2) {
    const size_t es = desc->precision == FORNAX_FP64 ? sizeof(double) : sizeof(float);
    if (hipMalloc(&ctx->stage_mem, (size_t)(1 + desc->ndim) * nz * desc->ngroups * es) != hipSuccess) {
      (void)hipFree(red);
      (void)hipFree(ctx->geo_mem);
      delete ctx;
      return FORNAX_ENOMEM;
    }
  }
  // adjoint tiling (FORNAX_M1_ADJ_TILE="TXB,TM" overrides the default, read here once) and
  // ghost buffers (the adjoint supports 1-D and 2-D Cartesian grids)
  ctx->adj_txb = 0;
  ctx->adj_tm = 0;
  if (const char* env = std::getenv("FORNAX_M1_ADJ_TILE")) {
    int x = 0, y = 0;
    if (std::sscanf(env, "%d,%d", &x, &y) == 2 && x >= 4 && y >= 1) {
      ctx->adj_txb = x;
      ctx->adj_tm = y;
    }
  }
  for (int d = 0; d < 3; ++d) {
    ctx->adj_gbuf[d] = nullptr;
    ctx->adj_gplane[d] = (int)(nz / desc->n[d]);
  }
  if (desc->coord == FORNAX_CARTESIAN && desc->ndim <= 2) {
    for (int d = 0; d < desc->ndim; ++d) {
      size_t bytes = (size_t)4 * ctx->adj_gplane[d] * desc->ngroups * (desc->ndim + 2) * sizeof(double);
      if (hipMalloc((void**)&ctx->adj_gbuf[d], bytes) != hipSuccess) {
        for (int e = 0; e < d; ++e) (void)hipFree(ctx->adj_gbuf[e]);
        if (ctx->stage_mem) (void)hipFree(ctx->stage_mem);
        (void)hipFree(red);
        (void)hipFree(ctx->geo_mem);
        delete ctx;
        return FORNAX_ENOMEM;
      }
    }
  }
  *out = ctx;
  return FORNAX_OK;
}

int fornax_m1_destroy(fornax_m1_ctx* ctx) {
  if (!ctx) return FORNAX_EINVAL;
  (void)hipFree(ctx->geo_mem);
  (void)hipFree(ctx->p_energy);
  for (int d = 0; d < 3; ++d)
    if (ctx->adj_gbuf[d]) (void)hipFree(ctx->adj_gbuf[d]);
  if (ctx->stage_mem) (void)hipFree(ctx->stage_mem);
  if (ctx->mat_tab) (void)hipFree(ctx->mat_tab);
  if (ctx->vel_nu) (void)hipFree(ctx->vel_nu);
  delete ctx;
  return FORNAX_OK;
}

double fornax_m1_max_dt(const fornax_m1_ctx* ctx, double cfl) {
  if (!ctx || !(cfl > 0.0)) return (double)FORNAX_EINVAL;
  return cfl * ctx->max_dt1;
}

static int check_state(const fornax_m1_ctx* ctx, const fornax_m1_state* s) {
  if (!s || !s->E) return FORNAX_EINVAL;
  size_t al = ctx->desc.precision == FORNAX_FP64 ? 8 : 4;
  if (!aligned(s->E, al)) return FORNAX_EINVAL;
  for (int k = 0; k < ctx->desc.ndim; ++k)
    if (!s->F[k] || !aligned(s->F[k], al)) return FORNAX_EINVAL;
  return FORNAX_OK;
}

static int check_coeffs(const fornax_m1_ctx* ctx, const fornax_m1_coeffs* cf) {
  if (!cf || !cf->kappa || !cf->sigma || !cf->B) return FORNAX_EINVAL;
  size_t al = ctx->desc.precision == FORNAX_FP64 ? 8 : 4;
  if (!aligned(cf->kappa, al) || !aligned(cf->sigma, al) || !aligned(cf->B, al)) return FORNAX_EINVAL;
  return FORNAX_OK;
}

static bool needs_inflow(const fornax_m1_desc& d) {
  for (int k = 0; k < d.ndim; ++k)
    if (d.bc_lo[k] == FORNAX_BC_INFLOW || d.bc_hi[k] == FORNAX_BC_INFLOW) return true;
  return false;
}

static bool overlaps(const fornax_m1_ctx* ctx, const fornax_m1_state* a, const fornax_m1_state* b) {
  const void* pa[4] = {a->E, a->F[0], a->F[1], a->F[2]};
  const void* pb[4] = {b->E, b->F[0], b->F[1], b->F[2]};
  for (int i = 0; i <= ctx->desc.ndim; ++i)
    for (int j = 0; j <= ctx->desc.ndim; ++j)
      if (pa[i] && pa[i] == pb[j]) return true;
  return false;
}

int fornax_m1_step(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                   const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_diag* diag,
                   void* stream) {
  if (!ctx) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, in)) || (rc = check_state(ctx, out)) || (rc = check_coeffs(ctx, cf))) return rc;
  if (overlaps(ctx, in, out)) return FORNAX_EINVAL;
  if (needs_inflow(ctx->desc) != (inflow != nullptr)) return FORNAX_EINVAL;
  if (!(dt > 0.0) || dt > ctx->max_dt1 * (1.0 + 1e-12)) return FORNAX_ECFL;
  return fm1_launch_step(ctx, in, out, cf, inflow, dt, diag, (hipStream_t)stream);
}

int fornax_m1_step_noalloc(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                           const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_diag* diag,
                           void* stream) {
  if (!ctx) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, in)) || (rc = check_state(ctx, out)) || (rc = check_coeffs(ctx, cf))) return rc;
  if (overlaps(ctx, in, out)) return FORNAX_EINVAL;
  if (needs_inflow(ctx->desc) != (inflow != nullptr)) return FORNAX_EINVAL;
  if (!(dt > 0.0) || dt > ctx->max_dt1 * (1.0 + 1e-12)) return FORNAX_ECFL;
  return fm1_launch_step_noalloc(ctx, in, out, cf, inflow, dt, diag, (hipStream_t)stream);
}

int fornax_m1_flux(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_coeffs* cf, const double* inflow,
                   void* face_flux[3], void* stream) {
  if (!ctx || !face_flux) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, in)) || (rc = check_coeffs(ctx, cf))) return rc;
  if (needs_inflow(ctx->desc) != (inflow != nullptr)) return FORNAX_EINVAL;
  for (int d = 0; d < ctx->desc.ndim; ++d)
    if (!face_flux[d]) return FORNAX_EINVAL;
  return fm1_launch_flux(ctx, in, cf, inflow, face_flux, (hipStream_t)stream);
}

int fornax_m1_source(fornax_m1_ctx* ctx, fornax_m1_state* inout, const fornax_m1_coeffs* cf, double dt,
                     double* dE_matter, void* stream) {
  if (!ctx) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, inout)) || (rc = check_coeffs(ctx, cf))) return rc;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return FORNAX_EINVAL;
  return fm1_launch_source(ctx, inout, cf, dt, dE_matter, (hipStream_t)stream);
}

int fornax_m1_adjoint(fornax_m1_ctx* ctx, const fornax_m1_state* Un, const fornax_m1_state* Unp1,
                      const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_state* lam_np1,
                      fornax_m1_state* lam_n, void* dkappa_accum, void* stream) {
  if (!ctx || !dkappa_accum || !Unp1) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, Un)) || (rc = check_state(ctx, lam_np1)) || (rc = check_state(ctx, lam_n)) ||
      (rc = check_coeffs(ctx, cf)) || (rc = check_state(ctx, Unp1)))
    return rc;
  if (overlaps(ctx, lam_n, lam_np1) || overlaps(ctx, lam_n, Un) || overlaps(ctx, lam_n, Unp1)) return FORNAX_EINVAL;
  if (needs_inflow(ctx->desc) != (inflow != nullptr)) return FORNAX_EINVAL;
  if (!(dt > 0.0) || dt > ctx->max_dt1 * (1.0 + 1e-12)) return FORNAX_ECFL;
  return fm1_launch_adjoint(ctx, Un, Unp1, cf, inflow, dt, lam_np1, lam_n, dkappa_accum, (hipStream_t)stream);
}

int fornax_m1_transport(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                        const fornax_m1_coeffs* cf, const double* inflow, double dt, void* stream) {
  if (!ctx || !cf || !cf->kappa || !cf->sigma) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, in)) || (rc = check_state(ctx, out))) return rc;
  const size_t al = ctx->desc.precision == FORNAX_FP64 ? 8 : 4;
  if (!aligned(cf->kappa, al) || !aligned(cf->sigma, al) || (cf->B && !aligned(cf->B, al))) return FORNAX_EINVAL;
  if (overlaps(ctx, in, out)) return FORNAX_EINVAL;
  if (needs_inflow(ctx->desc) != (inflow != nullptr)) return FORNAX_EINVAL;
  if (!(dt > 0.0) || dt > ctx->max_dt1 * (1.0 + 1e-12)) return FORNAX_ECFL;
  return fm1_launch_transport(ctx, in, out, cf, inflow, dt, (hipStream_t)stream);
}

int fornax_m1_set_matter_model(fornax_m1_ctx* ctx, const fornax_m1_matter_model* mm) {
  if (!ctx || !mm || !mm->nu_edge || !mm->nu_c || !mm->kg) return FORNAX_EINVAL;
  const int G = ctx->desc.ngroups;
  if (mm->ngroups != G) return FORNAX_EINVAL;
  if (G > 64) return FORNAX_EUNSUPPORTED;
  if (!(mm->a_rad > 0.0) || !std::isfinite(mm->a_rad) || !(mm->tol > 0.0) || !(mm->tol < 1.0) ||
      mm->max_newton < 0)
    return FORNAX_EINVAL;
  if (!(mm->nu_edge[0] >= 0.0) || !std::isfinite(mm->nu_edge[0])) return FORNAX_EINVAL;
  for (int g = 0; g < G; ++g) {
    if (!(mm->nu_edge[g + 1] > mm->nu_edge[g])) return FORNAX_EINVAL;
    if (g + 1 < G && !std::isfinite(mm->nu_edge[g + 1])) return FORNAX_EINVAL;
    if (!(mm->nu_c[g] > 0.0) || !std::isfinite(mm->nu_c[g]) || !(mm->kg[g] >= 0.0) || !std::isfinite(mm->kg[g]))
      return FORNAX_EINVAL;
  }
  std::vector<double> tab((size_t)3 * G + 1);
  for (int g = 0; g <= G; ++g) tab[g] = mm->nu_edge[g];
  for (int g = 0; g < G; ++g) {
    tab[G + 1 + g] = mm->nu_c[g];
    tab[2 * G + 1 + g] = mm->kg[g];
  }
  if (!ctx->mat_tab && hipMalloc((void**)&ctx->mat_tab, tab.size() * sizeof(double)) != hipSuccess) {
    ctx->mat_tab = nullptr;
    return FORNAX_ENOMEM;
  }
  if (hipMemcpy(ctx->mat_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return FORNAX_EDEVICE;
  ctx->mat_a = mm->a_rad;
  ctx->mat_tol = mm->tol;
  ctx->mat_maxn = mm->max_newton;
  return FORNAX_OK;
}

// ---- velocity-dependent terms ----
int fornax_m1_set_group_edges(fornax_m1_ctx* ctx, const double* nu_edge) {
  if (!ctx || !nu_edge) return FORNAX_EINVAL;
  const int G = ctx->desc.ngroups;
  if (!(nu_edge[0] >= 0.0)) return FORNAX_EINVAL;
  for (int g = 0; g < G; ++g)
    if (!(nu_edge[g + 1] > nu_edge[g]) || !std::isfinite(nu_edge[g + 1])) return FORNAX_EINVAL;
  if (!ctx->vel_nu && hipMalloc((void**)&ctx->vel_nu, (size_t)(G + 1) * sizeof(double)) != hipSuccess) {
    ctx->vel_nu = nullptr;
    return FORNAX_ENOMEM;
  }
  if (hipMemcpy(ctx->vel_nu, nu_edge, (size_t)(G + 1) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return FORNAX_EDEVICE;
  return FORNAX_OK;
}

static int check_velocity(const fornax_m1_ctx* ctx, const fornax_m1_velocity* vel) {
  if (!vel) return FORNAX_EINVAL;
  const size_t al = ctx->desc.precision == FORNAX_FP64 ? 8 : 4;
  for (int d = 0; d < ctx->desc.ndim; ++d)
    if (!vel->v[d] || !aligned(vel->v[d], al)) return FORNAX_EINVAL;
  return FORNAX_OK;
}

int fornax_m1_step_velocity(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                            const fornax_m1_coeffs* cf, const double* inflow, const fornax_m1_velocity* vel, double dt,
                            const fornax_m1_diag* diag, void* stream) {
  if (!ctx) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, in)) || (rc = check_state(ctx, out)) || (rc = check_coeffs(ctx, cf)) ||
      (rc = check_velocity(ctx, vel)))
    return rc;
  if (!ctx->vel_nu) return FORNAX_EINVAL;
  if (overlaps(ctx, in, out)) return FORNAX_EINVAL;
  if (needs_inflow(ctx->desc) != (inflow != nullptr)) return FORNAX_EINVAL;
  const fornax_m1_desc& D = ctx->desc;
  if (D.integrator != FORNAX_EULER || D.limiter == FORNAX_LIMITER_PPM || D.wavespeed != FORNAX_WAVESPEED_LIGHT ||
      D.ngroups > fm1::BLOCK)
    return FORNAX_EUNSUPPORTED;
  if (!(dt > 0.0) || dt > ctx->max_dt1 * (1.0 + 1e-12)) return FORNAX_ECFL;
  return fm1_launch_step_velocity(ctx, in, out, cf, inflow, vel, dt, diag, (hipStream_t)stream);
}

int fornax_m1_lab_frame(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_velocity* vel, double* E_lab,
                        double* F_lab[3], void* stream) {
  if (!ctx || !E_lab || !F_lab) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, in)) || (rc = check_velocity(ctx, vel))) return rc;
  if (!aligned(E_lab, 8)) return FORNAX_EINVAL;
  for (int d = 0; d < ctx->desc.ndim; ++d)
    if (!F_lab[d] || !aligned(F_lab[d], 8)) return FORNAX_EINVAL;
  return fm1_launch_lab_frame(ctx, in, vel, E_lab, F_lab, (hipStream_t)stream);
}

static int check_matter(const fornax_m1_ctx* ctx, const fornax_m1_matter* m) {
  if (!ctx->mat_tab) return FORNAX_EINVAL;
  if (!m || !m->cv || !m->kappa0 || !m->T) return FORNAX_EINVAL;
  if (!aligned(m->cv, 8) || !aligned(m->kappa0, 8) || !aligned(m->T, 8)) return FORNAX_EINVAL;
  return FORNAX_OK;
}

int fornax_m1_matter_coeffs(fornax_m1_ctx* ctx, const fornax_m1_matter* m, void* kappa_out, void* B_out,
                            void* stream) {
  if (!ctx || !kappa_out || !B_out) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_matter(ctx, m))) return rc;
  const size_t al = ctx->desc.precision == FORNAX_FP64 ? 8 : 4;
  if (!aligned(kappa_out, al) || !aligned(B_out, al) || kappa_out == B_out) return FORNAX_EINVAL;
  return fm1_launch_matter_coeffs(ctx, m, kappa_out, B_out, (hipStream_t)stream);
}

int fornax_m1_matter_source(fornax_m1_ctx* ctx, fornax_m1_state* inout, const void* sigma,
                            const fornax_m1_matter* m, double dt, double* dE_matter, int32_t* iters, void* stream) {
  if (!ctx || !sigma) return FORNAX_EINVAL;
  int rc;
  if ((rc = check_state(ctx, inout)) || (rc = check_matter(ctx, m))) return rc;
  const size_t al = ctx->desc.precision == FORNAX_FP64 ? 8 : 4;
  if (!aligned(sigma, al) || (dE_matter && !aligned(dE_matter, 8)) || (iters && !aligned(iters, 4)))
    return FORNAX_EINVAL;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return FORNAX_EINVAL;
  return fm1_launch_matter_source(ctx, inout, sigma, m, dt, dE_matter, iters, (hipStream_t)stream);
}

int fornax_m1_copy_probe(void* dst, const void* src, int64_t nbytes, void* stream) {
  if (!dst || !src || nbytes < 0 || (nbytes % 16) != 0 || !aligned(dst, 16) || !aligned(src, 16))
    return FORNAX_EINVAL;
  return fm1_launch_copy(dst, src, nbytes, (hipStream_t)stream);
}

}  // extern "C"
