// m1_matter.hip -- the radiation-matter energy exchange (Interaction Terms: the inner
// backward-Euler update of every group, eq:be_update, inside the outer solve for the matter
// temperature; photons: one equation) and the matter model's opacities and emission.
//
// Layout: a zone's groups on consecutive lanes (lanes per zone = the power of two >= G, at
// most 64, so a zone never spans two waves); the outer iteration is uniform over a zone's
// lanes and the group sums are butterfly reductions among them.  Everything in double.

#include <hip/hip_runtime.h>

#include <cmath>

#include "m1_internal.h"

namespace fm1 {

namespace {

constexpr int MBLOCK = 256;

struct MatterTab {
  const double* nu_edge;   // [G + 1]
  const double* nu_c;      // [G]
  const double* kg;        // [G]
  double a_rad, tol;
  int maxn;
};

template <typename S>
struct MatterArgs {
  S* E;
  S* F[3];
  const S* sig;
  const double* cv;
  const double* kappa0;
  double* T;
  double* dEm;
  int* iters;
  MatterTab tab;
  int G, ndim, lg;      // lanes per zone = 1 << lg
  int64_t nzones;
  double c, dt;
};

// x^3 / (e^x - 1) integrated from 0 to x (x below the split), from the expansion of
// x / (e^x - 1) in Bernoulli numbers: x^3 (1/3 - x/8 + sum_j b_j x^(2j)),
// b_j = B_2j / ((2j)! (2j + 3)), summed by Horner's rule in x^2.
__device__ __forceinline__ double planck_low(double x) {
  const double y = x * x;
  double p = -236364091.0 / (1693824136731743669452800000.0 * 27.0);
  p = p * y + 77683.0 / (14101100039391805440000.0 * 25.0);
  p = p * y - 174611.0 / (802857662698291200000.0 * 23.0);
  p = p * y + 43867.0 / (5109094217170944000.0 * 21.0);
  p = p * y - 3617.0 / (10670622842880000.0 * 19.0);
  p = p * y + 1.0 / (74724249600.0 * 17.0);
  p = p * y - 691.0 / (1307674368000.0 * 15.0);
  p = p * y + 1.0 / (47900160.0 * 13.0);
  p = p * y - 1.0 / (1209600.0 * 11.0);
  p = p * y + 1.0 / (30240.0 * 9.0);
  p = p * y - 1.0 / (720.0 * 7.0);
  p = p * y + 1.0 / (12.0 * 5.0);
  return x * y * (1.0 / 3.0 - x * 0.125 + y * p);
}

// 1/n for the terms of the exponential series
__constant__ double c_recip[64] = {
    1.0,        1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,  1.0 / 6,  1.0 / 7,  1.0 / 8,  1.0 / 9,  1.0 / 10, 1.0 / 11,
    1.0 / 12,   1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17, 1.0 / 18, 1.0 / 19, 1.0 / 20, 1.0 / 21, 1.0 / 22,
    1.0 / 23,   1.0 / 24, 1.0 / 25, 1.0 / 26, 1.0 / 27, 1.0 / 28, 1.0 / 29, 1.0 / 30, 1.0 / 31, 1.0 / 32, 1.0 / 33,
    1.0 / 34,   1.0 / 35, 1.0 / 36, 1.0 / 37, 1.0 / 38, 1.0 / 39, 1.0 / 40, 1.0 / 41, 1.0 / 42, 1.0 / 43, 1.0 / 44,
    1.0 / 45,   1.0 / 46, 1.0 / 47, 1.0 / 48, 1.0 / 49, 1.0 / 50, 1.0 / 51, 1.0 / 52, 1.0 / 53, 1.0 / 54, 1.0 / 55,
    1.0 / 56,   1.0 / 57, 1.0 / 58, 1.0 / 59, 1.0 / 60, 1.0 / 61, 1.0 / 62, 1.0 / 63, 1.0 / 64};

// x^3 / (e^x - 1) integrated from x to infinity (x at or above the split; +inf gives 0):
// sum over n of the closed-form integral of x^3 e^(-n x), the powers e^(-n x) by products.
__device__ __forceinline__ double planck_high(double x) {
  if (!(x < INFINITY)) return 0.0;
  const double q = exp(-x);
  const double x2 = x * x, x3 = x2 * x;
  double qn = 1.0, s = 0.0;
  for (int n = 0; n < 64; ++n) {
    qn *= q;
    const double r = c_recip[n];
    const double term = qn * r * (x3 + r * (3.0 * x2 + r * (6.0 * x + 6.0 * r)));
    s += term;
    if (term <= 1e-18 * s) break;
  }
  return s;
}

constexpr double PLANCK_SPLIT = 1.5;

// one edge's value in the form the group integrals need: the integral from 0 below the
// split, the integral to infinity from the split on
__device__ __forceinline__ double planck_edge(double x) { return x < PLANCK_SPLIT ? planck_low(x) : planck_high(x); }

// integral of x^3 / (e^x - 1) over [a, b] (0 <= a <= b <= inf) from the edge values va, vb
// (planck_edge), without subtracting two nearly equal integrals; hs = planck_low(split),
// hh = planck_high(split)
__device__ __forceinline__ double planck_part_v(double a, double b, double va, double vb, double hs, double hh) {
  if (b < PLANCK_SPLIT) return vb - va;
  if (a >= PLANCK_SPLIT) return va - vb;
  return (hs - va) + (hh - vb);
}

__device__ __forceinline__ double planck_part(double a, double b, double hs, double hh) {
  return planck_part_v(a, b, planck_edge(a), planck_edge(b), hs, hh);
}

// the value v of the lane whose byte address (4 x lane) is addr
__device__ __forceinline__ double lane_value(int addr, double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// sum of v over the 2^lg lanes of a zone
__device__ __forceinline__ double zone_sum(double v, int lg) {
  for (int o = 1; o < (1 << lg); o <<= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename S>
__global__ void __launch_bounds__(MBLOCK) k_matter_coeffs(MatterArgs<S> a, S* kap_out, S* B_out) {
  const int64_t i = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
  if (i >= a.nzones * a.G) return;
  const int64_t z = i / a.G;
  const int g = (int)(i - z * a.G);
  const double T = a.T[z];
  const double hs = planck_low(PLANCK_SPLIT), hh = planck_high(PLANCK_SPLIT);
  const double kap = a.kappa0[z] * a.tab.kg[g] / sqrt(T) * -expm1(-a.tab.nu_c[g] / T);
  const double T2 = T * T;
  const double B = a.tab.a_rad * T2 * T2 * (15.0 / (M_PI * M_PI * M_PI * M_PI)) *
                   planck_part(a.tab.nu_edge[g] / T, a.tab.nu_edge[g + 1] / T, hs, hh);
  kap_out[i] = (S)kap;
  B_out[i] = (S)B;
}

template <typename S>
__global__ void __launch_bounds__(MBLOCK) k_matter_source(MatterArgs<S> a) {
  const int64_t gt = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
  const int64_t z = gt >> a.lg;
  const int g = (int)(gt & ((1 << a.lg) - 1));
  if (z >= a.nzones) return;   // whole zones leave together
  const bool on = g < a.G;
  const int gg = on ? g : 0;
  const int64_t zg = z * a.G + gg;
  const double Em = on ? (double)a.E[zg] : 0.0;
  const double cv = a.cv[z], k0 = a.kappa0[z], Tm = a.T[z];
  const double kq = on ? k0 * a.tab.kg[gg] : 0.0;
  const double nuc = a.tab.nu_c[gg], nhi = a.tab.nu_edge[gg + 1];
  const double cdt = a.c * a.dt;
  const double hs = planck_low(PLANCK_SPLIT), hh = planck_high(PLANCK_SPLIT);
  const double pnorm = a.tab.a_rad * 15.0 / (M_PI * M_PI * M_PI * M_PI);

  // the group's opacity and inner update at temperature T; r(T) summed over the zone.  A lane
  // evaluates the Planck integral at its group's lower edge and takes the upper edge's value
  // from the next lane (the zone's last lane evaluates its upper edge itself; lanes past the
  // last group evaluate the top edge)
  const int lpz = 1 << a.lg;
  const double nedge = a.tab.nu_edge[g < a.G ? g : a.G];
  const double ntop = a.tab.nu_edge[a.G];
  const int up = (((int)threadIdx.x + 1) & 63) << 2;   // byte address of the next lane (a zone's
                                                          // last lane does not use it)
  auto inner = [&](double T, double& kap) {
    const double iT = 1.0 / T;
    kap = kq * sqrt(iT) * -expm1(-nuc * iT);
    const double xa = nedge * iT;
    const double va = planck_edge(xa);
    const double vn = lane_value(up, va);
    const double xb = nhi * iT;
    const double vb = (g == lpz - 1) ? planck_edge(ntop * iT) : vn;
    const double T2 = T * T;
    const double B = pnorm * T2 * T2 * planck_part_v(xa, xb, va, vb, hs, hh);
    return (Em + cdt * kap * B) / (1.0 + cdt * kap);
  };
  auto residual = [&](double T) {
    double kap;
    const double E = inner(T, kap);
    return cv * (T - Tm) + zone_sum(on ? E - Em : 0.0, a.lg);
  };

  // outer solve: Newton with a forward-difference derivative and backtracking, then bisection
  double T = Tm, r = residual(Tm), T1 = Tm;
  int it_out = 0;
  bool done = false;
  for (int it = 0; it < a.tab.maxn && !done; ++it) {
    const double h = 1e-7 * T;
    const double J = (residual(T + h) - r) / h;
    if (!(J > 0.0)) break;
    const double d = -r / J;
    if (fabs(d) <= a.tab.tol * T) {
      T1 = T + d;
      it_out = it + 1;
      done = true;
      break;
    }
    double lam = 1.0, Tn = T, rn = r;
    bool ok = false;
    for (int ls = 0; ls <= 10; ++ls) {
      Tn = T + lam * d;
      if (Tn > 0.0) {
        rn = residual(Tn);
        if (fabs(rn) < fabs(r)) {
          ok = true;
          break;
        }
      }
      lam *= 0.5;
    }
    if (!ok) break;
    const bool conv = fabs(Tn - T) <= a.tab.tol * Tn;
    T = Tn;
    r = rn;
    if (conv) {
      T1 = T;
      it_out = it + 1;
      done = true;
    }
  }
  if (!done) {
    const double esum = zone_sum(on ? fmax(Em, 0.0) : 0.0, a.lg);
    double lo = 0.0, hi = Tm + esum / cv;
    int steps = 0;
    while (hi - lo > 1e-13 * hi && steps < 400) {
      const double mid = 0.5 * (lo + hi);
      if (residual(mid) > 0.0)
        hi = mid;
      else
        lo = mid;
      ++steps;
    }
    T1 = 0.5 * (lo + hi);
    it_out = -steps;
  }

  // the groups at T^{n+1}, the fluxes with the new opacity
  if (on) {
    double kap;
    const double E1 = inner(T1, kap);
    a.E[zg] = (S)E1;
    const double den = 1.0 + cdt * (kap + (double)a.sig[zg]);
    for (int k = 0; k < a.ndim; ++k) a.F[k][zg] = (S)((double)a.F[k][zg] / den);
  }
  if (g == 0) {
    a.T[z] = T1;
    if (a.dEm) a.dEm[z] = cv * (T1 - Tm);
    if (a.iters) a.iters[z] = it_out;
  }
}

template <typename S>
void fill_matter(const fornax_m1_ctx* ctx, MatterArgs<S>& a, const fornax_m1_matter* m) {
  const int G = ctx->desc.ngroups;
  a.G = G;
  a.ndim = ctx->desc.ndim;
  int lg = 0;
  while ((1 << lg) < G) ++lg;
  a.lg = lg;
  a.nzones = (int64_t)ctx->desc.n[0] * ctx->desc.n[1] * ctx->desc.n[2];
  a.c = ctx->desc.c;
  a.cv = m->cv;
  a.kappa0 = m->kappa0;
  a.T = m->T;
  a.tab.nu_edge = ctx->mat_tab;
  a.tab.nu_c = ctx->mat_tab + (G + 1);
  a.tab.kg = ctx->mat_tab + (2 * G + 1);
  a.tab.a_rad = ctx->mat_a;
  a.tab.tol = ctx->mat_tol;
  a.tab.maxn = ctx->mat_maxn;
  a.dEm = nullptr;
  a.iters = nullptr;
  a.sig = nullptr;
  a.E = nullptr;
  for (int k = 0; k < 3; ++k) a.F[k] = nullptr;
}

template <typename S>
int launch_matter_coeffs_t(fornax_m1_ctx* ctx, const fornax_m1_matter* m, void* kap, void* B, hipStream_t st) {
  MatterArgs<S> a;
  fill_matter<S>(ctx, a, m);
  const int64_t n = a.nzones * a.G;
  if (n == 0) return FORNAX_OK;
  hipLaunchKernelGGL(k_matter_coeffs<S>, dim3((unsigned)((n + MBLOCK - 1) / MBLOCK)), dim3(MBLOCK), 0, st, a, (S*)kap,
                     (S*)B);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

template <typename S>
int launch_matter_source_t(fornax_m1_ctx* ctx, fornax_m1_state* io, const void* sigma, const fornax_m1_matter* m,
                           double dt, double* dEm, int* iters, hipStream_t st) {
  MatterArgs<S> a;
  fill_matter<S>(ctx, a, m);
  a.E = (S*)io->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) a.F[k] = (S*)io->F[k];
  a.sig = (const S*)sigma;
  a.dt = dt;
  a.dEm = dEm;
  a.iters = iters;
  const int64_t n = a.nzones << a.lg;
  if (n == 0) return FORNAX_OK;
  hipLaunchKernelGGL(k_matter_source<S>, dim3((unsigned)((n + MBLOCK - 1) / MBLOCK)), dim3(MBLOCK), 0, st, a);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

}  // namespace

}  // namespace fm1

int fm1_launch_matter_coeffs(fornax_m1_ctx* ctx, const fornax_m1_matter* m, void* kap, void* B, hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64) return fm1::launch_matter_coeffs_t<double>(ctx, m, kap, B, stream);
  return fm1::launch_matter_coeffs_t<float>(ctx, m, kap, B, stream);
}

int fm1_launch_matter_source(fornax_m1_ctx* ctx, fornax_m1_state* io, const void* sigma, const fornax_m1_matter* m,
                             double dt, double* dEm, int* iters, hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return fm1::launch_matter_source_t<double>(ctx, io, sigma, m, dt, dEm, iters, stream);
  return fm1::launch_matter_source_t<float>(ctx, io, sigma, m, dt, dEm, iters, stream);
}
