// m1_kernels.hip -- gfx950 kernels of libfornax_m1 (one explicit transport + implicit
// interaction step of the multigroup M1 radiation moments, static medium).
//
// Method (Skinner et al. 2019, FORNAX):
//   finite-volume update, eq:finite_vol; linear reconstruction in the volume coordinate,
//   eq:recon_constraints with n = 1, minmod limited; M1 closure; HLL fluxes with the
//   asymptotic-diffusion correction of the energy flux, eq:hll / eq:epsilon; geometric source
//   terms of the covariant flux equation with the overrides eq:angmom / eq:grad2P;
//   backward-Euler interaction update eq:be_update and the flux update that follows it.
// Readings of details the paper leaves open (all shared with the library's documentation):
//   wavespeeds +-c (physical), i.e. +-c/h_d in x^d; tau_cell = mean (kappa + sigma) of the
//   two zones times their mean proper width; epsilon on the energy flux only; a zone whose
//   face state in direction d is not realizable (E <= 0 or |F^| > cE) is piecewise constant
//   in d; emissivity j = c kappa B; f^2 clamped to 1, Eddington value for E <= 0.
//
// Layout: structure of arrays, zone-group index ((k n1 + j) n0 + i) G + g, group innermost,
// so a block of whole zones reads and writes contiguous runs of every component.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "m1_device.h"
#include "m1_internal.h"
#include "m1_step.h"

namespace fm1 {

// second stage of the diagnostics reduction: one block of 1024 threads, each summing a fixed
// stride of the block partials (independent loads in flight), then the waves in order
// (deterministic, no atomics)
constexpr int FIN_THREADS = 1024;
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(const double* p_energy, const double* p_maxf2,
                                                           const int* p_nun, const int* p_nnp, int nb, double* energy,
                                                           double* maxf, int* nun, int* nnp) {
  __shared__ double sa[FIN_THREADS / 64], sb[FIN_THREADS / 64];
  __shared__ int su[FIN_THREADS / 64], sp[FIN_THREADS / 64];
  const int t = threadIdx.x;
  double ea = 0.0, mb = 0.0;
  int ua = 0, pa = 0;
#pragma unroll 4
  for (int b = t; b < nb; b += FIN_THREADS) {
    ea += p_energy[b];
    mb = fmax(mb, p_maxf2[b]);
    ua += p_nun[b];
    pa += p_nnp[b];
  }
  for (int off = 32; off > 0; off >>= 1) {
    ea += __shfl_xor(ea, off);
    mb = fmax(mb, __shfl_xor(mb, off));
    ua += __shfl_xor(ua, off);
    pa += __shfl_xor(pa, off);
  }
  if ((t & 63) == 0) {
    sa[t >> 6] = ea;
    sb[t >> 6] = mb;
    su[t >> 6] = ua;
    sp[t >> 6] = pa;
  }
  __syncthreads();
  if (t == 0) {
    double e = 0.0, m = 0.0;
    int u = 0, p = 0;
    for (int k = 0; k < FIN_THREADS / 64; ++k) {
      e += sa[k];
      m = fmax(m, sb[k]);
      u += su[k];
      p += sp[k];
    }
    if (energy) *energy = e;
    if (maxf) *maxf = sqrt(m);
    if (nun) *nun = u;
    if (nnp) *nnp = p;
  }
}

// ------------------------------------------------------------------------------------------
// Face fluxes only: one thread per face-group along direction d.
// ------------------------------------------------------------------------------------------
template <typename S, typename R, bool SPH, int ND>
__global__ void __launch_bounds__(BLOCK) k_flux(StepArgs<S> a, Geo<R> geo, int d, S* out) {
  int m[3] = {a.n[0], a.n[1], a.n[2]};
  m[d] += 1;
  const int64_t nfg = (int64_t)m[0] * m[1] * m[2] * a.G;
  const int64_t id = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (id >= nfg) return;
  const int grp = (int)(id % a.G);
  const int64_t f = id / a.G;
  int idx[3] = {(int)(f % m[0]), (int)((f / m[0]) % m[1]), (int)(f / ((int64_t)m[0] * m[1]))};
  const int fi = idx[d];
  // zones of the row: use an in-range index for the d position (fetch replaces it)
  int base[3] = {idx[0], idx[1], idx[2]};
  base[d] = 0;
  R q[4][4], ksL, ksR;
  for (int o = -2; o <= 1; ++o)
    fetch<S, R, SPH, ND>(a, geo, d, fi + o, base[0], base[1], base[2], grp, q[o + 2],
                         o == -1 ? &ksL : (o == 0 ? &ksR : nullptr));
  R fl[4];
  face_flux<S, R, SPH, ND>(a, geo, d, fi, base[0], base[1], reinterpret_cast<const R(*)[4]>(&q[0][0]), ksL, ksR,
                           fl);
  const int nc = 1 + ND;
  for (int c = 0; c < nc; ++c) out[id * nc + c] = (S)fl[c];
}

// ------------------------------------------------------------------------------------------
// Implicit interaction update alone (in place), double arithmetic.
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(BLOCK) k_source(StepArgs<S> a) {
  const int G = a.G;
  const int lz = threadIdx.x / G, grp = threadIdx.x - lz * G;
  const int64_t z = (int64_t)blockIdx.x * a.zones_per_block + lz;
  const bool act = (lz < a.zones_per_block) && (z < a.nzones);
  double dz = 0.0;
  if (act) {
    const int64_t zg = z * G + grp;
    const double kd = (double)a.kap[zg], sd = (double)a.sig[zg], Bd = (double)a.B[zg];
    const double c = a.c, dt = a.dt;
    const double Em = (double)a.E[zg];
    const double E1 = (Em + dt * (c * kd * Bd)) / (1.0 + (c * dt) * kd);
    const double fden = 1.0 + (c * dt) * (kd + sd);
    const S E1s = (S)E1;
    a.Eo[zg] = E1s;
    for (int cc = 0; cc < a.ndim; ++cc) a.Fo[cc][zg] = (S)((double)a.F[cc][zg] / fden);
    dz = (double)E1s - Em;
  }
  if (!a.dEm) return;
  __shared__ double sh[BLOCK];
  sh[threadIdx.x] = dz;
  __syncthreads();
  if (act && grp == 0) {
    double s = 0.0;
    for (int g2 = 0; g2 < G; ++g2) s += sh[threadIdx.x + g2];
    a.dEm[z] = -s;
  }
}

// dE_matter of every zone from the partial sums of the group blocks of the step tile, in
// group-block order.
__global__ void __launch_bounds__(BLOCK) k_dem_sum(const double* __restrict__ part, int nparts, int64_t nz,
                                                   double* __restrict__ dEm) {
  const int64_t z = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (z >= nz) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * nz + z];
  dEm[z] = -s;
}

__global__ void __launch_bounds__(BLOCK) k_copy(float4* __restrict__ dst, const float4* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) dst[i] = src[i];
}

}  // namespace fm1

using namespace fm1;

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
namespace fm1 {

template <typename S>
void fill_args(const fornax_m1_ctx* ctx, StepArgs<S>& a, const fornax_m1_coeffs* cf, const double* inflow,
               double dt) {
  const fornax_m1_desc& D = ctx->desc;
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
  a.zones_per_block = BLOCK / D.ngroups;
  a.nzones = (int64_t)D.n[0] * D.n[1] * D.n[2];
  a.c = D.c;
  a.dt = dt;
  a.f2_fp64 = D.f_fp64 * D.f_fp64;
  a.inflow = inflow;
  a.kap = (const S*)cf->kappa;
  a.sig = (const S*)cf->sigma;
  a.B = (const S*)cf->B;
  a.E = nullptr;
  a.Eo = nullptr;
  for (int k = 0; k < 3; ++k) {
    a.F[k] = nullptr;
    a.Fo[k] = nullptr;
  }
  a.dEm = nullptr;
  a.dzp = nullptr;
  a.src = 1;
  a.Ea = nullptr;
  for (int k = 0; k < 3; ++k) a.Fa[k] = nullptr;
  a.p_energy = nullptr;
  a.p_maxf2 = nullptr;
  a.p_nun = nullptr;
  a.p_nnp = nullptr;
}
template void fill_args<double>(const fornax_m1_ctx*, StepArgs<double>&, const fornax_m1_coeffs*, const double*,
                                double);
template void fill_args<float>(const fornax_m1_ctx*, StepArgs<float>&, const fornax_m1_coeffs*, const double*,
                               double);

}  // namespace fm1

namespace {

template <typename S, typename R>
int launch_step_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, fornax_m1_state* out,
                  const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_diag* diag,
                  const StepScratch& sc, hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, inflow, dt);
  a.E = (const S*)in->E;
  a.Eo = (S*)out->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) {
    a.F[k] = (const S*)in->F[k];
    a.Fo[k] = (S*)out->F[k];
  }
  bool want = diag && (diag->energy_total || diag->max_f || diag->n_unrealizable || diag->n_nonpositive);
  if (diag) a.dEm = diag->dE_matter;
  a.dzp = sc.dzp;
  if (want) {
    a.p_energy = sc.p_energy;
    a.p_maxf2 = sc.p_maxf2;
    a.p_nun = sc.p_nun;
    a.p_nnp = sc.p_nnp;
  }
  if (ctx->desc.integrator == FORNAX_SSPRK2) {
    // stage 1: U* = U^n + dt L(U^n) into the context's stage storage, no interaction update
    StepArgs<S> a1 = a;
    const size_t nzg = (size_t)a.nzones * a.G;
    S* st_E = (S*)sc.stage;
    a1.Eo = st_E;
    for (int k = 0; k < 3; ++k) a1.Fo[k] = (k < ctx->desc.ndim) ? st_E + (1 + k) * nzg : nullptr;
    a1.src = 0;
    a1.dEm = nullptr;
    a1.p_energy = a1.p_maxf2 = nullptr;
    a1.p_nun = a1.p_nnp = nullptr;
    const int rc1 = launch_tiled<S, R>(ctx, geo, a1, st);
    if (rc1 != FORNAX_OK) return rc1;
    // stage 2 reads U* and averages with U^n: U^- = (U^n + U* + dt L(U*)) / 2
    a.Ea = a.E;
    for (int k = 0; k < 3; ++k) a.Fa[k] = a.F[k];
    a.E = a1.Eo;
    for (int k = 0; k < 3; ++k) a.F[k] = a1.Fo[k];
  }
  const int rc = launch_tiled<S, R>(ctx, geo, a, st);
  if (rc != FORNAX_OK) return rc;
  const int nb = ctx->last_tile->nblocks;
  if (a.dEm && ctx->last_tile->ngb > 1) {
    hipLaunchKernelGGL(k_dem_sum, dim3((unsigned)((a.nzones + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, a.dzp,
                       ctx->last_tile->ngb, a.nzones, a.dEm);
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  if (want) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, st, sc.p_energy, sc.p_maxf2, sc.p_nun,
                       sc.p_nnp, nb,
                       diag->energy_total, diag->max_f, diag->n_unrealizable, diag->n_nonpositive);
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  return FORNAX_OK;
}

// The explicit transport alone: the step kernel without the interaction update (the state
// the interaction update would start from, U^-).  B is not used; the kernels still load it,
// so a missing B reads the opacity array instead.
template <typename S, typename R>
int launch_transport_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, fornax_m1_state* out,
                       const fornax_m1_coeffs* cf, const double* inflow, double dt, hipStream_t st) {
  fornax_m1_coeffs c2 = *cf;
  if (!c2.B) c2.B = c2.kappa;
  StepArgs<S> a;
  fill_args<S>(ctx, a, &c2, inflow, dt);
  a.src = 0;
  a.E = (const S*)in->E;
  a.Eo = (S*)out->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) {
    a.F[k] = (const S*)in->F[k];
    a.Fo[k] = (S*)out->F[k];
  }
  if (ctx->desc.integrator == FORNAX_SSPRK2) {
    StepArgs<S> a1 = a;
    const size_t nzg = (size_t)a.nzones * a.G;
    S* st_E = (S*)ctx->stage_mem;
    a1.Eo = st_E;
    for (int k = 0; k < 3; ++k) a1.Fo[k] = (k < ctx->desc.ndim) ? st_E + (1 + k) * nzg : nullptr;
    const int rc1 = launch_tiled<S, R>(ctx, geo, a1, st);
    if (rc1 != FORNAX_OK) return rc1;
    a.Ea = a.E;
    for (int k = 0; k < 3; ++k) a.Fa[k] = a.F[k];
    a.E = a1.Eo;
    for (int k = 0; k < 3; ++k) a.F[k] = a1.Fo[k];
  }
  return launch_tiled<S, R>(ctx, geo, a, st);
}

template <typename S, typename R>
int launch_flux_t(fornax_m1_ctx* ctx, const Geo<R>& geo, const fornax_m1_state* in, const fornax_m1_coeffs* cf,
                  const double* inflow, void* face_flux[3], hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, inflow, 0.0);
  a.E = (const S*)in->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) a.F[k] = (const S*)in->F[k];
  const bool sph = ctx->desc.coord == FORNAX_SPHERICAL_LOGR;
  for (int d = 0; d < ctx->desc.ndim; ++d) {
    int64_t m[3] = {a.n[0], a.n[1], a.n[2]};
    m[d] += 1;
    int64_t nfg = m[0] * m[1] * m[2] * a.G;
    dim3 grid((unsigned)((nfg + BLOCK - 1) / BLOCK));
    S* out = (S*)face_flux[d];
    const int nd = ctx->desc.ndim;
#define FM1_FLUX(SPHV, NDV) hipLaunchKernelGGL((k_flux<S, R, SPHV, NDV>), grid, dim3(BLOCK), 0, st, a, geo, d, out)
    if (sph) {
      if (nd == 1) FM1_FLUX(true, 1);
      else if (nd == 2) FM1_FLUX(true, 2);
      else FM1_FLUX(true, 3);
    } else {
      if (nd == 1) FM1_FLUX(false, 1);
      else if (nd == 2) FM1_FLUX(false, 2);
      else FM1_FLUX(false, 3);
    }
#undef FM1_FLUX
    if (hipGetLastError() != hipSuccess) return FORNAX_EDEVICE;
  }
  return FORNAX_OK;
}

template <typename S>
int launch_source_t(fornax_m1_ctx* ctx, fornax_m1_state* io, const fornax_m1_coeffs* cf, double dt, double* dEm,
                    hipStream_t st) {
  StepArgs<S> a;
  fill_args<S>(ctx, a, cf, nullptr, dt);
  a.E = (const S*)io->E;
  a.Eo = (S*)io->E;
  for (int k = 0; k < ctx->desc.ndim; ++k) {
    a.F[k] = (const S*)io->F[k];
    a.Fo[k] = (S*)io->F[k];
  }
  a.dEm = dEm;
  hipLaunchKernelGGL(k_source<S>, dim3(ctx->nblocks_step), dim3(BLOCK), 0, st, a);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

}  // namespace

int fm1_launch_step(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out, const fornax_m1_coeffs* cf,
                    const double* inflow, double dt, const fornax_m1_diag* diag, hipStream_t stream) {
  const StepScratch sc{ctx->p_energy, ctx->p_maxf2, ctx->p_nun, ctx->p_nnp, ctx->dzp, ctx->stage_mem};
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_step_t<double, double>(ctx, ctx->geo_d, in, out, cf, inflow, dt, diag, sc, stream);
  return launch_step_t<float, float>(ctx, ctx->geo_f, in, out, cf, inflow, dt, diag, sc, stream);
}

// ------------------------------------------------------------------------------------------
// Static scratch of fornax_m1_step_noalloc: one array per device for the callers that cannot
// allocate.  In host code `scratch` names a host-side stand-in: kernels and copies take the
// device address obtained once per device with hipGetSymbolAddress (g_scratch_ptr).
// ------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FORNAX_M1_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int fm1_static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return FORNAX_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return FORNAX_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return FORNAX_EDEVICE;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FORNAX_EDEVICE;
  g_scratch_ptr[device] = ptr;
  return FORNAX_OK;
}

int fm1_launch_step_noalloc(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                            const fornax_m1_coeffs* cf, const double* inflow, double dt, const fornax_m1_diag* diag,
                            hipStream_t stream) {
  // the address was set up when a context was first created on this device
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
  }
  if (!base) return FORNAX_EDEVICE;
  // layout: the partials of every block the step kernels may launch, the dE_matter partials of
  // split group blocks (when dE_matter is asked for), the Runge-Kutta stage; each part 256-byte
  // aligned (no part needs clearing: every launch writes what it reads)
  const fornax_m1_desc& D = ctx->desc;
  const size_t nb = ctx->nb_partials;
  const size_t nz = (size_t)D.n[0] * D.n[1] * D.n[2];
  const size_t es = D.precision == FORNAX_FP64 ? sizeof(double) : sizeof(float);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  const size_t o_energy = off;
  off += al(nb * sizeof(double));
  const size_t o_maxf2 = off;
  off += al(nb * sizeof(double));
  const size_t o_nun = off;
  off += al(nb * sizeof(int));
  const size_t o_nnp = off;
  off += al(nb * sizeof(int));
  const size_t ngb = (size_t)std::max(std::max(ctx->tile.ngb, ctx->tile_v1.ngb), ctx->c3.ngb);
  const bool need_dzp = diag && diag->dE_matter && ngb > 1;
  const size_t o_dzp = off;
  if (need_dzp) off += al(ngb * nz * sizeof(double));
  const bool need_stage = D.integrator == FORNAX_SSPRK2;
  const size_t o_stage = off;
  if (need_stage) off += al((size_t)(1 + D.ndim) * nz * D.ngroups * es);
  if (off > (size_t)FORNAX_M1_NOALLOC_SCRATCH_BYTES) return FORNAX_ESCRATCH;
  char* b = (char*)base;
  const StepScratch sc{(double*)(b + o_energy), (double*)(b + o_maxf2), (int*)(b + o_nun), (int*)(b + o_nnp),
                       need_dzp ? (double*)(b + o_dzp) : nullptr,
                       need_stage ? (void*)(b + o_stage) : nullptr};
  if (D.precision == FORNAX_FP64)
    return launch_step_t<double, double>(ctx, ctx->geo_d, in, out, cf, inflow, dt, diag, sc, stream);
  return launch_step_t<float, float>(ctx, ctx->geo_f, in, out, cf, inflow, dt, diag, sc, stream);
}

int fm1_launch_transport(fornax_m1_ctx* ctx, const fornax_m1_state* in, fornax_m1_state* out,
                         const fornax_m1_coeffs* cf, const double* inflow, double dt, hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_transport_t<double, double>(ctx, ctx->geo_d, in, out, cf, inflow, dt, stream);
  return launch_transport_t<float, float>(ctx, ctx->geo_f, in, out, cf, inflow, dt, stream);
}

int fm1_launch_flux(fornax_m1_ctx* ctx, const fornax_m1_state* in, const fornax_m1_coeffs* cf, const double* inflow,
                    void* face_flux[3], hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64)
    return launch_flux_t<double, double>(ctx, ctx->geo_d, in, cf, inflow, face_flux, stream);
  return launch_flux_t<float, float>(ctx, ctx->geo_f, in, cf, inflow, face_flux, stream);
}

int fm1_launch_source(fornax_m1_ctx* ctx, fornax_m1_state* inout, const fornax_m1_coeffs* cf, double dt, double* dEm,
                      hipStream_t stream) {
  if (ctx->desc.precision == FORNAX_FP64) return launch_source_t<double>(ctx, inout, cf, dt, dEm, stream);
  return launch_source_t<float>(ctx, inout, cf, dt, dEm, stream);
}

int fm1_launch_finalize(const double* p_energy, const double* p_maxf2, const int* p_nun, const int* p_nnp, int nb,
                        const fornax_m1_diag* diag, hipStream_t stream) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, stream, p_energy, p_maxf2, p_nun, p_nnp, nb,
                     diag->energy_total, diag->max_f, diag->n_unrealizable, diag->n_nonpositive);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}

int fm1_launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t stream) {
  int64_t n = nbytes / 16;
  if (n == 0) return FORNAX_OK;
  // one 16-byte element per thread over a grid that covers the array (on MI355X this moves
  // 1-4 GiB at about 6.2 TB/s, ahead of a grid-stride loop over 8192 blocks at 4.5-4.7 TB/s
  // and of hipMemcpyAsync at 4.7-5.1 TB/s); the loop only runs past 2^31 - 1 blocks
  int64_t blocks = (n + BLOCK - 1) / BLOCK;
  if (blocks > 0x7fffffff) blocks = 0x7fffffff;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(BLOCK), 0, stream, (float4*)dst, (const float4*)src, n);
  return hipGetLastError() == hipSuccess ? FORNAX_OK : FORNAX_EDEVICE;
}
