// Real-time propagation of a block (Sec. "Real-time TDDFT", Eq. (td_ks)):
// i S~ d psi / dt = H~ psi, one Crank-Nicolson step per call with H~ held
// fixed over the step,
//   (S~ + i tau H~) psi(t + dt) = (S~ - i tau H~) psi(t),   tau = dt / 2,
// plus the delta kick psi -> exp(-i kappa . r) psi and the pseudo-density
// dipole that the propagation records.
//
// The linear system is solved band by band with conjugate orthogonal
// conjugate gradients (COCG): for k = 0 the operators are real symmetric, so
// M = S~ + i tau H~ is complex symmetric and the CG recurrences hold with the
// unconjugated bilinear form (x, y) = sum_g x_g y_g. Each iteration applies
// M once through the library's own H~/S~ kernels (projections, Delta.P, the
// fused stencil with both add-backs) and then runs three streaming passes
// over the block; every band carries its own scalars on the device. The
// bilinear forms and norms are formed as per-(band, chunk) partials in a
// fixed order and summed per band in chunk order, so the iteration is
// reproducible. The host reads the residual norms after each iteration
// (one synchronisation per M application) to stop.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace gfd {

namespace {

constexpr int TD_CH = 64;     // chunks per band for the partial sums
constexpr int TD_PART = 4;    // doubles per (band, chunk) partial

struct TdWs {
  z64 *b, *r, *p, *q, *sp;    // [nb][Ng]
  double *part;               // [nb][TD_CH][TD_PART]
  z64 *rho, *alpha, *beta;    // [nb]
  double *bn2, *rn2;          // [nb]
  double *host;               // pinned [2 nb]
};

int chunks_for(int64_t ng) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(TD_CH, (ng + 4095) / 4096)));
}

__device__ inline z64 mul_i(double t, z64 a) { return z64{-t * a.y, t * a.x}; }  // i t a

// block of 256 lanes: sums v[0..3] over the workgroup into part (lane 0)
__device__ inline void wg_sum4(double v0, double v1, double v2, double v3, double *out) {
  __shared__ double red[4][256];
  red[0][threadIdx.x] = v0;
  red[1][threadIdx.x] = v1;
  red[2][threadIdx.x] = v2;
  red[3][threadIdx.x] = v3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = red[c][0];
}

// chunk range of workgroup (blockIdx.x) of band blockIdx.y
__device__ inline void chunk_range(int64_t ng, int64_t &lo, int64_t &hi) {
  const int64_t per = (ng + gridDim.x - 1) / gridDim.x;
  lo = static_cast<int64_t>(blockIdx.x) * per;
  hi = std::min(ng, lo + per);
}

// b = Sx - i tau Hx; r = b - M x = -2 i tau Hx; p = r.
// partials: (r, r) (re, im), |b|^2, |r|^2
__global__ __launch_bounds__(256) void k_td_init(const z64 *__restrict__ Hx,
                                                 const z64 *__restrict__ Sx, z64 *__restrict__ b,
                                                 z64 *__restrict__ r, z64 *__restrict__ p,
                                                 double tau, int64_t ng, double *__restrict__ part) {
  int64_t lo, hi;
  chunk_range(ng, lo, hi);
  const int64_t base = static_cast<int64_t>(blockIdx.y) * ng;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int64_t g = lo + threadIdx.x; g < hi; g += 256) {
    const z64 h = Hx[base + g], s = Sx[base + g];
    const z64 bb = s - mul_i(tau, h);
    const z64 rr = mul_i(-2.0 * tau, h);
    b[base + g] = bb;
    r[base + g] = rr;
    p[base + g] = rr;
    const z64 rr2 = rr * rr;
    s0 += rr2.x;
    s1 += rr2.y;
    s2 += bb.x * bb.x + bb.y * bb.y;
    s3 += rr.x * rr.x + rr.y * rr.y;
  }
  wg_sum4(s0, s1, s2, s3, part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * TD_PART);
}

// q = Sp + i tau Hp (into Hp); partials: (p, q)
__global__ __launch_bounds__(256) void k_td_q(const z64 *__restrict__ p, z64 *__restrict__ Hp,
                                              const z64 *__restrict__ Sp, double tau, int64_t ng,
                                              double *__restrict__ part) {
  int64_t lo, hi;
  chunk_range(ng, lo, hi);
  const int64_t base = static_cast<int64_t>(blockIdx.y) * ng;
  double s0 = 0, s1 = 0;
  for (int64_t g = lo + threadIdx.x; g < hi; g += 256) {
    const z64 q = Sp[base + g] + mul_i(tau, Hp[base + g]);
    Hp[base + g] = q;
    const z64 pq = p[base + g] * q;
    s0 += pq.x;
    s1 += pq.y;
  }
  wg_sum4(s0, s1, 0.0, 0.0, part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * TD_PART);
}

// x += alpha p; r -= alpha q; partials: (r, r), |r|^2
__global__ __launch_bounds__(256) void k_td_update(z64 *__restrict__ x, z64 *__restrict__ r,
                                                   const z64 *__restrict__ p,
                                                   const z64 *__restrict__ q,
                                                   const z64 *__restrict__ alpha, int64_t ng,
                                                   double *__restrict__ part) {
  int64_t lo, hi;
  chunk_range(ng, lo, hi);
  const int64_t base = static_cast<int64_t>(blockIdx.y) * ng;
  const z64 a = alpha[blockIdx.y];
  double s0 = 0, s1 = 0, s3 = 0;
  for (int64_t g = lo + threadIdx.x; g < hi; g += 256) {
    x[base + g] = x[base + g] + a * p[base + g];
    const z64 rr = r[base + g] - a * q[base + g];
    r[base + g] = rr;
    const z64 rr2 = rr * rr;
    s0 += rr2.x;
    s1 += rr2.y;
    s3 += rr.x * rr.x + rr.y * rr.y;
  }
  wg_sum4(s0, s1, 0.0, s3, part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * TD_PART);
}

// p = r + beta p
__global__ __launch_bounds__(256) void k_td_dir(const z64 *__restrict__ r, z64 *__restrict__ p,
                                                const z64 *__restrict__ beta, int64_t ng) {
  int64_t lo, hi;
  chunk_range(ng, lo, hi);
  const int64_t base = static_cast<int64_t>(blockIdx.y) * ng;
  const z64 bt = beta[blockIdx.y];
  for (int64_t g = lo + threadIdx.x; g < hi; g += 256) p[base + g] = r[base + g] + bt * p[base + g];
}

__device__ inline z64 zdiv(z64 a, z64 b) {
  const double d = b.x * b.x + b.y * b.y;
  if (!(d > 0.0)) return z64{0.0, 0.0};  // breakdown or a converged band: no step
  return z64{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// per band, chunk partials summed in chunk order. mode 0 (after init):
// rho = s01, bn2 = s2, rn2 = s3; mode 1: alpha = rho / s01; mode 2 (after
// the update): beta = s01 / rho, rho = s01, rn2 = s3
__global__ __launch_bounds__(256) void k_td_scalars(const double *__restrict__ part, int nch,
                                                    int nb, int mode, z64 *__restrict__ rho,
                                                    z64 *__restrict__ alpha, z64 *__restrict__ beta,
                                                    double *__restrict__ bn2,
                                                    double *__restrict__ rn2) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= nb) return;
  double s[4] = {0, 0, 0, 0};
  for (int c = 0; c < nch; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] += part[(static_cast<int64_t>(n) * nch + c) * TD_PART + e];
  const z64 s01{s[0], s[1]};
  if (mode == 0) {
    rho[n] = s01;
    bn2[n] = s[2];
    rn2[n] = s[3];
  } else if (mode == 1) {
    alpha[n] = zdiv(rho[n], s01);
  } else {
    beta[n] = zdiv(s01, rho[n]);
    rho[n] = s01;
    rn2[n] = s[3];
  }
}

// psi *= exp(-i kappa . r), r = (i h0, j h1, l h2)
__global__ __launch_bounds__(256) void k_td_kick(z64 *__restrict__ psi, int64_t ng, int n1, int n2,
                                                 double k0, double k1, double k2) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= ng) return;
  const int l = static_cast<int>(g % n2);
  const int64_t t = g / n2;
  const int j = static_cast<int>(t % n1), i = static_cast<int>(t / n1);
  const double arg = -(k0 * i + k1 * j + k2 * l);
  double sn, cs;
  sincos(arg, &sn, &cs);
  const int64_t o = static_cast<int64_t>(blockIdx.y) * ng + g;
  psi[o] = psi[o] * z64{cs, sn};
}

// partials of f_n sum_g x_c(g) |psi_n(g)|^2, c = 0..2
__global__ __launch_bounds__(256) void k_td_dipole(const z64 *__restrict__ psi,
                                                   const double *__restrict__ f, int64_t ng, int n1,
                                                   int n2, double h0, double h1, double h2,
                                                   double *__restrict__ part) {
  int64_t lo, hi;
  chunk_range(ng, lo, hi);
  const int64_t base = static_cast<int64_t>(blockIdx.y) * ng;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int64_t g = lo + threadIdx.x; g < hi; g += 256) {
    const z64 v = psi[base + g];
    const double d = v.x * v.x + v.y * v.y;
    const int l = static_cast<int>(g % n2);
    const int64_t t = g / n2;
    const int j = static_cast<int>(t % n1), i = static_cast<int>(t / n1);
    s0 += i * h0 * d;
    s1 += j * h1 * d;
    s2 += l * h2 * d;
  }
  const double fn = f[blockIdx.y];
  wg_sum4(fn * s0, fn * s1, fn * s2, 0.0,
          part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * TD_PART);
}

// d[c] = dV sum over bands, then chunks, in order
__global__ void k_td_dipole_sum(const double *__restrict__ part, int nb, int nch, double dV,
                                double *__restrict__ d) {
  const int c = threadIdx.x;
  if (c >= 3) return;
  double s = 0.0;
  for (int64_t i = 0; i < static_cast<int64_t>(nb) * nch; ++i) s += part[i * TD_PART + c];
  d[c] = dV * s;
}

int ensure_td_ws(gpaw_sys *s, TdWs &w) {
  const int64_t blk = static_cast<int64_t>(s->max_bands) * s->ng;
  const size_t need = 5 * blk * sizeof(z64) +
                      static_cast<size_t>(s->max_bands) * TD_CH * TD_PART * sizeof(double) +
                      3 * s->max_bands * sizeof(z64) + 2 * s->max_bands * sizeof(double);
  if (s->td_bytes < need) {
    if (s->td) (void)hipFree(s->td);
    if (s->td_host) (void)hipHostFree(s->td_host);
    s->td = nullptr;
    s->td_host = nullptr;
    s->td_bytes = 0;
    if (hipMalloc(&s->td, need) != hipSuccess ||
        hipHostMalloc(&s->td_host, 2 * s->max_bands * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      if (s->td) (void)hipFree(s->td);
      s->td = nullptr;
      return fail(GPAW_ENOMEM, "time-propagation workspace: device allocation failed");
    }
    s->td_bytes = need;
  }
  char *c = static_cast<char *>(s->td);
  z64 *z = reinterpret_cast<z64 *>(c);
  w.b = z;
  w.r = z + blk;
  w.p = z + 2 * blk;
  w.q = z + 3 * blk;
  w.sp = z + 4 * blk;
  w.part = reinterpret_cast<double *>(z + 5 * blk);
  w.rho = reinterpret_cast<z64 *>(w.part + static_cast<int64_t>(s->max_bands) * TD_CH * TD_PART);
  w.alpha = w.rho + s->max_bands;
  w.beta = w.alpha + s->max_bands;
  w.bn2 = reinterpret_cast<double *>(w.beta + s->max_bands);
  w.rn2 = w.bn2 + s->max_bands;
  w.host = static_cast<double *>(s->td_host);
  return GPAW_OK;
}

int apply_HS_block(gpaw_sys *s, const void *x, int nb, void *Hx, void *Sx, hipStream_t st) {
  int rc;
  const void *X = nullptr, *XS = nullptr;
  if (s->np > 0) {
    if ((rc = launch_project(s, x, nb, s->ws.P, st)) != GPAW_OK) return rc;
    if ((rc = launch_dmat2(s, s->ws.P, nb, s->ws.X, s->ws.XS, st)) != GPAW_OK) return rc;
    X = s->ws.X;
    XS = s->ws.XS;
  }
  return launch_stencil(s, x, nb, X, Hx, st, XS, Sx);
}

int check_td(const gpaw_sys *s, int32_t nb, const void *psi) {
  if (!s) return fail(GPAW_EINVAL, "system is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != s->device)
    return fail(GPAW_EINVAL, "current HIP device differs from the system's device");
  if (nb < 1 || nb > s->max_bands) return fail(GPAW_ESHAPE, "nb outside [1, max_bands]");
  if (!psi) return fail(GPAW_EINVAL, "psi must not be NULL");
  if (s->dtype != GPAW_C128)
    return fail(GPAW_EDTYPE, "time propagation needs complex128 wave functions");
  return GPAW_OK;
}

}  // namespace
}  // namespace gfd

using namespace gfd;

extern "C" {

int gpaw_td_kick(gpaw_sys *s, void *psi, int32_t nb, const double *kappa, void *stream) {
  int rc = check_td(s, nb, psi);
  if (rc != GPAW_OK) return rc;
  if (!kappa) return fail(GPAW_EINVAL, "kappa must not be NULL");
  const dim3 grid(static_cast<unsigned>((s->ng + 255) / 256), static_cast<unsigned>(nb));
  k_td_kick<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<z64 *>(psi), s->ng, s->n[1], s->n[2], kappa[0] * s->h[0], kappa[1] * s->h[1],
      kappa[2] * s->h[2]);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_td_kick");
}

int gpaw_td_dipole(gpaw_sys *s, const void *psi, int32_t nb, const double *f, double *d,
                   void *stream) {
  int rc = check_td(s, nb, psi);
  if (rc != GPAW_OK) return rc;
  if (!f || !d) return fail(GPAW_EINVAL, "f and d must not be NULL");
  TdWs w;
  if ((rc = ensure_td_ws(s, w)) != GPAW_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nch = chunks_for(s->ng);
  k_td_dipole<<<dim3(nch, nb), 256, 0, st>>>(static_cast<const z64 *>(psi), f, s->ng, s->n[1],
                                             s->n[2], s->h[0], s->h[1], s->h[2], w.part);
  k_td_dipole_sum<<<1, 64, 0, st>>>(w.part, nb, nch, s->dV, d);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_td_dipole");
}

int gpaw_td_propagate(gpaw_sys *s, void *psi, int32_t nb, double dt, double tol,
                      int32_t max_iter, int32_t *iters, double *rel_residual, void *stream) {
  int rc = check_td(s, nb, psi);
  if (rc != GPAW_OK) return rc;
  if (s->k[0] != 0.0 || s->k[1] != 0.0 || s->k[2] != 0.0)
    return fail(GPAW_EINVAL, "time propagation needs k = 0 (real symmetric operators)");
  if (!std::isfinite(dt) || !(tol >= 0.0) || max_iter < 1)
    return fail(GPAW_EINVAL, "finite dt, tol >= 0 and max_iter >= 1 required");
  TdWs w;
  if ((rc = ensure_td_ws(s, w)) != GPAW_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double tau = 0.5 * dt;
  const int nch = chunks_for(s->ng);
  const dim3 grid(nch, nb);
  const unsigned sgrid = static_cast<unsigned>((nb + 255) / 256);
  z64 *x = static_cast<z64 *>(psi);
  auto residual = [&](double *out) -> int {
    hipError_t e = hipMemcpyAsync(w.host, w.bn2, 2 * s->max_bands * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gpaw_td_propagate");
    double worst = 0.0;
    for (int n = 0; n < nb; ++n) {
      const double b2 = w.host[n], r2 = w.host[s->max_bands + n];
      const double rel = b2 > 0.0 ? std::sqrt(r2 / b2) : std::sqrt(r2);
      if (!(rel <= worst)) worst = rel;  // a NaN stays the worst
    }
    *out = worst;
    return GPAW_OK;
  };
  // right-hand side and the first residual from psi(t) (the initial guess)
  if ((rc = apply_HS_block(s, x, nb, w.q, w.sp, st)) != GPAW_OK) return rc;
  k_td_init<<<grid, 256, 0, st>>>(w.q, w.sp, w.b, w.r, w.p, tau, s->ng, w.part);
  k_td_scalars<<<sgrid, 256, 0, st>>>(w.part, nch, nb, 0, w.rho, w.alpha, w.beta, w.bn2, w.rn2);
  double rel = 0.0;
  if ((rc = residual(&rel)) != GPAW_OK) return rc;
  int32_t it = 0;
  while (rel > tol && it < max_iter) {
    if ((rc = apply_HS_block(s, w.p, nb, w.q, w.sp, st)) != GPAW_OK) return rc;
    k_td_q<<<grid, 256, 0, st>>>(w.p, w.q, w.sp, tau, s->ng, w.part);
    k_td_scalars<<<sgrid, 256, 0, st>>>(w.part, nch, nb, 1, w.rho, w.alpha, w.beta, w.bn2, w.rn2);
    k_td_update<<<grid, 256, 0, st>>>(x, w.r, w.p, w.q, w.alpha, s->ng, w.part);
    k_td_scalars<<<sgrid, 256, 0, st>>>(w.part, nch, nb, 2, w.rho, w.alpha, w.beta, w.bn2, w.rn2);
    k_td_dir<<<grid, 256, 0, st>>>(w.r, w.p, w.beta, s->ng);
    ++it;
    if ((rc = residual(&rel)) != GPAW_OK) return rc;
  }
  if (iters) *iters = it;
  if (rel_residual) *rel_residual = rel;
  if (!std::isfinite(rel)) return fail(GPAW_ENONFINITE, "gpaw_td_propagate: non-finite residual");
  if (rel > tol) return fail(GPAW_ENOCONV, "gpaw_td_propagate: COCG did not reach tol");
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_td_propagate");
}

}  // extern "C"
