// Multigrid Poisson solver for finite systems (Sec. "Solving the Kohn-Sham
// equation": iterative multigrid Poisson solvers with Jacobi smoothing; the
// potential vanishes on the cell boundary of a finite system) and the grid
// transfers it is built from (interpolation between uniform grids is one of
// the C hot spots of Sec. "Developer's perspective").
//
// nabla^2 phi = -4 pi rho on the N0 x N1 x N2 interior points of a
// zero-boundary box (values past the faces are zero, also for the 6th-order
// stencil's reach of three points). Levels halve odd sizes, N = 2 m + 1 to
// m, coarse point j on fine point 2 j + 1 (0-based); restriction is full
// weighting (1/4, 1/2, 1/4 per axis), interpolation trilinear. A V-cycle
// runs two weighted-Jacobi sweeps (omega = 0.8) before and after the coarse
// correction; the coarsest level (an even axis, or one below 3 points) gets
// 20 x its largest axis sweeps. The host drives the cycles and stops at the
// requested relative residual.
//
// The grids of this solver are small next to the wave-function blocks (one
// potential per system), and they stay resident in the XCDs' L2 and the
// Infinity Cache across a sweep; every kernel is one lane per output point
// with coalesced rows along the contiguous axis. The coarsest level's many
// sweeps run in one workgroup with the level in LDS (one barrier per sweep)
// when it fits, instead of one launch per sweep.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace gfd {

namespace {

constexpr double PW0 = -49.0 / 18.0, PW1 = 1.5, PW2 = -0.15, PW3 = 1.0 / 90.0;
constexpr double JACOBI_OMEGA = 0.8;
constexpr int PRE_SWEEPS = 2, POST_SWEEPS = 2;  // even: the result lands in phi

struct Dims {
  int n0, n1, n2;
  double i0, i1, i2;  // 1 / h_c^2
};

__device__ inline double at(const double *f, const Dims &d, int x, int y, int z) {
  return (x >= 0 && x < d.n0 && y >= 0 && y < d.n1 && z >= 0 && z < d.n2)
             ? f[(static_cast<int64_t>(x) * d.n1 + y) * d.n2 + z]
             : 0.0;
}

__device__ inline double lap_at(const double *f, const Dims &d, int x, int y, int z) {
  const double c = f[(static_cast<int64_t>(x) * d.n1 + y) * d.n2 + z];
  double sx = PW0 * c, sy = PW0 * c, sz = PW0 * c;
  sx += PW1 * (at(f, d, x + 1, y, z) + at(f, d, x - 1, y, z));
  sx += PW2 * (at(f, d, x + 2, y, z) + at(f, d, x - 2, y, z));
  sx += PW3 * (at(f, d, x + 3, y, z) + at(f, d, x - 3, y, z));
  sy += PW1 * (at(f, d, x, y + 1, z) + at(f, d, x, y - 1, z));
  sy += PW2 * (at(f, d, x, y + 2, z) + at(f, d, x, y - 2, z));
  sy += PW3 * (at(f, d, x, y + 3, z) + at(f, d, x, y - 3, z));
  sz += PW1 * (at(f, d, x, y, z + 1) + at(f, d, x, y, z - 1));
  sz += PW2 * (at(f, d, x, y, z + 2) + at(f, d, x, y, z - 2));
  sz += PW3 * (at(f, d, x, y, z + 3) + at(f, d, x, y, z - 3));
  return sx * d.i0 + sy * d.i1 + sz * d.i2;
}

// mode 0: out = A f (zero-boundary Laplacian); mode 1: out = rhs - A f
// (the residual); mode 2: out = f + w (rhs - A f) (a weighted Jacobi sweep,
// w = omega / diag(A))
__global__ __launch_bounds__(256) void k_zlap(const double *__restrict__ f,
                                              const double *__restrict__ rhs,
                                              double *__restrict__ out, Dims d, int mode,
                                              double w) {
  const int64_t ng = static_cast<int64_t>(d.n0) * d.n1 * d.n2;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= ng) return;
  const int z = static_cast<int>(g % d.n2);
  const int64_t r = g / d.n2;
  const int y = static_cast<int>(r % d.n1), x = static_cast<int>(r / d.n1);
  const double a = lap_at(f, d, x, y, z);
  if (mode == 0) out[g] = a;
  else if (mode == 1) out[g] = rhs[g] - a;
  else out[g] = f[g] + w * (rhs[g] - a);
}

// All sweeps of the coarsest level in one workgroup: phi, the scratch and
// the right-hand side live in LDS, one barrier per sweep. Each sweep does
// the same arithmetic as k_zlap's mode 2, so the result equals that of one
// launch per sweep bit for bit. Used up to one point per lane: past that a
// sweep in one workgroup costs more than a launch over the whole chip
// (measured: a 14 x 14 x 19 coarsest level took 2.9 ms per V-cycle this way
// against 1.7 ms with a launch per sweep).
constexpr int COARSE_LDS_POINTS = 1024;  // 3 x 1024 doubles = 24 KiB of LDS
__global__ __launch_bounds__(1024) void k_coarse_sweeps(double *__restrict__ phi,
                                                        const double *__restrict__ rhs, Dims d,
                                                        int sweeps, double w) {
  extern __shared__ double lds[];
  const int npts = d.n0 * d.n1 * d.n2;
  double *a = lds, *b = lds + npts, *f = lds + 2 * npts;
  for (int g = threadIdx.x; g < npts; g += 1024) {
    a[g] = phi[g];
    f[g] = rhs[g];
  }
  __syncthreads();
  for (int s = 0; s < sweeps; ++s) {
    const double *src = (s & 1) ? b : a;
    double *dst = (s & 1) ? a : b;
    for (int g = threadIdx.x; g < npts; g += 1024) {
      const int z = g % d.n2, r = g / d.n2;
      const int y = r % d.n1, x = r / d.n1;
      const double lap = lap_at(src, d, x, y, z);
      dst[g] = src[g] + w * (f[g] - lap);
    }
    __syncthreads();
  }
  const double *res = (sweeps & 1) ? b : a;
  for (int g = threadIdx.x; g < npts; g += 1024) phi[g] = res[g];
}

// coarse[j] = sum over the 27 fine neighbours of fine point 2 j + 1 of
// prod_c (1/4, 1/2, 1/4)[d_c] fine
__global__ __launch_bounds__(256) void k_restrict(const double *__restrict__ fine,
                                                  double *__restrict__ coarse, Dims fd, Dims cd) {
  const int64_t nc = static_cast<int64_t>(cd.n0) * cd.n1 * cd.n2;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= nc) return;
  const int z = static_cast<int>(g % cd.n2);
  const int64_t r = g / cd.n2;
  const int y = static_cast<int>(r % cd.n1), x = static_cast<int>(r / cd.n1);
  const int fx = 2 * x + 1, fy = 2 * y + 1, fz = 2 * z + 1;
  const double w[3] = {0.25, 0.5, 0.25};
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double sa = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double *row = fine + ((static_cast<int64_t>(fx + a - 1) * fd.n1 + (fy + b - 1)) * fd.n2);
      const double sb = 0.25 * row[fz - 1] + 0.5 * row[fz] + 0.25 * row[fz + 1];
      sa += w[b] * sb;
    }
    acc += w[a] * sa;
  }
  coarse[g] = acc;
}

// fine[i] (+)= sum_j prod_c p(i_c, j_c) coarse[j], p = 1 on the coarse point,
// 1/2 next to it, zero past the faces
__global__ __launch_bounds__(256) void k_interp(const double *__restrict__ coarse,
                                                double *__restrict__ fine, Dims fd, Dims cd,
                                                int accumulate) {
  const int64_t nf = static_cast<int64_t>(fd.n0) * fd.n1 * fd.n2;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= nf) return;
  const int z = static_cast<int>(g % fd.n2);
  const int64_t r = g / fd.n2;
  const int y = static_cast<int>(r % fd.n1), x = static_cast<int>(r / fd.n1);
  // per axis: (coarse index, weight) pairs; 0-based fine i sits on coarse
  // (i - 1) / 2 when i is odd, between (i - 2) / 2 and i / 2 when even
  int jx[2], jy[2], jz[2];
  double wx[2], wy[2], wz[2];
  auto axis = [](int i, int m, int *j, double *w) {
    if (i & 1) {
      j[0] = (i - 1) / 2;
      w[0] = 1.0;
      j[1] = j[0];
      w[1] = 0.0;
    } else {
      j[0] = i / 2 - 1;
      j[1] = i / 2;
      w[0] = j[0] >= 0 ? 0.5 : 0.0;
      w[1] = j[1] < m ? 0.5 : 0.0;
      j[0] = std::max(j[0], 0);
      j[1] = std::min(j[1], m - 1);
    }
  };
  axis(x, cd.n0, jx, wx);
  axis(y, cd.n1, jy, wy);
  axis(z, cd.n2, jz, wz);
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double wt = wx[a] * wy[b] * wz[c];
        if (wt != 0.0) acc += wt * coarse[(static_cast<int64_t>(jx[a]) * cd.n1 + jy[b]) * cd.n2 + jz[c]];
      }
  fine[g] = accumulate ? fine[g] + acc : acc;
}

// out[g] = s * in[g]
__global__ __launch_bounds__(256) void k_scale(const double *__restrict__ in,
                                               double *__restrict__ out, int64_t n, double s) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g < n) out[g] = s * in[g];
}

__global__ __launch_bounds__(256) void k_fill0(double *__restrict__ out, int64_t n) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g < n) out[g] = 0.0;
}

// sum of squares: workgroup partials (grid-stride, fixed order), then one
// workgroup adds them in index order, so the sum is reproducible
constexpr int NRM_WGS = 1024;
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ x, int64_t n,
                                               double *__restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; g < n;
       g += static_cast<int64_t>(gridDim.x) * 256)
    s += x[g] * x[g];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int np,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

Dims dims_of(const int32_t *n, const double *h) {
  return Dims{n[0], n[1], n[2], 1.0 / (h[0] * h[0]), 1.0 / (h[1] * h[1]), 1.0 / (h[2] * h[2])};
}

bool coarsens(const int32_t *n) {
  for (int c = 0; c < 3; ++c)
    if (n[c] < 3 || n[c] % 2 == 0) return false;
  return true;
}

int check_dims(const int32_t *n, const double *h) {
  if (!n) return fail(GPAW_EINVAL, "grid sizes are NULL");
  for (int c = 0; c < 3; ++c) {
    if (n[c] < 1) return fail(GPAW_ESHAPE, "grid sizes must be positive");
    if (h && !(h[c] > 0.0)) return fail(GPAW_EINVAL, "grid spacings must be positive");
  }
  if (static_cast<int64_t>(n[0]) * n[1] * n[2] > (int64_t{1} << 31))
    return fail(GPAW_ESHAPE, "grid larger than 2^31 points");
  return GPAW_OK;
}

}  // namespace

struct PoissonLevel {
  int32_t n[3];
  double h[3];
  int64_t ng;
  double *f = nullptr, *phi = nullptr, *tmp = nullptr;  // phi of level 0 is the caller's
};

}  // namespace gfd

struct gpaw_poisson {
  std::vector<gfd::PoissonLevel> lv;
  bool coarse_lds_ok = false;  // the coarsest level's sweeps may run in one workgroup
  double *part = nullptr;   // norm partials [NRM_WGS]
  double *norm = nullptr;   // [2]: |f|^2, |r|^2
  double *host = nullptr;   // pinned [2]
};

namespace gfd {
namespace {

int zlap(const PoissonLevel &L, const double *f, const double *rhs, double *out, int mode,
         hipStream_t st) {
  const Dims d = dims_of(L.n, L.h);
  const double diag = PW0 * (d.i0 + d.i1 + d.i2);
  k_zlap<<<blocks_for(L.ng), 256, 0, st>>>(f, rhs, out, d, mode, JACOBI_OMEGA / diag);
  return GPAW_OK;
}

// even number of Jacobi sweeps, phi -> tmp -> phi
void sweeps(PoissonLevel &L, double *phi, int count, hipStream_t st) {
  for (int s = 0; s < count; s += 2) {
    zlap(L, phi, L.f, L.tmp, 2, st);
    zlap(L, L.tmp, L.f, phi, 2, st);
  }
}

void vcycle(gpaw_poisson *p, size_t l, double *phi, hipStream_t st) {
  PoissonLevel &L = p->lv[l];
  if (l + 1 == p->lv.size()) {
    const int mx = std::max({L.n[0], L.n[1], L.n[2]});
    const int count = 20 * mx;  // even
    if (L.ng <= COARSE_LDS_POINTS && p->coarse_lds_ok) {
      const Dims d = dims_of(L.n, L.h);
      const double diag = PW0 * (d.i0 + d.i1 + d.i2);
      k_coarse_sweeps<<<1, 1024, 3 * L.ng * sizeof(double), st>>>(phi, L.f, d, count,
                                                                  JACOBI_OMEGA / diag);
    } else {
      sweeps(L, phi, count, st);
    }
    return;
  }
  PoissonLevel &C = p->lv[l + 1];
  sweeps(L, phi, PRE_SWEEPS, st);
  zlap(L, phi, L.f, L.tmp, 1, st);
  k_restrict<<<blocks_for(C.ng), 256, 0, st>>>(L.tmp, C.f, dims_of(L.n, L.h), dims_of(C.n, C.h));
  k_fill0<<<blocks_for(C.ng), 256, 0, st>>>(C.phi, C.ng);
  vcycle(p, l + 1, C.phi, st);
  k_interp<<<blocks_for(L.ng), 256, 0, st>>>(C.phi, phi, dims_of(L.n, L.h), dims_of(C.n, C.h), 1);
  sweeps(L, phi, POST_SWEEPS, st);
}

void sumsq(gpaw_poisson *p, const double *x, int64_t n, double *out, hipStream_t st) {
  const int wgs = static_cast<int>(std::min<int64_t>(NRM_WGS, (n + 255) / 256));
  k_sumsq<<<wgs, 256, 0, st>>>(x, n, p->part);
  k_sum_parts<<<1, 256, 0, st>>>(p->part, wgs, out);
}

void free_poisson(gpaw_poisson *p) {
  if (!p) return;
  for (size_t l = 0; l < p->lv.size(); ++l) {
    (void)hipFree(p->lv[l].f);
    if (l > 0) (void)hipFree(p->lv[l].phi);
    (void)hipFree(p->lv[l].tmp);
  }
  (void)hipFree(p->part);
  (void)hipFree(p->norm);
  if (p->host) (void)hipHostFree(p->host);
  delete p;
}

}  // namespace
}  // namespace gfd

using namespace gfd;

extern "C" {

int gpaw_poisson_create(const int32_t *n, const double *h, gpaw_poisson **out) {
  if (!out) return fail(GPAW_EINVAL, "gpaw_poisson_create: out is NULL");
  *out = nullptr;
  if (!h) return fail(GPAW_EINVAL, "gpaw_poisson_create: h is NULL");
  int rc = check_dims(n, h);
  if (rc != GPAW_OK) return rc;
  gpaw_poisson *p = new gpaw_poisson();
  int32_t cn[3] = {n[0], n[1], n[2]};
  double ch[3] = {h[0], h[1], h[2]};
  for (;;) {
    PoissonLevel L;
    for (int c = 0; c < 3; ++c) {
      L.n[c] = cn[c];
      L.h[c] = ch[c];
    }
    L.ng = static_cast<int64_t>(cn[0]) * cn[1] * cn[2];
    p->lv.push_back(L);
    if (!coarsens(cn)) break;
    for (int c = 0; c < 3; ++c) {
      cn[c] = (cn[c] - 1) / 2;
      ch[c] *= 2.0;
    }
  }
  hipError_t e = hipSuccess;
  for (size_t l = 0; l < p->lv.size() && e == hipSuccess; ++l) {
    PoissonLevel &L = p->lv[l];
    e = hipMalloc(&L.f, sizeof(double) * L.ng);
    if (e == hipSuccess && l > 0) e = hipMalloc(&L.phi, sizeof(double) * L.ng);
    if (e == hipSuccess) e = hipMalloc(&L.tmp, sizeof(double) * L.ng);
  }
  if (e == hipSuccess) e = hipMalloc(&p->part, sizeof(double) * NRM_WGS);
  if (e == hipSuccess)
    p->coarse_lds_ok =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_coarse_sweeps),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            3 * COARSE_LDS_POINTS * sizeof(double)) == hipSuccess;
  (void)hipGetLastError();
  if (e == hipSuccess) e = hipMalloc(&p->norm, sizeof(double) * 2);
  if (e == hipSuccess) e = hipHostMalloc(&p->host, sizeof(double) * 2);
  if (e != hipSuccess) {
    free_poisson(p);
    (void)hipGetLastError();
    return fail(GPAW_ENOMEM, "gpaw_poisson_create: device allocation failed");
  }
  *out = p;
  return GPAW_OK;
}

int gpaw_poisson_solve(gpaw_poisson *p, const double *rho, double *phi, double tol,
                       int32_t max_cycles, int32_t *cycles, double *rel_residual, void *stream) {
  if (!p || !rho || !phi) return fail(GPAW_EINVAL, "gpaw_poisson_solve: NULL argument");
  if (rho == phi) return fail(GPAW_EALIAS, "gpaw_poisson_solve: rho and phi alias");
  if (!(tol >= 0.0) || max_cycles < 1)
    return fail(GPAW_EINVAL, "gpaw_poisson_solve: tol >= 0 and max_cycles >= 1 required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  PoissonLevel &L0 = p->lv[0];
  k_scale<<<blocks_for(L0.ng), 256, 0, st>>>(rho, L0.f, L0.ng, -4.0 * M_PI);
  sumsq(p, L0.f, L0.ng, p->norm, st);
  int32_t it = 0;
  double rel = 0.0;
  for (; it < max_cycles;) {
    vcycle(p, 0, phi, st);
    ++it;
    zlap(L0, phi, L0.f, L0.tmp, 1, st);
    sumsq(p, L0.tmp, L0.ng, p->norm + 1, st);
    hipError_t e = hipMemcpyAsync(p->host, p->norm, sizeof(double) * 2, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gpaw_poisson_solve");
    rel = p->host[0] > 0.0 ? std::sqrt(p->host[1] / p->host[0]) : std::sqrt(p->host[1]);
    if (!(rel > tol)) break;  // converged (or a non-finite residual: stop)
  }
  if (cycles) *cycles = it;
  if (rel_residual) *rel_residual = rel;
  if (!std::isfinite(rel)) return fail(GPAW_ENONFINITE, "gpaw_poisson_solve: non-finite residual");
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_poisson_solve");
}

void gpaw_poisson_destroy(gpaw_poisson *p) { free_poisson(p); }

int gpaw_poisson_levels(const gpaw_poisson *p, int32_t *levels) {
  if (!p || !levels) return fail(GPAW_EINVAL, "gpaw_poisson_levels: NULL argument");
  *levels = static_cast<int32_t>(p->lv.size());
  return GPAW_OK;
}

int gpaw_laplacian_zero(const int32_t *n, const double *h, const double *f, double *out,
                        void *stream) {
  if (!f || !out || !h) return fail(GPAW_EINVAL, "gpaw_laplacian_zero: NULL argument");
  if (f == out) return fail(GPAW_EALIAS, "gpaw_laplacian_zero: f and out alias");
  int rc = check_dims(n, h);
  if (rc != GPAW_OK) return rc;
  PoissonLevel L;
  for (int c = 0; c < 3; ++c) {
    L.n[c] = n[c];
    L.h[c] = h[c];
  }
  L.ng = static_cast<int64_t>(n[0]) * n[1] * n[2];
  zlap(L, f, nullptr, out, 0, static_cast<hipStream_t>(stream));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_laplacian_zero");
}

int gpaw_grid_restrict(const int32_t *nf, const double *fine, double *coarse, void *stream) {
  if (!fine || !coarse) return fail(GPAW_EINVAL, "gpaw_grid_restrict: NULL argument");
  int rc = check_dims(nf, nullptr);
  if (rc != GPAW_OK) return rc;
  if (!coarsens(nf)) return fail(GPAW_ESHAPE, "gpaw_grid_restrict: every axis must be odd and >= 3");
  const int32_t nc[3] = {(nf[0] - 1) / 2, (nf[1] - 1) / 2, (nf[2] - 1) / 2};
  const double one[3] = {1.0, 1.0, 1.0};
  const int64_t ngc = static_cast<int64_t>(nc[0]) * nc[1] * nc[2];
  k_restrict<<<blocks_for(ngc), 256, 0, static_cast<hipStream_t>(stream)>>>(
      fine, coarse, dims_of(nf, one), dims_of(nc, one));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_grid_restrict");
}

int gpaw_grid_interpolate(const int32_t *nf, const double *coarse, double *fine,
                          int32_t accumulate, void *stream) {
  if (!fine || !coarse) return fail(GPAW_EINVAL, "gpaw_grid_interpolate: NULL argument");
  int rc = check_dims(nf, nullptr);
  if (rc != GPAW_OK) return rc;
  if (!coarsens(nf))
    return fail(GPAW_ESHAPE, "gpaw_grid_interpolate: every fine axis must be odd and >= 3");
  const int32_t nc[3] = {(nf[0] - 1) / 2, (nf[1] - 1) / 2, (nf[2] - 1) / 2};
  const double one[3] = {1.0, 1.0, 1.0};
  const int64_t ngf = static_cast<int64_t>(nf[0]) * nf[1] * nf[2];
  k_interp<<<blocks_for(ngf), 256, 0, static_cast<hipStream_t>(stream)>>>(
      coarse, fine, dims_of(nf, one), dims_of(nc, one), accumulate ? 1 : 0);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_grid_interpolate");
}

}  // extern "C"
