// Generalised symmetric eigenproblem of the subspace, H C = S C diag(eps),
// in FP64 on the device (Cholesky and diagonalisation of the subspace
// matrices, Sec. "Parallelization"; SCF step (1), Sec. "Solving the
// Kohn-Sham equation").
//
// Pipeline (real symmetric, nb <= 128):
//   k_eig_reduce  (1 workgroup, 1024 lanes, matrix in LDS)
//       S <- (S+S^T)/2;  S = L L^T (right-looking, one barrier per column);
//       Linv = L^-1 (column-parallel forward substitution, 8 lanes per column);
//       A = Linv ((H+H^T)/2) Linv^T;  A <- (A+A^T)/2;
//       Householder tridiagonalisation A = Q T Q^T (reflectors kept for later).
//   k_eig_values  (one wavefront per eigenvalue)
//       T splits where |e_i| <= eps (|d_i| + |d_i+1|); each eigenvalue is found
//       in its unreduced block by 65-way multisection on Sturm counts.
//   k_eig_vectors (one lane per eigenvalue, LDS scratch)
//       inverse iteration on the block with a pivoted tridiagonal LU; shifts of
//       eigenvalues closer than 10 eps ||T|| are pulled apart by that amount.
//   k_eig_finish  (1 workgroup)
//       Newton-Schulz steps Z <- Z (3I - Z^T Z)/2 until Z^T Z = I to 1e-8
//       (each step squares the defect); back-transform U = Q Z; eigen-order by
//       value; C = Linv^T U.
#include <algorithm>
#include <cfloat>
#include <mutex>

#include "internal.h"

namespace gfd {

namespace {

constexpr int EIG_T = 1024;
constexpr int EIG_NMAX = 128;
constexpr int VEC_T = 16;  // lanes (eigenvectors) per inverse-iteration workgroup

struct EigWs {
  double *Linv, *T1, *V, *Z, *Z2, *tau, *d, *e, *lam;
};

EigWs eig_layout(double *base, int n) {
  const size_t nn = static_cast<size_t>(n) * n;
  EigWs w;
  w.Linv = base;
  w.T1 = w.Linv + nn;
  w.V = w.T1 + nn;
  w.Z = w.V + nn;
  w.Z2 = w.Z + nn;
  w.tau = w.Z2 + nn;
  w.d = w.tau + n;
  w.e = w.d + n;
  w.lam = w.e + n;
  return w;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}
__device__ inline double wave_min(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

__device__ inline bool split_at(const double *d, const double *e, int i) {
  return fabs(e[i]) <= DBL_EPSILON * (fabs(d[i]) + fabs(d[i + 1]));
}

// ------------------------------------------------------------------ reduce
__global__ __launch_bounds__(EIG_T) void k_eig_reduce(const double *__restrict__ H,
                                                      const double *__restrict__ S, int n,
                                                      EigWs w, int32_t *info) {
  extern __shared__ double sm[];
  const int lda = n + 1;
  double *A = sm;              // [n][lda]
  double *vv = A + n * lda;    // Householder vector
  double *pp = vv + n;         // tau * A v
  double *dinv = pp + n;       // 1 / L_jj
  double *red = dinv + n;      // 16 wavefront partials
  double *scal = red + 16;     // tau of the current step
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  for (int idx = tid; idx < n * n; idx += EIG_T) {
    const int i = idx / n, j = idx - i * n;
    A[i * lda + j] = 0.5 * (S[i * n + j] + S[j * n + i]);
  }
  __syncthreads();

  // Cholesky, lower. Column j is scaled one step late so that the trailing
  // update of step j and the scaling of column j-1 touch disjoint entries.
  int failed = 0;
  double prev_rs = 0.0;
  for (int j = 0; j < n; ++j) {
    const double djj = A[j * lda + j];
    if (!(djj > 0.0)) {
      failed = j + 1;
      break;
    }
    if (j > 0)
      for (int i = j + tid; i < n; i += EIG_T) A[i * lda + j - 1] *= prev_rs;
    const int m = n - j - 1;
    const double inv = 1.0 / djj;
    for (int idx = tid; idx < m * m; idx += EIG_T) {
      const int ii = idx / m, cc = idx - ii * m;
      if (cc <= ii) {
        const int i = j + 1 + ii, c = j + 1 + cc;
        A[i * lda + c] -= A[i * lda + j] * A[c * lda + j] * inv;
      }
    }
    prev_rs = 1.0 / sqrt(djj);
    __syncthreads();
  }
  if (failed) {
    if (tid == 0) *info = failed;
    return;
  }
  for (int j = tid; j < n; j += EIG_T) {
    const double r = sqrt(A[j * lda + j]);
    A[j * lda + j] = r;
    dinv[j] = 1.0 / r;
  }
  __syncthreads();

  // Linv: column col by 8 lanes; lane s keeps x_{8t+s} in xr[t]
  {
    const int col = tid >> 3, s = tid & 7;
    double xr[EIG_NMAX / 8];
#pragma unroll
    for (int t = 0; t < EIG_NMAX / 8; ++t) xr[t] = 0.0;
    if (col < n) {
      for (int i = col; i < n; ++i) {
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < EIG_NMAX / 8; ++t) {
          const int kk = 8 * t + s;
          if (kk >= col && kk < i) part += A[i * lda + kk] * xr[t];
        }
        part += __shfl_xor(part, 1);
        part += __shfl_xor(part, 2);
        part += __shfl_xor(part, 4);
        const double xi = (i == col) ? dinv[i] : -part * dinv[i];
#pragma unroll
        for (int t = 0; t < EIG_NMAX / 8; ++t)
          if (8 * t + s == i) xr[t] = xi;
      }
#pragma unroll
      for (int t = 0; t < EIG_NMAX / 8; ++t) {
        const int row = 8 * t + s;
        if (row < n) w.Linv[row * n + col] = xr[t];
      }
    }
  }
  __syncthreads();

  // Hs in LDS; T1 = Hs Linv^T (global); A = Linv T1 (LDS)
  for (int idx = tid; idx < n * n; idx += EIG_T) {
    const int i = idx / n, j = idx - i * n;
    A[i * lda + j] = 0.5 * (H[i * n + j] + H[j * n + i]);
  }
  __syncthreads();
  {
    const int i0 = (tid >> 5) * 4, j0 = (tid & 31) * 4;
    if (i0 < n && j0 < n) {
      double acc[4][4] = {};
      const int kmax = min(n, j0 + 4);
      for (int kk = 0; kk < kmax; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = (i0 + r < n) ? A[(i0 + r) * lda + kk] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = (j0 + c < n) ? w.Linv[(j0 + c) * n + kk] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (i0 + r < n && j0 + c < n) w.T1[(i0 + r) * n + j0 + c] = acc[r][c];
    }
  }
  __syncthreads();
  {
    const int i0 = (tid >> 5) * 4, j0 = (tid & 31) * 4;
    if (i0 < n && j0 < n) {
      double acc[4][4] = {};
      const int kmax = min(n, i0 + 4);
      for (int kk = 0; kk < kmax; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = (i0 + r < n) ? w.Linv[(i0 + r) * n + kk] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = (j0 + c < n) ? w.T1[kk * n + j0 + c] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (i0 + r < n && j0 + c < n) A[(i0 + r) * lda + j0 + c] = acc[r][c];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += EIG_T) {
    const int i = idx / n, j = idx - i * n;
    if (i < j) {
      const double avg = 0.5 * (A[i * lda + j] + A[j * lda + i]);
      A[i * lda + j] = avg;
      A[j * lda + i] = avg;
    }
  }
  __syncthreads();

  // Householder tridiagonalisation, reflector k acts on rows/columns k+1..n-1
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    if (wave == 0) {
      double xn2 = 0.0;
      for (int r = k + 2 + lane; r < n; r += 64) {
        const double x = A[r * lda + k];
        xn2 += x * x;
      }
      xn2 = wave_sum(xn2);
      const double alpha = A[(k + 1) * lda + k];
      double beta, tau, scl;
      if (xn2 == 0.0) {
        beta = alpha;
        tau = 0.0;
        scl = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scl = 1.0 / (alpha - beta);
      }
      for (int r = k + 1 + lane; r < n; r += 64) {
        const double vr = (r == k + 1) ? 1.0 : A[r * lda + k] * scl;
        vv[r] = vr;
        w.V[k * n + r] = vr;
      }
      if (lane == 0) {
        scal[0] = tau;
        w.tau[k] = tau;
        w.d[k] = A[k * lda + k];
        w.e[k] = beta;
      }
    }
    __syncthreads();
    const double tau = scal[0];
    {
      const int r = k + 1 + (tid >> 3), s = tid & 7;
      double part = 0.0;
      if (r < n)
        for (int c = k + 1 + s; c < n; c += 8) part += A[r * lda + c] * vv[c];
      part += __shfl_xor(part, 1);
      part += __shfl_xor(part, 2);
      part += __shfl_xor(part, 4);
      double contrib = 0.0;
      if (r < n && s == 0) {
        const double p = tau * part;
        pp[r] = p;
        contrib = p * vv[r];
      }
      contrib = wave_sum(contrib);
      if (lane == 0) red[wave] = contrib;
    }
    __syncthreads();
    {
      double pv = 0.0;
      for (int q = 0; q < EIG_T / 64; ++q) pv += red[q];
      const double K = -0.5 * tau * pv;
      for (int idx = tid; idx < m * m; idx += EIG_T) {
        const int ii = idx / m, cc = idx - ii * m;
        const int r = k + 1 + ii, c = k + 1 + cc;
        const double wr = pp[r] + K * vv[r], wc = pp[c] + K * vv[c];
        A[r * lda + c] -= vv[r] * wc + wr * vv[c];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      w.d[n - 2] = A[(n - 2) * lda + n - 2];
      w.e[n - 2] = A[(n - 1) * lda + n - 2];
    }
    w.d[n - 1] = A[(n - 1) * lda + n - 1];
    *info = 0;
  }
}

// ------------------------------------------------------------------ values
__global__ __launch_bounds__(256) void k_eig_values(int n, EigWs w, const int32_t *info) {
  if (*info != 0) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double *d = w.d, *e = w.e;
  int lo = j, hi = j;
  while (lo > 0 && !split_at(d, e, lo - 1)) --lo;
  while (hi < n - 1 && !split_at(d, e, hi)) ++hi;
  const int li = j - lo;
  double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
  for (int i = lo + lane; i <= hi; i += 64) {
    const double off = (i > lo ? fabs(e[i - 1]) : 0.0) + (i < hi ? fabs(e[i]) : 0.0);
    gl = fmin(gl, d[i] - off);
    gu = fmax(gu, d[i] + off);
    if (i < hi) emax2 = fmax(emax2, e[i] * e[i]);
  }
  gl = wave_min(gl);
  gu = wave_max(gu);
  emax2 = wave_max(emax2);
  const double tn = fmax(fabs(gl), fabs(gu));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  double a = gl - (2.0 * DBL_EPSILON * tn + 2.0 * pivmin);
  double b = gu + (2.0 * DBL_EPSILON * tn + 2.0 * pivmin);
  for (int it = 0; it < 64; ++it) {
    const double width = b - a;
    if (width <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + pivmin) break;
    const double x = a + width * ((lane + 1) / 65.0);
    int cnt = 0;
    double q = 1.0;
    for (int i = lo; i <= hi; ++i) {
      double t = d[i] - x;
      if (i > lo) t -= e[i - 1] * e[i - 1] / q;
      if (fabs(t) < pivmin) t = -pivmin;
      cnt += (t < 0.0);
      q = t;
    }
    // eigenvalue li lies at or above x exactly when fewer than li+1 lie below x
    const double na = wave_max(cnt <= li ? x : -DBL_MAX);
    const double nb = wave_min(cnt > li ? x : DBL_MAX);
    a = fmax(a, na);
    b = fmin(b, nb);
  }
  if (lane == 0) w.lam[j] = 0.5 * (a + b);
}

// ------------------------------------------------------------------ vectors
__device__ inline double start_value(int j, int i) {
  uint64_t z = (static_cast<uint64_t>(j) << 32) + static_cast<uint64_t>(i) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(VEC_T) void k_eig_vectors(int n, EigWs w, const int32_t *info) {
  if (*info != 0) return;
  extern __shared__ double sv[];
  const int t = threadIdx.x;
  const int j = blockIdx.x * VEC_T + t;
  if (j >= n) return;
  // per-lane scratch, lane-interleaved: u0, u1, u2, y
  double *u0 = sv + 0 * n * VEC_T + t;
  double *u1 = sv + 1 * n * VEC_T + t;
  double *u2 = sv + 2 * n * VEC_T + t;
  double *y = sv + 3 * n * VEC_T + t;
#define AT(p, i) (p)[(i) * VEC_T]
  const double *d = w.d, *e = w.e;
  int lo = j, hi = j;
  while (lo > 0 && !split_at(d, e, lo - 1)) --lo;
  while (hi < n - 1 && !split_at(d, e, hi)) ++hi;
  const int m = hi - lo + 1;
  double tn = 0.0;
  for (int i = lo; i <= hi; ++i)
    tn = fmax(tn, fabs(d[i]) + (i > lo ? fabs(e[i - 1]) : 0.0) + (i < hi ? fabs(e[i]) : 0.0));
  const double pert = 10.0 * DBL_EPSILON * fmax(tn, DBL_MIN);
  int ties = 0;
  for (int i = j; i > lo && w.lam[i] - w.lam[i - 1] < pert; --i) ++ties;
  const double x = w.lam[j - ties] + ties * pert;
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);

  for (int i = 0; i < m; ++i) AT(y, i) = start_value(j, i);
  for (int iter = 0; iter < 3; ++iter) {
    // LU with partial pivoting of (T_block - x I), forward-eliminating y
    double c0 = d[lo] - x, c1 = (m > 1) ? e[lo] : 0.0;
    for (int i = 0; i + 1 < m; ++i) {
      const double n0 = e[lo + i], n1 = d[lo + i + 1] - x;
      const double n2 = (i + 2 < m) ? e[lo + i + 1] : 0.0;
      const double yi = AT(y, i), yn = AT(y, i + 1);
      if (fabs(n0) > fabs(c0)) {
        const double l = c0 / n0;
        AT(u0, i) = n0;
        AT(u1, i) = n1;
        AT(u2, i) = n2;
        AT(y, i) = yn;
        AT(y, i + 1) = yi - l * yn;
        c0 = c1 - l * n1;
        c1 = -l * n2;
      } else {
        const double l = (c0 != 0.0) ? n0 / c0 : 0.0;
        AT(u0, i) = c0;
        AT(u1, i) = c1;
        AT(u2, i) = 0.0;
        AT(y, i + 1) = yn - l * yi;
        c0 = n1 - l * c1;
        c1 = n2;
      }
    }
    AT(u0, m - 1) = c0;
    // back substitution with tiny pivots replaced by +-eps ||T||
    double y1 = 0.0, y2 = 0.0, ymax = 0.0;
    for (int i = m - 1; i >= 0; --i) {
      double p = AT(u0, i);
      if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
      double s = AT(y, i);
      if (i + 1 < m) s -= AT(u1, i) * y1;
      if (i + 2 < m) s -= AT(u2, i) * y2;
      const double yi = s / p;
      AT(y, i) = yi;
      y2 = y1;
      y1 = yi;
      ymax = fmax(ymax, fabs(yi));
    }
    const double sc = 1.0 / fmax(ymax, DBL_MIN);
    for (int i = 0; i < m; ++i) AT(y, i) *= sc;
  }
  double nrm = 0.0, big = 0.0;
  int ibig = 0;
  for (int i = 0; i < m; ++i) {
    const double v = AT(y, i);
    nrm += v * v;
    if (fabs(v) > big) {
      big = fabs(v);
      ibig = i;
    }
  }
  const double sc = copysign(1.0 / sqrt(nrm), AT(y, ibig));
  for (int i = 0; i < n; ++i)
    w.Z[static_cast<int64_t>(i) * n + j] = (i >= lo && i <= hi) ? AT(y, i - lo) * sc : 0.0;
#undef AT
}

// ------------------------------------------------------------------ finish
// out = In * M with M = 1.5 I - 0.5 G, all n x n row-major in global memory
__device__ void ns_step(const double *In, const double *G, double *Out, int n, int tid) {
  const int i0 = (tid >> 5) * 4, j0 = (tid & 31) * 4;
  if (i0 >= n || j0 >= n) return;
  double acc[4][4] = {};
  for (int kk = 0; kk < n; ++kk) {
    double a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = (i0 + r < n) ? In[(i0 + r) * n + kk] : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      b[c] = (j0 + c < n) ? ((kk == j0 + c ? 1.5 : 0.0) - 0.5 * G[kk * n + j0 + c]) : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (i0 + r < n && j0 + c < n) Out[(i0 + r) * n + j0 + c] = acc[r][c];
}

// G = Z^T Z; returns max |G - I| over the workgroup (all lanes)
__device__ double gram(const double *Z, double *G, int n, int tid, double *red) {
  const int i0 = (tid >> 5) * 4, j0 = (tid & 31) * 4;
  double dev = 0.0;
  if (i0 < n && j0 < n) {
    double acc[4][4] = {};
    for (int r = 0; r < n; ++r) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = (i0 + q < n) ? Z[r * n + i0 + q] : 0.0;
        b[q] = (j0 + q < n) ? Z[r * n + j0 + q] : 0.0;
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i0 + p < n && j0 + q < n) {
          G[(i0 + p) * n + j0 + q] = acc[p][q];
          dev = fmax(dev, fabs(acc[p][q] - ((i0 + p == j0 + q) ? 1.0 : 0.0)));
        }
  }
  dev = wave_max(dev);
  if ((tid & 63) == 0) red[tid >> 6] = dev;
  __syncthreads();
  double all = 0.0;
  for (int q = 0; q < EIG_T / 64; ++q) all = fmax(all, red[q]);
  __syncthreads();
  return all;
}

__global__ __launch_bounds__(EIG_T) void k_eig_finish(int n, EigWs w, double *__restrict__ eps,
                                                      double *__restrict__ C,
                                                      int32_t *__restrict__ info) {
  if (*info != 0) return;
  __shared__ double red[EIG_T / 64];
  __shared__ int rank[EIG_NMAX];
  const int tid = threadIdx.x;
  double *Z = w.Z, *Z2 = w.Z2;
  double *G = w.T1;  // T1 is free after the reduction
  bool ok = false;
  for (int it = 0; it < 8; ++it) {
    const double dev = gram(Z, G, n, tid, red);
    if (!(dev < 0.3)) break;
    ns_step(Z, G, Z2, n, tid);
    __syncthreads();
    double *tmp = Z;
    Z = Z2;
    Z2 = tmp;
    if (dev <= 1e-8) {
      ok = true;
      break;
    }
  }
  if (!ok) {
    if (tid == 0) *info = -1;
    return;
  }
  // eigen-order: rank of each slot by (value, slot)
  for (int j = tid; j < n; j += EIG_T) {
    const double lj = w.lam[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
      const double li = w.lam[i];
      r += (li < lj) || (li == lj && i < j);
    }
    rank[j] = r;
  }
  // back-transform each column of Z: 8 lanes per column, rows 8t+s in registers
  {
    const int col = tid >> 3, s = tid & 7;
    double zr[EIG_NMAX / 8];
#pragma unroll
    for (int t = 0; t < EIG_NMAX / 8; ++t) {
      const int row = 8 * t + s;
      zr[t] = (col < n && row < n) ? Z[row * n + col] : 0.0;
    }
    if (col < n) {
      for (int k = n - 3; k >= 0; --k) {
        const double tk = w.tau[k];
        const double *vk = w.V + static_cast<int64_t>(k) * n;
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < EIG_NMAX / 8; ++t) {
          const int row = 8 * t + s;
          if (row > k && row < n) part += vk[row] * zr[t];
        }
        part += __shfl_xor(part, 1);
        part += __shfl_xor(part, 2);
        part += __shfl_xor(part, 4);
        const double f = tk * part;
#pragma unroll
        for (int t = 0; t < EIG_NMAX / 8; ++t) {
          const int row = 8 * t + s;
          if (row > k && row < n) zr[t] -= f * vk[row];
        }
      }
    }
    __syncthreads();  // every read of Z2/Z done before it is reused for U
#pragma unroll
    for (int t = 0; t < EIG_NMAX / 8; ++t) {
      const int row = 8 * t + s;
      if (col < n && row < n) Z2[row * n + col] = zr[t];
    }
  }
  __syncthreads();
  // C[m][rank j] = sum_{k >= m} Linv[k][m] U[k][j]
  {
    const double *U = Z2;
    const int i0 = (tid >> 5) * 4, j0 = (tid & 31) * 4;
    if (i0 < n && j0 < n) {
      double acc[4][4] = {};
      for (int kk = i0; kk < n; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = (i0 + r < n && kk >= i0 + r) ? w.Linv[kk * n + i0 + r] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = (j0 + c < n) ? U[kk * n + j0 + c] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (i0 + r < n && j0 + c < n) C[(i0 + r) * n + rank[j0 + c]] = acc[r][c];
    }
  }
  for (int j = tid; j < n; j += EIG_T) eps[rank[j]] = w.lam[j];
}

}  // namespace

size_t eig_ws_elems(int nmax, bool cplx) {
  const size_t n = static_cast<size_t>(std::min(nmax, EIG_NMAX));
  return (5 * n * n + 4 * n + 64) * (cplx ? 2 : 1);
}

int launch_eigh(const gpaw_sys *s, const void *H, const void *S, int nb, double *eps, void *C,
                int32_t *info, hipStream_t st) {
  if (s->dtype != GPAW_F64) return fail(GPAW_EDTYPE, "subspace eigensolver: complex not built yet");
  if (nb > EIG_NMAX) return fail(GPAW_ESHAPE, "subspace eigensolver supports nb <= 128");
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_eig_reduce),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  if (attr_err != hipSuccess) return hip_fail(attr_err, "hipFuncSetAttribute(k_eig_reduce)");
  const EigWs w = eig_layout(s->ws.eig, nb);
  const size_t lds1 = (static_cast<size_t>(nb) * (nb + 1) + 3 * nb + 17) * sizeof(double);
  k_eig_reduce<<<1, EIG_T, lds1, st>>>(static_cast<const double *>(H),
                                       static_cast<const double *>(S), nb, w, info);
  k_eig_values<<<(nb + 3) / 4, 256, 0, st>>>(nb, w, info);
  const size_t lds3 = static_cast<size_t>(4) * nb * VEC_T * sizeof(double);
  k_eig_vectors<<<(nb + VEC_T - 1) / VEC_T, VEC_T, lds3, st>>>(nb, w, info);
  k_eig_finish<<<1, EIG_T, 0, st>>>(nb, w, eps, static_cast<double *>(C), info);
  return GPAW_OK;
}

}  // namespace gfd
