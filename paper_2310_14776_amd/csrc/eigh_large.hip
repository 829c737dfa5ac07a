// Generalised Hermitian eigenproblem of the subspace for blocks too large
// for one workgroup's LDS (nb > 128 real, nb > 96 complex, up to 1024):
// the same method as eigh.hip (Cholesky and diagonalisation of the subspace
// matrices, Sec. "Parallelization"), with the matrices in global memory
// (L2/MALL resident) and every sequential step spread over the whole chip:
//   Cholesky       one launch per column (right-looking, lower), pivots
//                  recorded, columns scaled in one pass at the end;
//   Linv           one wavefront per column (forward substitution, the
//                  column held in registers, rows of L read from L2);
//   A = Linv H Linv^H, Newton-Schulz, C = Linv^H U: MFMA small-GEMM kernel;
//   tridiagonal    two launches per column: p = tau A v (one wavefront per
//                  row), then the rank-2 update of the trailing block with,
//                  in workgroup 0, the next column and its Householder
//                  vector (that column is left to workgroup 0 alone, so no
//                  workgroup reads a value another one is rewriting);
//   eigenvalues    as for small blocks (multisection, d/e in LDS);
//   eigenvectors   inverse iteration with the LU scratch in global memory;
//   back-transform one wavefront per column, reflectors read from L2.
#include <algorithm>
#include <cfloat>
#include <string>

#include "internal.h"

namespace gfd {

namespace {

constexpr int LNMAX = 1024;

__device__ inline double re_l(double a) { return a; }
__device__ inline double re_l(z64 a) { return a.x; }
__device__ inline double im_l(double) { return 0.0; }
__device__ inline double im_l(z64 a) { return a.y; }
__device__ inline double abs2_l(double a) { return a * a; }
__device__ inline double abs2_l(z64 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double cj_l(double a) { return a; }
__device__ inline z64 cj_l(z64 a) { return zconj(a); }
__device__ inline z64 mulr(z64 a, double s) { return z64{a.x * s, a.y * s}; }
__device__ inline double mulr(double a, double s) { return a * s; }
template <typename T> __device__ inline T rv(double r);
template <> __device__ inline double rv<double>(double r) { return r; }
template <> __device__ inline z64 rv<z64>(double r) { return z64{r, 0.0}; }

__device__ inline double wsum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ inline z64 wsum(z64 v) { return z64{wsum(v.x), wsum(v.y)}; }

// block-wide sum over 256 lanes (all lanes get the result)
template <typename T>
__device__ inline T block_sum(T v, T *red) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ Cholesky
// Step j: pivot d_j = A[j][j] (final after step j-1); trailing lower block
// A[r][c] -= A[r][j] conj(A[c][j]) / d_j for j < c <= r. Column j stays
// unscaled until k_lchol_scale.
template <typename T>
__global__ __launch_bounds__(256) void k_lchol_step(T *__restrict__ A, int n, int j,
                                                    double *__restrict__ piv, int32_t *info) {
  if (*info != 0) return;
  const double dj = re_l(A[static_cast<int64_t>(j) * n + j]);
  if (!(dj > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = j + 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) piv[j] = dj;
  const double inv = 1.0 / dj;
  const int m = n - j - 1;
  // 2-D tiles of 16 x 16 over the m x m trailing block, lower part only
  const int tiles = (m + 15) / 16;
  const int tile = blockIdx.x;
  const int ti = tile / tiles, tj = tile - (tile / tiles) * tiles;
  if (tj > ti) return;
  const int r = j + 1 + ti * 16 + (threadIdx.x >> 4), c = j + 1 + tj * 16 + (threadIdx.x & 15);
  if (r >= n || c > r) return;
  const T lr = A[static_cast<int64_t>(r) * n + j];
  const T lc = cj_l(A[static_cast<int64_t>(c) * n + j]);
  T &a = A[static_cast<int64_t>(r) * n + c];
  a = a - mulr(lr * lc, inv);
}

// L[r][j] = A[r][j] / sqrt(d_j) (r > j), L[j][j] = sqrt(d_j), upper part 0
template <typename T>
__global__ __launch_bounds__(256) void k_lchol_scale(T *__restrict__ A, int n,
                                                     const double *__restrict__ piv,
                                                     const int32_t *info) {
  if (*info != 0) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(idx / n), c = static_cast<int>(idx - static_cast<int64_t>(idx / n) * n);
  if (c > r) A[idx] = T{};
  else if (c == r) A[idx] = rv<T>(sqrt(piv[c]));
  else A[idx] = mulr(A[idx], 1.0 / sqrt(piv[c]));
}

// Linv column col = L^-1 e_col: one wavefront, lane s keeps rows 64t+s
template <typename T>
__global__ __launch_bounds__(64) void k_linv_col(const T *__restrict__ L, T *__restrict__ Linv,
                                                 int n, const int32_t *info) {
  if (*info != 0) return;
  const int col = blockIdx.x, s = threadIdx.x;
  constexpr int R = LNMAX / 64;
  T xr[R];
#pragma unroll
  for (int t = 0; t < R; ++t) xr[t] = T{};
  for (int i = col; i < n; ++i) {
    const T *Li = L + static_cast<int64_t>(i) * n;
    T part = T{};
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int k = 64 * t + s;
      if (k >= col && k < i) part = part + Li[k] * xr[t];
    }
    part = wsum(part);
    const double dinv = 1.0 / re_l(Li[i]);
    const T xi = (i == col) ? rv<T>(dinv) : mulr(part, -dinv);
#pragma unroll
    for (int t = 0; t < R; ++t)
      if (64 * t + s == i) xr[t] = xi;
  }
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = 64 * t + s;
    if (row < n) Linv[static_cast<int64_t>(row) * n + col] = xr[t];
  }
}

// ------------------------------------------------------------------ tridiagonal
// Householder vector of column k of A (rows k+1..n-1), one workgroup; the
// column values are passed in colv (already updated). Writes v into V[k],
// tau[k], e[k], and d[k] = re A[k][k] (passed as dkk).
template <typename T>
__device__ void house_col(const T *colv, double dkk, int k, int n, T *V, T *tau, double *d,
                          double *e, T *red) {
  double xn2 = 0.0;
  for (int r = k + 2 + threadIdx.x; r < n; r += 256) xn2 += abs2_l(colv[r]);
  xn2 = block_sum<double>(xn2, reinterpret_cast<double *>(red));
  const T alpha = colv[k + 1];
  const double ar = re_l(alpha);
  double beta;
  T tk, scl;
  if (xn2 == 0.0 && abs2_l(alpha) == ar * ar) {
    beta = ar;
    tk = T{};
    scl = T{};
  } else {
    beta = -copysign(sqrt(abs2_l(alpha) + xn2), ar);
    const T amb = alpha - rv<T>(beta);
    tk = mulr(amb, -1.0 / beta);
    scl = mulr(cj_l(amb), 1.0 / abs2_l(amb));
  }
  T *vk = V + static_cast<int64_t>(k) * n;
  for (int r = threadIdx.x; r < n; r += 256)
    vk[r] = (r <= k) ? T{} : ((r == k + 1) ? rv<T>(1.0) : colv[r] * scl);
  if (threadIdx.x == 0) {
    tau[k] = tk;
    d[k] = dkk;
    e[k] = beta;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trd_first(const T *__restrict__ A, int n, T *V, T *tau,
                                                   double *d, double *e, const int32_t *info) {
  if (*info != 0) return;
  __shared__ T red[4];
  extern __shared__ unsigned char smem[];
  T *colv = reinterpret_cast<T *>(smem);
  for (int r = threadIdx.x; r < n; r += 256) colv[r] = A[static_cast<int64_t>(r) * n];
  __syncthreads();
  house_col<T>(colv, re_l(colv[0]), 0, n, V, tau, d, e, red);
}

// p_r = tau_k sum_{c > k} A[r][c] v_c for r > k: one wavefront per row
template <typename T>
__global__ __launch_bounds__(256) void k_trd_symv(const T *__restrict__ A, int n, int k,
                                                  const T *__restrict__ V, const T *__restrict__ tau,
                                                  T *__restrict__ p, const int32_t *info) {
  if (*info != 0) return;
  const int r = k + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  const T *Ar = A + static_cast<int64_t>(r) * n;
  const T *vk = V + static_cast<int64_t>(k) * n;
  T acc0 = T{}, acc1 = T{};
  int c = k + 1 + lane;
  for (; c + 64 < n; c += 128) {
    acc0 = acc0 + Ar[c] * vk[c];
    acc1 = acc1 + Ar[c + 64] * vk[c + 64];
  }
  if (c < n) acc0 = acc0 + Ar[c] * vk[c];
  const T sum = wsum(acc0 + acc1);
  if (lane == 0) p[r] = tau[k] * sum;
}

// w = p + K v with K = -tau/2 (p^H v); A -= v w^H + w v^H on rows/cols >= k+2;
// workgroup 0 also updates column k+1 and forms the next Householder vector.
template <typename T>
__global__ __launch_bounds__(256) void k_trd_update(T *__restrict__ A, int n, int k, T *V, T *tau,
                                                    const T *__restrict__ p, double *d, double *e,
                                                    const int32_t *info) {
  if (*info != 0) return;
  __shared__ T red[4];
  extern __shared__ unsigned char smem[];
  const T *vk = V + static_cast<int64_t>(k) * n;
  T pv = T{};
  for (int r = k + 1 + threadIdx.x; r < n; r += 256) pv = pv + cj_l(p[r]) * vk[r];
  pv = block_sum<T>(pv, red);
  const T K = mulr(tau[k] * pv, -0.5);
  if (blockIdx.x == 0) {
    if (k + 2 < n) {
      // column k+1 after the update, rows k+1..n-1, then its reflector
      T *colv = reinterpret_cast<T *>(smem);
      const T wk1 = p[k + 1] + K * vk[k + 1];
      const T cv1 = cj_l(vk[k + 1]), cw1 = cj_l(wk1);
      for (int r = k + 1 + threadIdx.x; r < n; r += 256) {
        const T vr = vk[r], wr = p[r] + K * vk[r];
        T &a = A[static_cast<int64_t>(r) * n + k + 1];
        a = a - (vr * cw1 + wr * cv1);
        colv[r] = a;
      }
      __syncthreads();
      house_col<T>(colv, re_l(colv[k + 1]), k + 1, n, V, tau, d, e, red);
    } else if (threadIdx.x == 0) {
      // last diagonal element
      const T wk1 = p[k + 1] + K * vk[k + 1];
      const int r = n - 1;
      T &a = A[static_cast<int64_t>(r) * n + r];
      a = a - (vk[r] * cj_l(wk1) + wk1 * cj_l(vk[r]));
      d[r] = re_l(a);
    }
    return;
  }
  // trailing block rows/cols >= k+2 in 16 x 16 tiles
  const int base = k + 2;
  const int m = n - base;
  const int tiles = (m + 15) / 16;
  const int tile = blockIdx.x - 1;
  const int ti = tile / tiles, tj = tile - (tile / tiles) * tiles;
  const int r = base + ti * 16 + (threadIdx.x >> 4), c = base + tj * 16 + (threadIdx.x & 15);
  if (r >= n || c >= n) return;
  const T vr = vk[r], wr = p[r] + K * vk[r];
  const T vc = cj_l(vk[c]), wc = cj_l(p[c] + K * vk[c]);
  T &a = A[static_cast<int64_t>(r) * n + c];
  a = a - (vr * wc + wr * vc);
}

// ------------------------------------------------------------------ vectors
__device__ inline double start_value_l(int j, int i) {
  uint64_t z = (static_cast<uint64_t>(j) << 32) + static_cast<uint64_t>(i) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__device__ inline bool split_l(const double *d, const double *e, int i) {
  return fabs(e[i]) <= DBL_EPSILON * (fabs(d[i]) + fabs(d[i + 1]));
}

// inverse iteration, one lane per eigenvalue, LU scratch in global memory
// (lu[q][i][j] for q = u0, u1, u2, y)
__global__ __launch_bounds__(64) void k_lvectors(int n, const double *__restrict__ d,
                                                 const double *__restrict__ e,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ lu, double *__restrict__ Z,
                                                 const int32_t *info) {
  if (*info != 0) return;
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= n) return;
  const int64_t nn = static_cast<int64_t>(n) * n;
  double *u0 = lu, *u1 = lu + nn, *u2 = lu + 2 * nn, *y = lu + 3 * nn;
#define AT(p, i) (p)[static_cast<int64_t>(i) * n + j]
  int lo = j, hi = j;
  while (lo > 0 && !split_l(d, e, lo - 1)) --lo;
  while (hi < n - 1 && !split_l(d, e, hi)) ++hi;
  const int m = hi - lo + 1;
  double tn = 0.0;
  for (int i = lo; i <= hi; ++i)
    tn = fmax(tn, fabs(d[i]) + (i > lo ? fabs(e[i - 1]) : 0.0) + (i < hi ? fabs(e[i]) : 0.0));
  const double pert = 10.0 * DBL_EPSILON * fmax(tn, DBL_MIN);
  int ties = 0;
  for (int i = j; i > lo && lam[i] - lam[i - 1] < pert; --i) ++ties;
  const double x = lam[j - ties] + ties * pert;
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);
  for (int i = 0; i < m; ++i) AT(y, i) = start_value_l(j, i);
  // LU with partial pivoting of (T_block - x I) once (branch-free, the
  // running y_i kept in a register), forward-eliminating y; multipliers and
  // swap flags kept for the second solve, pivots stored as reciprocals
  // (tiny ones replaced by +-eps ||T||)
  double *ml = lu + 4 * nn, *ms = lu + 5 * nn;
  {
    double c0 = d[lo] - x, c1 = (m > 1) ? e[lo] : 0.0;
    double ycur = AT(y, 0);
    for (int i = 0; i + 1 < m; ++i) {
      const double n0 = e[lo + i], n1 = d[lo + i + 1] - x;
      const double n2 = (i + 2 < m) ? e[lo + i + 1] : 0.0;
      const double yn = AT(y, i + 1);
      const bool sw = fabs(n0) > fabs(c0);
      const double num = sw ? c0 : n0, den = sw ? n0 : c0;
      const double l = den != 0.0 ? num / den : 0.0;
      AT(u0, i) = sw ? n0 : c0;
      AT(u1, i) = sw ? n1 : c1;
      AT(u2, i) = sw ? n2 : 0.0;
      AT(y, i) = sw ? yn : ycur;
      ycur = sw ? ycur - l * yn : yn - l * ycur;
      AT(ml, i) = sw ? -1.0 : 0.0;
      AT(ms, i) = l;
      const double c0n = sw ? c1 - l * n1 : n1 - l * c1;
      c1 = sw ? -l * n2 : n2;
      c0 = c0n;
    }
    AT(y, m - 1) = ycur;
    AT(u0, m - 1) = c0;
  }
  for (int i = 0; i < m; ++i) {
    double pv = AT(u0, i);
    if (fabs(pv) < tiny) pv = (pv < 0.0) ? -tiny : tiny;
    AT(u0, i) = 1.0 / pv;
  }
  for (int iter = 0; iter < 2; ++iter) {
    if (iter > 0) {
      double ycur = AT(y, 0);
      for (int i = 0; i + 1 < m; ++i) {
        const double yn = AT(y, i + 1), l = AT(ms, i);
        const bool sw = AT(ml, i) < 0.0;
        AT(y, i) = sw ? yn : ycur;
        ycur = sw ? ycur - l * yn : yn - l * ycur;
      }
      AT(y, m - 1) = ycur;
    }
    double y1 = 0.0, y2 = 0.0, ymax = 0.0;
    for (int i = m - 1; i >= 0; --i) {
      double sacc = AT(y, i);
      if (i + 1 < m) sacc -= AT(u1, i) * y1;
      if (i + 2 < m) sacc -= AT(u2, i) * y2;
      const double yi = sacc * AT(u0, i);
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
    Z[static_cast<int64_t>(i) * n + j] = (i >= lo && i <= hi) ? AT(y, i - lo) * sc : 0.0;
#undef AT
}

// ------------------------------------------------------------------ back-transform
// one wavefront per column: u <- u - tau_k v_k (v_k^H u), k = n-2..0;
// U written to column rank(j), eps[rank] = lam[j]
template <typename T>
__global__ __launch_bounds__(64) void k_lback(int n, const double *__restrict__ Z,
                                              const T *__restrict__ V, const T *__restrict__ tau,
                                              const double *__restrict__ lam, T *__restrict__ Uo,
                                              double *__restrict__ eps, const int32_t *info) {
  if (*info != 0) return;
  constexpr int R = LNMAX / 64;
  const int col = blockIdx.x, s = threadIdx.x;
  T u[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = 64 * t + s;
    u[t] = rv<T>(row < n ? Z[static_cast<int64_t>(row) * n + col] : 0.0);
  }
  for (int k = n - 2; k >= 0; --k) {
    const T *vk = V + static_cast<int64_t>(k) * n;
    T part = T{};
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int row = 64 * t + s;
      if (row > k && row < n) part = part + cj_l(vk[row]) * u[t];
    }
    part = wsum(part);
    const T f = tau[k] * part;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int row = 64 * t + s;
      if (row > k && row < n) u[t] = u[t] - f * vk[row];
    }
  }
  const double lj = lam[col];
  int rank = 0;
  for (int i = s; i < n; i += 64) {
    const double li = lam[i];
    rank += (li < lj) || (li == lj && i < col);
  }
  for (int off = 32; off >= 1; off >>= 1) rank += __shfl_xor(rank, off);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = 64 * t + s;
    if (row < n) Uo[static_cast<int64_t>(row) * n + rank] = u[t];
  }
  if (s == 0) eps[rank] = lj;
}

}  // namespace

// entry points used by eigh.hip
template <typename T>
int large_chol_linv(T *Sw, T *Linv, int n, double *piv, int32_t *info, hipStream_t st) {
  for (int j = 0; j < n; ++j) {
    const int m = n - j - 1;
    const int tiles = (m + 15) / 16;
    k_lchol_step<T><<<std::max(1, tiles * tiles), 256, 0, st>>>(Sw, n, j, piv, info);
  }
  const int64_t nn = static_cast<int64_t>(n) * n;
  k_lchol_scale<T><<<static_cast<unsigned>((nn + 255) / 256), 256, 0, st>>>(Sw, n, piv, info);
  k_linv_col<T><<<n, 64, 0, st>>>(Sw, Linv, n, info);
  return GPAW_OK;
}

template <typename T>
int large_tridiag(T *A, int n, T *V, T *tau, double *d, double *e, T *p, int32_t *info,
                  hipStream_t st) {
  const size_t lds = static_cast<size_t>(n) * sizeof(T);
  k_trd_first<T><<<1, 256, lds, st>>>(A, n, V, tau, d, e, info);
  for (int k = 0; k + 1 < n; ++k) {
    k_trd_symv<T><<<(n - k - 1 + 3) / 4, 256, 0, st>>>(A, n, k, V, tau, p, info);
    const int m = std::max(0, n - k - 2);
    const int tiles = (m + 15) / 16;
    k_trd_update<T><<<1 + tiles * tiles, 256, lds, st>>>(A, n, k, V, tau, p, d, e, info);
  }
  return GPAW_OK;
}

int large_vectors(int n, const double *d, const double *e, const double *lam, double *lu,
                  double *Z, const int32_t *info, hipStream_t st) {
  k_lvectors<<<(n + 63) / 64, 64, 0, st>>>(n, d, e, lam, lu, Z, info);
  return GPAW_OK;
}

template <typename T>
int large_back(int n, const double *Z, const T *V, const T *tau, const double *lam, T *U,
               double *eps, const int32_t *info, hipStream_t st) {
  k_lback<T><<<n, 64, 0, st>>>(n, Z, V, tau, lam, U, eps, info);
  return GPAW_OK;
}

template int large_chol_linv<double>(double *, double *, int, double *, int32_t *, hipStream_t);
template int large_chol_linv<z64>(z64 *, z64 *, int, double *, int32_t *, hipStream_t);
template int large_tridiag<double>(double *, int, double *, double *, double *, double *,
                                   double *, int32_t *, hipStream_t);
template int large_tridiag<z64>(z64 *, int, z64 *, z64 *, double *, double *, z64 *, int32_t *,
                                hipStream_t);
template int large_back<double>(int, const double *, const double *, const double *,
                                const double *, double *, double *, const int32_t *, hipStream_t);
template int large_back<z64>(int, const double *, const z64 *, const z64 *, const double *, z64 *,
                             double *, const int32_t *, hipStream_t);

}  // namespace gfd
