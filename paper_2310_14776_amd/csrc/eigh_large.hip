// Generalised Hermitian eigenproblem of the subspace for blocks too large
// for one workgroup's LDS (nb > 128 real, nb > 96 complex, up to 1024):
// the same method as eigh.hip (Cholesky and diagonalisation of the subspace
// matrices, Sec. "Parallelization"), with the matrices in global memory
// (L2/MALL resident) and every sequential step spread over the whole chip:
//   Cholesky       blocked, right-looking, lower, two launches per panel
//                  of 32 columns, with L^-1 built block row by block row in
//                  the same launches;
//   A = Linv H Linv^H, Newton-Schulz, C = Linv^H U: MFMA small-GEMM kernel;
//   tridiagonal    two launches per column: p = tau A v (one wavefront per
//                  row), then the rank-2 update of the trailing block with,
//                  in workgroup 0, the next column and its Householder
//                  vector (that column is left to workgroup 0 alone, so no
//                  workgroup reads a value another one is rewriting);
//   eigenvalues    as for small blocks (multisection, d/e in LDS);
//   eigenvectors   inverse iteration, a few eigenvalues per workgroup with
//                  the LU scratch in LDS;
//   back-transform one wavefront per column, reflectors read from L2 one
//                  step ahead of their use.
#include <algorithm>
#include <cfloat>
#include <mutex>
#include <string>

#include "internal.h"

namespace gfd {

namespace {

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
__device__ inline double sel_l(bool c, double a, double b) { return c ? a : b; }
__device__ inline z64 sel_l(bool c, z64 a, z64 b) { return z64{c ? a.x : b.x, c ? a.y : b.y}; }
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
// Blocked right-looking Cholesky S = L L^H (lower) with the inverse L^-1
// formed block row by block row alongside, in panels of CB columns:
//   diagonal block  factored in LDS by one workgroup, which builds its
//                   inverse D with the same row operations applied to I,
//                   zeros the upper parts of its rows in L and L^-1 and
//                   records the pivots (the squared diagonal of L);
//   panel rows      L21 = A21 L11^-H, one thread per row (k_lchol_solve);
//   trailing block  A22 -= L21 L21^H on the lower tiles; the workgroup of
//                   the top-left tile factors that tile (the next diagonal
//                   block) straight from LDS (k_lchol_update);
//   L^-1 block row  (L^-1)_IJ = -D_I sum_{J <= K < I} L_IK (L^-1)_KJ, one
//                   workgroup per J < I, in the same launch as the trailing
//                   update (they touch disjoint parts of both matrices).
// Two launches per panel instead of one per column.
constexpr int CB = 32;       // panel width
constexpr int CBP = CB + 1;  // LDS row pitch

struct CholLds {
  double rdiag[CB];  // 1 / L_cc
  double pd[CB];     // pivots d_c = L_cc^2
};

// Factor the wb x wb block held in a (lower part) in place and build its
// inverse in m. Columns are eliminated unscaled: step c forms the unit-lower
// factor's column l_r = a_rc / d_c and applies row r -= l_r row c (r > c) to
// the trailing part of a (a_rk -= l_r conj(a_kc), k > c) and to m, which
// starts as the identity and so ends as the inverse of the unit-lower factor.
// Only rows below c and, in a, columns right of c change in step c, so one
// barrier per column suffices. At the end L_rk = a_rk / sqrt(d_k) and
// L^-1 = diag(1 / sqrt(d)) m. Returns the first failing column + 1 (pivot not
// positive, or NaN), else 0; uniform across the workgroup. The caller has
// synchronised after filling a (zeros outside the lower wb x wb part).
template <typename T>
__device__ int chol_block_lds(T *a, T *m, int wb, CholLds &cl) {
  const int tid = threadIdx.x, tr = tid / CB, k = tid - (tid / CB) * CB;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = tr + 8 * q;
    m[r * CBP + k] = r == k ? rv<T>(1.0) : T{};
  }
  __syncthreads();
  for (int c = 0; c < wb; ++c) {
    const double d = re_l(a[c * CBP + c]);
    if (!(d > 0.0)) return c + 1;
    const double inv = 1.0 / d;
    if (tid == 0) cl.pd[c] = d;
    const T akc = cj_l(a[k * CBP + c]), mck = m[c * CBP + k];
    // every element is read and written back (unchanged where not updated):
    // with conditional stores the compiler moves each load into its branch
    // and waits on them one by one; each element has one owner, and a value
    // written back unchanged is the value other threads may read
    T lr[4], ar[4], mr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = tr + 8 * q;
      lr[q] = a[r * CBP + c];
      ar[q] = a[r * CBP + k];
      mr[q] = m[r * CBP + k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = tr + 8 * q;
      const T l = mulr(lr[q], inv);
      const bool upd = r > c;
      a[r * CBP + k] = sel_l(upd && k > c, ar[q] - l * akc, ar[q]);
      m[r * CBP + k] = sel_l(upd && k <= c, mr[q] - l * mck, mr[q]);
    }
    __syncthreads();
  }
  if (tid < wb) cl.rdiag[tid] = 1.0 / sqrt(cl.pd[tid]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = tr + 8 * q;
    if (k <= r && r < wb) {
      a[r * CBP + k] = k == r ? rv<T>(sqrt(cl.pd[k])) : mulr(a[r * CBP + k], cl.rdiag[k]);
      m[r * CBP + k] = mulr(m[r * CBP + k], cl.rdiag[r]);
    }
  }
  __syncthreads();
  return 0;
}

// The diagonal block at row/column jb (width wb) sits in LDS a (lower part,
// trailing updates applied, zeros elsewhere): factor it, write L_bb, its
// inverse D_b (built in dm), the zeros right of the block in both matrices,
// the pivots, and info on failure.
template <typename T>
__device__ void chol_diag_finish(T *a, T *dm, CholLds &cl, T *__restrict__ A, T *__restrict__ Linv, int n,
                                 int jb, int wb, double *__restrict__ piv, int32_t *info) {
  const int tid = threadIdx.x;
  const int bad = chol_block_lds<T>(a, dm, wb, cl);
  if (bad) {
    if (tid == 0) *info = jb + bad;
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q, r = idx / CB, c = idx - (idx / CB) * CB;
    if (r < wb && c < wb) {
      const int64_t o = static_cast<int64_t>(jb + r) * n + jb + c;
      A[o] = c <= r ? a[r * CBP + c] : T{};
      Linv[o] = c <= r ? dm[r * CBP + c] : T{};
    }
  }
  const int right = n - jb - wb;
  for (int r = 0; r < wb; ++r)
    for (int c = tid; c < right; c += 256) {
      const int64_t o = static_cast<int64_t>(jb + r) * n + jb + wb + c;
      A[o] = T{};
      Linv[o] = T{};
    }
  if (tid < wb) piv[jb + tid] = cl.pd[tid];
}

// first diagonal block
template <typename T>
__global__ __launch_bounds__(256) void k_lchol_first(T *__restrict__ A, T *__restrict__ Linv, int n,
                                                     double *__restrict__ piv, int32_t *info) {
  if (*info != 0) return;
  __shared__ T a[CB * CBP], dm[CB * CBP];
  __shared__ CholLds cl;
  const int wb = min(CB, n);
  for (int idx = threadIdx.x; idx < CB * CB; idx += 256) {
    const int r = idx / CB, c = idx - (idx / CB) * CB;
    a[r * CBP + c] = (r < wb && c <= r) ? A[static_cast<int64_t>(r) * n + c] : T{};
  }
  __syncthreads();
  chol_diag_finish<T>(a, dm, cl, A, Linv, n, 0, wb, piv, info);
}

// L21 = A21 L11^-H for the rows below the panel at j0 (width CB): one row
// per thread, x_c = (a_c - sum_{k<c} x_k conj(L_ck)) / L_cc
template <typename T>
__global__ __launch_bounds__(256) void k_lchol_solve(T *__restrict__ A, int n, int j0,
                                                     const int32_t *info) {
  if (*info != 0) return;
  __shared__ T l[CB * CBP];
  __shared__ double rd[CB];
  for (int idx = threadIdx.x; idx < CB * CB; idx += 256) {
    const int r = idx / CB, c = idx - (idx / CB) * CB;
    l[r * CBP + c] = c <= r ? A[static_cast<int64_t>(j0 + r) * n + j0 + c] : T{};
  }
  __syncthreads();
  if (threadIdx.x < CB) rd[threadIdx.x] = 1.0 / re_l(l[threadIdx.x * CBP + threadIdx.x]);
  __syncthreads();
  const int r = j0 + CB + static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (r >= n) return;
  T *Ar = A + static_cast<int64_t>(r) * n + j0;
  T x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = Ar[c];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    T v = x[c];
#pragma unroll
    for (int k = 0; k < c; ++k) v = v - x[k] * cj_l(l[c * CBP + k]);
    x[c] = mulr(v, rd[c]);
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) Ar[c] = x[c];
}

// Workgroups [0, tt(tt+1)/2): lower tiles of the trailing block below the
// panel at j0 (tile 0 then factors the next diagonal block); the rest: block
// row I = j0 / CB of L^-1, one workgroup per block column J < I.
template <typename T>
__global__ __launch_bounds__(256) void k_lchol_update(T *__restrict__ A, T *__restrict__ Linv, int n,
                                                      int j0, int tt, double *__restrict__ piv,
                                                      int32_t *info) {
  if (*info != 0) return;
  __shared__ T ta[CB * CBP], tb[CB * CBP];
  __shared__ CholLds cl;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  const int w = min(CB, n - j0), j1 = j0 + w;
  const int ntri = tt * (tt + 1) / 2;
  const int bid = static_cast<int>(blockIdx.x);
  T acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = T{};
  if (bid < ntri) {
    int ti = 0, rest = bid;
    while (rest > ti) {
      rest -= ti + 1;
      ++ti;
    }
    const int tj = rest;
    const int r0 = j1 + ti * CB, c0 = j1 + tj * CB;
    for (int idx = tid; idx < CB * CB; idx += 256) {
      const int r = idx / CB, k = idx - (idx / CB) * CB;
      ta[r * CBP + k] = r0 + r < n ? A[static_cast<int64_t>(r0 + r) * n + j0 + k] : T{};
      tb[r * CBP + k] = c0 + r < n ? A[static_cast<int64_t>(c0 + r) * n + j0 + k] : T{};
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < CB; ++k) {
      const T bk = cj_l(tb[tx * CBP + k]);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = acc[q] + ta[(ty + 8 * q) * CBP + k] * bk;
    }
    const int c = c0 + tx;
    if (bid == 0) {
      // top-left tile = next diagonal block: update into LDS, factor there
      const int wb = min(CB, n - j1);
      __syncthreads();  // ta is reused
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rl = ty + 8 * q, r = r0 + rl;
        ta[rl * CBP + tx] = (r < n && c < n && tx <= rl) ? A[static_cast<int64_t>(r) * n + c] - acc[q] : T{};
      }
      __syncthreads();
      chol_diag_finish<T>(ta, tb, cl, A, Linv, n, j1, wb, piv, info);
      return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + ty + 8 * q;
      if (r < n && c < n && c <= r) {
        T &dst = A[static_cast<int64_t>(r) * n + c];
        dst = dst - acc[q];
      }
    }
    return;
  }
  const int I = j0 / CB, J = bid - ntri, cJ = J * CB;
  for (int K = J; K < I; ++K) {
    __syncthreads();
    for (int idx = tid; idx < CB * CB; idx += 256) {
      const int r = idx / CB, k = idx - (idx / CB) * CB;
      ta[r * CBP + k] = r < w ? A[static_cast<int64_t>(j0 + r) * n + K * CB + k] : T{};
      tb[r * CBP + k] = Linv[static_cast<int64_t>(K * CB + r) * n + cJ + k];
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < CB; ++k) {
      const T bk = tb[k * CBP + tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = acc[q] + ta[(ty + 8 * q) * CBP + k] * bk;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < CB * CB; idx += 256) {
    const int r = idx / CB, k = idx - (idx / CB) * CB;
    ta[r * CBP + k] = (r < w && k < w) ? Linv[static_cast<int64_t>(j0 + r) * n + j0 + k] : T{};
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) tb[(ty + 8 * q) * CBP + tx] = acc[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rl = ty + 8 * q;
    T v{};
#pragma unroll 8
    for (int k = 0; k < CB; ++k) v = v + ta[rl * CBP + k] * tb[k * CBP + tx];
    if (rl < w) Linv[static_cast<int64_t>(j0 + rl) * n + cJ + tx] = T{} - v;
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
  // trailing block rows/cols >= k+2 in 32 x 32 tiles, four elements per
  // lane (rows tid / 32 + 8 q of column tid % 32), so each workgroup's
  // reduction above serves 1024 elements
  const int base = k + 2;
  const int m = n - base;
  const int tiles = (m + 31) / 32;
  const int tile = blockIdx.x - 1;
  const int ti = tile / tiles, tj = tile - (tile / tiles) * tiles;
  const int c = base + tj * 32 + (threadIdx.x & 31);
  if (c >= n) return;
  const T vc = cj_l(vk[c]), wc = cj_l(p[c] + K * vk[c]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = base + ti * 32 + (threadIdx.x >> 5) + 8 * q;
    if (r < n) {
      const T vr = vk[r], wr = p[r] + K * vk[r];
      T &a = A[static_cast<int64_t>(r) * n + c];
      a = a - (vr * wc + wr * vc);
    }
  }
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
__global__ __launch_bounds__(64) void k_lvectors(int n, int L, const double *__restrict__ d,
                                                 const double *__restrict__ e,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ Z, const int32_t *info) {
  if (*info != 0) return;
  // L eigenvalues per workgroup (lanes 0..L-1), each with six n-long scratch
  // columns in LDS, interleaved by lane: the solves are sequential chains, so
  // their latency is that of LDS rather than of L2
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int j = blockIdx.x * L + lane;
  if (lane >= L || j >= n) return;
  const int nl = n * L;
  double *u0 = lds, *u1 = lds + nl, *u2 = lds + 2 * nl, *y = lds + 3 * nl;
#define AT(p, i) (p)[(i) * L + lane]
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
  double *ml = lds + 4 * nl, *ms = lds + 5 * nl;
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
template <typename T, int RR>
__global__ __launch_bounds__(64) void k_lback(int n, const double *__restrict__ Z,
                                              const T *__restrict__ V, const T *__restrict__ tau,
                                              const double *__restrict__ lam, T *__restrict__ Uo,
                                              double *__restrict__ eps, const int32_t *info) {
  if (*info != 0) return;
  // rows 64 t + s, t < RR (64 RR >= n); rows past n hold u = 0 and are never
  // updated; v_k is zero on rows <= k, so no row needs masking in the dot
  // product. The reflector of the next step is loaded while the current one
  // is applied (clamped, unconditional loads).
  const int col = blockIdx.x, s = threadIdx.x;
  T u[RR];
#pragma unroll
  for (int t = 0; t < RR; ++t) {
    const int row = 64 * t + s;
    u[t] = rv<T>(row < n ? Z[static_cast<int64_t>(row) * n + col] : 0.0);
  }
  auto load_v = [&](int k, T (&v)[RR], T &tk) {
    const int kc = k < 0 ? 0 : k;
    const T *vk = V + static_cast<int64_t>(kc) * n;
#pragma unroll
    for (int t = 0; t < RR; ++t) v[t] = vk[std::min(64 * t + s, n - 1)];
    tk = tau[kc];
  };
  auto apply = [&](const T (&v)[RR], T tk) {
    T part = T{};
#pragma unroll
    for (int t = 0; t < RR; ++t) part = part + cj_l(v[t]) * u[t];
    part = wsum(part);
    const T f = tk * part;
#pragma unroll
    for (int t = 0; t < RR; ++t) {
      u[t] = sel_l(64 * t + s < n, u[t] - f * v[t], u[t]);
    }
  };
  T va[RR], vb[RR], ta, tb;
  load_v(n - 2, va, ta);
  for (int k = n - 2; k >= 0; k -= 2) {
    load_v(k - 1, vb, tb);
    apply(va, ta);
    if (k - 1 < 0) break;
    load_v(k - 2, va, ta);
    apply(vb, tb);
  }
  const double lj = lam[col];
  int rank = 0;
  for (int i = s; i < n; i += 64) {
    const double li = lam[i];
    rank += (li < lj) || (li == lj && i < col);
  }
  for (int off = 32; off >= 1; off >>= 1) rank += __shfl_xor(rank, off);
#pragma unroll
  for (int t = 0; t < RR; ++t) {
    const int row = 64 * t + s;
    if (row < n) Uo[static_cast<int64_t>(row) * n + rank] = u[t];
  }
  if (s == 0) eps[rank] = lj;
}

}  // namespace

// entry points used by eigh.hip
template <typename T>
int large_chol_linv(T *Sw, T *Linv, int n, double *piv, int32_t *info, hipStream_t st) {
  k_lchol_first<T><<<1, 256, 0, st>>>(Sw, Linv, n, piv, info);
  for (int j0 = 0; j0 < n; j0 += CB) {
    const int below = n - j0 - CB;
    if (below > 0) k_lchol_solve<T><<<(below + 255) / 256, 256, 0, st>>>(Sw, n, j0, info);
    const int tt = below > 0 ? (below + CB - 1) / CB : 0;
    const int wgs = tt * (tt + 1) / 2 + j0 / CB;
    if (wgs > 0) k_lchol_update<T><<<wgs, 256, 0, st>>>(Sw, Linv, n, j0, tt, piv, info);
  }
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
    const int tiles = (m + 31) / 32;
    k_trd_update<T><<<1 + tiles * tiles, 256, lds, st>>>(A, n, k, V, tau, p, d, e, info);
  }
  return GPAW_OK;
}

int large_vectors(int n, const double *d, const double *e, const double *lam, double *lu,
                  double *Z, const int32_t *info, hipStream_t st) {
  (void)lu;  // the scratch lives in LDS
  constexpr size_t LDS_MAX = 160 * 1024;
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lvectors),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX);
  });
  if (attr_err != hipSuccess) return hip_fail(attr_err, "hipFuncSetAttribute(k_lvectors)");
  const size_t per_lane = 6 * static_cast<size_t>(n) * sizeof(double);
  const int L = static_cast<int>(std::max<size_t>(1, std::min<size_t>(64, LDS_MAX / per_lane)));
  k_lvectors<<<(n + L - 1) / L, 64, per_lane * L, st>>>(n, L, d, e, lam, Z, info);
  return GPAW_OK;
}

template <typename T>
int large_back(int n, const double *Z, const T *V, const T *tau, const double *lam, T *U,
               double *eps, const int32_t *info, hipStream_t st) {
  if (n <= 128) k_lback<T, 2><<<n, 64, 0, st>>>(n, Z, V, tau, lam, U, eps, info);
  else if (n <= 256) k_lback<T, 4><<<n, 64, 0, st>>>(n, Z, V, tau, lam, U, eps, info);
  else if (n <= 512) k_lback<T, 8><<<n, 64, 0, st>>>(n, Z, V, tau, lam, U, eps, info);
  else k_lback<T, 16><<<n, 64, 0, st>>>(n, Z, V, tau, lam, U, eps, info);
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
