// Generalised symmetric eigenproblem of the subspace, H C = S C diag(eps),
// in FP64 on the device (Cholesky and diagonalisation of the subspace
// matrices, Sec. "Parallelization"; SCF step (1), Sec. "Solving the
// Kohn-Sham equation").
//
// Pipeline (real symmetric, nb <= 128), all on one stream:
//   k_eig_chol     (1 workgroup, matrix in LDS) S <- (S+S^T)/2 = L L^T and
//                  Linv = L^-1, blocked by 16x16 tiles on FP64 MFMA;
//   k_small_gemm   A = Linv ((H+H^T)/2) Linv^T on FP64 MFMA (two products);
//   k_eig_tridiag  (1 workgroup, A in registers) Householder A = Q T Q^T;
//   k_eig_values   (one wavefront per eigenvalue) T splits where
//                  |e_i| <= eps (|d_i| + |d_i+1|); each eigenvalue is found in
//                  its unreduced block by 65-way multisection on Sturm counts;
//   k_eig_vectors  (one lane per eigenvalue) inverse iteration with a pivoted
//                  tridiagonal LU; shifts closer than 10 eps ||T|| are pulled
//                  apart by that amount;
//   k_cluster_orth modified Gram-Schmidt (twice) inside clusters of
//                  eigenvalues closer than 1e-7 ||T||;
//   refinement     one step (a second when the first leaves the Gram matrix
//                  more than 1e-13 from I) of the Ogita-Aishima eigenvector
//                  refinement on T: with G = Z^T Z and M = Z^T T Z it removes
//                  the orthogonality defect and every vector's part along
//                  eigenvectors at least 1e-2 ||T|| away;
//   k_eig_back     (8 lanes per column, reflectors in LDS) U = Q Z written
//                  in eigen-order; then C = Linv^T U on MFMA.
#include <algorithm>
#include <cfloat>
#include <mutex>
#include <string>

#include "internal.h"

namespace gfd {

template <typename T>
int large_chol_linv(T *Sw, T *Linv, int n, double *piv, int32_t *info, hipStream_t st);
template <typename T>
int large_tridiag(T *A, int n, T *V, T *tau, double *d, double *e, T *p, int32_t *info,
                  hipStream_t st);
int large_vectors(int n, const double *d, const double *e, const double *lam, double *lu,
                  double *Z, const int32_t *info, hipStream_t st);
template <typename T>
int large_back(int n, const double *Z, const T *V, const T *tau, const double *lam, T *U,
               double *eps, const int32_t *info, hipStream_t st);

namespace {

constexpr int EIG_T = 1024;
constexpr int EIG_NMAX = 128;
constexpr int EIG_LARGE_MAX = 1024;
constexpr int VEC_T = 8;  // lanes (eigenvectors) per inverse-iteration workgroup
constexpr int SG_T = 256;  // small-GEMM workgroup: four 16x16 output tiles
constexpr int CH_T = 512;  // blocked Cholesky: 8 wavefronts (256 VGPRs each)

typedef double d4 __attribute__((ext_vector_type(4)));

// Matrices Linv, T1, A, V and tau hold the system's scalar (double or
// complex); Z, Z2, G, d, e, lam are real. Pointers are to doubles.
struct EigWs {
  double *Linv, *T1, *A, *V, *Z, *Z2, *G, *tau, *d, *e, *lam;
  double *Sw, *piv, *p, *lu;  // blocks above the LDS limit only
  int32_t *cid;               // [n] first slot of each slot's eigenvalue cluster
  double *cltol;              // cluster tolerance CL_TOL ||T||
  int32_t *skip;              // nonzero: the second refinement step has nothing to do
};

size_t eig_layout_elems(int n, int sz, bool large) {
  const size_t nn = static_cast<size_t>(n) * n;
  size_t e = 4 * sz * nn + 3 * nn + sz * n + 3 * n;
  if (large) e += sz * nn + n + sz * n + 6 * nn;
  e += (n + 1) / 2 + 2;  // cluster ids and tolerance
  return e + 64;
}

// sz = doubles per scalar; large = include the global-memory path's buffers
EigWs eig_layout(double *base, int n, int sz, bool large) {
  const size_t nn = static_cast<size_t>(n) * n;
  EigWs w;
  w.Linv = base;
  w.T1 = w.Linv + sz * nn;
  w.A = w.T1 + sz * nn;
  w.V = w.A + sz * nn;
  w.Z = w.V + sz * nn;
  w.Z2 = w.Z + nn;
  w.G = w.Z2 + nn;
  w.tau = w.G + nn;
  w.d = w.tau + sz * n;
  w.e = w.d + n;
  w.lam = w.e + n;
  double *q = w.lam + n;
  w.Sw = w.piv = w.p = w.lu = nullptr;
  if (large) {
    w.Sw = q;
    w.piv = w.Sw + sz * nn;
    w.p = w.piv + n;
    w.lu = w.p + sz * n;
    q = w.lu + 6 * nn;
  }
  w.cltol = q;
  w.cid = reinterpret_cast<int32_t *>(q + 1);
  // the last double of the block (the layout keeps 64 spare at its end)
  w.skip = reinterpret_cast<int32_t *>(base + eig_layout_elems(n, sz, large) - 1);
  return w;
}


template <typename T> __host__ __device__ inline T *as(double *p) { return reinterpret_cast<T *>(p); }

// Wavefront reductions on DPP lane moves (gfx9 row permutations: lane ^ 1,
// lane ^ 2, half-row and row mirrors) plus readlane across the four rows;
// every lane gets the same value. The wavefront must be fully active.
template <int CTRL>
__device__ inline double dpp(double v) {
  const int2 u = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_mov_dpp(u.x, CTRL, 0xF, 0xF, false),
                                              __builtin_amdgcn_mov_dpp(u.y, CTRL, 0xF, 0xF, false)));
}
__device__ inline double lane_read(double v, int lane) {
  const int2 u = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(u.x, lane),
                                              __builtin_amdgcn_readlane(u.y, lane)));
}
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

__device__ inline double wave_sum(double v) {
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  v += dpp<DPP_HALF_MIRROR>(v);
  v += dpp<DPP_MIRROR>(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp<DPP_XOR1>(v));
  v = fmax(v, dpp<DPP_XOR2>(v));
  v = fmax(v, dpp<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp<DPP_MIRROR>(v));
  return fmax(fmax(lane_read(v, 0), lane_read(v, 16)), fmax(lane_read(v, 32), lane_read(v, 48)));
}
__device__ inline double wave_min(double v) {
  v = fmin(v, dpp<DPP_XOR1>(v));
  v = fmin(v, dpp<DPP_XOR2>(v));
  v = fmin(v, dpp<DPP_HALF_MIRROR>(v));
  v = fmin(v, dpp<DPP_MIRROR>(v));
  return fmin(fmin(lane_read(v, 0), lane_read(v, 16)), fmin(lane_read(v, 32), lane_read(v, 48)));
}

__device__ inline z64 wave_sum(z64 v) { return z64{wave_sum(v.x), wave_sum(v.y)}; }

// 8-lane group reductions (lanes 8q..8q+7, the half-rows)
__device__ inline double group8_sum(double v) {
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  v += dpp<DPP_HALF_MIRROR>(v);
  return v;
}
__device__ inline z64 group8_sum(z64 v) { return z64{group8_sum(v.x), group8_sum(v.y)}; }

// 1/x from the hardware estimate and two Newton steps (x != 0, finite)
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// real / complex helpers
__device__ inline double re_of(double a) { return a; }
__device__ inline double re_of(z64 a) { return a.x; }
__device__ inline double abs2(double a) { return a * a; }
__device__ inline double abs2(z64 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double cj(double a) { return a; }
__device__ inline z64 cj(z64 a) { return zconj(a); }
__device__ inline z64 operator*(z64 a, double s) { return z64{a.x * s, a.y * s}; }

template <typename T> __device__ inline T realv(double r);
template <> __device__ inline double realv<double>(double r) { return r; }
template <> __device__ inline z64 realv<z64>(double r) { return z64{r, 0.0}; }

template <typename T> struct EigMax;
template <> struct EigMax<double> { static constexpr int n = 128; };
template <> struct EigMax<z64> { static constexpr int n = 96; };

__device__ inline bool split_at(const double *d, const double *e, int i) {
  return fabs(e[i]) <= DBL_EPSILON * (fabs(d[i]) + fabs(d[i + 1]));
}

// ------------------------------------------------------------------ Cholesky
// S <- (S+S^H)/2 = L L^H and Linv = L^-1, blocked by 16x16 tiles in LDS.
// The matrix is padded to N = 16 ceil(n/16) with an identity block, so every
// tile is full. Right-looking over tile columns k:
//   wave 0   factors the diagonal tile (lane r owns row r, column values
//            broadcast by readlane) and overwrites it with its inverse;
//   panel    L_ik = A_ik L_kk^-H, one wavefront per tile (FP64 MFMA);
//   update   A_ij -= L_ik L_jk^H for k < j <= i, one wavefront per tile.
// Then block rows of Linv: X_ik = -L_ii^-1 sum_{j=k}^{i-1} L_ij X_jk, the
// blocks X_jk (j > k) kept transposed in the unused upper tile (k, j).

__device__ inline double rl(double v, int lane) {
  const int2 u = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(u.x, lane),
                                              __builtin_amdgcn_readlane(u.y, lane)));
}
__device__ inline z64 rl(z64 v, int lane) { return z64{rl(v.x, lane), rl(v.y, lane)}; }

// acc += op(A) op(B) over one 16-deep tile product on FP64 MFMA; fa(i, k) and
// fb(k, j) return the operand elements (complex: four real products).
template <typename T, typename FA, typename FB>
__device__ inline void tile_mma(d4 &accr, d4 &acci, FA fa, FB fb) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const T a = fa(i, 4 * ks + kq), b = fb(4 * ks + kq, i);
    if constexpr (St<T>::cplx) {
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(re_of(a), re_of(b), accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acci, 0, 0, 0);
    } else {
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(re_of(a), re_of(b), accr, 0, 0, 0);
    }
  }
}

template <typename T> __device__ inline T from_acc(const d4 &r, const d4 &i, int e);
template <> __device__ inline double from_acc<double>(const d4 &r, const d4 &, int e) { return r[e]; }
template <> __device__ inline z64 from_acc<z64>(const d4 &r, const d4 &i, int e) {
  return z64{r[e], i[e]};
}

// Wave 0: factor diagonal tile D (in LDS, stride lda) = L L^H and overwrite it
// with L^-1 (zeros above the diagonal). Returns j+1 of the first pivot that
// is not positive (uniform), else 0.
template <typename T>
__device__ inline int diag_factor_inverse(T *D, int lda) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  T row[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) row[c] = D[r * lda + c];
  double dinv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double d = rl(re_of(row[j]), j);
    if (!(d > 0.0)) return j + 1;
    // 1/sqrt(d) from the hardware estimate and two Newton steps, sqrt(d) as
    // d/sqrt(d): no division or square-root sequence on the chain
    double rs = __builtin_amdgcn_rsq(d);
    rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
    rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
    const double sd = d * rs;
    dinv[j] = rs;
    const T lrj = r > j ? row[j] * dinv[j] : (r == j ? realv<T>(sd) : T{});
    row[j] = lrj;
#pragma unroll
    for (int c = j + 1; c < 16; ++c) {
      const T lcj = rl(lrj, c);
      if (r >= c) row[c] = row[c] - lrj * cj(lcj);
    }
  }
  // L back to the tile; its row r is read again one element per step below
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) D[r * lda + c] = row[c];
  }
  // X = L^-1 by rows: X[i][:] = (e_i - sum_{m<i} L[i][m] X[m][:]) / L[i][i]
  T acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = realv<T>(c == r ? 1.0 : 0.0);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const T lri = D[r * lda + i];
    // row i is final: X[i][c] = acc[c] / L[i][i] in lane i
#pragma unroll
    for (int c = 0; c <= i; ++c) {
      const T xic = rl(acc[c] * dinv[i], i);
      if (r == i) acc[c] = xic;
      else if (r > i) acc[c] = acc[c] - lri * xic;
    }
  }
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) D[r * lda + c] = c <= r ? acc[c] : T{};
  }
  return 0;
}

template <typename T>
__device__ __forceinline__ void d_eig_chol(const T *__restrict__ S, int n, EigWs w,
                                                    int32_t *info) {
  extern __shared__ double sm[];
  const int NT = (n + 15) / 16, N = 16 * NT, lda = N + 1;
  T *A = reinterpret_cast<T *>(sm);
  int &fail_sh = *reinterpret_cast<int *>(A + N * lda);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  // lower triangle of (S + S^H)/2, identity on the padding; eight elements
  // per thread per round with their loads issued first
  for (int base = 0; base < N * N; base += 8 * CH_T) {
    T sa[8], sb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * CH_T + tid;
      const int r = idx / N, c = idx - (idx / N) * N;
      const bool in = idx < N * N && c <= r && r < n && c < n;
      sa[u] = in ? S[r * n + c] : T{};
      sb[u] = in ? S[c * n + r] : T{};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * CH_T + tid;
      const int r = idx / N, c = idx - (idx / N) * N;
      if (idx >= N * N || c > r) continue;
      A[r * lda + c] = (r < n && c < n) ? St<T>::scale(0.5, sa[u] + cj(sb[u])) : realv<T>(r == c ? 1.0 : 0.0);
    }
  }
  if (tid == 0) fail_sh = 0;
  __syncthreads();
  auto tile = [&](int bi, int bj) { return A + (16 * bi) * lda + 16 * bj; };

  for (int k = 0; k < NT; ++k) {
    if (wave == 0) {
      const int f = diag_factor_inverse<T>(tile(k, k), lda);
      if (f && lane == 0) fail_sh = 16 * k + f;
    }
    __syncthreads();
    if (fail_sh) break;
    // panel: L_ik = A_ik Dinv_k^H
    const T *Dk = tile(k, k);
    for (int i = k + 1 + wave; i < NT; i += CH_T / 64) {
      T *Ti = tile(i, k);
      d4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
      tile_mma<T>(ar, ai, [&](int r, int c) { return Ti[r * lda + c]; },
                  [&](int kk, int c) { return cj(Dk[c * lda + kk]); });
#pragma unroll
      for (int e = 0; e < 4; ++e) Ti[(lq + 4 * e) * lda + li] = from_acc<T>(ar, ai, e);
    }
    __syncthreads();
    // trailing update of the lower tiles (i, j), k < j <= i
    const int m = NT - k - 1;
    for (int t = wave; t < m * (m + 1) / 2; t += CH_T / 64) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= t) ++i;
      const int j = t - i * (i + 1) / 2;
      const T *Li = tile(k + 1 + i, k), *Lj = tile(k + 1 + j, k);
      T *Tij = tile(k + 1 + i, k + 1 + j);
      d4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
      tile_mma<T>(ar, ai, [&](int r, int c) { return Li[r * lda + c]; },
                  [&](int kk, int c) { return cj(Lj[c * lda + kk]); });
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        T *p = Tij + (lq + 4 * e) * lda + li;
        *p = *p - from_acc<T>(ar, ai, e);
      }
    }
    __syncthreads();
  }
  if (fail_sh) {
    if (tid == 0) *info = fail_sh <= n ? fail_sh : n;
    return;
  }
  // block rows of Linv; X_kk = tile(k,k), X_jk (j > k) transposed in tile(k, j)
  for (int i = 1; i < NT; ++i) {
    for (int k = wave; k < i; k += CH_T / 64) {
      d4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
      for (int j = k; j < i; ++j) {
        const T *Lij = tile(i, j);
        const T *X = tile(k, j);  // j == k: X_kk as stored; j > k: transposed
        if (j == k)
          tile_mma<T>(ar, ai, [&](int r, int c) { return Lij[r * lda + c]; },
                      [&](int kk, int c) { return X[kk * lda + c]; });
        else
          tile_mma<T>(ar, ai, [&](int r, int c) { return Lij[r * lda + c]; },
                      [&](int kk, int c) { return X[c * lda + kk]; });
      }
      // Y (16x16) into tile (k, i) transposed, then X_ik = -Dinv_i Y there
      T *Y = tile(k, i);
#pragma unroll
      for (int e = 0; e < 4; ++e) Y[li * lda + lq + 4 * e] = from_acc<T>(ar, ai, e);
      const T *Di = tile(i, i);
      d4 br = {0, 0, 0, 0}, bi = {0, 0, 0, 0};
      tile_mma<T>(br, bi, [&](int r, int c) { return Di[r * lda + c]; },
                  [&](int kk, int c) { return Y[c * lda + kk]; });
#pragma unroll
      for (int e = 0; e < 4; ++e)
        Y[li * lda + lq + 4 * e] = St<T>::scale(-1.0, from_acc<T>(br, bi, e));
    }
    __syncthreads();
  }
  T *Linv = as<T>(w.Linv);
  for (int idx = tid; idx < n * n; idx += CH_T) {
    const int r = idx / n, c = idx - (idx / n) * n;
    T v = T{};
    if (c <= r) {
      const int bi = r >> 4, bj = c >> 4;
      v = bi == bj ? tile(bi, bi)[(r & 15) * lda + (c & 15)]
                   : tile(bj, bi)[(c & 15) * lda + (r & 15)];
    }
    Linv[idx] = v;
  }
  if (tid == 0) *info = 0;
}

template <typename T>
__global__ __launch_bounds__(CH_T) void k_eig_chol(const T *__restrict__ S, int n, EigWs w,
                                                    int32_t *info) {
  d_eig_chol<T>(S, n, w, info);
}

// LDS bytes of k_eig_chol for an n x n block
template <typename T>
size_t chol_lds_bytes(int n) {
  const size_t N = 16 * ((n + 15) / 16);
  return N * (N + 1) * sizeof(T) + 16;
}

__global__ void k_set_info(int32_t *info) { *info = 0; }

// Y = (X + X^H)/2 for n x n row-major matrices (Y may equal X)
template <typename T>
__global__ __launch_bounds__(256) void k_hermitize(const T *X, T *Y, int n, const int32_t *info) {
  if (*info != 0) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(idx / n), c = static_cast<int>(idx - static_cast<int64_t>(r) * n);
  if (c < r) return;
  const T a = X[static_cast<int64_t>(r) * n + c], b = X[static_cast<int64_t>(c) * n + r];
  const T h = St<T>::scale(0.5, a + cj(b));
  Y[static_cast<int64_t>(r) * n + c] = h;
  Y[static_cast<int64_t>(c) * n + r] = cj(h);
}

// ------------------------------------------------------------------ small GEMM
// C = op(A) op(B) for n x n row-major matrices on FP64 MFMA, one 16x16 tile
// per wavefront. Operand modes:
//   A: 0 = A, 1 = A^H, 2 = (A + A^H)/2
//   B: 0 = B, 1 = B^H, 3 = 1.5 I - 0.5 B
template <int MODE, typename T>
__device__ inline T opval(const T *M, int r, int c, int n) {
  if constexpr (MODE == 0) return M[r * n + c];
  else if constexpr (MODE == 1) return cj(M[c * n + r]);
  else if constexpr (MODE == 2) return St<T>::scale(0.5, M[r * n + c] + cj(M[c * n + r]));
  else return realv<T>(r == c ? 1.5 : 0.0) - St<T>::scale(0.5, M[r * n + c]);
}

template <typename T, int AM, int BM>
__device__ __forceinline__ void d_small_gemm(const T *__restrict__ A,
                                                     const T *__restrict__ B,
                                                     T *__restrict__ C, int n,
                                                     const int32_t *info) {
  if (*info != 0) return;
  constexpr bool CX = St<T>::cplx;
  const int lane = threadIdx.x & 63;
  const int tiles_n = (n + 15) / 16;
  const int tile = blockIdx.x * (SG_T / 64) + (threadIdx.x >> 6);
  if (tile >= tiles_n * tiles_n) return;
  const int i0 = (tile / tiles_n) * 16, j0 = (tile % tiles_n) * 16;
  const int li = lane & 15, lk = lane >> 4;
  d4 accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
  const int r = i0 + li, c = j0 + li;
  // 64 k per round: all loads of a round are issued before its MFMAs
  for (int k0 = 0; k0 < n; k0 += 64) {
    T a[16], b[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + 4 * u + lk;
      a[u] = (r < n && k < n) ? opval<AM>(A, r, k, n) : T{};
      b[u] = (c < n && k < n) ? opval<BM>(B, k, c, n) : T{};
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if constexpr (CX) {
        const z64 au = a[u], bu = b[u];
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(au.x, bu.x, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-au.y, bu.y, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(au.x, bu.y, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(au.y, bu.x, acci, 0, 0, 0);
      } else {
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(re_of(a[u]), re_of(b[u]), accr, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int rr = i0 + lk + 4 * e, cc = j0 + li;
    if (rr < n && cc < n) {
      if constexpr (CX) C[rr * n + cc] = T{accr[e], acci[e]};
      else C[rr * n + cc] = accr[e];
    }
  }
}

template <typename T, int AM, int BM>
__global__ __launch_bounds__(SG_T) void k_small_gemm(const T *__restrict__ A,
                                                     const T *__restrict__ B,
                                                     T *__restrict__ C, int n,
                                                     const int32_t *info) {
  d_small_gemm<T, AM, BM>(A, B, C, n, info);
}

// ------------------------------------------------------------------ tridiagonal
// Householder A = Q T Q^H with H_k = I - tau_k v_k v_k^H chosen so that T is
// real symmetric (the sub-diagonal beta_k is real).
//
// Four wavefronts hold the whole (Hermitian, zero-padded) matrix in
// registers: lane (ty, tx) (32 x 8) owns rows ty + 32i and columns tx + 8j,
// RR x RC elements (4 x 16 real, 3 x 12 complex), so neither p = tau A v nor
// the rank-2 update A -= v w^H + w v^H touches LDS, and a row's partial
// products are summed over 8 lanes on DPP. A fifth wavefront builds the
// reflectors. Each step k:
//   A  (matrix waves) p over the live rows to LDS (zero at rows <= k); the
//      owners of row k+1 copy it, conjugated, to LDS as column k+1;
//   B  every wavefront forms K = -tau/2 p^H v (w = p + K v); the reflector
//      wave updates column k+1 (rows > k, two per lane, in registers) and
//      builds reflector k+1 from it while the matrix waves apply the rank-2
//      update to their rows > k;
// two barriers per step. Row blocks that are finished (all rows <= k) skip
// their arithmetic on wavefront-uniform branches.
constexpr int TRI_T = 320;

// 8-lane DPP sum (lanes 8q..8q+7; every lane of the group gets it)
__device__ inline z64 group8_sum_z(z64 v) { return z64{group8_sum(v.x), group8_sum(v.y)}; }
__device__ inline double sum8(double v) { return group8_sum(v); }
__device__ inline z64 sum8(z64 v) { return group8_sum_z(v); }
__device__ inline z64 lane_read(z64 v, int lane) { return z64{lane_read(v.x, lane), lane_read(v.y, lane)}; }

// a - x y and a + x y as fused multiply-adds
__device__ inline double fms(double a, double x, double y) { return fma(-x, y, a); }
__device__ inline z64 fms(z64 a, z64 x, z64 y) {
  return z64{fma(x.y, y.y, fma(-x.x, y.x, a.x)), fma(-x.y, y.x, fma(-x.x, y.y, a.y))};
}
__device__ inline double fmad(double a, double x, double y) { return fma(x, y, a); }
__device__ inline z64 fmad(z64 a, z64 x, z64 y) {
  return z64{fma(-x.y, y.y, fma(x.x, y.x, a.x)), fma(x.y, y.x, fma(x.x, y.y, a.y))};
}

// LDS shared by the two roles
template <typename T> struct TriLds {
  static constexpr int NM = EigMax<T>::n;
  T vb[2][NM];  // reflectors k and k+1 (zero at rows <= k and >= n)
  T pb[NM];     // p = tau A v (zero at rows <= k)
  T col[NM];    // column k+1
  T taus[NM];
  double dd[NM], ee[NM];
};

// Reflector k from x = column k at rows r0 = k + lane and r1 = r0 + 64 (one
// wavefront; row k is the diagonal): H = I - tau v v^H with v_k+1 = 1 maps
// x[k+1..] to (beta, 0, ..., 0), beta real. Writes v to vout and to row k of
// V (zeros at rows <= k and >= n), tau and beta to the tables.
template <typename T>
__device__ inline void tri_reflector(int n, int k, T x0, T x1, T *vout, TriLds<T> &L, T *Vg) {
  constexpr int NM = EigMax<T>::n;
  const int lane = threadIdx.x & 63;
  const int r0 = k + lane, r1 = r0 + 64;
  const double s2 = (lane >= 2 && r0 < n ? abs2(x0) : 0.0) + (r1 < n ? abs2(x1) : 0.0);
  const double xn2 = wave_sum(s2);
  const T alpha = lane_read(x0, 1);
  const double ar = re_of(alpha);
  double beta;
  T tn, scl;
  if (xn2 == 0.0 && abs2(alpha) == ar * ar) {
    beta = ar;
    tn = T{};
    scl = T{};
  } else {
    // beta = -sign(ar) sqrt(s2) and -1/beta from one reciprocal square root
    // (hardware estimate and two Newton steps); tau = (beta - alpha)/beta,
    // scl = 1/(alpha - beta)
    const double s2 = abs2(alpha) + xn2;
    double rs = __builtin_amdgcn_rsq(s2);
    rs = fma(0.5 * rs, fma(-s2 * rs, rs, 1.0), rs);
    rs = fma(0.5 * rs, fma(-s2 * rs, rs, 1.0), rs);
    beta = -copysign(s2 * rs, ar);
    const T amb = alpha - realv<T>(beta);
    tn = St<T>::scale(copysign(rs, ar), amb);
    scl = cj(amb) * rcp_nr(abs2(amb));
  }
  const T y0 = lane == 1 ? realv<T>(1.0) : (lane >= 2 && r0 < n ? x0 * scl : T{});
  const T y1 = r1 < n ? x1 * scl : T{};
  if (r0 < NM) vout[r0] = y0;
  if (r1 < NM) vout[r1] = y1;
  T *Vk = Vg + static_cast<int64_t>(k) * n;
  if (r0 < n) Vk[r0] = y0;
  if (r1 < n) Vk[r1] = y1;
  for (int r = lane; r < k; r += 64) Vk[r] = T{};
  if (lane == 0) {
    if (k > 0) vout[k - 1] = T{};  // left over from reflector k - 2
    L.taus[k] = tn;
    L.ee[k] = beta;
  }
}

template <typename T>
__device__ __forceinline__ void d_eig_tridiag(int n, EigWs w, const int32_t *info) {
  if (*info != 0) return;
  constexpr int NM = EigMax<T>::n, RR = NM / 32, RC = NM / 8;
  __shared__ TriLds<T> L;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  T *Vg = as<T>(w.V);
  // the two roles run separate loops with the same barriers
  if (wave < 4) {
    const int ty = tid >> 3, tx = tid & 7;
    const T *Ag = as<T>(w.A);
    // (A + A^H)/2, zero outside n x n
    T a[RR][RC];
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int r = ty + 32 * i, c = tx + 8 * j;
        const bool in = r < n && c < n;
        a[i][j] = in ? St<T>::scale(0.5, Ag[r * n + c] + cj(Ag[c * n + r])) : T{};
      }
    if (ty == 0)
#pragma unroll
      for (int j = 0; j < RC; ++j) L.col[tx + 8 * j] = cj(a[0][j]);
    __syncthreads();  // column 0 ready
    __syncthreads();  // reflector 0 ready
    for (int k = 0; k + 1 < n; ++k) {
      const T *v = L.vb[k & 1];
      const T tau = L.taus[k];
      const int c1 = k + 1;
      T vr[RR], vc[RC];
#pragma unroll
      for (int i = 0; i < RR; ++i) vr[i] = v[ty + 32 * i];
#pragma unroll
      for (int j = 0; j < RC; ++j) vc[j] = v[tx + 8 * j];
      // row c1 as it stands (conjugated: column c1) to LDS by its owners;
      // one uniform branch per candidate block, constant register indices
      if (ty == (c1 & 31)) {
        const int ib = c1 >> 5;
#pragma unroll
        for (int i = 0; i < RR; ++i)
          if (i == ib)
#pragma unroll
            for (int j = 0; j < RC; ++j) L.col[tx + 8 * j] = cj(a[i][j]);
      }
      // p = tau A v over the live row blocks (two accumulators per row)
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        if (32 * i + 31 <= k) continue;
        T s0 = T{}, s1 = T{};
#pragma unroll
        for (int j = 0; j < RC; j += 2) {
          s0 = fmad(s0, a[i][j], vc[j]);
          s1 = fmad(s1, a[i][j + 1], vc[j + 1]);
        }
        const T sum = sum8(s0 + s1);
        const int r = ty + 32 * i;
        if (tx == 0) L.pb[r] = r > k ? tau * sum : T{};
      }
      __syncthreads();  // p and column c1 ready
      // K = -tau/2 p^H v over all rows (p and v vanish at rows <= k)
      T pv = cj(L.pb[lane]) * v[lane];
      if (lane + 64 < NM) pv = pv + cj(L.pb[lane + 64]) * v[lane + 64];
      pv = wave_sum(pv);
      const T K = St<T>::scale(-0.5, tau * pv);
      // A -= v w^H + w v^H on the live row blocks (w vanishes at rows <= k)
      T wr[RR], wc[RC];
#pragma unroll
      for (int i = 0; i < RR; ++i) wr[i] = L.pb[ty + 32 * i] + K * vr[i];
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        wc[j] = cj(L.pb[tx + 8 * j] + K * vc[j]);
        vc[j] = cj(vc[j]);
      }
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        if (32 * i + 31 <= k) continue;
#pragma unroll
        for (int j = 0; j < RC; ++j) a[i][j] = fms(fms(a[i][j], vr[i], wc[j]), wr[i], vc[j]);
      }
      __syncthreads();  // reflector c1 ready, update done
    }
  } else {
    for (int idx = lane; idx < 2 * NM; idx += 64) L.vb[idx / NM][idx % NM] = T{};
    __syncthreads();  // column 0 ready
    if (n >= 2)
      tri_reflector<T>(n, 0, L.col[lane], lane + 64 < NM ? L.col[lane + 64] : T{}, L.vb[0], L, Vg);
    if (lane == 0) L.dd[0] = re_of(L.col[0]);
    __syncthreads();  // reflector 0 ready
    for (int k = 0; k + 1 < n; ++k) {
      const T *v = L.vb[k & 1];
      const T tau = L.taus[k];
      const int c1 = k + 1;
      __syncthreads();  // p and column c1 ready
      // column c1 on rows r0 = c1 + lane, r1 = r0 + 64 (v_c1 = 1: reflector
      // k starts with a unit entry): x = col - v conj(w_c1) - w, w = p + K v
      const int r0 = c1 + lane, r1 = r0 + 64;
      const T p0 = r0 < NM ? L.pb[r0] : T{}, p1 = r1 < NM ? L.pb[r1] : T{};
      const T v0 = r0 < NM ? v[r0] : T{}, v1 = r1 < NM ? v[r1] : T{};
      const T c0 = r0 < NM ? L.col[r0] : T{}, cc1 = r1 < NM ? L.col[r1] : T{};
      const T pc1 = L.pb[c1];
      const T pv = wave_sum(cj(p0) * v0 + cj(p1) * v1);
      const T K = St<T>::scale(-0.5, tau * pv);
      const T w1c = cj(pc1 + K);
      const T x0 = c0 - v0 * w1c - (p0 + K * v0);
      const T x1 = cc1 - v1 * w1c - (p1 + K * v1);
      if (lane == 0) L.dd[c1] = re_of(x0);
      if (c1 + 1 < n) tri_reflector<T>(n, c1, x0, x1, L.vb[(k + 1) & 1], L, Vg);
      __syncthreads();  // reflector c1 ready, update done
    }
  }
  T *tg = as<T>(w.tau);
  for (int i = tid; i < n; i += TRI_T) {
    w.d[i] = L.dd[i];
    w.e[i] = (i + 1 < n) ? L.ee[i] : 0.0;
    tg[i] = (i + 1 < n) ? L.taus[i] : T{};
    Vg[static_cast<int64_t>(n - 1) * n + i] = T{};  // no reflector n-1
  }
}

template <typename T>
__global__ __launch_bounds__(TRI_T) void k_eig_tridiag(int n, EigWs w, const int32_t *info) {
  d_eig_tridiag<T>(n, w, info);
}

// ------------------------------------------------------------------ values
// The workgroup stages T once: split points as ballot bit masks, and
// (d_i s, e_i-1^2 s^2) pairs for the Sturm recurrence, with s a power of two
// (exact) that brings the Gershgorin bound of the whole matrix below 1.
inline size_t values_lds_bytes(int n) { return (5 * static_cast<size_t>(n) + 1) * sizeof(double); }

__device__ __forceinline__ void d_eig_values(int n, const double *__restrict__ dg,
                                                    const double *__restrict__ eg,
                                                    double *__restrict__ lam_out,
                                                    const int32_t *__restrict__ info) {
  if (*info != 0) return;
  extern __shared__ double sdv[];
  double2 *de = reinterpret_cast<double2 *>(sdv);  // [n] (d_i s, e_i-1^2 s^2)
  double *d = sdv + 2 * n, *e = d + n, *e2 = e + n;
  __shared__ unsigned long long spm[EIG_LARGE_MAX / 64];  // split bits: bit i of word i / 64
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < n; i += 256) {
    d[i] = dg[i];
    e[i] = (i + 1 < n) ? eg[i] : 0.0;
    e2[i] = e[i] * e[i];
  }
  __syncthreads();
  {
    double g = 0.0;
    for (int i0 = 0; i0 < n; i0 += 256) {
      const int i = i0 + threadIdx.x;
      const bool sp = i + 1 < n && split_at(d, e, i);
      const unsigned long long bits = __ballot(sp);
      if (i < n) g = fmax(g, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + fabs(e[i]));
      if (lane == 0 && i0 + 64 * wv < n) spm[(i0 >> 6) + wv] = bits;
    }
    g = wave_max(g);
    if (lane == 0) red[wv] = g;
  }
  __syncthreads();
  int ex = 0;
  (void)frexp(fmax(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])), DBL_MIN), &ex);
  const double s = ldexp(1.0, -ex), s2 = s * s;
  for (int i = threadIdx.x; i < n; i += 256)
    de[i] = make_double2(d[i] * s, i > 0 ? e2[i - 1] * s2 : 0.0);
  __syncthreads();
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
  if (j >= n) return;
  // the unreduced block [lo, hi] of eigenvalue j from the split bits
  int lo = 0, hi = n - 1;
  for (int q = (j - 1) >> 6; j > 0 && q >= 0; --q) {
    unsigned long long bits = spm[q];
    const int top = (j - 1) & 63;
    if (q == (j - 1) >> 6 && top < 63) bits &= (2ull << top) - 1ull;
    if (bits) {
      lo = 64 * q + 63 - __builtin_clzll(bits) + 1;
      break;
    }
  }
  for (int q = j >> 6; 64 * q < n; ++q) {
    unsigned long long bits = spm[q];
    if (q == j >> 6) bits &= ~((1ull << (j & 63)) - 1ull);
    if (bits) {
      hi = 64 * q + __builtin_ctzll(bits);
      break;
    }
  }
  const int li = j - lo;
  double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
  for (int i = lo + lane; i <= hi; i += 64) {
    const double off = (i > lo ? fabs(e[i - 1]) : 0.0) + (i < hi ? fabs(e[i]) : 0.0);
    gl = fmin(gl, d[i] - off);
    gu = fmax(gu, d[i] + off);
    if (i < hi) emax2 = fmax(emax2, e2[i]);
  }
  gl = wave_min(gl);
  gu = wave_max(gu);
  emax2 = wave_max(emax2);
  // on the scaled T (|T| < 1) the leading minors grow by at most a factor 3
  // per step, so rescaling them is needed only every 8 steps
  const double tn = fmax(fabs(gl), fabs(gu)) * s;
  const double pivmin = DBL_MIN * fmax(1.0, emax2 * s2);
  double a = gl * s - (2.0 * DBL_EPSILON * tn + 2.0 * pivmin);
  double b = gu * s + (2.0 * DBL_EPSILON * tn + 2.0 * pivmin);
  const double d0 = de[lo].x;
  for (int it = 0; it < 64; ++it) {
    const double width = b - a;
    if (width <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + pivmin) break;
    // 65-way multisection: the number of eigenvalues below x = sign changes
    // along the leading minors P_i = (d_i - x) P_i-1 - e_i-1^2 P_i-2; an
    // exact zero takes the sign opposite to its predecessor
    const double x = a + width * ((lane + 1) / 65.0);
    double pm = 1.0, pc = d0 - x;
    bool neg = pc <= 0.0;
    int cnt = neg;
    auto sturm_step = [&](double2 q) {
      const double pn = fma(q.x - x, pc, -q.y * pm);
      const bool nn = (pn < 0.0) | ((pn == 0.0) & !neg);
      cnt += static_cast<int>(nn != neg);
      neg = nn;
      pm = pc;
      pc = pn;
    };
    int i = lo + 1;
    for (; i + 8 <= hi + 1; i += 8) {
      double2 qb[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) qb[q] = de[i + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) sturm_step(qb[q]);
      const double mag = fmax(fabs(pc), fabs(pm));
      const double sc = mag > 0x1p+400 ? 0x1p-400 : (mag < 0x1p-400 ? 0x1p+400 : 1.0);
      pm *= sc;
      pc *= sc;
    }
    for (; i <= hi; ++i) sturm_step(de[i]);
    // eigenvalue li lies at or above x exactly when at most li lie below x
    a = fmax(a, wave_max(cnt <= li ? x : -DBL_MAX));
    b = fmin(b, wave_min(cnt <= li ? DBL_MAX : x));
  }
  a /= s;
  b /= s;
  if (lane == 0) lam_out[j] = 0.5 * (a + b);
}

__global__ __launch_bounds__(256) void k_eig_values(int n, const double *__restrict__ dg,
                                                    const double *__restrict__ eg,
                                                    double *__restrict__ lam_out,
                                                    const int32_t *__restrict__ info) {
  d_eig_values(n, dg, eg, lam_out, info);
}

// ------------------------------------------------------------------ vectors
// Start vectors of inverse iteration: windows of one table of pseudo-random
// values in [-1, 1) (MurmurHash3's 32-bit finaliser of the index), window j
// starting at 61 j, so every eigenvector starts from a different vector.
constexpr int RV_N = 256;
__device__ inline double rv_value(unsigned q) {
  unsigned h = q * 0x9E3779B1u + 0x7F4A7C15u;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return static_cast<double>(h >> 8) * (1.0 / 8388608.0) - 1.0;
}


// LDS doubles of k_eig_vectors: d, e, lam, row sums, split words, the start
// table, then six per-lane arrays of n (interleaved by lane)
inline size_t vec_lds_doubles(int n) {
  return 4 * static_cast<size_t>(n) + 8 + RV_N + 6 * static_cast<size_t>(n) * VEC_T;
}

__device__ __forceinline__ void d_eig_vectors(int n, EigWs w, const int32_t *info) {
  if (*info != 0) return;
  extern __shared__ double sv[];
  double *d = sv, *e = sv + n, *lam = sv + 2 * n, *rs = sv + 3 * n;
  unsigned *spw = reinterpret_cast<unsigned *>(sv + 4 * n);  // split bits, 32 per word
  double *rv = sv + 4 * n + 8;
  double *scratch = rv + RV_N;
  const int t = threadIdx.x;
  // d, e, lam in rounds of eight loads per array and lane, all issued first
  for (int base = 0; base < n; base += 8 * VEC_T) {
    double a[8], b[8], c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * VEC_T + t;
      a[u] = idx < n ? w.d[idx] : 0.0;
      b[u] = idx < n ? w.e[idx] : 0.0;
      c[u] = idx < n ? w.lam[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * VEC_T + t;
      if (idx < n) {
        d[idx] = a[u];
        e[idx] = b[u];
        lam[idx] = c[u];
      }
    }
  }
  for (int q = t; q < RV_N; q += VEC_T) rv[q] = rv_value(static_cast<unsigned>(q));
  __syncthreads();
  // split points (the block boundary between i and i + 1) as bit words, and
  // the row sums |d_i| + |e_i-1| + |e_i| within the blocks
  const int nw = (n + 31) / 32;
  for (int q = t; q < nw; q += VEC_T) {
    unsigned bits = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      const int i = 32 * q + b;
      if (i + 1 < n && split_at(d, e, i)) bits |= 1u << b;
    }
    spw[q] = bits;
  }
  __syncthreads();
  auto split = [&](int i) { return (spw[i >> 5] >> (i & 31)) & 1u; };
  for (int i = t; i < n; i += VEC_T)
    rs[i] = fabs(d[i]) + (i > 0 && !split(i - 1) ? fabs(e[i - 1]) : 0.0) +
            (i + 1 < n && !split(i) ? fabs(e[i]) : 0.0);
  __syncthreads();
  const int j = blockIdx.x * VEC_T + t;
  if (j >= n) return;
  // the unreduced block [lo, hi] holding eigenvalue j: lo follows the last
  // split below j, hi is the first split at or above j
  int lo = 0, hi = n - 1;
  for (int q = (j - 1) >> 5; j > 0 && q >= 0; --q) {
    unsigned bits = spw[q];
    if (q == (j - 1) >> 5) bits &= (((j - 1) & 31) == 31) ? ~0u : ((2u << ((j - 1) & 31)) - 1u);
    if (bits) {
      lo = 32 * q + 31 - __builtin_clz(bits) + 1;
      break;
    }
  }
  for (int q = j >> 5; q < nw; ++q) {
    unsigned bits = spw[q];
    if (q == j >> 5) bits &= ~((1u << (j & 31)) - 1u);
    if (bits) {
      hi = 32 * q + __builtin_ctz(bits);
      break;
    }
  }
  const int m = hi - lo + 1;
  double tn = 0.0;
#pragma unroll 8
  for (int i = lo; i <= hi; ++i) tn = fmax(tn, rs[i]);
  const double pert = 10.0 * DBL_EPSILON * fmax(tn, DBL_MIN);
  int ties = 0;
  for (int i = j; i > lo && lam[i] - lam[i - 1] < pert; --i) ++ties;
  const double x = lam[j - ties] + ties * pert;
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);
  auto recip_pivot = [&](double p) {
    return rcp_nr(fabs(p) < tiny ? (p < 0.0 ? -tiny : tiny) : p);
  };
  const int r0 = (61 * j) & (RV_N - 1);  // start window

  double *u0 = scratch + 0 * n * VEC_T + t;  // reciprocal pivots
  double *u1 = scratch + 1 * n * VEC_T + t;
  double *u2 = scratch + 2 * n * VEC_T + t;
  double *y = scratch + 3 * n * VEC_T + t;
  int *sw_ = reinterpret_cast<int *>(scratch + 4 * n * VEC_T) + t;  // rows swapped
  double *ms = scratch + 5 * n * VEC_T + t;                        // row multipliers
#define AT(p, i) (p)[(i) * VEC_T]
  // LU with partial pivoting of (T_block - x I) once, forward-eliminating the
  // start vector; branch-free, since the lanes of a workgroup pivot
  // differently. Every recurrence keeps its running values in registers and
  // requests the next step's operands one step ahead, so no LDS round trip
  // sits on the chain.
  {
    double c0 = d[lo] - x, c1 = (m > 1) ? e[lo] : 0.0;
    double n0 = c1;
    double dcur = (m > 1) ? d[lo + 1] : 0.0, ecur = (m > 2) ? e[lo + 1] : 0.0;
    double ycur = rv[r0];
    double yn = rv[(r0 + 1) & (RV_N - 1)];
#pragma unroll 4
    for (int i = 0; i + 1 < m; ++i) {
      const double dnx = (i + 2 < m) ? d[lo + i + 2] : 0.0;
      const double enx = (i + 3 < m) ? e[lo + i + 2] : 0.0;
      const double ynx = rv[(r0 + i + 2) & (RV_N - 1)];
      const double n1 = dcur - x, n2 = ecur;
      const bool sw = fabs(n0) > fabs(c0);
      const double num = sw ? c0 : n0, den = sw ? n0 : c0;
      const double l = den != 0.0 ? num * rcp_nr(den) : 0.0;
      AT(u0, i) = recip_pivot(sw ? n0 : c0);
      AT(u1, i) = sw ? n1 : c1;
      AT(u2, i) = sw ? n2 : 0.0;
      AT(y, i) = sw ? yn : ycur;
      ycur = sw ? ycur - l * yn : yn - l * ycur;
      AT(sw_, i) = sw;
      AT(ms, i) = l;
      const double c0n = sw ? c1 - l * n1 : n1 - l * c1;
      c1 = sw ? -l * n2 : n2;
      c0 = c0n;
      n0 = ecur;
      dcur = dnx;
      ecur = enx;
      yn = ynx;
    }
    AT(y, m - 1) = ycur;
    AT(u0, m - 1) = recip_pivot(c0);
    AT(u1, m - 1) = 0.0;
    AT(u2, m - 1) = 0.0;
  }
  // back substitution with the reciprocal pivots, operands one step ahead;
  // returns the largest |y_i| and the squared norm, and the entry of largest
  // magnitude (lowest index among equals) in ybig
  auto back_solve = [&](double &nrm, double &ybig) {
    double y1 = 0.0, y2 = 0.0, ymax = 0.0, s2 = 0.0, yb = 0.0;
    double a0 = AT(u0, m - 1), a1 = AT(u1, m - 1), a2 = AT(u2, m - 1), ay = AT(y, m - 1);
#pragma unroll 4
    for (int i = m - 1; i >= 0; --i) {
      const int ip = i > 0 ? i - 1 : 0;
      const double b0 = AT(u0, ip), b1 = AT(u1, ip), b2 = AT(u2, ip), by = AT(y, ip);
      const double yi = (ay - a1 * y1 - a2 * y2) * a0;
      AT(y, i) = yi;
      y2 = y1;
      y1 = yi;
      if (fabs(yi) >= ymax) {
        ymax = fabs(yi);
        yb = yi;
      }
      s2 += yi * yi;
      a0 = b0;
      a1 = b1;
      a2 = b2;
      ay = by;
    }
    nrm = s2;
    ybig = yb;
    return ymax;
  };
  double nrm = 0.0, ybig = 0.0;
  const double sc = 1.0 / fmax(back_solve(nrm, ybig), DBL_MIN);
  // replay the forward elimination on the scaled first solution
  {
    double ycur = AT(y, 0) * sc;
    double yn = (m > 1) ? AT(y, 1) : 0.0, l = AT(ms, 0);
    int sw = AT(sw_, 0);
#pragma unroll 4
    for (int i = 0; i + 1 < m; ++i) {
      const int in = i + 2 < m ? i + 1 : i;
      const double ynn = AT(y, in + 1 < m ? in + 1 : in), lnx = AT(ms, in);
      const int swn = AT(sw_, in);
      const double ys = yn * sc;
      AT(y, i) = sw ? ys : ycur;
      ycur = sw ? ycur - l * ys : ys - l * ycur;
      yn = ynn;
      l = lnx;
      sw = swn;
    }
    AT(y, m - 1) = ycur;
  }
  back_solve(nrm, ybig);
  // unit 2-norm, largest component positive
  const double scl = copysign(1.0 / sqrt(nrm), ybig);
#pragma unroll 8
  for (int i = 0; i < n; ++i)
    w.Z[static_cast<int64_t>(i) * n + j] = (i >= lo && i <= hi) ? AT(y, i - lo) * scl : 0.0;
#undef AT
}

__global__ __launch_bounds__(VEC_T) void k_eig_vectors(int n, EigWs w, const int32_t *info) {
  d_eig_vectors(n, w, info);
}

// ------------------------------------------------------------------ orthogonality
// dev[slot] = max |G - I| (one workgroup); info = -1 when above the limit
// skip (optional): set to 1 when max |G - I| <= skip_limit (the vectors are
// already orthonormal to rounding, so the kernels that take skip as their
// status word do nothing) or when the status is not 0;
// gate (optional): the check does nothing while *gate is nonzero.
__device__ __forceinline__ void d_gram_check(const double *__restrict__ G, int n,
                                                     double limit, int32_t *info, int32_t *skip,
                                                     double skip_limit, const int32_t *gate) {
  if (*info != 0 || (gate && *gate != 0)) {
    if (skip && threadIdx.x == 0) *skip = 1;
    return;
  }
  __shared__ double red[16];
  double dev = 0.0;
  const int nn = n * n;
  for (int base = 0; base < nn; base += 1024 * 8) {
    double g[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = base + q * 1024 + threadIdx.x;
      g[q] = idx < nn ? G[idx] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = base + q * 1024 + threadIdx.x;
      if (idx < nn) {
        const int r = idx / n, c = idx - r * n;
        dev = fmax(dev, fabs(g[q] - (r == c ? 1.0 : 0.0)));
      }
    }
  }
  dev = wave_max(dev);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) {
    double all = 0.0;
    for (int q = 0; q < 16; ++q) all = fmax(all, red[q]);
    if (!(all <= limit)) *info = -1;
    if (skip) *skip = (all <= skip_limit || !(all <= limit)) ? 1 : 0;
  }
}

__global__ __launch_bounds__(1024) void k_gram_check(const double *__restrict__ G, int n,
                                                     double limit, int32_t *info, int32_t *skip,
                                                     double skip_limit, const int32_t *gate) {
  d_gram_check(G, n, limit, info, skip, skip_limit, gate);
}

// ------------------------------------------------------------------ clusters
// Inverse iteration separates the eigenvectors of one unreduced block of T
// only as far as the eigenvalue gaps allow: vectors whose eigenvalues lie
// within a few rounding units of ||T|| of each other (degenerate shells of a
// symmetric system, the close pairs of a Wilkinson matrix) come out nearly
// parallel. Slots of one block whose consecutive eigenvalue gaps are at most
// CL_TOL ||T|| form a cluster, and each cluster is orthonormalised by modified
// Gram-Schmidt in slot order, applied twice. Outside the clusters the vectors
// overlap by at most ~1e-8, which the refinement that follows removes.
// One workgroup; each wavefront takes whole clusters (lane r owns rows
// r + 64q of every column it touches, so its own stores are what it reads
// back).
constexpr double CL_TOL = 1e-7;
constexpr int CL_T = 256;
constexpr int CL_RPL = EIG_LARGE_MAX / 64;  // rows per lane
__device__ __forceinline__ void d_cluster_orth(int n, const double *__restrict__ d,
                                                       const double *__restrict__ e,
                                                       const double *__restrict__ lam,
                                                       double *__restrict__ Z,
                                                       int32_t *__restrict__ cid,
                                                       double *__restrict__ cltol,
                                                       const int32_t *__restrict__ info) {
  if (*info != 0) return;
  __shared__ unsigned char brk[EIG_LARGE_MAX];  // 1: slot j opens a new cluster
  __shared__ int list[EIG_LARGE_MAX / 2];       // clusters of >= 2 slots: first | last << 16
  __shared__ int nlist;
  __shared__ double red[CL_T / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double g = 0.0;
  for (int i = t; i < n; i += CL_T)
    g = fmax(g, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0));
  g = wave_max(g);
  if (lane == 0) red[wv] = g;
  if (t == 0) nlist = 0;
  __syncthreads();
  double tn = red[0];
#pragma unroll
  for (int q = 1; q < CL_T / 64; ++q) tn = fmax(tn, red[q]);
  const double tol = CL_TOL * tn;
  for (int j = t; j < n; j += CL_T)
    brk[j] = (j == 0 || split_at(d, e, j - 1) || !(lam[j] - lam[j - 1] <= tol)) ? 1 : 0;
  __syncthreads();
  // cluster id of every slot (its cluster's first slot) for the refinement
  for (int j = t; j < n; j += CL_T) {
    int b = j;
    while (brk[b] == 0) --b;
    cid[j] = b;
  }
  if (t == 0) *cltol = tol;
  for (int j = t; j < n; j += CL_T) {
    if (brk[j] == 0 && (j + 1 == n || brk[j + 1] == 1)) {
      int b = j;
      while (brk[b] == 0) --b;  // brk[0] == 1 ends the walk
      list[atomicAdd(&nlist, 1)] = b | (j << 16);
    }
  }
  __syncthreads();
  const int ncl = nlist;
  for (int c = wv; c < ncl; c += CL_T / 64) {  // wavefront-uniform
    const int b = list[c] & 0xFFFF, last = list[c] >> 16;
    for (int j = b; j <= last; ++j) {
      double zj[CL_RPL];
#pragma unroll
      for (int q = 0; q < CL_RPL; ++q) {
        const int r = lane + 64 * q;
        zj[q] = r < n ? Z[static_cast<int64_t>(r) * n + j] : 0.0;
      }
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = b; i < j; ++i) {
          double zi[CL_RPL], s = 0.0;
#pragma unroll
          for (int q = 0; q < CL_RPL; ++q) {
            const int r = lane + 64 * q;
            zi[q] = r < n ? Z[static_cast<int64_t>(r) * n + i] : 0.0;
            s = fma(zi[q], zj[q], s);
          }
          s = wave_sum(s);
#pragma unroll
          for (int q = 0; q < CL_RPL; ++q) zj[q] = fma(-s, zi[q], zj[q]);
        }
      }
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < CL_RPL; ++q) s = fma(zj[q], zj[q], s);
      s = wave_sum(s);
      // a vector lost to cancellation stays as it is; the Gram checks of the
      // refinement then report the failure
      const double sc = s > 1e-200 ? 1.0 / sqrt(s) : 1.0;
#pragma unroll
      for (int q = 0; q < CL_RPL; ++q) {
        const int r = lane + 64 * q;
        if (r < n) Z[static_cast<int64_t>(r) * n + j] = zj[q] * sc;
      }
    }
  }
}

__global__ __launch_bounds__(CL_T) void k_cluster_orth(int n, const double *__restrict__ d,
                                                       const double *__restrict__ e,
                                                       const double *__restrict__ lam,
                                                       double *__restrict__ Z,
                                                       int32_t *__restrict__ cid,
                                                       double *__restrict__ cltol,
                                                       const int32_t *__restrict__ info) {
  d_cluster_orth(n, d, e, lam, Z, cid, cltol, info);
}

// ------------------------------------------------------------------ refinement
// Eigenvector refinement of Ogita and Aishima (2018), one step, on the
// tridiagonal problem T z_j = lam_j z_j. With G = Z^T Z, M = Z^T (T Z) and
// R = I - G, every column becomes z_j + sum_i z_i E_ij with
//   E_ij = (M_ij + lam_j R_ij) / (lam_j - lam_i) for eigenvalues further
//          apart than RF_GAP ||T|| (and not in one Gram-Schmidt cluster);
//   E_ij = R_ij / 2 otherwise, and E_jj = R_jj / 2.
// A vector z_i = v_i + c v_j (v exact) gets E_ji = -c: the part along a
// distant eigenvector, which a symmetric orthogonalisation would only halve
// (leaving (lam_i - lam_j) c / 2 in Z^T T Z), is removed. M and R are formed
// in FP64, so M_ij + lam_j R_ij carries rounding of order eps |lam|; divided
// by a small gap it would inject errors larger than the ones corrected,
// hence the full correction only across gaps above RF_GAP ||T|| (rounding
// below ~1e-14 there). Across smaller gaps the leftover antisymmetric part
// contributes only gap x c to Z^T T Z, and the step is the symmetric
// (Newton-Schulz) orthogonalisation Z (3I - G) / 2.

// Y = T Z (T tridiagonal: diagonal d, off-diagonal e)
__device__ __forceinline__ void d_tri_apply(int n, const double *__restrict__ d,
                                                   const double *__restrict__ e,
                                                   const double *__restrict__ Z,
                                                   double *__restrict__ Y,
                                                   const int32_t *__restrict__ gate) {
  if (*gate != 0) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n);
  double y = d[i] * Z[idx];
  if (i > 0) y = fma(e[i - 1], Z[idx - n], y);
  if (i + 1 < n) y = fma(e[i], Z[idx + n], y);
  Y[idx] = y;
}

__global__ __launch_bounds__(256) void k_tri_apply(int n, const double *__restrict__ d,
                                                   const double *__restrict__ e,
                                                   const double *__restrict__ Z,
                                                   double *__restrict__ Y,
                                                   const int32_t *__restrict__ gate) {
  d_tri_apply(n, d, e, Z, Y, gate);
}

constexpr double RF_GAP = 1e-2;

// F = I + E from G and M (above)
__device__ __forceinline__ void d_refine_coef(int n, const double *__restrict__ G,
                                                     const double *__restrict__ M,
                                                     const double *__restrict__ lam,
                                                     const int32_t *__restrict__ cid,
                                                     const double *__restrict__ cltol,
                                                     double *__restrict__ F,
                                                     const int32_t *__restrict__ gate) {
  if (*gate != 0) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx - static_cast<int64_t>(i) * n);
  const double r = (i == j ? 1.0 : 0.0) - G[idx];
  const double gap = lam[j] - lam[i];
  double E = 0.5 * r;
  if (i != j && cid[i] != cid[j] && fabs(gap) > (RF_GAP / CL_TOL) * *cltol)
    E = (M[idx] + lam[j] * r) / gap;
  F[idx] = (i == j ? 1.0 : 0.0) + E;
}

__global__ __launch_bounds__(256) void k_refine_coef(int n, const double *__restrict__ G,
                                                     const double *__restrict__ M,
                                                     const double *__restrict__ lam,
                                                     const int32_t *__restrict__ cid,
                                                     const double *__restrict__ cltol,
                                                     double *__restrict__ F,
                                                     const int32_t *__restrict__ gate) {
  d_refine_coef(n, G, M, lam, cid, cltol, F, gate);
}

// ------------------------------------------------------------------ back-transform
// U = Q Z with Q = H_0 H_1 ... H_n-2, in blocks of KB reflectors in compact
// WY form: H_k0 ... H_k0+KB-1 = I - V_b T_b V_b^H with T_b upper triangular
// (tau_i on the diagonal, T(0:i, i) = -tau_i T(0:i, 0:i) V_b(:, 0:i)^H v_i).
// The workgroup first builds every T_b (8 lanes per block: Gram entries, then
// the triangular recurrence), then each column of Z (8 lanes, rows 8t+s in
// registers) takes the blocks last to first: W = V_b^H z (KB independent
// sums), z -= V_b (T_b W). U lands in column rank(j) of Uo, where rank orders
// the eigenvalues by (value, slot).
// (KB = 8 real, 4 complex: a block's reflector entries stay in registers)
template <typename T> struct BackKB { static constexpr int kb = St<T>::cplx ? 4 : 8; };
__host__ __device__ inline int tpk(int r, int c) { return c * (c + 1) / 2 + r; }

template <typename T>
size_t back_lds_bytes(int n) {
  constexpr int KB = BackKB<T>::kb, TP = KB * (KB + 1) / 2;
  const int nblk = (n - 1 + KB - 1) / KB;
  return (static_cast<size_t>(n) * EigMax<T>::n + n + static_cast<size_t>(nblk) * TP) * sizeof(T) +
         static_cast<size_t>(n) * sizeof(double);
}

template <typename T>
__device__ __forceinline__ void d_eig_back(int n, EigWs w, const double *__restrict__ Z,
                                                  T *__restrict__ Uo, double *__restrict__ eps,
                                                  const int32_t *info) {
  if (*info != 0) return;
  constexpr int NMAX = EigMax<T>::n, R = NMAX / 8, KB = BackKB<T>::kb, BK_TP = KB * (KB + 1) / 2;
  extern __shared__ double sv[];
  // reflector k in row k, rows padded to NMAX with zeros (so a lane's rows
  // past n read zeros with no bounds test)
  T *V = reinterpret_cast<T *>(sv);  // [n][NMAX]
  T *tau = V + n * NMAX;             // [n]
  T *Tm = tau + n;                   // [nblk][BK_TP]
  double *lam = reinterpret_cast<double *>(Tm + ((n - 1 + KB - 1) / KB) * BK_TP);  // [n]
  {
    const T *Vg = as<T>(w.V);
    const int tot = n * NMAX;
    for (int base = 0; base < tot; base += 16 * 128) {
      T u[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int idx = base + q * 128 + threadIdx.x;
        const int k = idx / NMAX, r = idx - k * NMAX;
        u[q] = idx < tot && r < n ? Vg[k * n + r] : T{};
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int idx = base + q * 128 + threadIdx.x;
        if (idx < tot) V[idx] = u[q];
      }
    }
  }
  copy_rounds(tau, as<T>(w.tau), n, threadIdx.x, 128);
  copy_rounds(lam, w.lam, n, threadIdx.x, 128);
  __syncthreads();
  const int nblk = (n - 1 + KB - 1) / KB;
  // T_b of every block: the 8 lanes of a group take one block, with rows
  // 8t+s of its reflectors in registers; the Gram entries G(r, c) = v_r^H v_c
  // (r < c) come from 8-lane sums, then every lane of the group runs the
  // triangular recurrence (unrolled, in registers) and lane 0 stores T_b
  for (int bb = 0; bb < nblk; bb += 128 / 8) {
    const int b = bb + (threadIdx.x >> 3), s = threadIdx.x & 7;
    if (b < nblk) {
      const int k0 = b * KB;
      T vb[KB][R];
#pragma unroll
      for (int i = 0; i < KB; ++i)
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int row = 8 * t + s;
          vb[i][t] = V[min(k0 + i, n - 1) * NMAX + row];
        }
      T G[KB][KB];
#pragma unroll
      for (int c = 1; c < KB; ++c)
#pragma unroll
        for (int r = 0; r < c; ++r) {
          T g = T{};
#pragma unroll
          for (int t = 0; t < R; ++t) g = g + cj(vb[r][t]) * vb[c][t];
          G[r][c] = group8_sum(g);
        }
      T Tb[KB][KB];
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        const T ti = (k0 + i < n - 1) ? tau[k0 + i] : T{};
#pragma unroll
        for (int r = 0; r < i; ++r) {
          T acc = T{};
#pragma unroll
          for (int c = r; c < i; ++c) acc = acc + Tb[r][c] * G[c][i];
          Tb[r][i] = St<T>::scale(-1.0, ti * acc);
        }
        Tb[i][i] = ti;
      }
      if (s == 0)
#pragma unroll
        for (int c = 0; c < KB; ++c)
#pragma unroll
          for (int r = 0; r <= c; ++r) Tm[b * BK_TP + tpk(r, c)] = Tb[r][c];
    }
  }
  __syncthreads();
  const int col = blockIdx.x * 16 + (threadIdx.x >> 3), s = threadIdx.x & 7;
  if (col >= n) return;
  T zr[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = 8 * t + s;
    zr[t] = realv<T>((row < n) ? Z[row * n + col] : 0.0);
  }
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * KB;
    // W = V_b^H z (row n - 1 of V, no reflector, is zero and stands in for
    // the reflectors past n - 2)
    T W[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const T *vk = V + min(k0 + i, n - 1) * NMAX;
      T pq[2] = {T{}, T{}};
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int row = 8 * t + s;
        pq[t & 1] = pq[t & 1] + cj(vk[row]) * zr[t];
      }
      W[i] = group8_sum(pq[0] + pq[1]);
    }
    // Y = T_b W
    const T *tb = Tm + b * BK_TP;
    T Y[KB];
#pragma unroll
    for (int r = 0; r < KB; ++r) {
      T acc = T{};
#pragma unroll
      for (int c = r; c < KB; ++c) acc = acc + tb[tpk(r, c)] * W[c];
      Y[r] = acc;
    }
    // z -= V_b Y
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const T *vk = V + min(k0 + i, n - 1) * NMAX;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int row = 8 * t + s;
        zr[t] = zr[t] - vk[row] * Y[i];
      }
    }
  }
  // rank of eigenvalue col by (value, slot): the 8 lanes count a share each
  const double lj = lam[col];
  int rank = 0;
  for (int i = s; i < n; i += 8) {
    const double li = lam[i];
    rank += (li < lj) || (li == lj && i < col);
  }
  rank += __shfl_xor(rank, 1);
  rank += __shfl_xor(rank, 2);
  rank += __shfl_xor(rank, 4);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int row = 8 * t + s;
    if (row < n) Uo[row * n + rank] = zr[t];
  }
  if (s == 0) eps[rank] = lj;
}

template <typename T>
__global__ __launch_bounds__(128) void k_eig_back(int n, EigWs w, const double *__restrict__ Z,
                                                  T *__restrict__ Uo, double *__restrict__ eps,
                                                  const int32_t *info) {
  d_eig_back<T>(n, w, Z, Uo, eps, info);
}



__device__ __forceinline__ void d_copy_gated(const double *__restrict__ src,
                                                    double *__restrict__ dst, int64_t count,
                                                    const int32_t *__restrict__ gate) {
  if (*gate != 0) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx < count) dst[idx] = src[idx];
}

__global__ __launch_bounds__(256) void k_copy_gated(const double *__restrict__ src,
                                                    double *__restrict__ dst, int64_t count,
                                                    const int32_t *__restrict__ gate) {
  d_copy_gated(src, dst, count, gate);
}

// Refined eigenvectors of T (from w.Z after the cluster step) into w.G.
// Step 1 always runs; its Gram matrix G' decides the second: none when
// max |G' - I| <= 1e-13 (w.skip set on the device, no host wait), and
// status -1 when above 1e-4 (or the first Gram matrix above 0.1), where the
// second-order step could not reach rounding level. Scratch: w.Z2, and w.T1
// (as doubles) for M; w.Z is overwritten.
void refine_vectors(int n, const EigWs &w, int32_t *info, hipStream_t st) {
  const int64_t nn = static_cast<int64_t>(n) * n;
  const unsigned eb = static_cast<unsigned>((nn + 255) / 256);
  const int tiles = ((n + 15) / 16) * ((n + 15) / 16);
  const unsigned sgb = static_cast<unsigned>((tiles + 3) / 4);
  double *M = w.T1;
  // step 1: G = Z^T Z, Y = T Z, M = Z^T Y, F = I + E, Z' = Z F (into G)
  k_small_gemm<double, 1, 0><<<sgb, SG_T, 0, st>>>(w.Z, w.Z, w.G, n, info);
  k_gram_check<<<1, 1024, 0, st>>>(w.G, n, 0.1, info, nullptr, 0.0, nullptr);
  k_tri_apply<<<eb, 256, 0, st>>>(n, w.d, w.e, w.Z, w.Z2, info);
  k_small_gemm<double, 1, 0><<<sgb, SG_T, 0, st>>>(w.Z, w.Z2, M, n, info);
  k_refine_coef<<<eb, 256, 0, st>>>(n, w.G, M, w.lam, w.cid, w.cltol, w.Z2, info);
  k_small_gemm<double, 0, 0><<<sgb, SG_T, 0, st>>>(w.Z, w.Z2, w.G, n, info);
  // step 2 on Z' (G' into w.Z), gated by w.skip
  k_small_gemm<double, 1, 0><<<sgb, SG_T, 0, st>>>(w.G, w.G, w.Z, n, info);
  k_gram_check<<<1, 1024, 0, st>>>(w.Z, n, 1e-4, info, w.skip, 1e-13, nullptr);
  k_tri_apply<<<eb, 256, 0, st>>>(n, w.d, w.e, w.G, w.Z2, w.skip);
  k_small_gemm<double, 1, 0><<<sgb, SG_T, 0, st>>>(w.G, w.Z2, M, n, w.skip);
  k_refine_coef<<<eb, 256, 0, st>>>(n, w.Z, M, w.lam, w.cid, w.cltol, w.Z2, w.skip);
  k_small_gemm<double, 0, 0><<<sgb, SG_T, 0, st>>>(w.G, w.Z2, w.Z, n, w.skip);
  k_copy_gated<<<eb, 256, 0, st>>>(w.Z, w.G, nn, w.skip);
}

// blocks above the LDS limit: global-memory pipeline (eigh_large.hip)
template <typename T>
int eigh_large_t(const gpaw_sys *s, const T *H, const T *S, int n, double *eps, T *C,
                 int32_t *info, hipStream_t st) {
  const int sz = St<T>::cplx ? 2 : 1;
  const EigWs w = eig_layout(s->ws.eig, n, sz, true);
  const int64_t nn = static_cast<int64_t>(n) * n;
  const unsigned eb = static_cast<unsigned>((nn + 255) / 256);
  const int tiles = ((n + 15) / 16) * ((n + 15) / 16);
  const unsigned sg_blocks = static_cast<unsigned>((tiles + 3) / 4);
  T *Sw = as<T>(w.Sw), *Linv = as<T>(w.Linv), *T1 = as<T>(w.T1), *Am = as<T>(w.A);
  T *V = as<T>(w.V), *tau = as<T>(w.tau), *p = as<T>(w.p), *U = as<T>(w.T1);
  k_set_info<<<1, 1, 0, st>>>(info);
  k_hermitize<T><<<eb, 256, 0, st>>>(S, Sw, n, info);
  large_chol_linv<T>(Sw, Linv, n, w.piv, info, st);
  k_small_gemm<T, 2, 1><<<sg_blocks, SG_T, 0, st>>>(H, Linv, T1, n, info);
  k_small_gemm<T, 0, 0><<<sg_blocks, SG_T, 0, st>>>(Linv, T1, Am, n, info);
  k_hermitize<T><<<eb, 256, 0, st>>>(Am, Am, n, info);
  large_tridiag<T>(Am, n, V, tau, w.d, w.e, p, info, st);
  k_eig_values<<<(n + 3) / 4, 256, values_lds_bytes(n), st>>>(n, w.d, w.e, w.lam, info);
  large_vectors(n, w.d, w.e, w.lam, w.lu, w.Z, info, st);
  k_cluster_orth<<<1, CL_T, 0, st>>>(n, w.d, w.e, w.lam, w.Z, w.cid, w.cltol, info);
  refine_vectors(n, w, info, st);
  large_back<T>(n, w.G, V, tau, w.lam, U, eps, info, st);
  k_small_gemm<T, 1, 0><<<sg_blocks, SG_T, 0, st>>>(Linv, U, C, n, info);
  return GPAW_OK;
}

template <typename T>
int eigh_t(const gpaw_sys *s, const void *H, const void *S, int nb, double *eps, void *C,
           int32_t *info, hipStream_t st) {
  constexpr int NMAX = EigMax<T>::n;
  if (nb > EIG_LARGE_MAX)
    return fail(GPAW_ESHAPE, "subspace eigensolver supports nb <= 1024");
  if (nb > NMAX)
    return eigh_large_t<T>(s, static_cast<const T *>(H), static_cast<const T *>(S), nb, eps,
                           static_cast<T *>(C), info, st);
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    const void *fns[] = {reinterpret_cast<const void *>(&k_eig_chol<T>),
                         reinterpret_cast<const void *>(&k_eig_back<T>)};
    for (const void *f : fns)
      if (attr_err == hipSuccess)
        attr_err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  if (attr_err != hipSuccess) return hip_fail(attr_err, "hipFuncSetAttribute(eigensolver)");
  const int n = nb;
  const int sz = St<T>::cplx ? 2 : 1;
  const EigWs w = eig_layout(s->ws.eig, n, sz, false);
  const T *Hd = static_cast<const T *>(H);
  const T *Sd = static_cast<const T *>(S);
  const int tiles = ((n + 15) / 16) * ((n + 15) / 16);
  const unsigned sg_blocks = static_cast<unsigned>((tiles + 3) / 4);
  T *Linv = reinterpret_cast<T *>(w.Linv), *T1 = reinterpret_cast<T *>(w.T1);
  T *Am = reinterpret_cast<T *>(w.A), *U = reinterpret_cast<T *>(w.T1);

  k_eig_chol<T><<<1, CH_T, chol_lds_bytes<T>(n), st>>>(Sd, n, w, info);
  // A = Linv ((H + H^H)/2) Linv^H
  k_small_gemm<T, 2, 1><<<sg_blocks, SG_T, 0, st>>>(Hd, Linv, T1, n, info);
  k_small_gemm<T, 0, 0><<<sg_blocks, SG_T, 0, st>>>(Linv, T1, Am, n, info);
  k_eig_tridiag<T><<<1, TRI_T, 0, st>>>(n, w, info);
  k_eig_values<<<(n + 3) / 4, 256, values_lds_bytes(n), st>>>(n, w.d, w.e, w.lam, info);
  k_eig_vectors<<<(n + VEC_T - 1) / VEC_T, VEC_T, vec_lds_doubles(n) * sizeof(double), st>>>(n, w,
                                                                                        info);
  k_cluster_orth<<<1, CL_T, 0, st>>>(n, w.d, w.e, w.lam, w.Z, w.cid, w.cltol, info);
  refine_vectors(n, w, info, st);
  // U = Q Z in eigen-order, then C = Linv^H U
  k_eig_back<T><<<(n + 15) / 16, 128, back_lds_bytes<T>(n), st>>>(
      n, w, w.G, U, eps, info);
  k_small_gemm<T, 1, 0><<<sg_blocks, SG_T, 0, st>>>(Linv, U, static_cast<T *>(C), n, info);
  return GPAW_OK;
}

// Cout = Linv^H with S = L L^H (the orthonormalising rotation: the block
// psi_out_n = sum_m Cout_mn psi_m has psi_out^H S~ psi_out = I)
template <typename T>
__global__ __launch_bounds__(256) void k_conj_transpose(const T *__restrict__ X, T *__restrict__ Y,
                                                        int n, const int32_t *info) {
  if (*info != 0) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(idx / n), c = static_cast<int>(idx - static_cast<int64_t>(r) * n);
  Y[idx] = cj(X[static_cast<int64_t>(c) * n + r]);
}

template <typename T>
int chol_inv_t(const gpaw_sys *s, const void *S, int n, void *Cout, int32_t *info, hipStream_t st) {
  constexpr int NMAX = EigMax<T>::n;
  if (n > EIG_LARGE_MAX) return fail(GPAW_ESHAPE, "orthonormalisation supports nb <= 1024");
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_eig_chol<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  if (attr_err != hipSuccess) return hip_fail(attr_err, "hipFuncSetAttribute(k_eig_chol)");
  const int sz = St<T>::cplx ? 2 : 1;
  const bool large = n > NMAX;
  const EigWs w = eig_layout(s->ws.eig, n, sz, large);
  const T *Sd = static_cast<const T *>(S);
  const int64_t nn = static_cast<int64_t>(n) * n;
  const unsigned eb = static_cast<unsigned>((nn + 255) / 256);
  if (!large) {
    k_eig_chol<T><<<1, CH_T, chol_lds_bytes<T>(n), st>>>(Sd, n, w, info);
  } else {
    k_set_info<<<1, 1, 0, st>>>(info);
    k_hermitize<T><<<eb, 256, 0, st>>>(Sd, as<T>(w.Sw), n, info);
    large_chol_linv<T>(as<T>(w.Sw), as<T>(w.Linv), n, w.piv, info, st);
  }
  k_conj_transpose<T><<<eb, 256, 0, st>>>(as<T>(w.Linv), static_cast<T *>(Cout), n, info);
  return GPAW_OK;
}

// ---------------------------------------------------------------------------
// Batched small eigensolves: the one-workgroup pipeline above for several
// systems of one scalar type in one chain of launches. Launch k covers every
// system (blockIdx.y = system) with the grid of the largest; a system's
// workgroups past its own grid for that stage leave at once, so each system
// runs exactly the single-system launches, in the same order, and its results
// equal those of its own call bit for bit. Independent systems then share
// one launch per stage instead of queueing one-workgroup launches behind
// each other.
struct EigJob {
  int n;
  EigWs w;
  const void *H, *S;
  double *eps;
  void *C;
  int32_t *info;
};

__device__ inline unsigned sg_grid(int n) {
  const int t = (n + 15) / 16;
  return static_cast<unsigned>((t * t + 3) / 4);
}
__device__ inline unsigned elem_grid(int n) {
  return static_cast<unsigned>((static_cast<int64_t>(n) * n + 255) / 256);
}

template <typename T>
__global__ __launch_bounds__(CH_T) void kb_eig_chol(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  d_eig_chol<T>(static_cast<const T *>(j.S), j.n, j.w, j.info);
}

// SEL picks the operands of one of the pipeline's small products (see
// eigh_t and refine_vectors for the single-system order)
template <typename T, int AM, int BM, int SEL>
__global__ __launch_bounds__(SG_T) void kb_small_gemm(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= sg_grid(j.n)) return;
  const EigWs &w = j.w;
  if constexpr (SEL == 0) d_small_gemm<T, AM, BM>(static_cast<const T *>(j.H), as<T>(w.Linv), as<T>(w.T1), j.n, j.info);
  if constexpr (SEL == 1) d_small_gemm<T, AM, BM>(as<T>(w.Linv), as<T>(w.T1), as<T>(w.A), j.n, j.info);
  if constexpr (SEL == 2) d_small_gemm<T, AM, BM>(as<T>(w.Linv), as<T>(w.T1), static_cast<T *>(j.C), j.n, j.info);
  if constexpr (SEL == 3) d_small_gemm<T, AM, BM>(w.Z, w.Z, w.G, j.n, j.info);
  if constexpr (SEL == 4) d_small_gemm<T, AM, BM>(w.Z, w.Z2, w.T1, j.n, j.info);
  if constexpr (SEL == 5) d_small_gemm<T, AM, BM>(w.Z, w.Z2, w.G, j.n, j.info);
  if constexpr (SEL == 6) d_small_gemm<T, AM, BM>(w.G, w.G, w.Z, j.n, j.info);
  if constexpr (SEL == 7) d_small_gemm<T, AM, BM>(w.G, w.Z2, w.T1, j.n, w.skip);
  if constexpr (SEL == 8) d_small_gemm<T, AM, BM>(w.G, w.Z2, w.Z, j.n, w.skip);
}

template <typename T>
__global__ __launch_bounds__(TRI_T) void kb_eig_tridiag(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  d_eig_tridiag<T>(j.n, j.w, j.info);
}

__global__ __launch_bounds__(256) void kb_eig_values(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= static_cast<unsigned>((j.n + 3) / 4)) return;
  d_eig_values(j.n, j.w.d, j.w.e, j.w.lam, j.info);
}

__global__ __launch_bounds__(VEC_T) void kb_eig_vectors(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= static_cast<unsigned>((j.n + VEC_T - 1) / VEC_T)) return;
  d_eig_vectors(j.n, j.w, j.info);
}

__global__ __launch_bounds__(CL_T) void kb_cluster_orth(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  d_cluster_orth(j.n, j.w.d, j.w.e, j.w.lam, j.w.Z, j.w.cid, j.w.cltol, j.info);
}

template <int STEP>
__global__ __launch_bounds__(1024) void kb_gram_check(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if constexpr (STEP == 0) d_gram_check(j.w.G, j.n, 0.1, j.info, nullptr, 0.0, nullptr);
  else d_gram_check(j.w.Z, j.n, 1e-4, j.info, j.w.skip, 1e-13, nullptr);
}

template <int STEP>
__global__ __launch_bounds__(256) void kb_tri_apply(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= elem_grid(j.n)) return;
  if constexpr (STEP == 0) d_tri_apply(j.n, j.w.d, j.w.e, j.w.Z, j.w.Z2, j.info);
  else d_tri_apply(j.n, j.w.d, j.w.e, j.w.G, j.w.Z2, j.w.skip);
}

template <int STEP>
__global__ __launch_bounds__(256) void kb_refine_coef(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= elem_grid(j.n)) return;
  const EigWs &w = j.w;
  if constexpr (STEP == 0) d_refine_coef(j.n, w.G, w.T1, w.lam, w.cid, w.cltol, w.Z2, j.info);
  else d_refine_coef(j.n, w.Z, w.T1, w.lam, w.cid, w.cltol, w.Z2, w.skip);
}

__global__ __launch_bounds__(256) void kb_copy_gated(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= elem_grid(j.n)) return;
  d_copy_gated(j.w.Z, j.w.G, static_cast<int64_t>(j.n) * j.n, j.w.skip);
}

template <typename T>
__global__ __launch_bounds__(128) void kb_eig_back(const EigJob *J) {
  const EigJob &j = J[blockIdx.y];
  if (blockIdx.x >= static_cast<unsigned>((j.n + 15) / 16)) return;
  d_eig_back<T>(j.n, j.w, j.w.G, as<T>(j.w.T1), j.eps, j.info);
}

template <typename T>
int eigh_batched_t(const EigBatchItem *items, int count, const void *jobs, hipStream_t st) {
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    const void *fns[] = {reinterpret_cast<const void *>(&kb_eig_chol<T>),
                         reinterpret_cast<const void *>(&kb_eig_back<T>)};
    for (const void *f : fns)
      if (attr_err == hipSuccess)
        attr_err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  if (attr_err != hipSuccess) return hip_fail(attr_err, "hipFuncSetAttribute(batched eigensolver)");
  int nmax = 1;
  for (int i = 0; i < count; ++i) nmax = std::max(nmax, items[i].nb);
  if (nmax > EigMax<T>::n) return fail(GPAW_ESHAPE, "batched eigensolver: nb above the one-workgroup limit");
  const EigJob *J = static_cast<const EigJob *>(jobs);
  const unsigned ny = static_cast<unsigned>(count);
  const int64_t nn = static_cast<int64_t>(nmax) * nmax;
  const unsigned eb = static_cast<unsigned>((nn + 255) / 256);
  const int tiles = ((nmax + 15) / 16) * ((nmax + 15) / 16);
  const unsigned sgb = static_cast<unsigned>((tiles + 3) / 4);
  kb_eig_chol<T><<<dim3(1, ny), CH_T, chol_lds_bytes<T>(nmax), st>>>(J);
  kb_small_gemm<T, 2, 1, 0><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_small_gemm<T, 0, 0, 1><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_eig_tridiag<T><<<dim3(1, ny), TRI_T, 0, st>>>(J);
  kb_eig_values<<<dim3((nmax + 3) / 4, ny), 256, values_lds_bytes(nmax), st>>>(J);
  kb_eig_vectors<<<dim3((nmax + VEC_T - 1) / VEC_T, ny), VEC_T,
                   vec_lds_doubles(nmax) * sizeof(double), st>>>(J);
  kb_cluster_orth<<<dim3(1, ny), CL_T, 0, st>>>(J);
  // eigenvector refinement, as refine_vectors
  kb_small_gemm<double, 1, 0, 3><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_gram_check<0><<<dim3(1, ny), 1024, 0, st>>>(J);
  kb_tri_apply<0><<<dim3(eb, ny), 256, 0, st>>>(J);
  kb_small_gemm<double, 1, 0, 4><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_refine_coef<0><<<dim3(eb, ny), 256, 0, st>>>(J);
  kb_small_gemm<double, 0, 0, 5><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_small_gemm<double, 1, 0, 6><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_gram_check<1><<<dim3(1, ny), 1024, 0, st>>>(J);
  kb_tri_apply<1><<<dim3(eb, ny), 256, 0, st>>>(J);
  kb_small_gemm<double, 1, 0, 7><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_refine_coef<1><<<dim3(eb, ny), 256, 0, st>>>(J);
  kb_small_gemm<double, 0, 0, 8><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  kb_copy_gated<<<dim3(eb, ny), 256, 0, st>>>(J);
  // U = Q Z in eigen-order, then C = Linv^H U
  kb_eig_back<T><<<dim3((nmax + 15) / 16, ny), 128, back_lds_bytes<T>(nmax), st>>>(J);
  kb_small_gemm<T, 1, 0, 2><<<dim3(sgb, ny), SG_T, 0, st>>>(J);
  return GPAW_OK;
}

}  // namespace

int launch_chol_inv(const gpaw_sys *s, const void *S, int nb, void *Cout, int32_t *info,
                    hipStream_t st) {
  if (is_complex(s->dtype)) return chol_inv_t<z64>(s, S, nb, Cout, info, st);
  return chol_inv_t<double>(s, S, nb, Cout, info, st);
}

size_t eig_ws_elems(int nmax, bool cplx) {
  const int small = cplx ? EigMax<z64>::n : EigMax<double>::n;
  const int n = std::min(nmax, EIG_LARGE_MAX);
  return eig_layout_elems(n, cplx ? 2 : 1, n > small);
}

int eig_small_max(bool cplx) { return cplx ? EigMax<z64>::n : EigMax<double>::n; }

size_t eig_job_bytes() { return sizeof(EigJob); }

int eigh_batched_prepare(const EigBatchItem *items, int count, void *jobs) {
  std::vector<EigJob> host(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    const EigBatchItem &it = items[i];
    const bool cplx = is_complex(it.s->dtype);
    if (it.nb < 1 || it.nb > eig_small_max(cplx))
      return fail(GPAW_ESHAPE, "batched eigensolver: nb outside [1, one-workgroup limit]");
    EigJob &j = host[static_cast<size_t>(i)];
    j.n = it.nb;
    j.w = eig_layout(it.s->ws.eig, it.nb, cplx ? 2 : 1, false);
    j.H = it.H;
    j.S = it.S;
    j.eps = it.eps;
    j.C = it.C;
    j.info = it.info;
  }
  if (count > 0) GFD_HIP(hipMemcpy(jobs, host.data(), host.size() * sizeof(EigJob), hipMemcpyHostToDevice));
  return GPAW_OK;
}

int launch_eigh_batched(const EigBatchItem *items, int count, bool cplx, const void *jobs,
                        hipStream_t st) {
  if (count == 0) return GPAW_OK;
  return cplx ? eigh_batched_t<z64>(items, count, jobs, st)
              : eigh_batched_t<double>(items, count, jobs, st);
}

int launch_eigh(const gpaw_sys *s, const void *H, const void *S, int nb, double *eps, void *C,
                int32_t *info, hipStream_t st) {
  if (s->dtype == GPAW_C128 || s->dtype == GPAW_C64) return eigh_t<z64>(s, H, S, nb, eps, C, info, st);
  return eigh_t<double>(s, H, S, nb, eps, C, info, st);
}

}  // namespace gfd
