// Subspace matrices and rotation (SCF step (1), Sec. "Solving the Kohn-Sham
// equation") on the FP64 matrix cores of gfx950.
//
// H_nm = dV sum_r psi_n(r) Hpsi_m(r) is a tall-skinny contraction (K = Ng up
// to millions, M = N = nb). Work splits over K across the whole chip; each
// workgroup (4 wavefronts) owns one 64x64 output tile of one matrix for one
// K-range, every wavefront accumulates the full tile over a quarter of the
// range with v_mfma_f64_16x16x4, and the four partial tiles are summed
// through LDS in a fixed order. A second kernel adds the K-range partials in
// a fixed order and applies dV, so the result is bitwise reproducible.
//
// MFMA operand layout (16x16x4, FP64): lane l supplies A[i = l%16][k = l/16]
// and B[k = l/16][j = l%16]; the accumulator element r of lane l is
// D[l/16 + 4r][l%16] (measured on gfx950). For the contraction each lane instead loads four
// consecutive k of its row (k = 4*(l/16) + s for the s-th MFMA): a
// permutation of the K index applied to both operands, which leaves the sum
// unchanged and turns each lane's loads into one contiguous 32-byte run.
//
// Rotation psi'_n = sum_m C_mn psi_m: output rows are bands, columns grid
// points; A[i][k] = C[k][i] (16 consecutive n of one row of C) and
// B[k][j] = psi[k][g0 + j] (16 consecutive grid points), so both operands
// and the output are read/written in 128-byte runs.
#include <algorithm>

#include "internal.h"

namespace gfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SUB_TILE = 64;

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// part[(split*nmat + mat)][nb][nb] = sum_{k in range} A[n][k] B_mat[m][k]
__global__ __launch_bounds__(256) void k_subspace_f64(const double *__restrict__ A,
                                                      const double *__restrict__ B0,
                                                      const double *__restrict__ B1,
                                                      double *__restrict__ part, int nb,
                                                      int64_t ng, int64_t kchunk, int tiles_n,
                                                      int nmat) {
  __shared__ d4 red[2][4][4][64];  // 2 wavefronts x 4x4 blocks x 64 lanes = 64 KB
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int mat = blockIdx.y;
  const double *B = mat ? B1 : B0;
  const int64_t kb = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t ke = std::min(ng, kb + kchunk);
  const int r = lane & 15, kq = lane >> 4;

  const double *ap[4];
  const double *bp[4];
  bool av[4], bv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ra = tm * SUB_TILE + q * 16 + r;
    const int rb = tn * SUB_TILE + q * 16 + r;
    av[q] = ra < nb;
    bv[q] = rb < nb;
    ap[q] = A + static_cast<int64_t>(av[q] ? ra : 0) * ng;
    bp[q] = B + static_cast<int64_t>(bv[q] ? rb : 0) * ng;
  }

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int64_t kg = kb + wave * 16; kg < ke; kg += 64) {
    const int64_t k = kg + 4 * kq;
    double a[4][4], b[4][4];
    if (kg + 16 <= ke) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a[q][s] = av[q] ? ap[q][k + s] : 0.0;
          b[q][s] = bv[q] ? bp[q][k + s] : 0.0;
        }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const bool in = k + s < ke;
          a[q][s] = (av[q] && in) ? ap[q][k + s] : 0.0;
          b[q][s] = (bv[q] && in) ? bp[q][k + s] : 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
  }

  // fixed-order sum of the four wavefronts' tiles: (w0 + w2) + (w1 + w3)
  if (wave >= 2)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[wave - 2][i][j][lane] = acc[i][j];
  __syncthreads();
  if (wave < 2)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += red[wave][i][j][lane];
  __syncthreads();
  if (wave == 1)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[0][i][j][lane] = acc[i][j];
  __syncthreads();
  if (wave == 0) {
    double *out = part + (static_cast<int64_t>(blockIdx.z) * nmat + mat) * nb * nb;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const d4 v = acc[i][j] + red[0][i][j][lane];
        const int col = tn * SUB_TILE + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = tm * SUB_TILE + i * 16 + (lane >> 4) + 4 * e;
          if (row < nb && col < nb) out[static_cast<int64_t>(row) * nb + col] = v[e];
        }
      }
  }
}

__global__ __launch_bounds__(256) void k_subspace_reduce(const double *__restrict__ part,
                                                         double *__restrict__ H,
                                                         double *__restrict__ S, int nb,
                                                         int nsplit, int nmat, double dV) {
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= nn * nmat) return;
  const int mat = static_cast<int>(idx / nn);
  const int64_t e = idx - mat * nn;
  double acc = 0.0;
  for (int s = 0; s < nsplit; ++s) acc += part[(static_cast<int64_t>(s) * nmat + mat) * nn + e];
  (mat ? S : H)[e] = dV * acc;
}

struct SplitPlan {
  int tiles_n, tiles;
  int nsplit;
  int64_t kchunk;
};

SplitPlan plan_subspace(int nb, int64_t ng, int nmat) {
  SplitPlan p;
  p.tiles_n = (nb + SUB_TILE - 1) / SUB_TILE;
  p.tiles = p.tiles_n * p.tiles_n;
  // aim at ~512 workgroups (two per CU) with at least 1024 K per workgroup
  const int64_t want = std::max<int64_t>(1, 512 / (p.tiles * nmat));
  const int64_t kmax_split = std::max<int64_t>(1, ng / 1024);
  int64_t nsplit = std::min(want, kmax_split);
  int64_t kchunk = (ng + nsplit - 1) / nsplit;
  kchunk = (kchunk + 63) / 64 * 64;
  p.kchunk = kchunk;
  p.nsplit = static_cast<int>((ng + kchunk - 1) / kchunk);
  return p;
}

// out[n][g] = sum_m C[m][n] src[m][g], rows n in the 128-row group blockIdx.y
__global__ __launch_bounds__(256) void k_rotate_f64(const double *__restrict__ C,
                                                    const double *__restrict__ src,
                                                    double *__restrict__ dst, int nb,
                                                    int64_t cols) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int64_t g0 = static_cast<int64_t>(blockIdx.x) * 128 + wave * 32;
  const int n0 = blockIdx.y * 128;
  int64_t gc[2];
  bool gv[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    gc[cb] = g0 + cb * 16 + j;
    gv[cb] = gc[cb] < cols;
  }
  d4 acc[8][2];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[i][c] = d4{0.0, 0.0, 0.0, 0.0};

  for (int m0 = 0; m0 < nb; m0 += 4) {
    const int m = m0 + kq;
    const bool mv = m < nb;
    double a[8], b[2];
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      const int n = n0 + rb * 16 + j;
      a[rb] = (mv && n < nb) ? C[static_cast<int64_t>(m) * nb + n] : 0.0;
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
      b[cb] = (mv && gv[cb]) ? src[static_cast<int64_t>(m) * cols + gc[cb]] : 0.0;
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mfma(a[rb], b[cb], acc[rb][cb]);
  }
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      if (!gv[cb]) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + rb * 16 + kq + 4 * e;
        if (n < nb) dst[static_cast<int64_t>(n) * cols + gc[cb]] = acc[rb][cb][e];
      }
    }
}

}  // namespace

size_t subspace_part_elems(const gpaw_sys *s, int nb) {
  // nsplit * tiles * nmat <= 512 whenever want >= 1, else nsplit = 1
  const int64_t bound = std::max<int64_t>(512 * SUB_TILE * SUB_TILE, 2 * int64_t(nb) * nb);
  return static_cast<size_t>(bound) * (s->dtype == GPAW_C128 ? 2 : 1);
}

int launch_subspace(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                    int nb, void *H, void *S, hipStream_t st) {
  if (s->dtype != GPAW_F64) return fail(GPAW_EDTYPE, "subspace matrices: complex not built yet");
  const int nmat = Spsi ? 2 : 1;
  const SplitPlan p = plan_subspace(nb, s->ng, nmat);
  const int64_t need = static_cast<int64_t>(p.nsplit) * nmat * nb * nb;
  if (need > static_cast<int64_t>(s->ws.part_elems))
    return fail(GPAW_EINVAL, "subspace workspace too small");
  dim3 grid(p.tiles, nmat, p.nsplit);
  k_subspace_f64<<<grid, 256, 0, st>>>(static_cast<const double *>(psi),
                                       static_cast<const double *>(Hpsi),
                                       static_cast<const double *>(Spsi ? Spsi : Hpsi),
                                       s->ws.part, nb, s->ng, p.kchunk, p.tiles_n, nmat);
  const int64_t tot = static_cast<int64_t>(nb) * nb * nmat;
  k_subspace_reduce<<<static_cast<unsigned>((tot + 255) / 256), 256, 0, st>>>(
      s->ws.part, static_cast<double *>(H), static_cast<double *>(S), nb, p.nsplit, nmat, s->dV);
  return GPAW_OK;
}

int launch_rotate(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                  void *dst, hipStream_t st) {
  if (s->dtype != GPAW_F64) return fail(GPAW_EDTYPE, "rotation: complex not built yet");
  if (cols == 0) return GPAW_OK;
  dim3 grid(static_cast<unsigned>((cols + 127) / 128), (nb + 127) / 128);
  k_rotate_f64<<<grid, 256, 0, st>>>(static_cast<const double *>(C),
                                     static_cast<const double *>(src),
                                     static_cast<double *>(dst), nb, cols);
  return GPAW_OK;
}

}  // namespace gfd
