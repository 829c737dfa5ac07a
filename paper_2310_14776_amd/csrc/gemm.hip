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
#include <type_traits>

#include "internal.h"

namespace gfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SUB_TILE = 64;

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Complex operands: conj(a) b = (ax bx + ay by) + i (ax by - ay bx) and
// a b = (ax bx - ay by) + i (ax by + ay bx), four real MFMAs each.
template <typename T> struct Cx;
template <> struct Cx<double> {
  static constexpr int parts = 1;
  __device__ static double re(double a) { return a; }
  __device__ static double im(double) { return 0.0; }
  __device__ static double make(double r, double) { return r; }
};
template <> struct Cx<z64> {
  static constexpr int parts = 2;
  __device__ static double re(z64 a) { return a.x; }
  __device__ static double im(z64 a) { return a.y; }
  __device__ static z64 make(double r, double i) { return z64{r, i}; }
};

// part[(split*nmat + mat)][nb][nb] = sum_{k in range} conj(A[n][k]) B_mat[m][k]
// BM x BM blocks of 16x16 per wavefront (a TILE x TILE output tile).
// four consecutive elements p[0..3] as 16-byte loads
template <typename T>
__device__ inline void load4(const T *p, T *v) {
  typedef double dv2 __attribute__((ext_vector_type(2)));
  constexpr int W = static_cast<int>(sizeof(T) * 4 / 16);
  dv2 w[W];
#pragma unroll
  for (int q = 0; q < W; ++q) w[q] = reinterpret_cast<const dv2 *>(p)[q];
  __builtin_memcpy(v, w, sizeof(T) * 4);
}

template <typename T, int BM, bool VEC>
__global__ __launch_bounds__(256) void k_subspace(const T *__restrict__ A, const T *__restrict__ B0,
                                                  const T *__restrict__ B1, T *__restrict__ part,
                                                  int nb, int64_t ng, int64_t kchunk, int tiles_n,
                                                  int nmat, int nsplit) {
  constexpr int TILE = 16 * BM;
  constexpr int NP = Cx<T>::parts;
  __shared__ d4 red[2][NP][BM][BM][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // workgroups are dealt to the 8 XCDs round-robin by id: give all tiles and
  // matrices of one K chunk the same id residue so they share that XCD's L2
  // (with fewer than 8 K chunks the plain order keeps every XCD busy)
  // H and S are Hermitian: only the tiles on and above the diagonal are
  // formed (the reduction mirrors the rest)
  const int tiles = tiles_n * (tiles_n + 1) / 2, TT = tiles * nmat;
  int split, tt;
  if (nsplit >= 8) {
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    split = (jj / TT) * 8 + xcd;
    tt = jj - (jj / TT) * TT;
  } else {
    split = blockIdx.x / TT;
    tt = blockIdx.x - split * TT;
  }
  if (split >= nsplit) return;
  const int mat = tt / tiles, tile = tt - mat * tiles;
  int tm = 0, rest = tile;
  while (rest >= tiles_n - tm) {
    rest -= tiles_n - tm;
    ++tm;
  }
  const int tn = tm + rest;
  const T *B = mat ? B1 : B0;
  const int64_t kb = static_cast<int64_t>(split) * kchunk;
  const int64_t ke = std::min(ng, kb + kchunk);
  const int r = lane & 15, kq = lane >> 4;

  // rows past nb are clamped to the last row: they only feed outputs that
  // are never stored
  const T *ap[BM];
  const T *bp[BM];
#pragma unroll
  for (int q = 0; q < BM; ++q) {
    ap[q] = A + static_cast<int64_t>(std::min(tm * TILE + q * 16 + r, nb - 1)) * ng;
    bp[q] = B + static_cast<int64_t>(std::min(tn * TILE + q * 16 + r, nb - 1)) * ng;
  }

  d4 acc[NP][BM][BM];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) acc[c][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  auto compute = [&](const T (&a)[BM][4], const T (&b)[BM][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) {
          const double ax = Cx<T>::re(a[i][s]), bx = Cx<T>::re(b[j][s]);
          acc[0][i][j] = mfma(ax, bx, acc[0][i][j]);
          if constexpr (NP == 2) {
            const double ay = Cx<T>::im(a[i][s]), by = Cx<T>::im(b[j][s]);
            acc[0][i][j] = mfma(ay, by, acc[0][i][j]);
            acc[NP - 1][i][j] = mfma(ax, by, acc[NP - 1][i][j]);
            acc[NP - 1][i][j] = mfma(-ay, bx, acc[NP - 1][i][j]);
          }
        }
  };
  // The wavefront's full 16-wide K steps run as a software pipeline: a ring
  // of D register buffers, each step's operands requested D steps before its
  // MFMAs. Every load in the ring is unconditional and in bounds (the
  // prefetch past the last step re-reads it), so no branch sits between a
  // load and its use and the waits count down instead of draining.
  const int64_t k0 = kb + wave * 16;
  const int64_t nfull = ke - k0 >= 16 ? (ke - k0 - 16) / 64 + 1 : 0;
  auto load_full = [&](int64_t t, T (&a)[BM][4], T (&b)[BM][4]) {
    const int64_t k = k0 + 64 * t + 4 * kq;
    if constexpr (VEC) {
      // four consecutive k of a row: 16-byte loads (rows 32-byte aligned)
#pragma unroll
      for (int q = 0; q < BM; ++q) {
        load4(ap[q] + k, a[q]);
        load4(bp[q] + k, b[q]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < BM; ++q)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a[q][s] = ap[q][k + s];
          b[q][s] = bp[q][k + s];
        }
    }
  };
  constexpr int D = 3;
  T a[D][BM][4], b[D][BM][4];
  if (nfull > 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) load_full(std::min<int64_t>(d, nfull - 1), a[d], b[d]);
  }
  for (int64_t t = 0; t < nfull; t += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (t + d < nfull) compute(a[d], b[d]);
      load_full(std::min<int64_t>(t + d + D, nfull - 1), a[d], b[d]);
    }
  }
  // at most one partial step (the end of the last K chunk): masked loads
  {
    const int64_t k = k0 + 64 * nfull + 4 * kq;
    if (k0 + 64 * nfull < ke) {
#pragma unroll
      for (int q = 0; q < BM; ++q)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const bool in = k + s < ke;
          a[0][q][s] = in ? ap[q][k + s] : T{};
          b[0][q][s] = in ? bp[q][k + s] : T{};
        }
      compute(a[0], b[0]);
    }
  }

  // fixed-order sum of the four wavefronts' tiles: (w0 + w2) + (w1 + w3)
  if (wave >= 2)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) red[wave - 2][c][i][j][lane] = acc[c][i][j];
  __syncthreads();
  if (wave < 2)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) acc[c][i][j] += red[wave][c][i][j][lane];
  __syncthreads();
  if (wave == 1)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) red[0][c][i][j][lane] = acc[c][i][j];
  __syncthreads();
  if (wave == 0) {
    T *out = part + (static_cast<int64_t>(split) * nmat + mat) * nb * nb;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) {
        const d4 vr = acc[0][i][j] + red[0][0][i][j][lane];
        const d4 vi = acc[NP - 1][i][j] + red[0][NP - 1][i][j][lane];
        const int col = tn * TILE + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = tm * TILE + i * 16 + (lane >> 4) + 4 * e;
          if (row < nb && col < nb) out[static_cast<int64_t>(row) * nb + col] = Cx<T>::make(vr[e], vi[e]);
        }
      }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_subspace_reduce(const T *__restrict__ part,
                                                         T *__restrict__ H, T *__restrict__ S,
                                                         int nb, int nsplit, int nmat, double dV,
                                                         int tile) {
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= nn * nmat) return;
  const int mat = static_cast<int>(idx / nn);
  const int64_t eo = idx - mat * nn;
  const int r = static_cast<int>(eo / nb), c = static_cast<int>(eo - static_cast<int64_t>(r) * nb);
  // entries of tiles below the diagonal were not formed: the thread of the
  // mirror entry writes them (as its conjugate)
  if (r / tile > c / tile) return;
  const bool mirror = r / tile < c / tile;
  const int64_t e = eo;
  // the partials are added in split order (bitwise reproducible), eight
  // loads in flight at a time
  T acc{};
  for (int s0 = 0; s0 < nsplit; s0 += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = s0 + u < nsplit ? part[(static_cast<int64_t>(s0 + u) * nmat + mat) * nn + e] : T{};
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s0 + u < nsplit) acc = acc + v[u];
  }
  const T val = St<T>::scale(dV, acc);
  T *M = mat ? S : H;
  M[eo] = val;
  if (mirror) M[static_cast<int64_t>(c) * nb + r] = Cx<T>::make(Cx<T>::re(val), -Cx<T>::im(val));
}

}  // namespace

int64_t balanced_splits(int64_t units, int64_t slots, double tile_s, double part_s,
                        int64_t max_split, int64_t k, int64_t min_k) {
  slots = std::max<int64_t>(1, slots);
  const int64_t hi = std::max<int64_t>(1, std::min({max_split, k / std::max<int64_t>(1, min_k),
                                                    int64_t{64}}));
  int64_t best = 1;
  double best_t = 0.0;
  for (int64_t ns = 1; ns <= hi; ++ns) {
    const int64_t w = (ns >= 8 ? (ns + 7) / 8 * 8 : ns) * units;
    const double rounds = static_cast<double>((w + slots - 1) / slots);
    const double t = rounds * tile_s / static_cast<double>(ns) + static_cast<double>(ns) * part_s;
    // a larger count must gain at least 1%
    if (ns == 1 || t < 0.99 * best_t) {
      best = ns;
      best_t = t;
    }
  }
  return best;
}

int64_t resident_slots(const void *kern, int threads, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess)
    return 512;
  return static_cast<int64_t>(std::max(1, cus)) * std::max(1, per_cu);
}

namespace {

struct SplitPlan {
  int tiles_n, tiles;
  int nsplit;
  int64_t kchunk;
};

// target > 0: about that many workgroups (a tuned launch shape); else the
// balanced count for the resident slots of the kernel (flops: of one tile
// over the whole K range; pbytes: partial sums of one split)
SplitPlan plan_subspace(int nb, int64_t ng, int nmat, int tile, int target, int64_t max_split,
                        int64_t slots, double tile_flops, double pbytes) {
  SplitPlan p;
  p.tiles_n = (nb + tile - 1) / tile;
  p.tiles = p.tiles_n * (p.tiles_n + 1) / 2;  // on and above the diagonal
  int64_t nsplit;
  if (target > 0) {
    target = std::min(target, 1024);
    // (with 8 or more splits the launch rounds them up to whole groups of
    // 8, so round down here to stay within the target)
    int64_t want = std::max<int64_t>(1, target / (p.tiles * nmat));
    if (want >= 8) want = want / 8 * 8;
    const int64_t kmax_split = std::max<int64_t>(1, ng / 1024);
    nsplit = std::max<int64_t>(1, std::min({want, kmax_split, max_split}));
  } else {
    // FP64 matrix cores at about 70% of peak, partial sums at 5 TB/s
    nsplit = balanced_splits(static_cast<int64_t>(p.tiles) * nmat, slots,
                             tile_flops * static_cast<double>(slots) / (0.7 * 78.6e12),
                             2.0 * pbytes / 5e12, max_split, ng, 1024);
  }
  int64_t kchunk = (ng + nsplit - 1) / nsplit;
  kchunk = (kchunk + 63) / 64 * 64;
  p.kchunk = kchunk;
  p.nsplit = static_cast<int>((ng + kchunk - 1) / kchunk);
  return p;
}

// out[n][g] = sum_m C[m][n] src[m][g]; each wavefront owns RB*16 rows (the
// row group blockIdx.y) by 32 columns; no conjugation (psi' = C^T psi).
template <typename T, int RB>
__global__ __launch_bounds__(256) void k_rotate(const T *__restrict__ C, const T *__restrict__ src,
                                                T *__restrict__ dst, int nb, int nout,
                                                int64_t cols, int upper) {
  constexpr int NP = Cx<T>::parts;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int64_t g0 = static_cast<int64_t>(blockIdx.x) * 128 + wave * 32;
  const int n0 = blockIdx.y * RB * 16;
  int64_t gc[2];
  bool gv[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    gc[cb] = g0 + cb * 16 + j;
    gv[cb] = gc[cb] < cols;
  }
  d4 acc[NP][RB][2];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[c][i][q] = d4{0.0, 0.0, 0.0, 0.0};

  // Clamped addresses keep every load unconditional and in bounds (branches
  // around loads would force a full wait at each loop turn): rows n >= nout
  // and columns g >= cols only feed outputs that are never stored, and the
  // steps past m = nb are zeroed on the src side where they are used. C is
  // nb x nb (row stride nb); the first nout of its columns are used.
  const T *cp[RB];
  const T *sp[2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) cp[rb] = C + std::min(n0 + rb * 16 + j, nout - 1);
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) sp[cb] = src + std::min<int64_t>(gc[cb], cols - 1);
  auto load_step = [&](int m0, T (&a)[RB], T (&b)[2]) {
    const int64_t m = std::min(m0 + kq, nb - 1);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[rb] = cp[rb][m * nb];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) b[cb] = sp[cb][m * cols];
  };
  // a ring of D steps in flight: step s is requested D steps before its
  // MFMAs run, so the HBM latency of the src stream hides behind them
  constexpr int D = 4;
  T a[D][RB], b[D][2];
#pragma unroll
  for (int d = 0; d < D; ++d) load_step(4 * d, a[d], b[d]);
  // an upper-triangular C (m <= n) needs rows m < n0 + RB*16 only
  const int mend = upper ? std::min(nb, n0 + RB * 16) : nb;
  for (int m0 = 0; m0 < mend; m0 += 4 * D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (m0 + 4 * d < mend) {
        const bool mv = m0 + 4 * d + kq < nb;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          if (!mv) b[d][cb] = T{};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            const double ax = Cx<T>::re(a[d][rb]), bx = Cx<T>::re(b[d][cb]);
            acc[0][rb][cb] = mfma(ax, bx, acc[0][rb][cb]);
            if constexpr (NP == 2) {
              const double ay = Cx<T>::im(a[d][rb]), by = Cx<T>::im(b[d][cb]);
              acc[0][rb][cb] = mfma(-ay, by, acc[0][rb][cb]);
              acc[NP - 1][rb][cb] = mfma(ax, by, acc[NP - 1][rb][cb]);
              acc[NP - 1][rb][cb] = mfma(ay, bx, acc[NP - 1][rb][cb]);
            }
          }
      }
      load_step(m0 + 4 * (d + D), a[d], b[d]);
    }
  }
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      if (!gv[cb]) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + rb * 16 + kq + 4 * e;
        if (n < nout)
          dst[static_cast<int64_t>(n) * cols + gc[cb]] =
              Cx<T>::make(acc[0][rb][cb][e], acc[NP - 1][rb][cb][e]);
      }
    }
}

// Rotation of a short-row matrix (the projections: cols = Np): one wavefront
// per 16 x 16 output tile, 64 m per round with all loads issued first.
template <typename T>
__global__ __launch_bounds__(256) void k_rot_small(const T *__restrict__ C, const T *__restrict__ src,
                                                   T *__restrict__ dst, int nb, int nout,
                                                   int64_t cols, int tiles_c, int upper) {
  constexpr int NP = Cx<T>::parts;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int tiles_n = (nout + 15) / 16;
  if (tile >= tiles_n * tiles_c) return;
  const int n0 = (tile / tiles_c) * 16;
  const int64_t c0 = static_cast<int64_t>(tile % tiles_c) * 16;
  const int i = lane & 15, lk = lane >> 4;
  d4 acc[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
  const int mend = upper ? std::min(nb, n0 + 16) : nb;  // upper-triangular C: m <= n
  for (int m0 = 0; m0 < mend; m0 += 64) {
    T a[16], b[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int m = m0 + 4 * u + lk;
      a[u] = (m < nb && n0 + i < nout) ? C[static_cast<int64_t>(m) * nb + n0 + i] : T{};
      b[u] = (m < nb && c0 + i < cols) ? src[static_cast<int64_t>(m) * cols + c0 + i] : T{};
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double ax = Cx<T>::re(a[u]), bx = Cx<T>::re(b[u]);
      acc[0] = mfma(ax, bx, acc[0]);
      if constexpr (NP == 2) {
        const double ay = Cx<T>::im(a[u]), by = Cx<T>::im(b[u]);
        acc[0] = mfma(-ay, by, acc[0]);
        acc[NP - 1] = mfma(ax, by, acc[NP - 1]);
        acc[NP - 1] = mfma(ay, bx, acc[NP - 1]);
      }
    }
  }
  if (c0 + i >= cols) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int n = n0 + lk + 4 * e;
    if (n < nout) dst[static_cast<int64_t>(n) * cols + c0 + i] = Cx<T>::make(acc[0][e], acc[NP - 1][e]);
  }
}

template <typename T>
int rotate_small_t(const void *C, const void *src, int nb, int nout, int64_t cols, void *dst,
                   hipStream_t st, bool upper) {
  const int tiles_c = static_cast<int>((cols + 15) / 16);
  const int64_t tiles = static_cast<int64_t>((nout + 15) / 16) * tiles_c;
  k_rot_small<T><<<static_cast<unsigned>((tiles + 3) / 4), 256, 0, st>>>(
      static_cast<const T *>(C), static_cast<const T *>(src), static_cast<T *>(dst), nb, nout,
      cols, tiles_c, upper ? 1 : 0);
  return GPAW_OK;
}

template <typename T, int BM>
int subspace_t(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi, int nb,
               void *H, void *S, hipStream_t st, double *pbuf, size_t pcap) {
  const int nmat = Spsi ? 2 : 1;
  const int64_t per_split = static_cast<int64_t>(nmat) * nb * nb * Cx<T>::parts;
  const int64_t max_split = static_cast<int64_t>(pcap) / per_split;
  if (max_split < 1) return fail(GPAW_ESHAPE, "subspace partial-sum buffer too small for nb");
  // rows are 32-byte aligned when Ng is a multiple of 4 (the tensors' bases are)
  const bool vec = (s->ng % 4) == 0 &&
                   (reinterpret_cast<uintptr_t>(psi) | reinterpret_cast<uintptr_t>(Hpsi) |
                    reinterpret_cast<uintptr_t>(Spsi ? Spsi : Hpsi)) % 32 == 0;
  const int64_t slots =
      resident_slots(vec ? reinterpret_cast<const void *>(&k_subspace<T, BM, true>)
                         : reinterpret_cast<const void *>(&k_subspace<T, BM, false>),
                     256, 0);
  const double tile_flops = 2.0 * Cx<T>::parts * Cx<T>::parts * (16.0 * BM) * (16.0 * BM) *
                            static_cast<double>(s->ng);
  const SplitPlan p =
      plan_subspace(nb, s->ng, nmat, 16 * BM, s->tune.sub_wgs, max_split, slots, tile_flops,
                    static_cast<double>(per_split) * sizeof(double));
  T *part = reinterpret_cast<T *>(pbuf);
  const int64_t sgroups = p.nsplit >= 8 ? (p.nsplit + 7) / 8 * 8 : p.nsplit;
  const int64_t wgs = sgroups * p.tiles * nmat;
  auto go = [&](auto vflag) {
    k_subspace<T, BM, decltype(vflag)::value><<<static_cast<unsigned>(wgs), 256, 0, st>>>(
        static_cast<const T *>(psi), static_cast<const T *>(Hpsi),
        static_cast<const T *>(Spsi ? Spsi : Hpsi), part, nb, s->ng, p.kchunk, p.tiles_n, nmat,
        p.nsplit);
  };
  if (vec) go(std::true_type{});
  else go(std::false_type{});
  const int64_t tot = static_cast<int64_t>(nb) * nb * nmat;
  k_subspace_reduce<T><<<static_cast<unsigned>((tot + 255) / 256), 256, 0, st>>>(
      part, static_cast<T *>(H), static_cast<T *>(S), nb, p.nsplit, nmat, s->dV, 16 * BM);
  return GPAW_OK;
}

template <typename T, int RB>
int rotate_t(const void *C, const void *src, int nb, int nout, int64_t cols, void *dst,
             hipStream_t st, bool upper) {
  dim3 grid(static_cast<unsigned>((cols + 127) / 128), (nout + RB * 16 - 1) / (RB * 16));
  k_rotate<T, RB><<<grid, 256, 0, st>>>(static_cast<const T *>(C), static_cast<const T *>(src),
                                        static_cast<T *>(dst), nb, nout, cols, upper ? 1 : 0);
  return GPAW_OK;
}

}  // namespace

size_t subspace_part_elems(const gpaw_sys *s, int nb) {
  if (s->dtype == GPAW_F32 || s->dtype == GPAW_C64) return split_part_elems(nb, s->dtype == GPAW_C64);
  // A tuned target keeps nsplit * tiles * nmat <= 1024 whenever that allows
  // one split, else nsplit = 1; the tiles formed are those on and above the
  // diagonal, T (T + 1) / 2 >= T^2 / 2 of them for T tiles a side, so
  // nsplit * nmat * nb^2 <= 2048 tile^2 (complex tiles are 32 x 32, a quarter
  // of the real 64 x 64). The balanced plan takes up to 64 splits of two
  // matrices, within 64 Mi doubles (512 MiB); past that it is capped to fit.
  const bool cplx = s->dtype == GPAW_C128;
  const int64_t tile = cplx ? 32 : SUB_TILE;
  const int64_t parts = cplx ? 2 : 1;
  const int64_t tuned = std::max<int64_t>(2048 * tile * tile, 2 * int64_t(nb) * nb) * parts;
  const int64_t balanced = std::min<int64_t>(64 * 2 * int64_t(nb) * nb * parts, int64_t{64} << 20);
  return static_cast<size_t>(std::max(tuned, balanced));
}

int launch_subspace(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                    int nb, void *H, void *S, hipStream_t st, double *part, size_t part_elems) {
  if (!part) {
    part = s->ws.part;
    part_elems = s->ws.part_elems;
  }
  if (s->dtype == GPAW_F32 || s->dtype == GPAW_C64)
    return launch_subspace_split(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
  if (s->dtype == GPAW_C128)
    return subspace_t<z64, 2>(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
  return subspace_t<double, 4>(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
}

int launch_rotate(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                  void *dst, hipStream_t st, bool upper, bool near_id, int nout) {
  if (cols == 0) return GPAW_OK;
  if (nout < 0) nout = nb;
  if (nout > nb || (upper && nout != nb)) return fail(GPAW_EINVAL, "rotation: nout > nb");
  if (s->dtype == GPAW_F32 || s->dtype == GPAW_C64) {
    if (nout != nb)
      return fail(GPAW_EDTYPE, "a rotation to fewer bands runs in FP64/complex128 only");
    return launch_rotate_split(s, C, src, nb, cols, dst, st, upper, near_id);
  }
  // short rows (projections): too few columns to fill the chip by column
  // tiles, so one wavefront per 16 x 16 output tile instead
  if (cols <= 4096) {
    if (s->dtype == GPAW_C128) return rotate_small_t<z64>(C, src, nb, nout, cols, dst, st, upper);
    return rotate_small_t<double>(C, src, nb, nout, cols, dst, st, upper);
  }
  if (s->dtype == GPAW_C128)
    return s->tune.rot_rb == 2 ? rotate_t<z64, 2>(C, src, nb, nout, cols, dst, st, upper)
                               : rotate_t<z64, 4>(C, src, nb, nout, cols, dst, st, upper);
  return s->tune.rot_rb == 4 ? rotate_t<double, 4>(C, src, nb, nout, cols, dst, st, upper)
                             : rotate_t<double, 8>(C, src, nb, nout, cols, dst, st, upper);
}

}  // namespace gfd
