// Subspace matrices and rotation (SCF step (1), Sec. "Solving the Kohn-Sham
// equation") on the FP64 matrix cores of gfx950.
//
// H_nm = dV sum_r psi_n(r) Hpsi_m(r) is a tall-skinny contraction (K = Ng up
// to millions, M = N = nb). Work splits over K across the whole chip, in
// K chunks whose count balances whole rounds of resident workgroups against
// the partial-sum traffic. Two kernels form one K chunk's partial tiles:
//   * k_subspace (narrow blocks, and real blocks): a workgroup (4 wavefronts)
//     owns one output tile of one matrix; every wavefront accumulates the
//     full tile over a quarter of the chunk from registers fed by 16-byte
//     global loads, and the four partial tiles are summed through LDS in a
//     fixed order;
//   * k_subspace_lds (complex blocks of 256 bands or more): a 64 x 64 tile
//     per workgroup, 2 x 2 wavefronts, operands staged in LDS once for all
//     four (half the global bytes per MFMA).
// Work items run K chunk by K chunk, each chunk's tiles in super-blocks, and
// each XCD takes a contiguous range of them, so the workgroups resident on
// one XCD read the same rows. A second kernel adds the K-chunk partials in a
// fixed order and applies dV, so the result is bitwise reproducible.
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
#include "tile_order.h"

namespace gfd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SUB_TILE = 64;

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Complex operands take three real MFMAs per complex product (Gauss's
// three-multiplication form), each into an accumulator of its own:
//   conj(a) b: T1 = ax bx, T2 = ay by, T3 = (ax - ay)(bx + by);
//              re = T1 + T2, im = T3 - T1 + T2
//   a b:       T1 = ax bx, T2 = ay by, T3 = (ax + ay)(bx + by);
//              re = T1 - T2, im = T3 - T1 - T2
// The operand sums are one vector add per fragment. The three sums are
// combined once, after the K loop; the rounding error stays of the order
// of the unit roundoff times sum |a||b|, as for the four-product form.
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
                                                  int nmat, int nsplit, int sb) {
  constexpr int TILE = 16 * BM;
  constexpr int NP = Cx<T>::parts;
  constexpr int NACC = NP == 2 ? 3 : 1;
  __shared__ d4 red[2][NP][BM][BM][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // H and S are Hermitian: only the tiles on and above the diagonal are
  // formed (the reduction mirrors the rest). Work items run K chunk by K
  // chunk, each chunk's tiles in super-block order.
  const int tiles = tiles_n * (tiles_n + 1) / 2, TT = tiles * nmat;
  const int64_t item = xcd_item();
  const int split = static_cast<int>(item / TT);
  if (split >= nsplit) return;
  int mat, tm, tn;
  tile_of(static_cast<int>(item - static_cast<int64_t>(split) * TT), tiles_n, nmat, sb, mat, tm,
          tn);
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

  d4 acc[NACC][BM][BM];
#pragma unroll
  for (int c = 0; c < NACC; ++c)
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) acc[c][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  auto compute = [&](const T (&a)[BM][4], const T (&b)[BM][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if constexpr (NP == 2) {
        double ad[BM], bs[BM];
#pragma unroll
        for (int i = 0; i < BM; ++i) ad[i] = Cx<T>::re(a[i][s]) - Cx<T>::im(a[i][s]);
#pragma unroll
        for (int j = 0; j < BM; ++j) bs[j] = Cx<T>::re(b[j][s]) + Cx<T>::im(b[j][s]);
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BM; ++j) {
            acc[0][i][j] = mfma(Cx<T>::re(a[i][s]), Cx<T>::re(b[j][s]), acc[0][i][j]);
            acc[1][i][j] = mfma(Cx<T>::im(a[i][s]), Cx<T>::im(b[j][s]), acc[1][i][j]);
            acc[2][i][j] = mfma(ad[i], bs[j], acc[2][i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BM; ++j)
            acc[0][i][j] = mfma(Cx<T>::re(a[i][s]), Cx<T>::re(b[j][s]), acc[0][i][j]);
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

  // the wavefront's real and imaginary parts from the three products
  d4 fin[NP][BM][BM];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BM; ++j) {
      if constexpr (NP == 2) {
        fin[0][i][j] = acc[0][i][j] + acc[1][i][j];
        fin[1][i][j] = (acc[2][i][j] - acc[0][i][j]) + acc[1][i][j];
      } else {
        fin[0][i][j] = acc[0][i][j];
      }
    }
  // fixed-order sum of the four wavefronts' tiles: (w0 + w2) + (w1 + w3)
  if (wave >= 2)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) red[wave - 2][c][i][j][lane] = fin[c][i][j];
  __syncthreads();
  if (wave < 2)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) fin[c][i][j] += red[wave][c][i][j][lane];
  __syncthreads();
  if (wave == 1)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) red[0][c][i][j][lane] = fin[c][i][j];
  __syncthreads();
  if (wave == 0) {
    T *out = part + (static_cast<int64_t>(split) * nmat + mat) * nb * nb;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) {
        const d4 vr = fin[0][i][j] + red[0][0][i][j][lane];
        const d4 vi = fin[NP - 1][i][j] + red[0][NP - 1][i][j][lane];
        const int col = tn * TILE + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = tm * TILE + i * 16 + (lane >> 4) + 4 * e;
          if (row < nb && col < nb) out[static_cast<int64_t>(row) * nb + col] = Cx<T>::make(vr[e], vi[e]);
        }
      }
  }
}

// The same contraction for wide blocks (nb >= 256): a workgroup owns a
// TILE x TILE output tile (TILE = 32 WM) of one matrix for one K chunk, its
// four wavefronts in a 2 x 2 layout each own 16WM x 16WM of it, and the
// A and B rows of each 16-wide K stage are staged once in LDS for all four
// (each row serves two wavefronts): per MFMA the workgroup reads half the
// global bytes of the register-only kernel above.
//
// Stage pipeline: the next stage's global loads are issued before the
// current stage is multiplied out of one of two LDS buffers, then written to
// the other; one barrier per stage. Loads are unconditional: past the end
// of the chunk a lane reads a row of zeros instead (an address select, no
// branch), so the last stage needs no separate path.
//
// LDS rows hold the stage's 16 values plus 16 bytes of padding, so the
// fragment reads of eight consecutive rows (one 128-bit LDS phase) and the
// staging writes hit disjoint banks.
__device__ __attribute__((aligned(64))) double zero_group[8] = {};  // four complex zeros

template <typename T, int WM, bool VEC>
__global__ __launch_bounds__(256) void k_subspace_lds(const T *__restrict__ A,
                                                      const T *__restrict__ B0,
                                                      const T *__restrict__ B1,
                                                      T *__restrict__ part, int nb, int64_t ng,
                                                      int64_t kchunk, int tiles_n, int nmat,
                                                      int nsplit, int sb) {
  constexpr int NP = Cx<T>::parts;
  constexpr int NACC = NP == 2 ? 3 : 1;
  constexpr int TILE = 32 * WM;
  constexpr int KS = 16;                                  // K values per stage
  constexpr int PITCH = KS + static_cast<int>(16 / sizeof(T));  // LDS row pitch (elements)
  constexpr int TPR = 256 / TILE;                         // staging threads per row
  constexpr int EPT = KS / TPR;                           // values per thread and row
  constexpr int GPT = EPT / 4;                            // groups of 4 per thread
  static_assert(TPR * EPT == KS && GPT * 4 == EPT, "staging layout");
  __shared__ __attribute__((aligned(16))) T sA[2][TILE * PITCH];
  __shared__ __attribute__((aligned(16))) T sB[2][TILE * PITCH];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;

  const int tiles = tiles_n * (tiles_n + 1) / 2, TT = tiles * nmat;
  const int64_t item = xcd_item();
  const int split = static_cast<int>(item / TT);
  if (split >= nsplit) return;  // whole workgroup: no barrier is reached
  int mat, tm, tn;
  tile_of(static_cast<int>(item - static_cast<int64_t>(split) * TT), tiles_n, nmat, sb, mat, tm,
          tn);
  const T *B = mat ? B1 : B0;
  const int64_t kb = static_cast<int64_t>(split) * kchunk;
  const int64_t ke = std::min(ng, kb + kchunk);
  const int nst = kb < ke ? static_cast<int>((ke - kb + KS - 1) / KS) : 0;

  // staging: thread -> row srow of the tile, values sk .. sk + EPT - 1 of
  // the stage (rows past nb are clamped: they feed outputs never stored)
  const int srow = tid / TPR, sk = (tid % TPR) * EPT;
  const T *ga = A + static_cast<int64_t>(std::min(tm * TILE + srow, nb - 1)) * ng;
  const T *gb = B + static_cast<int64_t>(std::min(tn * TILE + srow, nb - 1)) * ng;
  const T *zr = reinterpret_cast<const T *>(zero_group);
  auto gload = [&](int st, T (&va)[EPT], T (&vb)[EPT]) {
    const int64_t k0 = kb + static_cast<int64_t>(st) * KS + sk;
    if constexpr (VEC) {
      // groups of four values start at multiples of 4 and ke is one, so a
      // group is either inside the chunk or past it
#pragma unroll
      for (int g = 0; g < GPT; ++g) {
        const int64_t k = k0 + 4 * g;
        const bool in = k < ke;
        load4(in ? ga + k : zr, va + 4 * g);
        load4(in ? gb + k : zr, vb + 4 * g);
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int64_t k = k0 + e;
        const bool in = k < ke;
        va[e] = *(in ? ga + k : zr);
        vb[e] = *(in ? gb + k : zr);
      }
    }
  };
  auto lstore = [&](int buf, const T (&va)[EPT], const T (&vb)[EPT]) {
    T *pa = &sA[buf][srow * PITCH + sk];
    T *pb = &sB[buf][srow * PITCH + sk];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      pa[e] = va[e];
      pb[e] = vb[e];
    }
  };

  d4 acc[NACC][WM][WM];
#pragma unroll
  for (int c = 0; c < NACC; ++c)
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WM; ++j) acc[c][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // fragment reads: lane l takes row l % 16 of each 16-row block and the
  // four consecutive stage values 4 (l / 16) .. 4 (l / 16) + 3, the s-th of
  // which feeds the s-th MFMA (the same K permutation on both operands)
  const int fr = lane & 15, fk = 4 * (lane >> 4);
  auto compute = [&](int buf) {  // buf: LDS buffer, a run-time index
    T a[WM][4], b[WM][4];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const T *pa = &sA[buf][(wr * 16 * WM + i * 16 + fr) * PITCH + fk];
      const T *pb = &sB[buf][(wc * 16 * WM + i * 16 + fr) * PITCH + fk];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[i][e] = pa[e];
        b[i][e] = pb[e];
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if constexpr (NP == 2) {
        double ad[WM], bs[WM];
#pragma unroll
        for (int i = 0; i < WM; ++i) ad[i] = Cx<T>::re(a[i][s]) - Cx<T>::im(a[i][s]);
#pragma unroll
        for (int j = 0; j < WM; ++j) bs[j] = Cx<T>::re(b[j][s]) + Cx<T>::im(b[j][s]);
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WM; ++j) {
            acc[0][i][j] = mfma(Cx<T>::re(a[i][s]), Cx<T>::re(b[j][s]), acc[0][i][j]);
            acc[1][i][j] = mfma(Cx<T>::im(a[i][s]), Cx<T>::im(b[j][s]), acc[1][i][j]);
            acc[2][i][j] = mfma(ad[i], bs[j], acc[2][i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WM; ++j)
            acc[0][i][j] = mfma(Cx<T>::re(a[i][s]), Cx<T>::re(b[j][s]), acc[0][i][j]);
      }
    }
  };

  if (nst > 0) {
    T ra[EPT], rb[EPT];
    gload(0, ra, rb);
    lstore(0, ra, rb);
    __syncthreads();
    for (int t = 0; t < nst; ++t) {
      // the next stage's loads are in flight while this one is multiplied
      gload(t + 1, ra, rb);
      compute(t & 1);
      // keep the products ahead of the LDS writes, which wait for the loads
      __builtin_amdgcn_sched_barrier(0);
      lstore((t + 1) & 1, ra, rb);
      __syncthreads();
    }
  }

  T *out = part + (static_cast<int64_t>(split) * nmat + mat) * nb * nb;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WM; ++j) {
      const int col = tn * TILE + wc * 16 * WM + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = tm * TILE + wr * 16 * WM + i * 16 + (lane >> 4) + 4 * e;
        double re = acc[0][i][j][e], im = 0.0;
        if constexpr (NP == 2) {
          re = acc[0][i][j][e] + acc[1][i][j][e];
          im = (acc[2][i][j][e] - acc[0][i][j][e]) + acc[1][i][j][e];
        }
        if (row < nb && col < nb) out[static_cast<int64_t>(row) * nb + col] = Cx<T>::make(re, im);
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

// out[n][g] = sum_m C[m][n] src[m][g]; a workgroup owns RB*16 rows (a row
// group) by 128 columns (a column block), each wavefront 32 of the columns;
// no conjugation (psi' = C^T psi). Work items run column block by column
// block, the row groups of one block consecutively, so the workgroups that
// read the same src columns are resident on one XCD together and src comes
// from HBM about once.
template <typename T, int RB>
__global__ __launch_bounds__(256) void k_rotate(const T *__restrict__ C, const T *__restrict__ src,
                                                T *__restrict__ dst, int nb, int nout,
                                                int64_t cols, int upper, int rgroups,
                                                int64_t items) {
  constexpr int NP = Cx<T>::parts;
  constexpr int NACC = NP == 2 ? 3 : 1;
  const int64_t item = xcd_item();
  if (item >= items) return;
  const int64_t cblock = item / rgroups;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int64_t g0 = cblock * 128 + wave * 32;
  const int n0 = static_cast<int>(item - cblock * rgroups) * RB * 16;
  int64_t gc[2];
  bool gv[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    gc[cb] = g0 + cb * 16 + j;
    gv[cb] = gc[cb] < cols;
  }
  d4 acc[NACC][RB][2];
#pragma unroll
  for (int c = 0; c < NACC; ++c)
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
        if constexpr (NP == 2) {
          double as[RB], bs[2];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) as[rb] = Cx<T>::re(a[d][rb]) + Cx<T>::im(a[d][rb]);
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) bs[cb] = Cx<T>::re(b[d][cb]) + Cx<T>::im(b[d][cb]);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
              acc[0][rb][cb] = mfma(Cx<T>::re(a[d][rb]), Cx<T>::re(b[d][cb]), acc[0][rb][cb]);
              acc[1][rb][cb] = mfma(Cx<T>::im(a[d][rb]), Cx<T>::im(b[d][cb]), acc[1][rb][cb]);
              acc[2][rb][cb] = mfma(as[rb], bs[cb], acc[2][rb][cb]);
            }
        } else {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
              acc[0][rb][cb] = mfma(Cx<T>::re(a[d][rb]), Cx<T>::re(b[d][cb]), acc[0][rb][cb]);
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
        if (n >= nout) continue;
        double re = acc[0][rb][cb][e], im = 0.0;
        if constexpr (NP == 2) {
          re = acc[0][rb][cb][e] - acc[1][rb][cb][e];
          im = (acc[2][rb][cb][e] - acc[0][rb][cb][e]) - acc[1][rb][cb][e];
        }
        dst[static_cast<int64_t>(n) * cols + gc[cb]] = Cx<T>::make(re, im);
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

// BM: wavefront blocks of the register-only kernel; WM > 0: wavefront
// blocks of the LDS-staged kernel, used from nb >= 256 on (complex blocks:
// for real ones the register-only kernel measured faster)
template <typename T, int BM, int WM>
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
  using Kern = void (*)(const T *, const T *, const T *, T *, int, int64_t, int64_t, int, int, int,
                        int);
  Kern kern = vec ? &k_subspace<T, BM, true> : &k_subspace<T, BM, false>;
  int tile = 16 * BM;
  if constexpr (WM > 0) {
    if (nb >= 256) {
      kern = vec ? &k_subspace_lds<T, WM, true> : &k_subspace_lds<T, WM, false>;
      tile = 32 * WM;
    }
  }
  const int64_t slots = resident_slots(reinterpret_cast<const void *>(kern), 256, 0);
  // real MFMA flops of one tile over the whole K range (three real
  // products per complex one)
  const double tile_flops = 2.0 * (Cx<T>::parts == 2 ? 3.0 : 1.0) * tile * tile *
                            static_cast<double>(s->ng);
  const SplitPlan p =
      plan_subspace(nb, s->ng, nmat, tile, s->tune.sub_wgs, max_split, slots, tile_flops,
                    static_cast<double>(per_split) * sizeof(double));
  T *part = reinterpret_cast<T *>(pbuf);
  // one work item per (K chunk, tile, matrix); the grid is rounded up to
  // whole groups of 8 (one workgroup per XCD)
  const int64_t items = static_cast<int64_t>(p.nsplit) * p.tiles * nmat;
  const int64_t wgs = (items + 7) / 8 * 8;
  // super-blocks of about the workgroups one XCD holds at a time
  const int sb = super_block(slots, p.tiles_n);
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(wgs)), dim3(256), 0, st,
                     static_cast<const T *>(psi), static_cast<const T *>(Hpsi),
                     static_cast<const T *>(Spsi ? Spsi : Hpsi), part, nb, s->ng, p.kchunk,
                     p.tiles_n, nmat, p.nsplit, sb);
  const int64_t tot = static_cast<int64_t>(nb) * nb * nmat;
  k_subspace_reduce<T><<<static_cast<unsigned>((tot + 255) / 256), 256, 0, st>>>(
      part, static_cast<T *>(H), static_cast<T *>(S), nb, p.nsplit, nmat, s->dV, tile);
  return GPAW_OK;
}

template <typename T, int RB>
int rotate_t(const void *C, const void *src, int nb, int nout, int64_t cols, void *dst,
             hipStream_t st, bool upper) {
  const int rgroups = (nout + RB * 16 - 1) / (RB * 16);
  const int64_t items = (cols + 127) / 128 * rgroups;
  const int64_t wgs = (items + 7) / 8 * 8;
  k_rotate<T, RB><<<static_cast<unsigned>(wgs), 256, 0, st>>>(
      static_cast<const T *>(C), static_cast<const T *>(src), static_cast<T *>(dst), nb, nout,
      cols, upper ? 1 : 0, rgroups, items);
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
    return subspace_t<z64, 2, 2>(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
  return subspace_t<double, 4, 0>(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
}

namespace {
__global__ __launch_bounds__(256) void k_add_mat(const double *__restrict__ a,
                                                 double *__restrict__ acc, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) acc[i] += a[i];
}
}  // namespace

int launch_add_mat(const double *a, double *acc, int64_t n, hipStream_t st) {
  if (n <= 0) return GPAW_OK;
  k_add_mat<<<static_cast<unsigned>((n + 255) / 256), 256, 0, st>>>(a, acc, n);
  return GPAW_OK;
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
