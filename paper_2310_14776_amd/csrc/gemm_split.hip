// Precision form of the subspace contractions (SCF step (1), Sec. "Solving
// the Kohn-Sham equation"): single-precision wave functions, products on the
// BF16 matrix cores of gfx950 with FP32 accumulation promoted to FP64.
//
// Split: an FP32 value x is written exactly as x = hi + mid + lo with three
// BF16 numbers (hi keeps the leading 8 significant bits, mid the next 8, lo
// the last 8; each remainder is exact in FP32). A product a b is formed from
// the six partial products whose size is at least 2^-16 of a b
// (hh, hm, mh, hl, lh, mm); the dropped ones are below 2^-23 relative, under
// FP32 rounding. BF16 keeps FP32's exponent range, so no scaling pass over
// the data is needed. Each partial product is exact in FP32; the MFMA
// accumulates in FP32. The subspace matrices add the FP32 tile into FP64
// accumulators after every 32-term step: the rounding error of an FP32
// partial sum is 2^-24 of that sum, so long FP32 runs over positive terms
// (the diagonal of S_nm) would dominate the error. The rotation, whose output
// is FP32, promotes every 8 steps (256 terms).
//
// MFMA layout (16x16x32, BF16 in, FP32 out): lane l supplies A[i = l%16]
// [8 values of k] and B[8 values of k][j = l%16] from the same k set, and
// accumulator element r of lane l is D[4*(l/16) + r][l%16] (measured).
#include <algorithm>

#include "internal.h"

namespace gfd {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

struct Split8 {
  bf8 h, m, l;
};

__device__ inline __bf16 top_half(uint32_t u) {
  return __builtin_bit_cast(__bf16, static_cast<unsigned short>(u >> 16));
}

// bits of the BF16 value nearest to the finite FP32 value with bits u (ties to
// even), as the high half of an FP32 word
__device__ inline uint32_t bf16_rne(uint32_t u) {
  return (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
}

// Exact three-way BF16 split of eight FP32 values, x = hi + mid + lo, each
// part rounded to nearest: hi = bf16(x), mid = bf16(x - hi), lo = x - hi - mid
// (x - hi has at most 16 significant bits and lo at most 8, so every
// difference is exact). Rounding to nearest leaves the parts with either
// sign, so the products dropped from the six-term sum (mid*lo, lo*mid,
// lo*lo, below 2^-24 relative) carry no systematic bias.
__device__ inline Split8 split8(const float *x) {
  Split8 s;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t uh = bf16_rne(__float_as_uint(x[e]));
    const float r1 = x[e] - __uint_as_float(uh);
    const uint32_t um = bf16_rne(__float_as_uint(r1));
    const float r2 = r1 - __uint_as_float(um);
    s.h[e] = top_half(uh);
    s.m[e] = top_half(um);
    s.l[e] = top_half(__float_as_uint(r2));
  }
  return s;
}

__device__ inline f4 mm(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// sum of the six leading partial products a b into c
__device__ inline f4 mm6(const Split8 &a, const Split8 &b, f4 c) {
  c = mm(a.l, b.h, c);
  c = mm(a.h, b.l, c);
  c = mm(a.m, b.m, c);
  c = mm(a.m, b.h, c);
  c = mm(a.h, b.m, c);
  c = mm(a.h, b.h, c);
  return c;
}

template <typename T> struct Parts;
template <> struct Parts<float> {
  static constexpr int n = 1;
  __device__ static float re(float a) { return a; }
  __device__ static float im(float) { return 0.0f; }
};
template <> struct Parts<z32> {
  static constexpr int n = 2;
  __device__ static float re(z32 a) { return a.x; }
  __device__ static float im(z32 a) { return a.y; }
};

// part[(split*nmat + mat)][nb][nb] (double / complex double) =
//   sum_{k in range} conj(A[n][k]) B_mat[m][k]; BM x BM 16x16 blocks per wavefront
template <typename T, int BM>
__global__ __launch_bounds__(256) void k_subspace_split(const T *__restrict__ A,
                                                        const T *__restrict__ B0,
                                                        const T *__restrict__ B1,
                                                        double *__restrict__ part, int nb,
                                                        int64_t ng, int64_t kchunk, int tiles_n,
                                                        int nmat) {
  constexpr int TILE = 16 * BM;
  constexpr int NP = Parts<T>::n;
  __shared__ d4 red[2][NP][BM][BM][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int mat = blockIdx.y;
  const T *B = mat ? B1 : B0;
  const int64_t kb = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t ke = std::min(ng, kb + kchunk);
  const int r = lane & 15, kq = lane >> 4;

  const T *ap[BM];
  const T *bp[BM];
  bool av[BM], bv[BM];
#pragma unroll
  for (int q = 0; q < BM; ++q) {
    const int ra = tm * TILE + q * 16 + r;
    const int rb = tn * TILE + q * 16 + r;
    av[q] = ra < nb;
    bv[q] = rb < nb;
    ap[q] = A + static_cast<int64_t>(av[q] ? ra : 0) * ng;
    bp[q] = B + static_cast<int64_t>(bv[q] ? rb : 0) * ng;
  }
  d4 dacc[NP][BM][BM];
  f4 facc[NP][BM][BM];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) {
        dacc[c][i][j] = d4{0.0, 0.0, 0.0, 0.0};
        facc[c][i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
  // each wavefront takes every fourth 32-wide K step of the range
  for (int64_t kg = kb + wave * 32; kg < ke; kg += 128) {
    const int64_t k = kg + 8 * kq;
    Split8 sa[NP][BM], sb[NP][BM];
#pragma unroll
    for (int q = 0; q < BM; ++q) {
      float xr[8], xi[8], yr[8], yi[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool in = k + e < ke;
        const T a = (av[q] && in) ? ap[q][k + e] : T{};
        const T b = (bv[q] && in) ? bp[q][k + e] : T{};
        xr[e] = Parts<T>::re(a);
        xi[e] = Parts<T>::im(a);
        yr[e] = Parts<T>::re(b);
        yi[e] = Parts<T>::im(b);
      }
      sa[0][q] = split8(xr);
      sb[0][q] = split8(yr);
      if constexpr (NP == 2) {
        sa[1][q] = split8(xi);
        sb[1][q] = split8(yi);
      }
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) {
        // conj(a) b: re = ar br + ai bi, im = ar bi - ai br
        facc[0][i][j] = mm6(sa[0][i], sb[0][j], facc[0][i][j]);
        if constexpr (NP == 2) {
          facc[0][i][j] = mm6(sa[1][i], sb[1][j], facc[0][i][j]);
          facc[1][i][j] = mm6(sa[0][i], sb[1][j], facc[1][i][j]);
          Split8 nai = sa[1][i];
          nai.h = -nai.h;
          nai.m = -nai.m;
          nai.l = -nai.l;
          facc[1][i][j] = mm6(nai, sb[0][j], facc[1][i][j]);
        }
      }
    {
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BM; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) dacc[c][i][j][e] += static_cast<double>(facc[c][i][j][e]);
            facc[c][i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
          }
    }
  }
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) dacc[c][i][j][e] += static_cast<double>(facc[c][i][j][e]);

  // fixed-order sum of the four wavefronts' tiles: (w0 + w2) + (w1 + w3)
  if (wave >= 2)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) red[wave - 2][c][i][j][lane] = dacc[c][i][j];
  __syncthreads();
  if (wave < 2)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) dacc[c][i][j] += red[wave][c][i][j][lane];
  __syncthreads();
  if (wave == 1)
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BM; ++j) red[0][c][i][j][lane] = dacc[c][i][j];
  __syncthreads();
  if (wave == 0) {
    double *out = part + (static_cast<int64_t>(blockIdx.z) * nmat + mat) * nb * nb * NP;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BM; ++j) {
        const d4 vr = dacc[0][i][j] + red[0][0][i][j][lane];
        const d4 vi = dacc[NP - 1][i][j] + red[0][NP - 1][i][j][lane];
        const int col = tn * TILE + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = tm * TILE + i * 16 + 4 * (lane >> 4) + e;
          if (row < nb && col < nb) {
            const int64_t o = (static_cast<int64_t>(row) * nb + col) * NP;
            out[o] = vr[e];
            if constexpr (NP == 2) out[o + 1] = vi[e];
          }
        }
      }
  }
}

template <int NP>
__global__ __launch_bounds__(256) void k_split_reduce(const double *__restrict__ part,
                                                      double *__restrict__ H,
                                                      double *__restrict__ S, int nb, int nsplit,
                                                      int nmat, double dV) {
  const int64_t nn = static_cast<int64_t>(nb) * nb * NP;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= nn * nmat) return;
  const int mat = static_cast<int>(idx / nn);
  const int64_t e = idx - mat * nn;
  double acc = 0.0;
  for (int s = 0; s < nsplit; ++s) acc += part[(static_cast<int64_t>(s) * nmat + mat) * nn + e];
  (mat ? S : H)[e] = dV * acc;
}

// C (double / complex double, [nb][nb]) -> transposed BF16 planes
// Ct[p][n][m] for p = hi, mid, lo (and the imaginary part in planes 3..5)
template <int NP>
__global__ __launch_bounds__(256) void k_split_c(const double *__restrict__ C, __bf16 *__restrict__ Ct,
                                                 int nb) {
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= nn) return;
  const int m = static_cast<int>(idx / nb), n = static_cast<int>(idx - static_cast<int64_t>(m) * nb);
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    // three BF16 parts of the FP64 coefficient, each rounded to nearest from
    // the remainder in FP64 (the remainders are exact)
    const double x = C[idx * NP + c];
    const uint32_t uh = bf16_rne(__float_as_uint(static_cast<float>(x)));
    const double r1 = x - static_cast<double>(__uint_as_float(uh));
    const uint32_t um = bf16_rne(__float_as_uint(static_cast<float>(r1)));
    const double r2 = r1 - static_cast<double>(__uint_as_float(um));
    const uint32_t ul = bf16_rne(__float_as_uint(static_cast<float>(r2)));
    const int64_t t = static_cast<int64_t>(n) * nb + m;
    Ct[(3 * c + 0) * nn + t] = top_half(uh);
    Ct[(3 * c + 1) * nn + t] = top_half(um);
    Ct[(3 * c + 2) * nn + t] = top_half(ul);
  }
}

// out[n][g] = sum_m C[m][n] src[m][g] (no conjugation): A[i=n][k=m] from the
// transposed planes, B[k=m][j=g] split on the fly. Each wavefront owns
// RB*16 rows (row group blockIdx.y) by 32 columns.
template <typename T, int RB>
__global__ __launch_bounds__(256) void k_rotate_split(const __bf16 *__restrict__ Ct,
                                                      const T *__restrict__ src,
                                                      T *__restrict__ dst, int nb, int64_t cols) {
  constexpr int NP = Parts<T>::n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int64_t g0 = static_cast<int64_t>(blockIdx.x) * 128 + wave * 32;
  const int n0 = blockIdx.y * RB * 16;
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  int64_t gc[2];
  bool gv[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    gc[cb] = g0 + cb * 16 + j;
    gv[cb] = gc[cb] < cols;
  }
  d4 dacc[NP][RB][2];
  f4 facc[NP][RB][2];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        dacc[c][i][q] = d4{0.0, 0.0, 0.0, 0.0};
        facc[c][i][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
  int steps = 0;
  for (int m0 = 0; m0 < nb; m0 += 32) {
    const int mb = m0 + 8 * kq;
    Split8 sa[NP][RB], sb[NP][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int n = n0 + rb * 16 + j;
#pragma unroll
      for (int c = 0; c < NP; ++c) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool in = n < nb && mb + e < nb;
          const int64_t t = static_cast<int64_t>(n) * nb + mb + e;
          const __bf16 zero = top_half(0u);
          sa[c][rb].h[e] = in ? Ct[(3 * c + 0) * nn + t] : zero;
          sa[c][rb].m[e] = in ? Ct[(3 * c + 1) * nn + t] : zero;
          sa[c][rb].l[e] = in ? Ct[(3 * c + 2) * nn + t] : zero;
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      float xr[8], xi[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool in = gv[cb] && mb + e < nb;
        const T v = in ? src[static_cast<int64_t>(mb + e) * cols + gc[cb]] : T{};
        xr[e] = Parts<T>::re(v);
        xi[e] = Parts<T>::im(v);
      }
      sb[0][cb] = split8(xr);
      if constexpr (NP == 2) sb[1][cb] = split8(xi);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        // C psi: re = Cr pr - Ci pi, im = Cr pi + Ci pr
        facc[0][rb][cb] = mm6(sa[0][rb], sb[0][cb], facc[0][rb][cb]);
        if constexpr (NP == 2) {
          Split8 nci = sa[1][rb];
          nci.h = -nci.h;
          nci.m = -nci.m;
          nci.l = -nci.l;
          facc[0][rb][cb] = mm6(nci, sb[1][cb], facc[0][rb][cb]);
          facc[1][rb][cb] = mm6(sa[0][rb], sb[1][cb], facc[1][rb][cb]);
          facc[1][rb][cb] = mm6(sa[1][rb], sb[0][cb], facc[1][rb][cb]);
        }
      }
    if (++steps == 8) {
      steps = 0;
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int e = 0; e < 4; ++e) dacc[c][i][q][e] += static_cast<double>(facc[c][i][q][e]);
            facc[c][i][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
          }
    }
  }
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      if (!gv[cb]) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + rb * 16 + 4 * kq + e;
        if (n >= nb) continue;
        const double vr = dacc[0][rb][cb][e] + static_cast<double>(facc[0][rb][cb][e]);
        T out;
        if constexpr (NP == 2) {
          const double vi = dacc[1][rb][cb][e] + static_cast<double>(facc[1][rb][cb][e]);
          out = T{static_cast<float>(vr), static_cast<float>(vi)};
        } else {
          out = static_cast<float>(vr);
        }
        dst[static_cast<int64_t>(n) * cols + gc[cb]] = out;
      }
    }
}

struct SplitPlanS {
  int tiles_n, tiles, nsplit;
  int64_t kchunk;
};

SplitPlanS plan_split(int nb, int64_t ng, int nmat, int tile) {
  SplitPlanS p;
  p.tiles_n = (nb + tile - 1) / tile;
  p.tiles = p.tiles_n * p.tiles_n;
  const int64_t want = std::max<int64_t>(1, 512 / (p.tiles * nmat));
  const int64_t kmax_split = std::max<int64_t>(1, ng / 2048);
  const int64_t nsplit = std::min(want, kmax_split);
  int64_t kchunk = (ng + nsplit - 1) / nsplit;
  kchunk = (kchunk + 127) / 128 * 128;
  p.kchunk = kchunk;
  p.nsplit = static_cast<int>((ng + kchunk - 1) / kchunk);
  return p;
}

template <typename T, int BM>
int subspace_split_t(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                     int nb, void *H, void *S, hipStream_t st) {
  constexpr int NP = Parts<T>::n;
  const int nmat = Spsi ? 2 : 1;
  const SplitPlanS p = plan_split(nb, s->ng, nmat, 16 * BM);
  const int64_t need = static_cast<int64_t>(p.nsplit) * nmat * nb * nb * NP;
  if (need > static_cast<int64_t>(s->ws.part_elems))
    return fail(GPAW_EINVAL, "subspace workspace too small");
  dim3 grid(p.tiles, nmat, p.nsplit);
  k_subspace_split<T, BM><<<grid, 256, 0, st>>>(
      static_cast<const T *>(psi), static_cast<const T *>(Hpsi),
      static_cast<const T *>(Spsi ? Spsi : Hpsi), s->ws.part, nb, s->ng, p.kchunk, p.tiles_n,
      nmat);
  const int64_t tot = static_cast<int64_t>(nb) * nb * nmat * NP;
  k_split_reduce<NP><<<static_cast<unsigned>((tot + 255) / 256), 256, 0, st>>>(
      s->ws.part, static_cast<double *>(H), static_cast<double *>(S), nb, p.nsplit, nmat, s->dV);
  return GPAW_OK;
}

template <typename T, int RB>
int rotate_split_t(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                   void *dst, hipStream_t st) {
  constexpr int NP = Parts<T>::n;
  __bf16 *Ct = reinterpret_cast<__bf16 *>(s->ws.split);
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  k_split_c<NP><<<static_cast<unsigned>((nn + 255) / 256), 256, 0, st>>>(
      static_cast<const double *>(C), Ct, nb);
  dim3 grid(static_cast<unsigned>((cols + 127) / 128), (nb + RB * 16 - 1) / (RB * 16));
  k_rotate_split<T, RB><<<grid, 256, 0, st>>>(Ct, static_cast<const T *>(src),
                                              static_cast<T *>(dst), nb, cols);
  return GPAW_OK;
}

}  // namespace

size_t split_part_elems(int nb, bool cplx) {
  const int64_t tile = cplx ? 32 : 64;
  const int64_t bound = std::max<int64_t>(512 * tile * tile, 2 * int64_t(nb) * nb);
  return static_cast<size_t>(bound) * (cplx ? 2 : 1);
}

size_t split_c_bytes(int nb, bool cplx) {
  return static_cast<size_t>(nb) * nb * 3 * (cplx ? 2 : 1) * sizeof(__bf16);
}

int launch_subspace_split(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                          int nb, void *H, void *S, hipStream_t st) {
  if (s->dtype == GPAW_C64) return subspace_split_t<z32, 2>(s, psi, Hpsi, Spsi, nb, H, S, st);
  return subspace_split_t<float, 4>(s, psi, Hpsi, Spsi, nb, H, S, st);
}

int launch_rotate_split(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                        void *dst, hipStream_t st) {
  if (cols == 0) return GPAW_OK;
  if (s->dtype == GPAW_C64) return rotate_split_t<z32, 2>(s, C, src, nb, cols, dst, st);
  return rotate_split_t<float, 4>(s, C, src, nb, cols, dst, st);
}

}  // namespace gfd
