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
// is FP32, promotes every 256 terms (4 steps of 64).
//
// MFMA layout (16x16x32, BF16 in, FP32 out): lane l supplies A[i = l%16]
// [8 values of k] and B[8 values of k][j = l%16] from the same k set, and
// accumulator element r of lane l is D[4*(l/16) + r][l%16] (measured).
#include <algorithm>

#include "internal.h"
#include "tile_order.h"

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

// ---------------------------------------------------------------------------
// LDS-staged split products. A workgroup stages 32-wide K slices of both
// operands in LDS, splitting every element once into its three BF16 parts
// (planes h, m, l); the next slice is fetched from global memory while the
// matrix cores work on the current one. The planes are unpadded with their
// 16-byte chunks XOR-swizzled per row (swz32, swz64), so that both the
// staging stores (several chunks of a row, a pair of rows per 8 lanes) and
// the fragment reads (one chunk of 8 consecutive rows per 8 lanes) fall on
// distinct banks: the bank-conflict counter reads zero for them, against
// about 5 conflict cycles per LDS instruction with rows padded by 16 bytes.
// Workgroup ids are laid out so that the workgroups sharing an operand slice
// (same K chunk for the subspace products, same grid columns for the
// rotation) land on the same XCD and find it in that XCD's L2.
constexpr int KS = 32;

// offset (BF16 values) of 16-byte chunk c of row r: rows of 32 values (four
// chunks), chunk c ^ ((r >> 1) & 3) (rows alternate between the two halves
// of the banks; within 8 rows the swizzle separates the rest)
__device__ inline int swz32(int r, int c) { return r * 32 + 8 * (c ^ ((r >> 1) & 3)); }
// rows of 64 values (eight chunks), chunk c ^ s(r) with s(r) = 4 (r & 1) +
// ((r >> 1) & 3): the pair of rows a staging store covers gets complementary
// halves, eight consecutive rows distinct chunks
__device__ inline int swz64(int r, int c) { return r * 64 + 8 * (c ^ (((r & 1) << 2) | ((r >> 1) & 3))); }

__device__ inline void split_to(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
  const uint32_t uh = bf16_rne(__float_as_uint(x));
  const float r1 = x - __uint_as_float(uh);
  const uint32_t um = bf16_rne(__float_as_uint(r1));
  const float r2 = r1 - __uint_as_float(um);
  h = top_half(uh);
  m = top_half(um);
  l = top_half(__float_as_uint(r2));
}

// two FP32 values -> two BF16 values rounded to nearest even, the first in
// the low half (the hardware pair conversion, written out so that the
// operand order is explicit: the compiler's own vector form of it was found
// to return the first element's result for both on this toolchain)
__device__ inline uint32_t cvt2_bf16(float a, float b) {
  uint32_t r;
  asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// eight consecutive values (real or one part of complex) -> three planes,
// the same exact split as split_to (hi = bf16(x), mid = bf16(x - hi),
// lo = x - hi - mid, each remainder exact), two values per conversion
__device__ inline void split_store8(const float *x, __bf16 *ph, __bf16 *pm, __bf16 *pl) {
  uint32_t h[4], m[4], l[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t hq = cvt2_bf16(x[2 * q], x[2 * q + 1]);
    const float r0 = x[2 * q] - __uint_as_float(hq << 16);
    const float r1 = x[2 * q + 1] - __uint_as_float(hq & 0xFFFF0000u);
    const uint32_t mq = cvt2_bf16(r0, r1);
    const float s0 = r0 - __uint_as_float(mq << 16);
    const float s1 = r1 - __uint_as_float(mq & 0xFFFF0000u);
    h[q] = hq;
    m[q] = mq;
    l[q] = cvt2_bf16(s0, s1);  // exact: at most 8 significant bits
  }
  *reinterpret_cast<uint4 *>(ph) = make_uint4(h[0], h[1], h[2], h[3]);
  *reinterpret_cast<uint4 *>(pm) = make_uint4(m[0], m[1], m[2], m[3]);
  *reinterpret_cast<uint4 *>(pl) = make_uint4(l[0], l[1], l[2], l[3]);
}

// eight consecutive values -> their high BF16 parts only (the one-product
// rotation near the identity)
__device__ inline void hi_store8(const float *x, __bf16 *ph) {
  bf8 h;
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = top_half(bf16_rne(__float_as_uint(x[e])));
  *reinterpret_cast<bf8 *>(ph) = h;
}

// eight consecutive values p[0..7] (zero where e >= avail or !row_ok), as
// 16-byte loads when the address allows
template <typename T>
__device__ inline void load8(const T *p, bool row_ok, int64_t avail, T *v) {
  if (row_ok && avail >= 8 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    constexpr int W = static_cast<int>(sizeof(T) * 8 / 16);  // 16-byte words
    f4v w[W];
#pragma unroll
    for (int q = 0; q < W; ++q) w[q] = reinterpret_cast<const f4v *>(p)[q];
    __builtin_memcpy(v, w, sizeof(T) * 8);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (row_ok && e < avail) ? p[e] : T{};
  }
}

// hi_only: the high plane alone (the others are left unset)
__device__ inline Split8 frag(const __bf16 *plane0, int plane_stride, int off,
                              bool hi_only = false) {
  Split8 f;
  f.h = *reinterpret_cast<const bf8 *>(plane0 + off);
  if (!hi_only) {
    f.m = *reinterpret_cast<const bf8 *>(plane0 + plane_stride + off);
    f.l = *reinterpret_cast<const bf8 *>(plane0 + 2 * plane_stride + off);
  }
  return f;
}

// part[(split*nmat + mat)][nb][nb] (double / complex double) =
//   sum_{k in chunk} conj(A[n][k]) B_mat[m][k].
// Workgroup tile TM x TM (TM = 32 WT), four wavefronts in a 2 x 2 layout,
// each owning WT x WT 16x16 blocks; FP32 tiles are added into FP64
// accumulators after every 32-wide step.
template <typename T, int WT>
__global__ __launch_bounds__(256) void k_sub_lds(const T *__restrict__ A, const T *__restrict__ B0,
                                                 const T *__restrict__ B1, double *__restrict__ part,
                                                 int nb, int64_t ng, int64_t kchunk, int tiles_n,
                                                 int nmat, int nsplit, int sb) {
  constexpr int NP = Parts<T>::n;
  constexpr int TM = 32 * WT;
  constexpr int PS = TM * KS;  // plane stride (bf16): rows of KS values, unpadded
  constexpr int RPP = 256 / 4;   // rows staged per pass (4 threads x 8 values per row)
  __shared__ __attribute__((aligned(16))) __bf16 sA[3 * NP * PS];
  __shared__ __attribute__((aligned(16))) __bf16 sB[3 * NP * PS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
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
  const int nsteps = kb < ke ? static_cast<int>((ke - kb + KS - 1) / KS) : 0;

  // staging: thread -> row r0 + RPP*pass, values k = 8c..8c+7 of the slice
  const int sr = tid >> 2, sc = (tid & 3) * 8;
  constexpr int PASSES = TM / RPP;
  float ra[PASSES][NP][8], rbv[PASSES][NP][8];
  auto fetch = [&](int step) {
    const int64_t k0 = kb + static_cast<int64_t>(step) * KS + sc;
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int rowa = tm * TM + ps * RPP + sr, rowb = tn * TM + ps * RPP + sr;
      const T *pa = A + static_cast<int64_t>(rowa < nb ? rowa : 0) * ng;
      const T *pb = B + static_cast<int64_t>(rowb < nb ? rowb : 0) * ng;
      T va[8], vb[8];
      load8(pa + k0, rowa < nb, ke - k0, va);
      load8(pb + k0, rowb < nb, ke - k0, vb);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        ra[ps][0][e] = Parts<T>::re(va[e]);
        rbv[ps][0][e] = Parts<T>::re(vb[e]);
        if constexpr (NP == 2) {
          ra[ps][NP - 1][e] = Parts<T>::im(va[e]);
          rbv[ps][NP - 1][e] = Parts<T>::im(vb[e]);
        }
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        const int row = ps * RPP + sr;
        const int o = (c * 3) * PS + swz32(row, sc >> 3);
        split_store8(ra[ps][c], sA + o, sA + o + PS, sA + o + 2 * PS);
        split_store8(rbv[ps][c], sB + o, sB + o + PS, sB + o + 2 * PS);
      }
  };

  const int wr = wave >> 1, wc = wave & 1;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  d4 dacc[NP][WT][WT];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int j = 0; j < WT; ++j) dacc[c][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (nsteps > 0) fetch(0);
  for (int step = 0; step < nsteps; ++step) {
    __syncthreads();
    stage();
    __syncthreads();
    if (step + 1 < nsteps) fetch(step + 1);
    Split8 fa[NP][WT];
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int c = 0; c < NP; ++c)
        fa[c][i] = frag(sA + (c * 3) * PS, PS, swz32(wr * 16 * WT + i * 16 + fr, fk >> 3));
#pragma unroll
    for (int j = 0; j < WT; ++j) {
      Split8 fb[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c)
        fb[c] = frag(sB + (c * 3) * PS, PS, swz32(wc * 16 * WT + j * 16 + fr, fk >> 3));
#pragma unroll
      for (int i = 0; i < WT; ++i) {
        const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        // conj(a) b: re = ar br + ai bi, im = ar bi - ai br (the two parts of
        // im in tiles of their own, subtracted in FP64: no fragment negated)
        f4 re = mm6(fa[0][i], fb[0], z);
        if constexpr (NP == 2) {
          re = mm6(fa[1][i], fb[1], re);
          const f4 im1 = mm6(fa[0][i], fb[1], z);
          const f4 im2 = mm6(fa[1][i], fb[0], z);
#pragma unroll
          for (int e = 0; e < 4; ++e)
            dacc[1][i][j][e] += static_cast<double>(im1[e]) - static_cast<double>(im2[e]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) dacc[0][i][j][e] += static_cast<double>(re[e]);
      }
    }
  }

  double *out = part + (static_cast<int64_t>(split) * nmat + mat) * nb * nb * NP;
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) {
      const int col = tn * TM + wc * 16 * WT + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = tm * TM + wr * 16 * WT + i * 16 + 4 * (lane >> 4) + e;
        if (row < nb && col < nb) {
          const int64_t o = (static_cast<int64_t>(row) * nb + col) * NP;
          out[o] = dacc[0][i][j][e];
          if constexpr (NP == 2) out[o + 1] = dacc[NP - 1][i][j][e];
        }
      }
    }
}

template <int NP>
__global__ __launch_bounds__(256) void k_split_reduce(const double *__restrict__ part,
                                                      double *__restrict__ H,
                                                      double *__restrict__ S, int nb, int nsplit,
                                                      int nmat, double dV, int tile) {
  const int64_t nn = static_cast<int64_t>(nb) * nb * NP;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= nn * nmat) return;
  const int mat = static_cast<int>(idx / nn);
  const int64_t e = idx - mat * nn;
  const int64_t el = e / NP;
  const int c = static_cast<int>(e - el * NP);
  const int r = static_cast<int>(el / nb), q = static_cast<int>(el - static_cast<int64_t>(r) * nb);
  // entries of tiles below the diagonal were not formed: the thread of the
  // mirror entry writes them (as its conjugate)
  if (r / tile > q / tile) return;
  double acc = 0.0;
  for (int s = 0; s < nsplit; ++s) acc += part[(static_cast<int64_t>(s) * nmat + mat) * nn + e];
  double *M = mat ? S : H;
  M[e] = dV * acc;
  if (r / tile < q / tile) M[(static_cast<int64_t>(q) * nb + r) * NP + c] = c ? -dV * acc : dV * acc;
}

// flag = 1 when max |C - I| <= 2^-21: the rotation by C = I + E then needs only
// the high BF16 parts of E (their product error, about 2^-8 |E| per term, stays
// below the FP32 resolution of the result), else 0
template <int NP>
__global__ __launch_bounds__(1024) void k_offid_small(const double *__restrict__ C, int nb,
                                                      int32_t *__restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int64_t nn = static_cast<int64_t>(nb) * nb;
  bool big = false;
  for (int64_t idx = threadIdx.x; idx < nn; idx += 1024) {
    const int m = static_cast<int>(idx / nb), n = static_cast<int>(idx - static_cast<int64_t>(m) * nb);
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      const double e = C[idx * NP + c] - (c == 0 && m == n ? 1.0 : 0.0);
      big |= !(fabs(e) <= 0x1p-21);
    }
  }
  if (big) bad = 1;  // any lane; a plain LDS store of the same value
  __syncthreads();
  if (threadIdx.x == 0) *flag = bad ? 0 : 1;
}

// C (double / complex double, [nb][nb]) -> transposed BF16 planes
// Ct[p][n][m] for p = hi, mid, lo (and the imaginary part in planes 3..5),
// rows padded with zeros to nbp = nb rounded up to the 64-wide K step, so
// that every 16-byte row fragment a rotation step reads is in bounds.
// Cf (if set): the high parts once more, fragment-major for the column-panel
// rotation: block (part c, rows 16 rb.., K step ks) is 512 values in lane
// order, lane l = 16 fq + fr holding rows 16 rb + fr, values m = 32 ks +
// 8 fq .. +7, so that a wavefront reads a fragment as one contiguous 1 KB.
template <int NP>
__global__ __launch_bounds__(256) void k_split_c(const double *__restrict__ C, __bf16 *__restrict__ Ct,
                                                 int nb, int nbp, int minus_id,
                                                 __bf16 *__restrict__ Cf) {
  const int64_t np = static_cast<int64_t>(nb) * nbp;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= np) return;
  // idx = m nb + n, the element C[m][n] for m < nb
  const int m = static_cast<int>(idx / nb), n = static_cast<int>(idx - static_cast<int64_t>(m) * nb);
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    // three BF16 parts of the FP64 coefficient, each rounded to nearest from
    // the remainder in FP64 (the remainders are exact)
    // minus_id: the planes of C - I (the rotation then adds the source back)
    const double x = m < nb ? C[idx * NP + c] - (minus_id && c == 0 && m == n ? 1.0 : 0.0) : 0.0;
    const uint32_t uh = bf16_rne(__float_as_uint(static_cast<float>(x)));
    const double r1 = x - static_cast<double>(__uint_as_float(uh));
    const uint32_t um = bf16_rne(__float_as_uint(static_cast<float>(r1)));
    const double r2 = r1 - static_cast<double>(__uint_as_float(um));
    const uint32_t ul = bf16_rne(__float_as_uint(static_cast<float>(r2)));
    const int64_t t = static_cast<int64_t>(n) * nbp + m;
    Ct[(3 * c + 0) * np + t] = top_half(uh);
    Ct[(3 * c + 1) * np + t] = top_half(um);
    Ct[(3 * c + 2) * np + t] = top_half(ul);
    if (Cf) {
      const int64_t blk = (static_cast<int64_t>(c) * ((nb + 15) / 16) + (n >> 4)) * (nbp / 32) + (m >> 5);
      Cf[blk * 512 + (((m >> 3) & 3) * 16 + (n & 15)) * 8 + (m & 7)] = top_half(uh);
    }
  }
}

// out[n][g] = sum_m C[m][n] src[m][g] (no conjugation). A[i=n][k=m] comes
// from the pre-split transposed planes of C (rows padded to nbp); the src
// slice (KR rows m x TN columns g) is split once and stored column-major in
// LDS, so that the B fragment B[k=m][j=g] of a lane is eight consecutive
// values. FP32 tiles are added into FP64 accumulators every 4 steps (256
// terms). A step spans 64 values of m: with one wavefront per SIMD the
// loads of the next step are in flight during one step of matrix work, so
// the step is made long enough to keep many bytes in flight. The loads are
// unconditional (row, column and step indices clamped; clamped src rows meet
// zero padding in Ct, clamped output rows and columns are not stored).
// ADDSRC: Ct holds C - I and the result is src + (C - I)^T src. Two kernels
// are launched for it and the device decides which one works: when *fewer
// is nonzero (|C - I| small, see k_offid_small) the ONEP one multiplies the
// high BF16 parts only (one product instead of six; its LDS holds one plane
// per part, so four workgroups fit a CU), else the six-product one. Both are
// persistent (a resident-sized grid walks the output tiles, each XCD a
// contiguous range of them), so the one that exits costs one launch.
constexpr int KR = 64;     // K values per rotation step

template <typename T, int WT, bool ADDSRC, bool ONEP>
__global__ __launch_bounds__(256) void k_rot_lds(const __bf16 *__restrict__ Ct,
                                                 const T *__restrict__ src, T *__restrict__ dst,
                                                 int nb, int nbp, int64_t cols, int ntiles_n,
                                                 int64_t gtiles, int upper,
                                                 const int32_t *__restrict__ fewer) {
  constexpr int NP = Parts<T>::n;
  constexpr int TM = 32 * WT;
  constexpr int PS = TM * KR;  // plane stride: rows of KR values, swizzled (swz64)
  constexpr int NPL = ONEP ? 1 : 3;  // BF16 planes staged per part
  static_assert(ADDSRC || !ONEP, "one product only near the identity");
  __shared__ __attribute__((aligned(16))) __bf16 sA[NPL * NP * PS];
  __shared__ __attribute__((aligned(16))) __bf16 sB[NPL * NP * PS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (ADDSRC && ((*fewer != 0) != ONEP)) return;  // the other kernel's case
  // output tiles (column block gtile, row tile ntile), the row tiles of one
  // column block consecutive
  const int x = blockIdx.x & 7;
  int64_t it, it_end, it_step;
  if constexpr (ADDSRC) {
    const int64_t items = gtiles * ntiles_n, per = (items + 7) / 8;
    it = x * per + (blockIdx.x >> 3);
    it_end = std::min(items, (x + 1) * per);
    it_step = gridDim.x >> 3;
  } else {
    const int64_t jj = blockIdx.x >> 3;
    const int64_t gt = (jj / ntiles_n) * 8 + x;
    it = gt * ntiles_n + jj % ntiles_n;
    it_end = gt < gtiles ? it + 1 : it;
    it_step = 1;
  }
  for (; it < it_end; it += it_step) {
  const int ntile = static_cast<int>(it % ntiles_n);
  const int64_t gtile = it / ntiles_n;
  const int64_t np = static_cast<int64_t>(nb) * nbp;
  const int n0 = ntile * TM;
  const int64_t g0 = gtile * TM;
  // an upper-triangular C (m <= n) needs rows m < n0 + TM only
  const int mend = upper ? std::min(nb, n0 + TM) : nb;
  const int nsteps = (mend + KR - 1) / KR;

  // A staging: row n = n0 + tid/4 (+64 per pass), values m = sc..sc+7 and
  // sc+32..sc+39 per plane
  constexpr int PASSES = TM / 64;
  const int sr = tid >> 2, sc = (tid & 3) * 8;
  bf8 ca[PASSES][NP][3][2];
  // B staging: column g = g0 + (tid % TM), values m = bm .. bm+MPT-1
  constexpr int MPT = KR * TM / 256;  // real 32, complex 16
  const int bg = tid % TM, bm = (tid / TM) * MPT;
  float rb[NP][MPT];
  const T *srcg = src + std::min<int64_t>(g0 + bg, cols - 1);
  constexpr bool one = ONEP;
  auto fetch = [&](int step) {
    const int m0 = std::min(step, nsteps - 1) * KR;
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int n = std::min(n0 + ps * 64 + sr, nb - 1);
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int p = 0; p < 3; ++p)
          if (p == 0 || !one)  // one product: the high parts only
#pragma unroll
            for (int h = 0; h < 2; ++h)
              ca[ps][c][p][h] = *reinterpret_cast<const bf8 *>(
                  Ct + (3 * c + p) * np + static_cast<int64_t>(n) * nbp + m0 + sc + 32 * h);
    }
    if (m0 + KR <= nb) {  // a whole step of rows: no clamping, one row offset per value
      const T *rowp = srcg + static_cast<int64_t>(m0 + bm) * cols;
#pragma unroll
      for (int e = 0; e < MPT; ++e) {
        const T v = rowp[static_cast<int64_t>(e) * cols];
        rb[0][e] = Parts<T>::re(v);
        if constexpr (NP == 2) rb[NP - 1][e] = Parts<T>::im(v);
      }
    } else {
#pragma unroll
      for (int e = 0; e < MPT; ++e) {
        const int m = std::min(m0 + bm + e, nb - 1);
        const T v = srcg[static_cast<int64_t>(m) * cols];
        rb[0][e] = Parts<T>::re(v);
        if constexpr (NP == 2) rb[NP - 1][e] = Parts<T>::im(v);
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int p = 0; p < 3; ++p)
          if (p == 0 || !one)
#pragma unroll
            for (int h = 0; h < 2; ++h)
              *reinterpret_cast<bf8 *>(sA + (c * NPL + p) * PS +
                                       swz64(ps * 64 + sr, (sc >> 3) + 4 * h)) = ca[ps][c][p][h];
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int h = 0; h < MPT / 8; ++h) {
        const int o = (c * NPL) * PS + swz64(bg, (bm >> 3) + h);
        if constexpr (ONEP) hi_store8(rb[c] + 8 * h, sB + o);
        else split_store8(rb[c] + 8 * h, sB + o, sB + o + PS, sB + o + 2 * PS);
      }
  };

  const int wr = wave >> 1, wc = wave & 1;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  // complex: fx holds Ci pi, subtracted from the real part when the tile is
  // promoted (so that no fragment is negated)
  d4 dacc[NP][WT][WT];
  f4 facc[NP][WT][WT], fx[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) {
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        dacc[c][i][j] = d4{0.0, 0.0, 0.0, 0.0};
        facc[c][i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
      fx[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
  fetch(0);
  auto run_step = [&](int step) {
    __syncthreads();
    stage();
    __syncthreads();
    fetch(step + 1);  // clamped: the last one re-reads the final step, unused
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      Split8 fa[NP][WT];
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int c = 0; c < NP; ++c)
          fa[c][i] = frag(sA + (c * NPL) * PS, PS, swz64(wr * 16 * WT + i * 16 + fr, 4 * kh + (fk >> 3)),
                          one);
#pragma unroll
      for (int j = 0; j < WT; ++j) {
        Split8 fb[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c)
          fb[c] = frag(sB + (c * NPL) * PS, PS, swz64(wc * 16 * WT + j * 16 + fr, 4 * kh + (fk >> 3)),
                       one);
#pragma unroll
        for (int i = 0; i < WT; ++i) {
          // C psi: re = Cr pr - Ci pi, im = Cr pi + Ci pr
          if (ADDSRC && one) {
            facc[0][i][j] = mm(fa[0][i].h, fb[0].h, facc[0][i][j]);
            if constexpr (NP == 2) {
              fx[i][j] = mm(fa[1][i].h, fb[1].h, fx[i][j]);
              facc[1][i][j] = mm(fa[0][i].h, fb[1].h, facc[1][i][j]);
              facc[1][i][j] = mm(fa[1][i].h, fb[0].h, facc[1][i][j]);
            }
          } else {
            facc[0][i][j] = mm6(fa[0][i], fb[0], facc[0][i][j]);
            if constexpr (NP == 2) {
              fx[i][j] = mm6(fa[1][i], fb[1], fx[i][j]);
              facc[1][i][j] = mm6(fa[0][i], fb[1], facc[1][i][j]);
              facc[1][i][j] = mm6(fa[1][i], fb[0], facc[1][i][j]);
            }
          }
        }
      }
    }
  };
  // FP32 tiles into the FP64 accumulators after every 4 steps (the step loop
  // is unrolled by 4 so that this needs no test per step). The one-product
  // rotation sums terms of size 2^-21 |psi| and keeps its FP32 tile: its
  // rounding is far below that of the FP32 result.
  auto promote = [&]() {
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int j = 0; j < WT; ++j) {
#pragma unroll
        for (int c = 0; c < NP; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            double v = static_cast<double>(facc[c][i][j][e]);
            if (NP == 2 && c == 0) v -= static_cast<double>(fx[i][j][e]);
            dacc[c][i][j][e] += v;
          }
#pragma unroll
        for (int c = 0; c < NP; ++c) facc[c][i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        fx[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
  };
  int step = 0;
  if constexpr (!ONEP) {
    for (; step + 4 <= nsteps; step += 4) {
      run_step(step);
      run_step(step + 1);
      run_step(step + 2);
      run_step(step + 3);
      promote();
    }
  }
  for (; step < nsteps; ++step) run_step(step);
  if constexpr (!ONEP) promote();
#pragma unroll
  for (int i = 0; i < WT; ++i) {
    // ADDSRC: the source values of this row band are loaded together, from
    // clamped positions and without branches (a load inside the store's
    // bounds test would be waited for on its own)
    T sv[WT][4];
    if constexpr (ADDSRC) {
#pragma unroll
      for (int j = 0; j < WT; ++j) {
        const int64_t g = std::min<int64_t>(g0 + wc * 16 * WT + j * 16 + (lane & 15), cols - 1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = std::min(n0 + wr * 16 * WT + i * 16 + 4 * (lane >> 4) + e, nb - 1);
          sv[j][e] = src[static_cast<int64_t>(n) * cols + g];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < WT; ++j) {
      const int64_t g = g0 + wc * 16 * WT + j * 16 + (lane & 15);
      if (g >= cols) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + wr * 16 * WT + i * 16 + 4 * (lane >> 4) + e;
        if (n >= nb) continue;
        double vr = ONEP ? static_cast<double>(facc[0][i][j][e]) -
                               (NP == 2 ? static_cast<double>(fx[i][j][e]) : 0.0)
                         : dacc[0][i][j][e];
        double vi = ONEP ? facc[NP - 1][i][j][e] : dacc[NP - 1][i][j][e];
        if constexpr (ADDSRC) {
          vr += Parts<T>::re(sv[j][e]);
          if constexpr (NP == 2) vi += Parts<T>::im(sv[j][e]);
        }
        T o;
        if constexpr (NP == 2) o = T{static_cast<float>(vr), static_cast<float>(vi)};
        else o = static_cast<float>(vr);
        dst[static_cast<int64_t>(n) * cols + g] = o;
      }
    }
  }
  }  // output tiles
}
// The one-product rotation by an upper-triangular C = I + E (the case the
// orthonormality correction produces: E = L^-H - I, max |E| <= 2^-21) as a
// column-panel stream: each source value is read from HBM once and each
// output value written once. A workgroup owns TN grid columns and all nb
// output rows. It walks the rows in chunks of 8 wavefronts x 16 RB rows;
// the source rows of a chunk are loaded in the accumulator layout, kept in
// registers for the add-back, and their high BF16 parts appended to an LDS
// panel (column-major, [part][column][m], rows padded by 8 values so that
// the 16-byte fragment reads of 16 columns fall on distinct banks). Output
// row n only needs source rows m <= n, so a chunk only needs the panel rows
// written so far. E's fragments come from global memory through an NS-stage
// register ring, from a fragment-major copy of E's high parts (one
// contiguous 1 KB per fragment, so that each load touches the fewest cache
// lines; E is shared by every workgroup and stays in L2). The next chunk's source rows are loaded during
// the current chunk's products. Complex: re = Er sr - Ei si (the second
// term in an accumulator of its own, so no fragment is negated),
// im = Er si + Ei sr. The FP32 sums (terms of 2^-21 |src| and below) are
// added to the source in FP64 and rounded once.
constexpr int NEAR_PITCH_MAX = 1024 + 8;  // nb <= 1024

template <typename T, int TN, int RB, int NS>
__global__ __launch_bounds__(512) void k_rot_near(const __bf16 *__restrict__ Cf,
                                                  const T *__restrict__ src, T *__restrict__ dst,
                                                  int nb, int nbp, int64_t cols, int64_t gblocks,
                                                  const int32_t *__restrict__ fewer) {
  constexpr int NP = Parts<T>::n;
  constexpr int CB = TN / 16;
  constexpr int CHUNK = 128 * RB;  // rows per chunk: 8 wavefronts x RB blocks of 16
  static_assert(RB == 1 || RB == 2, "one or two row blocks per wavefront");
  static_assert((NS & (NS - 1)) == 0 && NS >= 2, "ring stages: a power of two");
  __shared__ __attribute__((aligned(16))) __bf16 pan[NP * TN * NEAR_PITCH_MAX];
  if (*fewer == 0) return;  // the six-product kernel's case
  const int pitch = nbp + 8;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, fr = lane & 15, fq = lane >> 4;
  const int nrb = (nb + 15) / 16, nks = nbp / 32;  // fragment blocks of Cf
  const int nk_all = (nb + 31) / 32;  // 32-wide K steps over all rows
  const int mrows = nk_all * 32;      // panel rows the products read
  const int nchunks = (nb + CHUNK - 1) / CHUNK;
  // each XCD a contiguous range of column blocks
  const int x = blockIdx.x & 7;
  const int64_t per = (gblocks + 7) / 8;
  const int64_t blk_end = std::min<int64_t>(gblocks, (x + 1) * per);
  const int64_t blk_step = gridDim.x >> 3;

  // first row of row block rb of this wavefront in chunk ci: blocks w and
  // 15 - w of the chunk's 16, so that every wavefront carries the same share
  // of the triangle
  auto rowblk = [&](int ci, int rb) { return ci * CHUNK + 16 * (rb == 0 ? wave : 15 - wave); };
  T sc[RB][CB][4], sn[RB][CB][4];
  auto load_src = [&](int64_t g0, int ci, T (&sv)[RB][CB][4]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = std::min(rowblk(ci, rb) + 4 * fq + e, nb - 1);
        const T *row = src + static_cast<int64_t>(n) * cols;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          sv[rb][cb][e] = row[std::min<int64_t>(g0 + 16 * cb + fr, cols - 1)];
      }
  };

  for (int64_t blk = x * per + (blockIdx.x >> 3); blk < blk_end; blk += blk_step) {
    const int64_t g0 = blk * TN;
    load_src(g0, 0, sc);
    for (int ci = 0; ci < nchunks; ++ci) {
      int r0[RB], nk[RB], nkmax = 0;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        r0[rb] = rowblk(ci, rb);
        // upper triangular: rows r0 .. r0 + 15 need m < r0 + 16
        nk[rb] = r0[rb] < nb ? std::min(nk_all, (r0[rb] + 16 + 31) / 32) : 0;
        nkmax = std::max(nkmax, nk[rb]);
      }
      // panel rows of this chunk: high parts, zero past nb
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int nbase = r0[rb] + 4 * fq;
        if (nbase < mrows) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int c = 0; c < NP; ++c) {
              uint32_t w[2];
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                uint32_t hv[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                  const int e = 2 * h + q;
                  const float v = c ? Parts<T>::im(sc[rb][cb][e]) : Parts<T>::re(sc[rb][cb][e]);
                  hv[q] = nbase + e < nb ? bf16_rne(__float_as_uint(v)) >> 16 : 0u;
                }
                w[h] = hv[0] | (hv[1] << 16);
              }
              *reinterpret_cast<uint2 *>(pan + (c * TN + 16 * cb + fr) * pitch + nbase) =
                  make_uint2(w[0], w[1]);
            }
        }
      }
      bf8 ring[NS][RB][NP];
      auto load_a = [&](int slot, int k) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          if (k < nk[rb])  // then r0 < nb
#pragma unroll
            for (int c = 0; c < NP; ++c)
              ring[slot][rb][c] = *reinterpret_cast<const bf8 *>(
                  Cf + ((static_cast<int64_t>(c) * nrb + (r0[rb] >> 4)) * nks + k) * 512 + 8 * lane);
      };
#pragma unroll
      for (int s = 0; s < NS - 1; ++s) load_a(s, s);
      __syncthreads();  // the chunk's panel rows are written
      if (ci + 1 < nchunks) load_src(g0, ci + 1, sn);

      f4 acc[RB][CB][NP == 2 ? 3 : 1];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int q = 0; q < (NP == 2 ? 3 : 1); ++q) acc[rb][cb][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int k0 = 0; k0 < nkmax; k0 += NS) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int k = k0 + s;
          load_a((s + NS - 1) & (NS - 1), k + NS - 1);
          if (k < nkmax) {
            bf8 b[CB][NP];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
              for (int c = 0; c < NP; ++c)
                b[cb][c] = *reinterpret_cast<const bf8 *>(pan + (c * TN + 16 * cb + fr) * pitch +
                                                          32 * k + 8 * fq);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
              if (k < nk[rb])
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                const bf8 ar = ring[s][rb][0];
                acc[rb][cb][0] = mm(ar, b[cb][0], acc[rb][cb][0]);
                if constexpr (NP == 2) {
                  const bf8 ai = ring[s][rb][1];
                  acc[rb][cb][1] = mm(ai, b[cb][1], acc[rb][cb][1]);
                  acc[rb][cb][2] = mm(ar, b[cb][1], acc[rb][cb][2]);
                  acc[rb][cb][2] = mm(ai, b[cb][0], acc[rb][cb][2]);
                }
              }
          }
        }
      }
      {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int64_t g = g0 + 16 * cb + fr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int n = r0[rb] + 4 * fq + e;
              if (n >= nb || g >= cols) continue;
              const T v = sc[rb][cb][e];
              T o;
              if constexpr (NP == 2) {
                const double re = static_cast<double>(Parts<T>::re(v)) +
                                  (static_cast<double>(acc[rb][cb][0][e]) -
                                   static_cast<double>(acc[rb][cb][1][e]));
                const double im = static_cast<double>(Parts<T>::im(v)) +
                                  static_cast<double>(acc[rb][cb][2][e]);
                o = T{static_cast<float>(re), static_cast<float>(im)};
              } else {
                o = static_cast<float>(static_cast<double>(v) +
                                       static_cast<double>(acc[rb][cb][0][e]));
              }
              dst[static_cast<int64_t>(n) * cols + g] = o;
            }
          }
      }
      if (ci + 1 < nchunks) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) sc[rb][cb][e] = sn[rb][cb][e];
      }
    }
    __syncthreads();  // every wavefront is done with the panel
  }
}

struct SplitPlanS {
  int tiles_n, tiles, nsplit;
  int64_t kchunk;
};

// split-K over ~512 workgroups, chunks a multiple of 32, split count a
// multiple of 8 (one group of splits per XCD)
// split count balanced over the resident workgroups (tile_flops: one tile
// over the whole K range, as BF16 products; pbytes: partials of one split)
SplitPlanS plan_split(int nb, int64_t ng, int nmat, int tile, int64_t max_split, int64_t slots,
                      double tile_flops, double pbytes) {
  SplitPlanS p;
  p.tiles_n = (nb + tile - 1) / tile;
  p.tiles = p.tiles_n * (p.tiles_n + 1) / 2;  // on and above the diagonal
  // BF16 matrix cores at about 30% of their peak, partial sums at 5 TB/s
  int64_t nsplit = balanced_splits(static_cast<int64_t>(p.tiles) * nmat, slots,
                                   tile_flops * static_cast<double>(slots) / (0.3 * 2.5e15),
                                   2.0 * pbytes / 5e12, max_split, ng, 256);
  int64_t kchunk = (ng + nsplit - 1) / nsplit;
  kchunk = (kchunk + KS - 1) / KS * KS;
  nsplit = (ng + kchunk - 1) / kchunk;
  p.kchunk = kchunk;
  p.nsplit = static_cast<int>(nsplit);
  return p;
}

template <typename T, int WT>
int subspace_split_t(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                     int nb, void *H, void *S, hipStream_t st, double *part, size_t pcap) {
  constexpr int NP = Parts<T>::n;
  const int nmat = Spsi ? 2 : 1;
  const int64_t per_split = static_cast<int64_t>(nmat) * nb * nb * NP;
  const int64_t max_split = static_cast<int64_t>(pcap) / per_split;
  if (max_split < 1) return fail(GPAW_ESHAPE, "subspace partial-sum buffer too small for nb");
  const int64_t slots =
      resident_slots(reinterpret_cast<const void *>(&k_sub_lds<T, WT>), 256, 0);
  // six BF16 products per real product, four real products per complex one
  const double tile_flops =
      6.0 * 2.0 * NP * NP * (32.0 * WT) * (32.0 * WT) * static_cast<double>(s->ng);
  const SplitPlanS p = plan_split(nb, s->ng, nmat, 32 * WT, max_split, slots, tile_flops,
                                  static_cast<double>(per_split) * sizeof(double));
  // one work item per (K chunk, tile, matrix), the grid rounded up to whole
  // groups of 8 (one workgroup per XCD)
  const int64_t items = static_cast<int64_t>(p.nsplit) * p.tiles * nmat;
  const int64_t wgs = (items + 7) / 8 * 8;
  k_sub_lds<T, WT><<<static_cast<unsigned>(wgs), 256, 0, st>>>(
      static_cast<const T *>(psi), static_cast<const T *>(Hpsi),
      static_cast<const T *>(Spsi ? Spsi : Hpsi), part, nb, s->ng, p.kchunk, p.tiles_n,
      nmat, p.nsplit, super_block(slots, p.tiles_n));
  const int64_t tot = static_cast<int64_t>(nb) * nb * nmat * NP;
  k_split_reduce<NP><<<static_cast<unsigned>((tot + 255) / 256), 256, 0, st>>>(
      part, static_cast<double *>(H), static_cast<double *>(S), nb, p.nsplit, nmat, s->dV,
      32 * WT);
  return GPAW_OK;
}

template <typename T, int WT>
int rotate_split_t(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                   void *dst, hipStream_t st, bool upper, bool near_id) {
  constexpr int NP = Parts<T>::n;
  constexpr int TM = 32 * WT;
  __bf16 *Ct = reinterpret_cast<__bf16 *>(s->ws.split);
  const int nbp = (nb + KR - 1) / KR * KR;
  const int64_t np = static_cast<int64_t>(nb) * nbp;
  const double *Cd = static_cast<const double *>(C);
  // near the identity: rotate by C - I and add the source back, with one
  // BF16 product per pair when |C - I| is small enough (decided on the device)
  if (near_id) k_offid_small<NP><<<1, 1024, 0, st>>>(Cd, nb, s->ws.flag);
  // the column-panel rotation (upper triangular, near the identity, nb <=
  // 1024) reads a fragment-major copy of the high parts, stored after Ct
  const bool panel = near_id && upper && nbp + 8 <= NEAR_PITCH_MAX;
  __bf16 *Cf = panel ? Ct + 3 * NP * np : nullptr;
  k_split_c<NP><<<static_cast<unsigned>((np + 255) / 256), 256, 0, st>>>(Cd, Ct, nb, nbp,
                                                                        near_id ? 1 : 0, Cf);
  const int ntiles_n = (nb + TM - 1) / TM;
  const int64_t gtiles = (cols + TM - 1) / TM;
  const int64_t wgs = (gtiles + 7) / 8 * 8 * ntiles_n;
  if (near_id) {
    // both persistent kernels, resident-sized grids (whole groups of 8); the
    // device's flag lets exactly one of them work. The one-product kernel
    // takes 128 x 128 tiles (complex too: it keeps no FP64 accumulators),
    // so each staged source column serves twice the rows.
    constexpr int WT1 = WT < 4 ? 4 : WT;
    constexpr int TM1 = 32 * WT1;
    auto grid_of = [&](const void *k, int64_t items) {
      const int64_t r = std::max<int64_t>(8, resident_slots(k, 256, 0) / 8 * 8);
      return static_cast<unsigned>(std::min(r, (items + 7) / 8 * 8));
    };
    const int nt1 = (nb + TM1 - 1) / TM1;
    const int64_t gt1 = (cols + TM1 - 1) / TM1;
    auto *k1 = &k_rot_lds<T, WT1, true, true>;
    auto *k6 = &k_rot_lds<T, WT, true, false>;
    if (panel) {
      // upper triangular (the orthonormality correction): the column-panel
      // stream, 32 complex or 64 real columns per workgroup
      constexpr int TNP = NP == 2 ? 32 : 64, RBP = NP == 2 ? 1 : 2;
      auto *kp = &k_rot_near<T, TNP, RBP, 4>;
      const int64_t gb = (cols + TNP - 1) / TNP;
      const int64_t r = std::max<int64_t>(8, resident_slots(reinterpret_cast<const void *>(kp), 512, 0) / 8 * 8);
      kp<<<static_cast<unsigned>(std::min(r, (gb + 7) / 8 * 8)), 512, 0, st>>>(
          Cf, static_cast<const T *>(src), static_cast<T *>(dst), nb, nbp, cols, gb, s->ws.flag);
    } else {
      k1<<<grid_of(reinterpret_cast<const void *>(k1), gt1 * nt1), 256, 0, st>>>(
          Ct, static_cast<const T *>(src), static_cast<T *>(dst), nb, nbp, cols, nt1, gt1,
          upper ? 1 : 0, s->ws.flag);
    }
    k6<<<grid_of(reinterpret_cast<const void *>(k6), gtiles * ntiles_n), 256, 0, st>>>(
        Ct, static_cast<const T *>(src), static_cast<T *>(dst), nb, nbp, cols, ntiles_n, gtiles,
        upper ? 1 : 0, s->ws.flag);
  } else {
    k_rot_lds<T, WT, false, false><<<static_cast<unsigned>(wgs), 256, 0, st>>>(
        Ct, static_cast<const T *>(src), static_cast<T *>(dst), nb, nbp, cols, ntiles_n, gtiles,
        upper ? 1 : 0, nullptr);
  }
  return GPAW_OK;
}

}  // namespace

size_t split_part_elems(int nb, bool cplx) {
  // up to 64 splits of two matrices, within 64 Mi doubles (512 MiB); past
  // that the split count is capped to fit
  const int64_t tile = cplx ? 64 : 128;
  const int64_t parts = cplx ? 2 : 1;
  const int64_t small = std::max<int64_t>(1024 * tile * tile, 16 * int64_t(nb) * nb) * parts;
  const int64_t balanced = std::min<int64_t>(64 * 2 * int64_t(nb) * nb * parts, int64_t{64} << 20);
  return static_cast<size_t>(std::max(small, balanced));
}

size_t split_c_bytes(int nb, bool cplx) {
  // three planes per part, then the fragment-major copy of the high parts
  // (rows rounded up to 16)
  const size_t nbp = static_cast<size_t>((nb + KR - 1) / KR * KR);
  const size_t parts = cplx ? 2 : 1;
  return (static_cast<size_t>(nb) * 3 + static_cast<size_t>((nb + 15) / 16 * 16)) * nbp * parts *
         sizeof(__bf16);
}

int launch_subspace_split(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                          int nb, void *H, void *S, hipStream_t st, double *part,
                          size_t part_elems) {
  if (s->dtype == GPAW_C64)
    return subspace_split_t<z32, 2>(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
  return subspace_split_t<float, 4>(s, psi, Hpsi, Spsi, nb, H, S, st, part, part_elems);
}

int launch_rotate_split(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                        void *dst, hipStream_t st, bool upper, bool near_id) {
  if (cols == 0) return GPAW_OK;
  if (s->dtype == GPAW_C64)
    return rotate_split_t<z32, 2>(s, C, src, nb, cols, dst, st, upper, near_id);
  return rotate_split_t<float, 4>(s, C, src, nb, cols, dst, st, upper, near_id);
}

}  // namespace gfd
