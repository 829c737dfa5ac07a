// Projector overlaps <p~^a_i|psi_n> (the projections of Eq. (dh)) and the
// per-atom contraction Delta^a P^a that feeds the add-back.
//
// Projection: one workgroup per (atom, group of bands). Lanes stride over the
// atom's sphere entries (sorted by grid index, so neighbouring lanes gather
// neighbouring z points), keep the ni x NBG partial sums in registers, and
// reduce them across the wavefront with cross-lane shuffles and across the
// four wavefronts through LDS in a fixed order (bitwise reproducible).
#include <algorithm>

#include "internal.h"

namespace gfd {

namespace {

template <typename T> struct Red;
template <> struct Red<double> {
  __device__ static double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
  }
};
template <> struct Red<z64> {
  __device__ static z64 wave_sum(z64 v) {
    for (int off = 32; off >= 1; off >>= 1) {
      v.x += __shfl_xor(v.x, off);
      v.y += __shfl_xor(v.y, off);
    }
    return v;
  }
};

template <typename T, int NI, int NBG>
__global__ __launch_bounds__(256) void k_project(const T *__restrict__ psi, T *__restrict__ P,
                                                 const int32_t *__restrict__ a_start,
                                                 const int32_t *__restrict__ e_g,
                                                 const T *__restrict__ e_q, int64_t nent,
                                                 int64_t ng, int nb, int ni, int np, double dV) {
  const int atom = blockIdx.x;
  const int b0 = blockIdx.y * NBG;
  const int e0 = a_start[atom], e1 = a_start[atom + 1];
  T acc[NBG][NI];
#pragma unroll
  for (int b = 0; b < NBG; ++b)
#pragma unroll
    for (int i = 0; i < NI; ++i) acc[b][i] = St<T>::zero();

  for (int e = e0 + static_cast<int>(threadIdx.x); e < e1; e += 256) {
    const int64_t g = e_g[e];
    T q[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) q[i] = (i < ni) ? St<T>::conj(e_q[i * nent + e]) : St<T>::zero();
#pragma unroll
    for (int b = 0; b < NBG; ++b) {
      if (b0 + b < nb) {
        const T p = psi[static_cast<int64_t>(b0 + b) * ng + g];
#pragma unroll
        for (int i = 0; i < NI; ++i) acc[b][i] = acc[b][i] + St<T>::mul(q[i], p);
      }
    }
  }

  __shared__ T red[4][NBG * NI];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < NBG; ++b)
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const T r = Red<T>::wave_sum(acc[b][i]);
      if (lane == 0) red[wave][b * NI + i] = r;
    }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NBG * NI; idx += 256) {
    const int b = idx / NI, i = idx - b * NI;
    if (b0 + b < nb && i < ni)
      P[static_cast<int64_t>(b0 + b) * np + atom * ni + i] =
          St<T>::scale(dV, (red[0][idx] + red[1][idx]) + (red[2][idx] + red[3][idx]));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dmat(const double *__restrict__ D, const T *__restrict__ P,
                                              T *__restrict__ X, int64_t total, int ni, int np) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t n = idx / np;
  const int ai = static_cast<int>(idx - n * np);
  const int a = ai / ni, i = ai - a * ni;
  const double *Da = D + (static_cast<int64_t>(a) * ni + i) * ni;
  const T *Pa = P + n * np + a * ni;
  T acc = St<T>::zero();
  for (int j = 0; j < ni; ++j) acc = acc + St<T>::scale(Da[j], Pa[j]);
  X[idx] = acc;
}

template <typename T, int NI, int NBG>
void project_t(const gpaw_sys *s, const void *psi, int nb, void *P, hipStream_t st) {
  dim3 grid(s->natoms, (nb + NBG - 1) / NBG);
  k_project<T, NI, NBG><<<grid, 256, 0, st>>>(
      static_cast<const T *>(psi), static_cast<T *>(P), s->tab.a_start, s->tab.e_g,
      static_cast<const T *>(s->tab.e_q), s->tab.nent, s->ng, nb, s->ni, s->np, s->dV);
}

}  // namespace

int launch_project(const gpaw_sys *s, const void *psi, int nb, void *P, hipStream_t st) {
  if (s->np == 0) return GPAW_OK;
  const bool cplx = s->dtype == GPAW_C128;
  if (s->ni == 13) {
    if (cplx) project_t<z64, 13, 2>(s, psi, nb, P, st);
    else project_t<double, 13, 4>(s, psi, nb, P, st);
  } else {
    if (cplx) project_t<z64, 32, 1>(s, psi, nb, P, st);
    else project_t<double, 32, 1>(s, psi, nb, P, st);
  }
  return GPAW_OK;
}

int launch_dmat(const gpaw_sys *s, const double *D, const void *P, int nb, void *X,
                hipStream_t st) {
  if (s->np == 0) return GPAW_OK;
  const int64_t total = static_cast<int64_t>(nb) * s->np;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  if (s->dtype == GPAW_C128)
    k_dmat<z64><<<blocks, 256, 0, st>>>(D, static_cast<const z64 *>(P), static_cast<z64 *>(X),
                                        total, s->ni, s->np);
  else
    k_dmat<double><<<blocks, 256, 0, st>>>(D, static_cast<const double *>(P),
                                           static_cast<double *>(X), total, s->ni, s->np);
  return GPAW_OK;
}

}  // namespace gfd
