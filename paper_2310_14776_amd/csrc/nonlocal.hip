// Projector overlaps <p~^a_i|psi_n> (the projections of Eq. (dh)) and the
// per-atom contraction Delta^a P^a that feeds the add-back.
//
// Projection: one workgroup per (atom, group of bands). Lanes stride over the
// atom's sphere entries (sorted by grid index, so neighbouring lanes gather
// neighbouring z points), evaluate the projector values of their entry once
// for all bands of the group, keep the ni x NBG partial sums in registers,
// and reduce them across the wavefront with cross-lane shuffles and across
// the four wavefronts through LDS in a fixed order (bitwise reproducible).
#include <algorithm>

#include "proj.h"

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
                                                 const short4 *__restrict__ e_xyz,
                                                 const double *__restrict__ pos,
                                                 const ProjDev *__restrict__ pjp,
                                                 int64_t ng, int nb, int np, double dV) {
  typename PJSel<NI>::type pj = PJSel<NI>::get(pjp);
  // per-axis image phases in LDS (complex only): divergent indices stay off
  // global memory
  __shared__ z64 phs[48];
  if (St<T>::cplx) {
    for (int idx = threadIdx.x; idx < 48; idx += 256) phs[idx] = pjp->ph[idx / 16][idx % 16];
    __syncthreads();
  }
  const int atom = blockIdx.x;
  const int b0 = blockIdx.y * NBG;
  const int e0 = a_start[atom], e1 = a_start[atom + 1];
  const double R0 = pos[3 * atom], R1 = pos[3 * atom + 1], R2 = pos[3 * atom + 2];
  using A = typename St<T>::Acc;
  A acc[NBG][NI];
#pragma unroll
  for (int b = 0; b < NBG; ++b)
#pragma unroll
    for (int i = 0; i < NI; ++i) acc[b][i] = St<A>::zero();

  for (int e = e0 + static_cast<int>(threadIdx.x); e < e1; e += 256) {
    const int64_t g = e_g[e];
    const short4 u = e_xyz[e];
    A p[NBG];
#pragma unroll
    for (int b = 0; b < NBG; ++b)
      p[b] = St<T>::widen((b0 + b < nb) ? psi[static_cast<int64_t>(b0 + b) * ng + g] : St<T>::zero());
    double pv[NI];
    if constexpr (NI == 13) eval_proj13(pj, u.x * pj.h[0] - R0, u.y * pj.h[1] - R1, u.z * pj.h[2] - R2, pv);
    else eval_proj<NI>(pj, u.x * pj.h[0] - R0, u.y * pj.h[1] - R1, u.z * pj.h[2] - R2, pv);
    if (St<T>::cplx) {
      // conj(q) psi = p(r) conj(exp(-2 pi i k.w)) psi
      const int c = u.w;
      const z64 ph = zconj(phs[((c >> 8) & 15)] * phs[16 + ((c >> 4) & 15)] * phs[32 + (c & 15)]);
#pragma unroll
      for (int b = 0; b < NBG; ++b) p[b] = St<A>::phase(p[b], ph);
    }
#pragma unroll
    for (int b = 0; b < NBG; ++b)
#pragma unroll
      for (int i = 0; i < NI; ++i) acc[b][i] = acc[b][i] + St<A>::scale(pv[i], p[b]);
  }

  __shared__ A red[4][NBG * NI];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < NBG; ++b)
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const A r = Red<A>::wave_sum(acc[b][i]);
      if (lane == 0) red[wave][b * NI + i] = r;
    }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NBG * NI; idx += 256) {
    const int b = idx / NI, i = idx - b * NI;
    const int ni = NI == 13 ? 13 : pjp->ni;
    if (b0 + b < nb && i < ni)
      P[static_cast<int64_t>(b0 + b) * np + atom * ni + i] = St<T>::narrow(
          St<A>::scale(dV, (red[0][idx] + red[1][idx]) + (red[2][idx] + red[3][idx])));
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
  using A = typename St<T>::Acc;
  A acc = St<A>::zero();
  for (int j = 0; j < ni; ++j) acc = acc + St<A>::scale(Da[j], St<T>::widen(Pa[j]));
  X[idx] = St<T>::narrow(acc);
}

template <typename T, int NI, int NBG>
void project_t(const gpaw_sys *s, const void *psi, int nb, void *P, hipStream_t st) {
  dim3 grid(s->natoms, (nb + NBG - 1) / NBG);
  k_project<T, NI, NBG><<<grid, 256, 0, st>>>(
      static_cast<const T *>(psi), static_cast<T *>(P), s->tab.a_start, s->tab.e_g,
      s->tab.e_xyz, s->tab.pos, s->tab.proj, s->ng, nb, s->np, s->dV);
}

}  // namespace

int launch_project(const gpaw_sys *s, const void *psi, int nb, void *P, hipStream_t st) {
  if (s->np == 0) return GPAW_OK;
  const bool std13 = s->ni == 13 && s->proj.std13;
  switch (s->dtype) {
    case GPAW_C128:
      if (std13 && s->tune.prj_nbg == 1) project_t<z64, 13, 1>(s, psi, nb, P, st);
      else if (std13) project_t<z64, 13, 2>(s, psi, nb, P, st);
      else project_t<z64, 32, 1>(s, psi, nb, P, st);
      break;
    case GPAW_F32:
      std13 ? project_t<float, 13, 4>(s, psi, nb, P, st) : project_t<float, 32, 1>(s, psi, nb, P, st);
      break;
    case GPAW_C64:
      std13 ? project_t<z32, 13, 2>(s, psi, nb, P, st) : project_t<z32, 32, 1>(s, psi, nb, P, st);
      break;
    default:
      if (std13 && s->tune.prj_nbg == 2) project_t<double, 13, 2>(s, psi, nb, P, st);
      else if (std13 && s->tune.prj_nbg == 8) project_t<double, 13, 8>(s, psi, nb, P, st);
      else if (std13) project_t<double, 13, 4>(s, psi, nb, P, st);
      else project_t<double, 32, 1>(s, psi, nb, P, st);
  }
  return GPAW_OK;
}

// X = Delta H . P and XS = Delta S . P in one launch (one read of P)
template <typename T>
__global__ __launch_bounds__(256) void k_dmat2(const double *__restrict__ DH,
                                               const double *__restrict__ DS,
                                               const T *__restrict__ P, T *__restrict__ X,
                                               T *__restrict__ XS, int64_t total, int ni, int np) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t n = idx / np;
  const int ai = static_cast<int>(idx - n * np);
  const int a = ai / ni, i = ai - a * ni;
  const int64_t drow = (static_cast<int64_t>(a) * ni + i) * ni;
  const T *Pa = P + n * np + a * ni;
  using A = typename St<T>::Acc;
  A h = St<A>::zero(), sv = St<A>::zero();
  for (int j = 0; j < ni; ++j) {
    const A pj = St<T>::widen(Pa[j]);
    h = h + St<A>::scale(DH[drow + j], pj);
    sv = sv + St<A>::scale(DS[drow + j], pj);
  }
  X[idx] = St<T>::narrow(h);
  XS[idx] = St<T>::narrow(sv);
}

template <typename T>
void dmat2_t(const gpaw_sys *s, const void *P, int nb, void *X, void *XS, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(nb) * s->np;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  k_dmat2<T><<<blocks, 256, 0, st>>>(s->dH, s->dS, static_cast<const T *>(P), static_cast<T *>(X),
                                     static_cast<T *>(XS), total, s->ni, s->np);
}

int launch_dmat2(const gpaw_sys *s, const void *P, int nb, void *X, void *XS, hipStream_t st) {
  if (s->np == 0) return GPAW_OK;
  switch (s->dtype) {
    case GPAW_C128: dmat2_t<z64>(s, P, nb, X, XS, st); break;
    case GPAW_F32: dmat2_t<float>(s, P, nb, X, XS, st); break;
    case GPAW_C64: dmat2_t<z32>(s, P, nb, X, XS, st); break;
    default: dmat2_t<double>(s, P, nb, X, XS, st);
  }
  return GPAW_OK;
}

template <typename T>
void dmat_t(const gpaw_sys *s, const double *D, const void *P, int nb, void *X, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(nb) * s->np;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  k_dmat<T><<<blocks, 256, 0, st>>>(D, static_cast<const T *>(P), static_cast<T *>(X), total,
                                    s->ni, s->np);
}

int launch_dmat(const gpaw_sys *s, const double *D, const void *P, int nb, void *X,
                hipStream_t st) {
  if (s->np == 0) return GPAW_OK;
  switch (s->dtype) {
    case GPAW_C128: dmat_t<z64>(s, D, P, nb, X, st); break;
    case GPAW_F32: dmat_t<float>(s, D, P, nb, X, st); break;
    case GPAW_C64: dmat_t<z32>(s, D, P, nb, X, st); break;
    default: dmat_t<double>(s, D, P, nb, X, st);
  }
  return GPAW_OK;
}

}  // namespace gfd
