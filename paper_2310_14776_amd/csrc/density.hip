// Pseudo density and atomic density matrices of a block (Sec. "Projector
// augmented-wave method", Eq. (atomicdensitymatrix); steps (3)-(4) of the
// SCF loop consume them):
//   n~(r)    = sum_n f_n |psi~_n(r)|^2,
//   D^a_ii'  = sum_n f_n <psi~_n|p~^a_i> <p~^a_i'|psi~_n>
//            = sum_n f_n conj(P_n,ai) P_n,ai'.
// k_density: one lane per grid point, bands in fixed order, eight loads in
// flight per lane, FP64 sums (every dtype); the kernel streams the block
// once, so it is bound by HBM. k_dmat_density: one workgroup per atom, one
// lane per (i, i') entry, bands in fixed order.
#include "internal.h"

namespace gfd {
namespace {

__device__ inline double abs2_d(double a) { return a * a; }
__device__ inline double abs2_d(float a) { return static_cast<double>(a) * a; }
__device__ inline double abs2_d(z64 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double abs2_d(z32 a) {
  return static_cast<double>(a.x) * a.x + static_cast<double>(a.y) * a.y;
}

template <typename T>
__global__ __launch_bounds__(256) void k_density(const T *__restrict__ psi,
                                                 const double *__restrict__ f, int nb,
                                                 int64_t ng, double *__restrict__ n_out) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= ng) return;
  double acc = 0.0;
  int b = 0;
  for (; b + 8 <= nb; b += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = psi[static_cast<int64_t>(b + u) * ng + g];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(f[b + u], abs2_d(v[u]), acc);
  }
  for (; b < nb; ++b) acc = fma(f[b], abs2_d(psi[static_cast<int64_t>(b) * ng + g]), acc);
  n_out[g] = acc;
}

// D[a][i][j] in the matrix dtype M (double or z64) from P of dtype T
template <typename T, typename M>
__global__ __launch_bounds__(256) void k_dmat_density(const T *__restrict__ P,
                                                      const double *__restrict__ f, int nb,
                                                      int np, int ni, M *__restrict__ D) {
  const int a = blockIdx.x, t = threadIdx.x;
  if (t >= ni * ni) return;
  const int i = t / ni, j = t - (t / ni) * ni;
  const T *pi = P + a * ni + i, *pj = P + a * ni + j;
  M acc = St<M>::zero();
  for (int n = 0; n < nb; ++n) {
    const M x = St<T>::widen(pi[static_cast<int64_t>(n) * np]);
    const M y = St<T>::widen(pj[static_cast<int64_t>(n) * np]);
    acc = acc + St<M>::scale(f[n], St<M>::conj(x) * y);
  }
  D[static_cast<int64_t>(a) * ni * ni + t] = acc;
}

template <typename T, typename M>
int density_t(const gpaw_sys *s, const void *psi, int nb, const double *f, const void *P,
              double *n_out, void *D_out, hipStream_t st) {
  if (n_out)
    k_density<T><<<static_cast<unsigned>((s->ng + 255) / 256), 256, 0, st>>>(
        static_cast<const T *>(psi), f, nb, s->ng, n_out);
  if (D_out && s->natoms > 0)
    k_dmat_density<T, M><<<s->natoms, 256, 0, st>>>(static_cast<const T *>(P), f, nb, s->np,
                                                     s->ni, static_cast<M *>(D_out));
  return GPAW_OK;
}

}  // namespace

int launch_density(const gpaw_sys *s, const void *psi, int nb, const double *f, const void *P,
                   double *n_out, void *D_out, hipStream_t st) {
  switch (s->dtype) {
    case GPAW_C128: return density_t<z64, z64>(s, psi, nb, f, P, n_out, D_out, st);
    case GPAW_F32: return density_t<float, double>(s, psi, nb, f, P, n_out, D_out, st);
    case GPAW_C64: return density_t<z32, z64>(s, psi, nb, f, P, n_out, D_out, st);
    default: return density_t<double, double>(s, psi, nb, f, P, n_out, D_out, st);
  }
}

}  // namespace gfd
