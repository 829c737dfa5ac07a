// One block Davidson step around the subspace step (SCF step (2), Sec.
// "Solving the Kohn-Sham equation"; the iterative Davidson eigensolver of
// Sec. "Parallelization"). Reading (the paper gives no formulas): from Ritz
// vectors psi_n with Ritz values eps_n,
//   corrections  d_n(r) = -(H~psi_n - eps_n S~psi_n)(r) / p_n(r),
//                p_n(r) = max(t0 + v(r) - eps_n, t0 / 2),
//                t0 = (1/2)(49/18) sum_c 1/h_c^2 (the diagonal of the FD
//                kinetic operator: a positive diagonal preconditioner);
//   Rayleigh-Ritz on span{psi, d} (2 nb vectors) with the step's own kernels
//   (projections, H~ and S~ in one pass, subspace matrices, FP64 eigensolve)
//   and the rotation to the lowest nb Ritz vectors.
// k_precond is one HBM pass (read H~psi and S~psi, write d), v from L2.
#include "internal.h"

namespace gfd {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_precond(const T *__restrict__ Hpsi,
                                                 const T *__restrict__ Spsi,
                                                 const double *__restrict__ eps,
                                                 const double *__restrict__ v, double t0,
                                                 int64_t ng, T *__restrict__ out) {
  const int n = blockIdx.y;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= ng) return;
  const double e = eps[n];
  const int64_t i = static_cast<int64_t>(n) * ng + g;
  using A = typename St<T>::Acc;
  const A r = St<T>::widen(Hpsi[i]) - St<A>::scale(e, St<T>::widen(Spsi[i]));
  const double p = fmax(t0 + v[g] - e, 0.5 * t0);
  out[i] = St<T>::narrow(St<A>::scale(-1.0 / p, r));
}

template <typename T>
void precond_t(const gpaw_sys *s, const void *Hpsi, const void *Spsi, const double *eps, int nb,
               void *out, hipStream_t st) {
  double t0 = 0.0;
  for (int c = 0; c < 3; ++c) t0 += 1.0 / (s->h[c] * s->h[c]);
  t0 *= 0.5 * (49.0 / 18.0);
  const dim3 grid(static_cast<unsigned>((s->ng + 255) / 256), static_cast<unsigned>(nb));
  k_precond<T><<<grid, 256, 0, st>>>(static_cast<const T *>(Hpsi), static_cast<const T *>(Spsi),
                                     eps, s->v, t0, s->ng, static_cast<T *>(out));
}

}  // namespace

int launch_precond(const gpaw_sys *s, const void *Hpsi, const void *Spsi, const double *eps,
                   int nb, void *out, hipStream_t st) {
  switch (s->dtype) {
    case GPAW_C128: precond_t<z64>(s, Hpsi, Spsi, eps, nb, out, st); break;
    case GPAW_F32: precond_t<float>(s, Hpsi, Spsi, eps, nb, out, st); break;
    case GPAW_C64: precond_t<z32>(s, Hpsi, Spsi, eps, nb, out, st); break;
    default: precond_t<double>(s, Hpsi, Spsi, eps, nb, out, st); break;
  }
  return GPAW_OK;
}

}  // namespace gfd
