// Stencil kernels instantiated for FP64 real blocks (see stencil_impl.h).
#include "stencil_impl.h"

namespace gfd {

int launch_stencil_f64(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                       hipStream_t st, const void *XS, void *outS) {
  const bool std13 = s->ni == 13 && s->proj.std13;
  const bool two = stencil_ppl(s) == 2;
  // 2 bands per workgroup: the seven-plane window holds 16 bytes per point and plane
  if (std13)
    return two ? plane_t<double, false, 2, 13, 2>(s, psi, nb, X, out, st, XS, outS)
               : plane_t<double, false, 2, 13, 1>(s, psi, nb, X, out, st, XS, outS);
  return two ? plane_t<double, false, 2, PROJ_MAX_NI, 2>(s, psi, nb, X, out, st, XS, outS)
             : plane_t<double, false, 2, PROJ_MAX_NI, 1>(s, psi, nb, X, out, st, XS, outS);
}

}  // namespace gfd
