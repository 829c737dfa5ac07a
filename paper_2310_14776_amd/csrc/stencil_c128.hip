// Stencil kernels instantiated for complex128 (Bloch) blocks (see stencil_impl.h).
#include "stencil_impl.h"

namespace gfd {

int launch_stencil_c128(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                       hipStream_t st, const void *XS, void *outS) {
  const bool std13 = s->ni == 13 && s->proj.std13;
  const bool two = stencil_ppl(s) == 2;
  // 1 band per workgroup: the seven-plane window holds 16 bytes per point and plane
  if (std13)
    return two ? plane_t<z64, true, 1, 13, 2>(s, psi, nb, X, out, st, XS, outS)
               : plane_t<z64, true, 1, 13, 1>(s, psi, nb, X, out, st, XS, outS);
  return two ? plane_t<z64, true, 1, PROJ_MAX_NI, 2>(s, psi, nb, X, out, st, XS, outS)
             : plane_t<z64, true, 1, PROJ_MAX_NI, 1>(s, psi, nb, X, out, st, XS, outS);
}

}  // namespace gfd
