// Dispatch of the FD stencil (H~psi, S~psi) and of S~ alone by dtype; the
// kernels are in stencil_impl.h.
#include "stencil_impl.h"

namespace gfd {

std::vector<std::pair<int, int>> stencil_tiles(const gpaw_sys *s, int keep) {
  return tile_candidates(s->n[1], s->n[2], stencil_ppl(s), static_cast<size_t>(keep));
}

int launch_stencil(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st, const void *XS, void *outS) {
  switch (s->dtype) {
    case GPAW_C128: return launch_stencil_c128(s, psi, nb, X, out, st, XS, outS);
    case GPAW_F32: return launch_stencil_f32(s, psi, nb, X, out, st, XS, outS);
    case GPAW_C64: return launch_stencil_c64(s, psi, nb, X, out, st, XS, outS);
    default: return launch_stencil_f64(s, psi, nb, X, out, st, XS, outS);
  }
}

int launch_apply_S(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st) {
  const bool std13 = s->ni == 13 && s->proj.std13;
  switch (s->dtype) {
    case GPAW_C128:
      return std13 ? apply_S_t<z64, 8, 13>(s, psi, nb, X, out, st)
                   : apply_S_t<z64, 8, PROJ_MAX_NI>(s, psi, nb, X, out, st);
    case GPAW_F32:
      return std13 ? apply_S_t<float, 16, 13>(s, psi, nb, X, out, st)
                   : apply_S_t<float, 16, PROJ_MAX_NI>(s, psi, nb, X, out, st);
    case GPAW_C64:
      return std13 ? apply_S_t<z32, 8, 13>(s, psi, nb, X, out, st)
                   : apply_S_t<z32, 8, PROJ_MAX_NI>(s, psi, nb, X, out, st);
    default:
      return std13 ? apply_S_t<double, 16, 13>(s, psi, nb, X, out, st)
                   : apply_S_t<double, 16, PROJ_MAX_NI>(s, psi, nb, X, out, st);
  }
}

}  // namespace gfd
