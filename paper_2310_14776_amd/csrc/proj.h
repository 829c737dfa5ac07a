// Device evaluation of the projector functions p~^a_i at a grid point.
//
// Channel (l, sigma, rc): N r^l exp(-r^2/2sigma^2) (1-(r/rc)^2)^2 Y_lm for
// r < rc, N = [Gamma(l+3/2) sigma^(2l+3)/2]^(-1/2), real harmonics in the
// order (1), (y, z, x), (xy, yz, 3z^2-r^2, xz, x^2-y^2) with the
// normalisations 1/(2 sqrt(pi)), sqrt(3/4pi), (1/2)sqrt(15/pi),
// (1/4)sqrt(5/pi), (1/4)sqrt(15/pi). The kernels recompute these values at
// every use instead of streaming a table of them: a few dozen FP64 operations
// per (point, atom) pair, shared by all bands a lane handles, replace
// 8*ni bytes of table traffic per band.
#pragma once

#include "internal.h"

namespace gfd {

// Entry code of the point-major list: atom << 12 | (wx+8) << 8 | (wy+8) << 4 | (wz+8);
// the unwrapped grid index along axis c is (folded index) + w_c n_c.
__host__ __device__ inline int32_t pack_code(int atom, int wx, int wy, int wz) {
  return (atom << 12) | ((wx + 8) << 8) | ((wy + 8) << 4) | (wz + 8);
}

// r^l Y_lm for harmonic slot 0..8 at displacement (x, y, z), r2 = r^2
__device__ inline double solid_slot(int slot, double x, double y, double z, double r2) {
  constexpr double c0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
  constexpr double c1 = 0.48860251190291992;   // sqrt(3/(4 pi))
  constexpr double c2 = 1.0925484305920792;    // (1/2) sqrt(15/pi)
  constexpr double c20 = 0.31539156525252005;  // (1/4) sqrt(5/pi)
  constexpr double c22 = 0.54627421529603959;  // (1/4) sqrt(15/pi)
  switch (slot) {
    case 0: return c0;
    case 1: return c1 * y;
    case 2: return c1 * z;
    case 3: return c1 * x;
    case 4: return c2 * x * y;
    case 5: return c2 * y * z;
    case 6: return c20 * (3.0 * z * z - r2);
    case 7: return c2 * x * z;
    default: return c22 * (x * x - y * y);
  }
}

// radial factor N exp(-r^2/2sigma^2) (1 - r^2/rc^2)^2 of channel c (0 beyond rc)
__device__ inline double radial(const ProjDev &P, int c, double r2) {
  const double s2 = r2 * P.rc2inv[c];
  if (!(s2 < 1.0)) return 0.0;
  const double t = 1.0 - s2;
  return P.norm[c] * exp(-r2 * P.a2[c]) * (t * t);
}

// same, with the Gaussian of channel 0 or 1 (whose sigma channel c shares)
__device__ inline double radial_shared(const ProjDev &P, int c, double r2, double E0, double E1) {
  const double s2 = r2 * P.rc2inv[c];
  const double t = 1.0 - s2;
  const double E = P.same_sigma[c] == 0 ? E0 : E1;
  return s2 < 1.0 ? P.norm[c] * E * (t * t) : 0.0;
}

// Values of all NI projectors of one atom at displacement (x, y, z).
// NI == 13 is the channel layout l = (0, 0, 1, 1, 2) with the last three
// channels sharing the sigma of channel 0 or 1; any other layout takes the
// generic path (NI = PROJ_MAX_NI, entries beyond ni are zero).
template <int NI>
__device__ inline void eval_proj(const ProjDev &P, double x, double y, double z, double *out) {
  const double r2 = x * x + y * y + z * z;
  if constexpr (NI == 13) {
    constexpr double c0 = 0.28209479177387814;
    constexpr double c1 = 0.48860251190291992;
    constexpr double c2 = 1.0925484305920792;
    constexpr double c20 = 0.31539156525252005;
    constexpr double c22 = 0.54627421529603959;
    const double E0 = exp(-r2 * P.a2[0]), E1 = exp(-r2 * P.a2[1]);
    double r0 = 0.0, r1 = 0.0;
    {
      const double s0 = r2 * P.rc2inv[0], s1 = r2 * P.rc2inv[1];
      if (s0 < 1.0) r0 = P.norm[0] * E0 * (1.0 - s0) * (1.0 - s0);
      if (s1 < 1.0) r1 = P.norm[1] * E1 * (1.0 - s1) * (1.0 - s1);
    }
    const double rp = radial_shared(P, 2, r2, E0, E1), rq = radial_shared(P, 3, r2, E0, E1),
                 rd = radial_shared(P, 4, r2, E0, E1);
    out[0] = r0 * c0;
    out[1] = r1 * c0;
    const double py = c1 * y, pz = c1 * z, px = c1 * x;
    out[2] = rp * py;
    out[3] = rp * pz;
    out[4] = rp * px;
    out[5] = rq * py;
    out[6] = rq * pz;
    out[7] = rq * px;
    out[8] = rd * (c2 * x * y);
    out[9] = rd * (c2 * y * z);
    out[10] = rd * (c20 * (3.0 * z * z - r2));
    out[11] = rd * (c2 * x * z);
    out[12] = rd * (c22 * (x * x - y * y));
  } else {
#pragma unroll
    for (int i = 0; i < NI; ++i)
      out[i] = (i < P.ni) ? radial(P, P.ch[i], r2) * solid_slot(P.ym[i], x, y, z, r2) : 0.0;
  }
}

// Parameters of the straight-line layout copied once per kernel into
// registers (uniform values), so the inner loops issue no scalar loads.
struct Proj13 {
  double norm[5], rc2inv[5], a2[2];
  bool sel1[5];  // channel c uses the Gaussian of channel 1 (else of channel 0)
  int n[3];
  double h[3];
};

__device__ inline Proj13 load_proj13(const ProjDev &P) {
  Proj13 q;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    q.norm[c] = P.norm[c];
    q.rc2inv[c] = P.rc2inv[c];
    q.sel1[c] = c == 1 || (c >= 2 && P.same_sigma[c] == 1);
  }
  q.a2[0] = P.a2[0];
  q.a2[1] = P.a2[1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    q.n[c] = P.n[c];
    q.h[c] = P.h[c];
  }
  return q;
}

// the 13 projector values of one atom at displacement (x, y, z)
__device__ inline void eval_proj13(const Proj13 &P, double x, double y, double z, double *out) {
  constexpr double c0 = 0.28209479177387814;
  constexpr double c1 = 0.48860251190291992;
  constexpr double c2 = 1.0925484305920792;
  constexpr double c20 = 0.31539156525252005;
  constexpr double c22 = 0.54627421529603959;
  const double r2 = x * x + y * y + z * z;
  const double E0 = exp(-r2 * P.a2[0]), E1 = exp(-r2 * P.a2[1]);
  double rad[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double s2 = r2 * P.rc2inv[c];
    const double t = 1.0 - s2;
    rad[c] = s2 < 1.0 ? P.norm[c] * (P.sel1[c] ? E1 : E0) * (t * t) : 0.0;
  }
  out[0] = rad[0] * c0;
  out[1] = rad[1] * c0;
  const double py = c1 * y, pz = c1 * z, px = c1 * x;
  out[2] = rad[2] * py;
  out[3] = rad[2] * pz;
  out[4] = rad[2] * px;
  out[5] = rad[3] * py;
  out[6] = rad[3] * pz;
  out[7] = rad[3] * px;
  out[8] = rad[4] * (c2 * x * y);
  out[9] = rad[4] * (c2 * y * z);
  out[10] = rad[4] * (c20 * (3.0 * z * z - r2));
  out[11] = rad[4] * (c2 * x * z);
  out[12] = rad[4] * (c22 * (x * x - y * y));
}

// Projector parameters as the kernels hold them: a register copy for the
// 13-projector layout, the device table otherwise.
template <int NI> struct PJSel {
  using type = const ProjDev &;
  __device__ static const ProjDev &get(const ProjDev *p) { return *p; }
};
template <> struct PJSel<13> {
  using type = Proj13;
  __device__ static Proj13 get(const ProjDev *p) { return load_proj13(*p); }
};

// Bloch phase exp(-2 pi i k.w) of an image shift w (grid-cell units).
__device__ inline z64 image_phase(const ProjDev &P, int wx, int wy, int wz) {
  return P.ph[0][wx + 8] * P.ph[1][wy + 8] * P.ph[2][wz + 8];
}

}  // namespace gfd
