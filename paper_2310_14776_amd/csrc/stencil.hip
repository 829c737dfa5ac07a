// (T + v + non-local) applied to a block: the FD kinetic stencil of the
// grid representation (Sec. "Wave-function representations"), the local
// potential and the projector add-back of Eq. (dh); and the overlap
// operator S~ = 1 + sum |p> Delta S <p|.
//
// Kernel shape (gfx950): a workgroup of 256 lanes owns 256 consecutive points
// of one y-z plane (flattened, z contiguous, so every load is coalesced) for
// one band, and marches along x over a segment of planes. The x neighbours
// live in a 7-deep register queue per lane; the y and z neighbours come from
// an LDS copy of the current plane slice widened by three rows on each side.
// Periodic/Bloch folding happens at load time (x and y) and when a z
// neighbour crosses its row (z). The non-local add-back is fused into the
// store: each covered grid point sums q^a_i(r) (Delta.P)^a_i over the atoms
// whose spheres reach it, so H~psi leaves the kernel in one HBM pass.
#include <algorithm>

#include "internal.h"

namespace gfd {

namespace {

constexpr int ST_THREADS = 256;

struct StencilGeom {
  int n0, n1, n2;
  double c0;                  // centre coefficient summed over the three axes
  double cx[3], cy[3], cz[3]; // -1/2 w_d / h_c^2, d = 1..3
  z64 phx[7], phy[7], phz[7]; // Bloch phase to the power w = -3..3
  int xseg;
};

struct AddArgs {
  const int32_t *g2u;
  const int32_t *u_start;
  const int32_t *pm_atom;
  const void *pm_q;
  const void *X;
  int64_t nent;
  int ni, np;
};

// floor(a / b) for b > 0 and small |a / b| (|quotient| <= 3 in every use)
__device__ inline int fold_count(int a, int b) {
  int w = 0;
  while (a >= b) { a -= b; ++w; }
  while (a < 0) { a += b; --w; }
  return w;
}

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

__device__ inline int clamp3(int w) { return w < -3 ? -3 : (w > 3 ? 3 : w); }

template <typename T>
__device__ inline T addback_at(const AddArgs &ab, int64_t g, int band) {
  T acc = St<T>::zero();
  const int u = ab.g2u[g];
  if (u < 0) return acc;
  const int e0 = ab.u_start[u], e1 = ab.u_start[u + 1];
  const T *q = static_cast<const T *>(ab.pm_q);
  const T *X = static_cast<const T *>(ab.X) + static_cast<int64_t>(band) * ab.np;
  for (int e = e0; e < e1; ++e) {
    const T *Xa = X + ab.pm_atom[e] * ab.ni;
    for (int i = 0; i < ab.ni; ++i) acc = acc + St<T>::mul(q[i * ab.nent + e], Xa[i]);
  }
  return acc;
}

template <typename T, bool BLOCH, bool ADD>
__global__ __launch_bounds__(ST_THREADS) void k_stencil(const T *__restrict__ psi,
                                                        T *__restrict__ out,
                                                        const double *__restrict__ v,
                                                        StencilGeom G, AddArgs ab) {
  extern __shared__ unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  const int n0 = G.n0, n1 = G.n1, n2 = G.n2;
  const int plane = n1 * n2;
  const int halo = 3 * n2;
  const int t = threadIdx.x;
  const int start = blockIdx.x * ST_THREADS;
  const int band = blockIdx.y;
  const int64_t bstride = static_cast<int64_t>(n0) * plane;
  const T *src = psi + band * bstride;
  T *dst = out + band * bstride;
  const int x0 = blockIdx.z * G.xseg;
  const int x1 = min(n0, x0 + G.xseg);

  // this lane's slot of the flattened plane, folded into the cell
  const int f = start + t;
  const int wy = floor_div(f, plane);
  const int pw = f - wy * plane;
  const bool active = f < plane;
  const int z = pw % n2;

  auto load = [&](int x, int p, int wyy) -> T {
    const int wx = fold_count(x, n0);
    T val = src[static_cast<int64_t>(x - wx * n0) * plane + p];
    if (BLOCH) val = St<T>::phase(val, G.phx[clamp3(wx) + 3] * G.phy[clamp3(wyy) + 3]);
    return val;
  };

  T q[7];
#pragma unroll
  for (int d = 0; d < 6; ++d) q[d] = load(x0 + d - 3, pw, wy);

  for (int x = x0; x < x1; ++x) {
    q[6] = load(x + 3, pw, wy);
    __syncthreads();  // previous plane's LDS reads are done
    for (int i = t; i < 2 * halo; i += ST_THREADS) {
      const int ff = (i < halo) ? (start - halo + i) : (start + ST_THREADS + (i - halo));
      const int w = floor_div(ff, plane);
      lds[(i < halo) ? i : i + ST_THREADS] = load(x, ff - w * plane, w);
    }
    lds[halo + t] = q[3];
    __syncthreads();
    if (active) {
      const T *L = lds + halo + t;
      const T c = q[3];
      const int64_t g = static_cast<int64_t>(x) * plane + f;
      T acc = St<T>::scale(G.c0 + v[g], c);
#pragma unroll
      for (int d = 1; d <= 3; ++d) {
        acc = acc + St<T>::scale(G.cx[d - 1], q[3 + d] + q[3 - d]);
        acc = acc + St<T>::scale(G.cy[d - 1], L[d * n2] + L[-d * n2]);
        const int wp = fold_count(z + d, n2), wm = fold_count(z - d, n2);
        T vp = L[d - wp * n2];
        T vm = L[-d - wm * n2];
        if (BLOCH) {
          vp = St<T>::phase(vp, G.phz[clamp3(wp) + 3]);
          vm = St<T>::phase(vm, G.phz[clamp3(wm) + 3]);
        }
        acc = acc + St<T>::scale(G.cz[d - 1], vp + vm);
      }
      if (ADD) acc = acc + addback_at<T>(ab, g, band);
      dst[g] = acc;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) q[d] = q[d + 1];
  }
}

template <typename T, bool ADD>
__global__ __launch_bounds__(256) void k_apply_S(const T *__restrict__ psi, T *__restrict__ out,
                                                 int64_t ng, AddArgs ab) {
  const int band = blockIdx.y;
  const int64_t base = static_cast<int64_t>(band) * ng;
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; g < ng;
       g += static_cast<int64_t>(gridDim.x) * 256) {
    T val = psi[base + g];
    if (ADD) val = val + addback_at<T>(ab, g, band);
    out[base + g] = val;
  }
}

// 6th-order central second-difference weights (h^2 d^2/dx^2)
constexpr double kW[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};

StencilGeom make_geom(const gpaw_sys *s, int nb) {
  StencilGeom G;
  G.n0 = s->n[0];
  G.n1 = s->n[1];
  G.n2 = s->n[2];
  double *cc[3] = {G.cx, G.cy, G.cz};
  G.c0 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double f = -0.5 / (s->h[c] * s->h[c]);
    G.c0 += f * kW[0];
    for (int d = 1; d <= 3; ++d) cc[c][d - 1] = f * kW[d];
  }
  z64 *ph[3] = {G.phx, G.phy, G.phz};
  for (int c = 0; c < 3; ++c) {
    const z64 p = s->phase[c];
    z64 pw = zmake(1.0, 0.0);
    ph[c][3] = pw;
    for (int w = 1; w <= 3; ++w) {
      pw = pw * p;
      ph[c][3 + w] = pw;
      ph[c][3 - w] = zconj(pw);
    }
  }
  const int plane = s->n[1] * s->n[2];
  const int chunks = (plane + ST_THREADS - 1) / ST_THREADS;
  const int64_t wgs = static_cast<int64_t>(chunks) * nb;
  int nseg = static_cast<int>((2048 + wgs - 1) / wgs);
  nseg = std::max(1, std::min(nseg, std::max(1, s->n[0] / 8)));
  G.xseg = (s->n[0] + nseg - 1) / nseg;
  return G;
}

AddArgs make_add(const gpaw_sys *s, const void *X) {
  AddArgs ab;
  ab.g2u = s->tab.g2u;
  ab.u_start = s->tab.u_start;
  ab.pm_atom = s->tab.pm_atom;
  ab.pm_q = s->tab.pm_q;
  ab.X = X;
  ab.nent = s->tab.nent;
  ab.ni = s->ni;
  ab.np = s->np;
  return ab;
}

template <typename T, bool BLOCH>
int stencil_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st) {
  const StencilGeom G = make_geom(s, nb);
  const AddArgs ab = make_add(s, X);
  const int plane = s->n[1] * s->n[2];
  const size_t lds = (ST_THREADS + 6 * static_cast<size_t>(s->n[2])) * sizeof(T);
  if (lds > 65536) return fail(GPAW_EINVAL, "n[2] too large for the stencil's LDS tile");
  dim3 grid((plane + ST_THREADS - 1) / ST_THREADS, nb, (s->n[0] + G.xseg - 1) / G.xseg);
  if (X)
    k_stencil<T, BLOCH, true><<<grid, ST_THREADS, lds, st>>>(
        static_cast<const T *>(psi), static_cast<T *>(out), s->v, G, ab);
  else
    k_stencil<T, BLOCH, false><<<grid, ST_THREADS, lds, st>>>(
        static_cast<const T *>(psi), static_cast<T *>(out), s->v, G, ab);
  return GPAW_OK;
}

template <typename T>
int apply_S_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st) {
  const AddArgs ab = make_add(s, X);
  const int64_t blocks = std::min<int64_t>((s->ng + 255) / 256, 4096);
  dim3 grid(static_cast<unsigned>(blocks), nb);
  if (X)
    k_apply_S<T, true><<<grid, 256, 0, st>>>(static_cast<const T *>(psi), static_cast<T *>(out),
                                             s->ng, ab);
  else
    k_apply_S<T, false><<<grid, 256, 0, st>>>(static_cast<const T *>(psi),
                                              static_cast<T *>(out), s->ng, ab);
  return GPAW_OK;
}

}  // namespace

int launch_stencil(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st) {
  if (s->dtype == GPAW_C128) return stencil_t<z64, true>(s, psi, nb, X, out, st);
  return stencil_t<double, false>(s, psi, nb, X, out, st);
}

int launch_apply_S(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st) {
  if (s->dtype == GPAW_C128) return apply_S_t<z64>(s, psi, nb, X, out, st);
  return apply_S_t<double>(s, psi, nb, X, out, st);
}

}  // namespace gfd
