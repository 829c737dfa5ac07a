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

#include "proj.h"

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
  const int32_t *estart;   // [Ng+1] point-major entry ranges
  const int32_t *pm_code;  // atom << 12 | image code
  const double *pos;       // [natoms][3]
  const void *X;           // [nb][Np] Delta.P
  const ProjDev *pj;
  int np;
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

// Non-local add-back for NB bands at grid point g = (ix, iy, iz):
// acc[b] += sum_entries phase * sum_i p_i(r) X[b][atom*ni + i]. The projector
// values of an entry are evaluated once and reused for every band; X rows
// of the band group come from LDS (Xs, row stride ldx) or global memory.
template <typename T, int NI, int NB>
__device__ inline void addback_group(const AddArgs &ab, int64_t g, int ix, int iy, int iz,
                                     const T *Xs, int ldx, int b0, int nb, T *acc) {
  const int e0 = ab.estart[g], e1 = ab.estart[g + 1];
  const ProjDev &pj = *ab.pj;
  for (int e = e0; e < e1; ++e) {
    const int code = ab.pm_code[e];
    const int a = code >> 12;
    const int wx = ((code >> 8) & 15) - 8, wy = ((code >> 4) & 15) - 8, wz = (code & 15) - 8;
    const double *R = ab.pos + 3 * a;
    double pv[NI];
    eval_proj<NI>(pj, (ix + wx * pj.n[0]) * pj.h[0] - R[0], (iy + wy * pj.n[1]) * pj.h[1] - R[1],
                  (iz + wz * pj.n[2]) * pj.h[2] - R[2], pv);
    z64 ph = zmake(1.0, 0.0);
    if (St<T>::cplx) ph = image_phase(pj, wx, wy, wz);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b0 + b >= nb) continue;
      const T *Xb = Xs + static_cast<int64_t>(b) * ldx + a * pj.ni;
      T sum = St<T>::zero();
#pragma unroll
      for (int i = 0; i < NI; ++i)
        if (i < pj.ni) sum = sum + St<T>::scale(pv[i], Xb[i]);
      acc[b] = acc[b] + St<T>::phase(sum, ph);
    }
  }
}

// Copies the band group's X rows into LDS (rows b >= nb are left unset).
template <typename T, int NB>
__device__ inline void stage_x(const AddArgs &ab, int b0, int nb, T *xs) {
  const T *X = static_cast<const T *>(ab.X);
  const int tot = NB * ab.np;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int b = idx / ab.np;
    if (b0 + b < nb) xs[idx] = X[static_cast<int64_t>(b0) * ab.np + idx];
  }
}

constexpr int HALO_SLOTS = 4;  // 6*n2 <= 4*256, i.e. n2 <= 170

template <typename T, bool BLOCH, bool ADD, bool XLDS, int NI, int NB>
__global__ __launch_bounds__(ST_THREADS) void k_stencil(const T *__restrict__ psi,
                                                        T *__restrict__ out,
                                                        const double *__restrict__ v,
                                                        StencilGeom G, AddArgs ab, int nb) {
  extern __shared__ unsigned char smem[];
  const int n0 = G.n0, n2 = G.n2;
  const int plane = G.n1 * n2;
  const int halo = 3 * n2;
  const int span = ST_THREADS + 2 * halo;  // LDS slots per band
  T *lds = reinterpret_cast<T *>(smem);
  const int t = threadIdx.x;
  const int start = blockIdx.x * ST_THREADS;
  const int b0 = blockIdx.y * NB;
  const int64_t bstride = static_cast<int64_t>(n0) * plane;
  const int x0 = blockIdx.z * G.xseg;
  const int x1 = min(n0, x0 + G.xseg);

  // this lane's slot of the flattened plane, folded into the cell
  const int f = start + t;
  const int wy = floor_div(f, plane);
  const int pw = f - wy * plane;
  const bool active = f < plane;
  const int y = pw / n2;
  const int z = pw - y * n2;
  z64 ph_self = G.phy[clamp3(wy) + 3];
  // X rows of this band group (after the plane tiles in LDS)
  const T *Xs = static_cast<const T *>(ab.X) + static_cast<int64_t>(b0) * ab.np;
  if (ADD && XLDS) {
    T *xs = lds + NB * span;
    stage_x<T, NB>(ab, b0, nb, xs);
    Xs = xs;
  }

  // halo slots this lane fills for every plane: folded index and y phase
  int hp[HALO_SLOTS], hl[HALO_SLOTS];
  z64 hph[HALO_SLOTS];
#pragma unroll
  for (int s = 0; s < HALO_SLOTS; ++s) {
    const int i = t + s * ST_THREADS;
    hl[s] = -1;
    hp[s] = 0;
    hph[s] = zmake(1.0, 0.0);
    if (i < 2 * halo) {
      const int ff = (i < halo) ? (start - halo + i) : (start + ST_THREADS + (i - halo));
      const int w = floor_div(ff, plane);
      hp[s] = ff - w * plane;
      hl[s] = (i < halo) ? i : i + ST_THREADS;
      hph[s] = G.phy[clamp3(w) + 3];
    }
  }
  // z neighbours: LDS offsets and phases (fixed per lane)
  int zo[6];
  z64 zph[6];
#pragma unroll
  for (int d = 1; d <= 3; ++d) {
    const int wp = fold_count(z + d, n2), wm = fold_count(z - d, n2);
    zo[2 * (d - 1)] = d - wp * n2;
    zo[2 * (d - 1) + 1] = -d - wm * n2;
    zph[2 * (d - 1)] = G.phz[clamp3(wp) + 3];
    zph[2 * (d - 1) + 1] = G.phz[clamp3(wm) + 3];
  }

  auto plane_of = [&](int x, z64 &ph) -> int64_t {
    const int wx = fold_count(x, n0);
    ph = G.phx[clamp3(wx) + 3];
    return static_cast<int64_t>(x - wx * n0) * plane;
  };

  T q[NB][7];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    z64 ph;
    const int64_t off = plane_of(x0 + d - 3, ph);
    const z64 pt = ph * ph_self;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      T val = St<T>::zero();
      if (b0 + b < nb) val = psi[(b0 + b) * bstride + off + pw];
      q[b][d] = BLOCH ? St<T>::phase(val, pt) : val;
    }
  }

  for (int x = x0; x < x1; ++x) {
    {
      z64 ph;
      const int64_t off = plane_of(x + 3, ph);
      const z64 pt = ph * ph_self;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        T val = St<T>::zero();
        if (b0 + b < nb) val = psi[(b0 + b) * bstride + off + pw];
        q[b][6] = BLOCH ? St<T>::phase(val, pt) : val;
      }
    }
    __syncthreads();  // previous plane's LDS reads are done
    {
      z64 ph;
      const int64_t off = plane_of(x, ph);
#pragma unroll
      for (int s = 0; s < HALO_SLOTS; ++s) {
        if (hl[s] < 0) continue;
        const z64 pt = ph * hph[s];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          T val = St<T>::zero();
          if (b0 + b < nb) val = psi[(b0 + b) * bstride + off + hp[s]];
          lds[b * span + hl[s]] = BLOCH ? St<T>::phase(val, pt) : val;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) lds[b * span + halo + t] = q[b][3];
    __syncthreads();
    if (active) {
      const int64_t g = static_cast<int64_t>(x) * plane + f;
      T acc[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = St<T>::zero();
      if (ADD) addback_group<T, NI, NB>(ab, g, x, y, z, Xs, ab.np, b0, nb, acc);
      const double cv = G.c0 + v[g];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const T *L = lds + b * span + halo + t;
        T r = acc[b] + St<T>::scale(cv, q[b][3]);
#pragma unroll
        for (int d = 1; d <= 3; ++d) {
          r = r + St<T>::scale(G.cx[d - 1], q[b][3 + d] + q[b][3 - d]);
          r = r + St<T>::scale(G.cy[d - 1], L[d * n2] + L[-d * n2]);
          T vp = L[zo[2 * (d - 1)]], vm = L[zo[2 * (d - 1) + 1]];
          if (BLOCH) {
            vp = St<T>::phase(vp, zph[2 * (d - 1)]);
            vm = St<T>::phase(vm, zph[2 * (d - 1) + 1]);
          }
          r = r + St<T>::scale(G.cz[d - 1], vp + vm);
        }
        if (b0 + b < nb) out[(b0 + b) * bstride + g] = r;
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int d = 0; d < 6; ++d) q[b][d] = q[b][d + 1];
  }
}

// S~psi: one lane per grid point, NB bands per workgroup
template <typename T, bool ADD, bool XLDS, int NI, int NB>
__global__ __launch_bounds__(256) void k_apply_S(const T *__restrict__ psi, T *__restrict__ out,
                                                 int64_t ng, int nb, AddArgs ab) {
  extern __shared__ unsigned char smem[];
  const int b0 = blockIdx.y * NB;
  const T *Xs = static_cast<const T *>(ab.X) + static_cast<int64_t>(b0) * ab.np;
  if (ADD && XLDS) {
    T *xs = reinterpret_cast<T *>(smem);
    stage_x<T, NB>(ab, b0, nb, xs);
    __syncthreads();
    Xs = xs;
  }
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= ng) return;
  T acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = St<T>::zero();
  if (ADD) {
    const int n1 = ab.pj->n[1], n2 = ab.pj->n[2];
    const int plane = n1 * n2;
    const int ix = static_cast<int>(g / plane);
    const int r = static_cast<int>(g - static_cast<int64_t>(ix) * plane);
    const int iy = r / n2, iz = r - iy * n2;
    addback_group<T, NI, NB>(ab, g, ix, iy, iz, Xs, ab.np, b0, nb, acc);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b)
    if (b0 + b < nb) {
      const int64_t idx = static_cast<int64_t>(b0 + b) * ng + g;
      out[idx] = psi[idx] + acc[b];
    }
}

// 6th-order central second-difference weights (h^2 d^2/dx^2)
constexpr double kW[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};

StencilGeom make_geom(const gpaw_sys *s, int nb) {  // nb: band groups
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
  nseg = std::max(1, std::min(nseg, std::max(1, s->n[0] / 16)));
  G.xseg = (s->n[0] + nseg - 1) / nseg;
  return G;
}

AddArgs make_add(const gpaw_sys *s, const void *X) {
  AddArgs ab;
  ab.estart = s->tab.estart;
  ab.pm_code = s->tab.pm_code;
  ab.pos = s->tab.pos;
  ab.X = X;
  ab.pj = s->tab.proj;
  ab.np = s->np;
  return ab;
}

constexpr size_t XLDS_MAX = 32 * 1024;

template <typename T, bool BLOCH, int NB, int NI>
int stencil_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st) {
  const int ngroups = (nb + NB - 1) / NB;
  const StencilGeom G = make_geom(s, ngroups);
  const AddArgs ab = make_add(s, X);
  const int plane = s->n[1] * s->n[2];
  if (6 * s->n[2] > HALO_SLOTS * ST_THREADS)
    return fail(GPAW_EINVAL, "n[2] > 170 is not supported by the stencil tile");
  const size_t tile = static_cast<size_t>(NB) * (ST_THREADS + 6 * s->n[2]) * sizeof(T);
  const size_t xbytes = static_cast<size_t>(NB) * s->np * sizeof(T);
  const bool xlds = X && xbytes <= XLDS_MAX / 2;
  const size_t lds = tile + (xlds ? xbytes : 0);
  dim3 grid((plane + ST_THREADS - 1) / ST_THREADS, ngroups, (s->n[0] + G.xseg - 1) / G.xseg);
  const T *ps = static_cast<const T *>(psi);
  T *po = static_cast<T *>(out);
  if (!X)
    k_stencil<T, BLOCH, false, false, NI, NB><<<grid, ST_THREADS, lds, st>>>(ps, po, s->v, G, ab, nb);
  else if (xlds)
    k_stencil<T, BLOCH, true, true, NI, NB><<<grid, ST_THREADS, lds, st>>>(ps, po, s->v, G, ab, nb);
  else
    k_stencil<T, BLOCH, true, false, NI, NB><<<grid, ST_THREADS, lds, st>>>(ps, po, s->v, G, ab, nb);
  return GPAW_OK;
}

template <typename T, int NB, int NI>
int apply_S_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st) {
  const AddArgs ab = make_add(s, X);
  dim3 grid(static_cast<unsigned>((s->ng + 255) / 256), (nb + NB - 1) / NB);
  const size_t xbytes = static_cast<size_t>(NB) * s->np * sizeof(T);
  const bool xlds = X && xbytes <= XLDS_MAX;
  const T *ps = static_cast<const T *>(psi);
  T *po = static_cast<T *>(out);
  if (!X)
    k_apply_S<T, false, false, NI, NB><<<grid, 256, 0, st>>>(ps, po, s->ng, nb, ab);
  else if (xlds)
    k_apply_S<T, true, true, NI, NB><<<grid, 256, xbytes, st>>>(ps, po, s->ng, nb, ab);
  else
    k_apply_S<T, true, false, NI, NB><<<grid, 256, 0, st>>>(ps, po, s->ng, nb, ab);
  return GPAW_OK;
}

}  // namespace

int launch_stencil(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st) {
  const bool std13 = s->ni == 13 && s->proj.std13;
  if (s->dtype == GPAW_C128)
    return std13 ? stencil_t<z64, true, 2, 13>(s, psi, nb, X, out, st)
                 : stencil_t<z64, true, 2, PROJ_MAX_NI>(s, psi, nb, X, out, st);
  return std13 ? stencil_t<double, false, 4, 13>(s, psi, nb, X, out, st)
               : stencil_t<double, false, 4, PROJ_MAX_NI>(s, psi, nb, X, out, st);
}

int launch_apply_S(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st) {
  const bool std13 = s->ni == 13 && s->proj.std13;
  if (s->dtype == GPAW_C128)
    return std13 ? apply_S_t<z64, 8, 13>(s, psi, nb, X, out, st)
                 : apply_S_t<z64, 8, PROJ_MAX_NI>(s, psi, nb, X, out, st);
  return std13 ? apply_S_t<double, 16, 13>(s, psi, nb, X, out, st)
               : apply_S_t<double, 16, PROJ_MAX_NI>(s, psi, nb, X, out, st);
}

}  // namespace gfd
