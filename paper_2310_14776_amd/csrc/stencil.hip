// (T + v + non-local) applied to a block: the FD kinetic stencil of the
// grid representation (Sec. "Wave-function representations"), the local
// potential and the projector add-back of Eq. (dh); and the overlap
// operator S~ = 1 + sum |p> Delta S <p|.
//
// Kernel shape (gfx950): a workgroup of 256 lanes owns 256 consecutive points
// of one y-z plane (flattened, z contiguous, so every load is coalesced) for
// a group of bands, and marches along x over a segment of planes. The x
// neighbours live in a 7-deep register queue per lane and band; the y and z
// neighbours are read straight from the current plane, which the wavefronts
// of the workgroup have just brought into L1/L2, so the kernel needs no LDS
// tile and no barrier. Periodic/Bloch folding of every neighbour offset is
// worked out once per lane. The non-local add-back is fused into the store:
// each covered grid point sums q^a_i(r) (Delta.P)^a_i over the atoms whose
// spheres reach it, so H~psi leaves the kernel in one HBM pass.
#include <algorithm>
#include <type_traits>

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
  int chunks, ngroups, nseg;  // plane chunks of 256 points, band groups, x segments
};

struct AddArgs {
  const int4 *pinfo;       // [Ng] first three entry codes, count << 24 | first index
  const int32_t *pm_code;  // atom << 12 | image code
  const double *pos;       // [natoms][3]
  const void *X;           // [nb][Np] Delta.P
  const void *XS;          // [nb][Np] Delta S.P when S~psi is formed in the same pass
  const ProjDev *pj;
  int np;
  int natoms;
};

constexpr int POS_LDS_MAX = 1024;  // atoms whose positions are staged in LDS

// floor(a / b) for b > 0 and small |a / b| (|quotient| <= 3 in every use)
__device__ inline int fold_count(int a, int b) {
  int w = 0;
  while (a >= b) { a -= b; ++w; }
  while (a < 0) { a += b; --w; }
  return w;
}

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

__device__ inline int clamp3(int w) { return w < -3 ? -3 : (w > 3 ? 3 : w); }

// Non-local add-back for NB bands at grid point (ix, iy, iz) whose entry
// summary is pi: acc[b] += sum_entries phase * sum_i p_i(r) X[b][atom*ni + i].
// The projector values of an entry are evaluated once and reused for every
// band; X rows of the band group and the atom positions come from LDS when
// they fit (generic pointers otherwise).
template <typename T, int NI, int NB, bool S2, typename PJ>
__device__ inline void addback_group(const AddArgs &ab, const PJ &pj, int4 pi, int ix, int iy,
                                     int iz, const double *pos, const z64 *phs, const T *Xs,
                                     const T *XSs, int ldx, int ni, int b0, int nb,
                                     typename St<T>::Acc *acc, typename St<T>::Acc *accS) {
  using A = typename St<T>::Acc;
  constexpr bool FIXED = NI == 13;
  const int cnt = static_cast<int>(static_cast<unsigned>(pi.w) >> 24);
  const int first = pi.w & 0xFFFFFF;
  for (int j = 0; j < cnt; ++j) {
    const int code = j == 0 ? pi.x : (j == 1 ? pi.y : (j == 2 ? pi.z : ab.pm_code[first + j]));
    const int a = code >> 12;
    const int wx = ((code >> 8) & 15) - 8, wy = ((code >> 4) & 15) - 8, wz = (code & 15) - 8;
    const double *R = pos + 3 * a;
    const double dx = (ix + wx * pj.n[0]) * pj.h[0] - R[0];
    const double dy = (iy + wy * pj.n[1]) * pj.h[1] - R[1];
    const double dz = (iz + wz * pj.n[2]) * pj.h[2] - R[2];
    double pv[NI];
    if constexpr (FIXED) eval_proj13(pj, dx, dy, dz, pv);
    else eval_proj<NI>(pj, dx, dy, dz, pv);
    z64 ph = zmake(1.0, 0.0);
    if (St<T>::cplx) ph = phs[wx + 8] * phs[16 + wy + 8] * phs[32 + wz + 8];
    const T *Xa = Xs + a * (FIXED ? 13 : ni);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b0 + b >= nb) continue;
      const T *Xb = Xa + static_cast<int64_t>(b) * ldx;
      A sum = St<A>::zero();
#pragma unroll
      for (int i = 0; i < NI; ++i)
        if (FIXED || i < ni) sum = sum + St<A>::scale(pv[i], St<T>::widen(Xb[i]));
      acc[b] = acc[b] + St<A>::phase(sum, ph);
      if constexpr (S2) {
        // the overlap's add-back from the same projector values
        const T *XSb = XSs + a * (FIXED ? 13 : ni) + static_cast<int64_t>(b) * ldx;
        A sumS = St<A>::zero();
#pragma unroll
        for (int i = 0; i < NI; ++i)
          if (FIXED || i < ni) sumS = sumS + St<A>::scale(pv[i], St<T>::widen(XSb[i]));
        accS[b] = accS[b] + St<A>::phase(sumS, ph);
      }
    }
  }
}

// Per-axis image phases exp(-2 pi i k_c w), w = -8..7, into LDS (complex only)
__device__ inline const z64 *stage_phases(const AddArgs &ab, z64 *lds) {
  for (int idx = threadIdx.x; idx < 48; idx += blockDim.x) lds[idx] = ab.pj->ph[idx / 16][idx % 16];
  return lds;
}

// Atom positions into LDS (when they fit), else the global array.
__device__ inline const double *stage_pos(const AddArgs &ab, double *lds_pos, int natoms_lds) {
  if (!lds_pos) return ab.pos;
  for (int idx = threadIdx.x; idx < 3 * natoms_lds; idx += blockDim.x) lds_pos[idx] = ab.pos[idx];
  return lds_pos;
}

// Copies the band group's X rows into LDS (rows b >= nb are left unset); the
// rows of a group are contiguous in X
template <typename T, int NB>
__device__ inline void stage_x(const AddArgs &ab, int b0, int nb, T *xs, const void *Xsrc) {
  const T *X = static_cast<const T *>(Xsrc) + static_cast<int64_t>(b0) * ab.np;
  const int rows = nb - b0 < NB ? nb - b0 : NB;
  copy_rounds(xs, X, rows * ab.np, static_cast<int>(threadIdx.x), static_cast<int>(blockDim.x));
}

// SOUT: S~psi = psi + sum q^a (Delta S P)^a is formed in the same pass (the
// projector values and psi at the point are shared) and stored to outS.
template <typename T, bool BLOCH, bool ADD, bool XLDS, int NI, int NB, bool SOUT>
__global__ __launch_bounds__(ST_THREADS) void k_stencil(const T *__restrict__ psi,
                                                        T *__restrict__ out,
                                                        T *__restrict__ outS,
                                                        const double *__restrict__ v,
                                                        StencilGeom G, AddArgs ab, int nb) {
  extern __shared__ unsigned char smem[];
  const int n0 = G.n0, n1 = G.n1, n2 = G.n2;
  const int plane = n1 * n2;
  const int t = threadIdx.x;
  // Workgroups are dealt to the 8 XCDs round-robin by id. All plane chunks of
  // one (band group, x segment) get the same id residue, so the halo rows
  // they read from each other come from the same XCD's L2.
  // (with fewer than 8 such columns the plain order keeps every XCD busy)
  const int ncols = G.ngroups * G.nseg;
  int chunk, col;
  if (ncols >= 8) {
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    chunk = jj % G.chunks;
    col = (jj / G.chunks) * 8 + xcd;
  } else {
    chunk = blockIdx.x % G.chunks;
    col = blockIdx.x / G.chunks;
  }
  if (col >= ncols) return;
  const int grp = col % G.ngroups, seg = col / G.ngroups;
  const int b0 = grp * NB;
  const int64_t bstride = static_cast<int64_t>(n0) * plane;
  const int x0 = seg * G.xseg;
  const int x1 = min(n0, x0 + G.xseg);

  // X rows of this band group and the atom positions, staged in LDS
  const T *Xs = static_cast<const T *>(ab.X) + static_cast<int64_t>(b0) * ab.np;
  const T *XSs = SOUT && ADD ? static_cast<const T *>(ab.XS) + static_cast<int64_t>(b0) * ab.np
                             : nullptr;
  const double *pos = ab.pos;
  const z64 *phs = nullptr;
  if (ADD) {
    T *after = reinterpret_cast<T *>(smem);
    if (St<T>::cplx) {
      phs = stage_phases(ab, reinterpret_cast<z64 *>(smem));
      after = reinterpret_cast<T *>(smem + 48 * sizeof(z64));
    }
    if (XLDS) {
      stage_x<T, NB>(ab, b0, nb, after, ab.X);
      Xs = after;
      after += NB * ab.np;
      if (SOUT) {
        stage_x<T, NB>(ab, b0, nb, after, ab.XS);
        XSs = after;
        after += NB * ab.np;
      }
    }
    pos = stage_pos(ab, ab.natoms <= POS_LDS_MAX ? reinterpret_cast<double *>(after) : nullptr,
                    ab.natoms);
    __syncthreads();
  }
  typename PJSel<NI>::type pj = PJSel<NI>::get(ab.pj);
  const int ni = NI == 13 ? 13 : ab.pj->ni;
  const int f = chunk * ST_THREADS + t;
  if (f >= plane) return;
  const int y = f / n2, z = f - (f / n2) * n2;

  // in-plane neighbour offsets (folded) and Bloch phases: y +-d, z +-d
  int yo[6], zo[6];
  z64 yph[6], zph[6];
#pragma unroll
  for (int d = 1; d <= 3; ++d) {
#pragma unroll
    for (int sgn = 0; sgn < 2; ++sgn) {
      const int dd = sgn ? -d : d;
      const int wy = fold_count(y + dd, n1), wz = fold_count(z + dd, n2);
      yo[2 * (d - 1) + sgn] = (y + dd - wy * n1) * n2 + z;
      zo[2 * (d - 1) + sgn] = y * n2 + (z + dd - wz * n2);
      yph[2 * (d - 1) + sgn] = G.phy[clamp3(wy) + 3];
      zph[2 * (d - 1) + sgn] = G.phz[clamp3(wz) + 3];
    }
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
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      T val = St<T>::zero();
      if (b0 + b < nb) val = psi[(b0 + b) * bstride + off + f];
      q[b][d] = BLOCH ? St<T>::narrow(St<typename St<T>::Acc>::phase(St<T>::widen(val), ph)) : val;
    }
  }

  for (int x = x0; x < x1; ++x) {
    {
      z64 ph;
      const int64_t off = plane_of(x + 3, ph);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        T val = St<T>::zero();
        if (b0 + b < nb) val = psi[(b0 + b) * bstride + off + f];
        q[b][6] = BLOCH ? St<T>::narrow(St<typename St<T>::Acc>::phase(St<T>::widen(val), ph)) : val;
      }
    }
    const int64_t xoff = static_cast<int64_t>(x) * plane;
    const int64_t g = xoff + f;
    using A = typename St<T>::Acc;
    A acc[NB], accS[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[b] = St<A>::zero();
      accS[b] = St<A>::zero();
    }
    if (ADD)
      addback_group<T, NI, NB, SOUT>(ab, pj, ab.pinfo[g], x, y, z, pos, phs, Xs, XSs, ab.np, ni,
                                     b0, nb, acc, accS);
    const double cv = G.c0 + v[g];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b0 + b >= nb) continue;
      const T *Pb = psi + (b0 + b) * bstride + xoff;
      A r = acc[b] + St<A>::scale(cv, St<T>::widen(q[b][3]));
#pragma unroll
      for (int d = 1; d <= 3; ++d) {
        const int ip = 2 * (d - 1), im = ip + 1;
        A yp = St<T>::widen(Pb[yo[ip]]), ym = St<T>::widen(Pb[yo[im]]);
        A zp = St<T>::widen(Pb[zo[ip]]), zm = St<T>::widen(Pb[zo[im]]);
        if (BLOCH) {
          yp = St<A>::phase(yp, yph[ip]);
          ym = St<A>::phase(ym, yph[im]);
          zp = St<A>::phase(zp, zph[ip]);
          zm = St<A>::phase(zm, zph[im]);
        }
        r = r + St<A>::scale(G.cx[d - 1], St<T>::widen(q[b][3 + d]) + St<T>::widen(q[b][3 - d]));
        r = r + St<A>::scale(G.cy[d - 1], yp + ym);
        r = r + St<A>::scale(G.cz[d - 1], zp + zm);
      }
      out[(b0 + b) * bstride + g] = St<T>::narrow(r);
      if (SOUT) outS[(b0 + b) * bstride + g] = St<T>::narrow(St<T>::widen(q[b][3]) + accS[b]);
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
  const double *pos = ab.pos;
  const z64 *phs = nullptr;
  if (ADD) {
    T *after = reinterpret_cast<T *>(smem);
    if (St<T>::cplx) {
      phs = stage_phases(ab, reinterpret_cast<z64 *>(smem));
      after = reinterpret_cast<T *>(smem + 48 * sizeof(z64));
    }
    if (XLDS) {
      stage_x<T, NB>(ab, b0, nb, after, ab.X);
      Xs = after;
      after += NB * ab.np;
    }
    pos = stage_pos(ab, ab.natoms <= POS_LDS_MAX ? reinterpret_cast<double *>(after) : nullptr,
                    ab.natoms);
    __syncthreads();
  }
  typename PJSel<NI>::type pj = PJSel<NI>::get(ab.pj);
  const int ni = NI == 13 ? 13 : ab.pj->ni;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (g >= ng) return;
  using A = typename St<T>::Acc;
  A acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = St<A>::zero();
  if (ADD) {
    const int n1 = pj.n[1], n2 = pj.n[2];
    const int plane = n1 * n2;
    const int ix = static_cast<int>(g / plane);
    const int r = static_cast<int>(g - static_cast<int64_t>(ix) * plane);
    const int iy = r / n2, iz = r - iy * n2;
    addback_group<T, NI, NB, false>(ab, pj, ab.pinfo[g], ix, iy, iz, pos, phs, Xs, nullptr,
                                    ab.np, ni, b0, nb, acc, nullptr);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b)
    if (b0 + b < nb) {
      const int64_t idx = static_cast<int64_t>(b0 + b) * ng + g;
      out[idx] = St<T>::narrow(St<T>::widen(psi[idx]) + acc[b]);
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
  // The x march is latency-bound: split x into segments until the grid has
  // ~4096 workgroups, keeping segments >= 6 planes (each segment first reads
  // the 6 planes around its start).
  const int plane = s->n[1] * s->n[2];
  const int chunks = (plane + ST_THREADS - 1) / ST_THREADS;
  const int64_t wgs = static_cast<int64_t>(chunks) * nb;
  int nseg = static_cast<int>((4096 + wgs - 1) / wgs);
  nseg = std::max(1, std::min(nseg, std::max(1, s->n[0] / 6)));
  if (s->tune.st_nseg > 0) nseg = std::min(s->tune.st_nseg, s->n[0]);
  G.xseg = (s->n[0] + nseg - 1) / nseg;
  G.chunks = chunks;
  G.ngroups = nb;
  G.nseg = (s->n[0] + G.xseg - 1) / G.xseg;
  return G;
}

AddArgs make_add(const gpaw_sys *s, const void *X, const void *XS = nullptr) {
  AddArgs ab;
  ab.pinfo = s->tab.pinfo;
  ab.pm_code = s->tab.pm_code;
  ab.pos = s->tab.pos;
  ab.X = X;
  ab.XS = XS;
  ab.pj = s->tab.proj;
  ab.np = s->np;
  ab.natoms = s->natoms;
  return ab;
}

constexpr size_t XLDS_MAX = 32 * 1024;

template <typename T, bool BLOCH, int NB, int NI>
int stencil_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st, const void *XS = nullptr, void *outS = nullptr) {
  const int ngroups = (nb + NB - 1) / NB;
  const StencilGeom G = make_geom(s, ngroups);
  const AddArgs ab = make_add(s, X, XS);
  const bool sout = outS != nullptr;
  const size_t tile = 0;
  const size_t xbytes = static_cast<size_t>(NB) * s->np * sizeof(T) * (sout ? 2 : 1);
  const bool xlds = X && xbytes <= XLDS_MAX;
  const size_t pbytes = (X && s->natoms <= POS_LDS_MAX) ? 3 * sizeof(double) * s->natoms : 0;
  const size_t phb = (X && St<T>::cplx) ? 48 * sizeof(z64) : 0;
  const size_t lds = tile + phb + (xlds ? xbytes : 0) + pbytes;
  const int64_t cols = static_cast<int64_t>(G.ngroups) * G.nseg;
  const unsigned grid = static_cast<unsigned>((cols >= 8 ? (cols + 7) / 8 * 8 : cols) * G.chunks);
  const T *ps = static_cast<const T *>(psi);
  T *po = static_cast<T *>(out);
  T *pso = static_cast<T *>(outS);
  auto go = [&](auto sflag) {
    constexpr bool SO = decltype(sflag)::value;
    if (!X)
      k_stencil<T, BLOCH, false, false, NI, NB, SO><<<grid, ST_THREADS, lds, st>>>(ps, po, pso, s->v,
                                                                                  G, ab, nb);
    else if (xlds)
      k_stencil<T, BLOCH, true, true, NI, NB, SO><<<grid, ST_THREADS, lds, st>>>(ps, po, pso, s->v,
                                                                                G, ab, nb);
    else
      k_stencil<T, BLOCH, true, false, NI, NB, SO><<<grid, ST_THREADS, lds, st>>>(ps, po, pso, s->v,
                                                                                 G, ab, nb);
  };
  if (sout) go(std::true_type{});
  else go(std::false_type{});
  return GPAW_OK;
}

template <typename T, int NB, int NI>
int apply_S_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st) {
  const AddArgs ab = make_add(s, X);
  dim3 grid(static_cast<unsigned>((s->ng + 255) / 256), (nb + NB - 1) / NB);
  const size_t xbytes = static_cast<size_t>(NB) * s->np * sizeof(T);
  const bool xlds = X && xbytes <= XLDS_MAX;
  const size_t pbytes = (X && s->natoms <= POS_LDS_MAX) ? 3 * sizeof(double) * s->natoms : 0;
  const T *ps = static_cast<const T *>(psi);
  T *po = static_cast<T *>(out);
  const size_t phb = (X && St<T>::cplx) ? 48 * sizeof(z64) : 0;
  if (!X)
    k_apply_S<T, false, false, NI, NB><<<grid, 256, 0, st>>>(ps, po, s->ng, nb, ab);
  else if (xlds)
    k_apply_S<T, true, true, NI, NB><<<grid, 256, phb + xbytes + pbytes, st>>>(ps, po, s->ng, nb, ab);
  else
    k_apply_S<T, true, false, NI, NB><<<grid, 256, phb + pbytes, st>>>(ps, po, s->ng, nb, ab);
  return GPAW_OK;
}

}  // namespace

int launch_stencil(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st, const void *XS, void *outS) {
  const bool std13 = s->ni == 13 && s->proj.std13;
  switch (s->dtype) {
    case GPAW_C128:
      // one band per lane with projectors (shorter add-back per wave), two without
      if (std13 && (s->tune.st_nb == 1 || (s->tune.st_nb == 0 && X)))
        return stencil_t<z64, true, 1, 13>(s, psi, nb, X, out, st, XS, outS);
      return std13 ? stencil_t<z64, true, 2, 13>(s, psi, nb, X, out, st, XS, outS)
                   : stencil_t<z64, true, 2, PROJ_MAX_NI>(s, psi, nb, X, out, st, XS, outS);
    case GPAW_F32:
      return std13 ? stencil_t<float, false, 4, 13>(s, psi, nb, X, out, st, XS, outS)
                   : stencil_t<float, false, 4, PROJ_MAX_NI>(s, psi, nb, X, out, st, XS, outS);
    case GPAW_C64:
      return std13 ? stencil_t<z32, true, 2, 13>(s, psi, nb, X, out, st, XS, outS)
                   : stencil_t<z32, true, 2, PROJ_MAX_NI>(s, psi, nb, X, out, st, XS, outS);
    default:
      // two bands per lane with projectors, four without
      if (std13 && (s->tune.st_nb == 2 || (s->tune.st_nb == 0 && X)))
        return stencil_t<double, false, 2, 13>(s, psi, nb, X, out, st, XS, outS);
      return std13 ? stencil_t<double, false, 4, 13>(s, psi, nb, X, out, st, XS, outS)
                   : stencil_t<double, false, 4, PROJ_MAX_NI>(s, psi, nb, X, out, st, XS, outS);
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
