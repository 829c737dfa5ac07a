// (T + v + non-local) applied to a block: the FD kinetic stencil of the
// grid representation (Sec. "Wave-function representations"), the local
// potential and the projector add-back of Eq. (dh); and the overlap
// operator S~ = 1 + sum |p> Delta S <p|.
//
// Kernel shape (gfx950), k_plane: a workgroup of 512 lanes owns a tile of
// TY x TZ points of the y-z plane (up to 512 PPL, PPL per lane) for NB
// bands and marches along x over a segment of planes. Per plane it
//   * keeps every owned point's x neighbours (planes x-3..x+3) in registers,
//     fed from a ring of loads issued PF planes ahead of use;
//   * writes the owned values of the current plane, and a 3-point halo
//     around the tile (loaded PF planes ahead, Bloch phases of wrapped
//     neighbours applied at the load), into one of two LDS buffers;
//   * after one barrier reads the y and z neighbours from LDS.
// So each grid value is read from HBM about once per band (plus the halo,
// which neighbouring tiles of the same column bring into the XCD's L2 at
// the same time), and the only other memory instructions are the two
// stores. The march is unrolled by the ring length PF + 1, so every ring
// slot index is a compile-time constant; the seven-plane window shifts by
// register moves of values whose loads have completed.
// The non-local add-back is fused into the store: each covered grid point
// sums q^a_i(r) (Delta.P)^a_i over the atoms whose spheres reach it, so
// H~psi (and S~psi with it) leaves the kernel in one HBM pass.
//
// This header holds the kernels and their host launch templates; each
// stencil_<dtype>.hip instantiates them for one dtype (compiled in
// parallel), stencil.hip dispatches.
#pragma once

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "proj.h"

namespace gfd {

namespace {

constexpr int PT_THREADS = 512;             // lanes per workgroup
constexpr int PT_CELLS = 1600;              // LDS cells per band buffer: (TY + 6)(TZ + 6)
constexpr int PT_PF = 2;                    // planes loaded ahead of use

struct PlaneGeom {
  int n0, n1, n2;
  double c0;                  // centre coefficient summed over the three axes
  double cx[3], cy[3], cz[3]; // -1/2 w_d / h_c^2, d = 1..3
  z64 phx[7], phy[7], phz[7]; // Bloch phase to the power w = -3..3
  int TY, TZ, LS;             // tile rows (y), columns (z), LDS row stride TZ + 6
  int tiles_z, tiles;         // tiles per plane
  int xseg, nseg, ngroups;    // planes per x segment, x segments, band groups
  int zbc;                    // zero boundary: values past the faces are zero
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
  double rcmax;  // largest projector cut-off radius
  int cap;       // k_plane: atoms whose X rows a workgroup stages in LDS
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

// Pointers with their address space spelled out, so that the LDS and the
// global-memory paths of the add-back stay two code paths with their own
// load instructions (a merged path through a generic pointer uses flat
// loads, which make every wait cover both counters). The host pass of the
// compiler sees plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using lds_cptr = const __attribute__((address_space(3))) T *;
template <typename T> using glb_cptr = const __attribute__((address_space(1))) T *;
#else
template <typename T> using lds_cptr = const T *;
template <typename T> using glb_cptr = const T *;
#endif

// Non-local add-back for NB bands at grid point (ix, iy, iz) whose entry
// summary is pi: acc[b] += sum_entries phase * sum_i p_i(r) X[b][atom*ni + i].
// The projector values of an entry are evaluated once and reused for every
// band.
//
// SLOT: slot[a] >= 0 (LDS) places atom a's position in lpos[3 slot] and its
// rows in Xl/XSl (row [b][slot][i], band stride ldl); atoms without a slot,
// or every atom without SLOT, read pos and Xs/XSs (band stride ldx,
// atom-major inside a band).
//
// Values read from global memory on the rare paths (entry codes past the
// three carried in pi, atoms without a slot) are waited for inside their
// branch: the empty asm statements take them as operands, so the wait is
// placed there and not where the paths join, where it would also wait for
// every prefetched load of the caller.
template <typename T, int NI, int NB, bool S2, typename PJ, bool SLOT = false, bool XG = false>
__device__ inline void addback_group(const AddArgs &ab, const PJ &pj, int4 pi, int ix, int iy,
                                     int iz, const double *pos, const z64 *phs, const T *Xs,
                                     const T *XSs, int ldx, int ni, int b0, int nb,
                                     typename St<T>::Acc *acc, typename St<T>::Acc *accS,
                                     const int *slot = nullptr, const double *lpos = nullptr,
                                     const T *Xl = nullptr, const T *XSl = nullptr,
                                     int ldl = 0) {
  using A = typename St<T>::Acc;
  constexpr bool FIXED = NI == 13;
  const int stride = FIXED ? 13 : ni;
  auto entry = [&](int code) {
    const int a = code >> 12;
    const int wx = ((code >> 8) & 15) - 8, wy = ((code >> 4) & 15) - 8, wz = (code & 15) - 8;
    int sl = -1;
    if constexpr (SLOT) sl = slot[a];
    double R0, R1, R2;
    if (sl >= 0) {
      R0 = lpos[3 * sl];
      R1 = lpos[3 * sl + 1];
      R2 = lpos[3 * sl + 2];
    } else {
      R0 = pos[3 * a];
      R1 = pos[3 * a + 1];
      R2 = pos[3 * a + 2];
      asm volatile("" : "+v"(R0), "+v"(R1), "+v"(R2));
    }
    const double dx = (ix + wx * pj.n[0]) * pj.h[0] - R0;
    const double dy = (iy + wy * pj.n[1]) * pj.h[1] - R1;
    const double dz = (iz + wz * pj.n[2]) * pj.h[2] - R2;
    double pv[NI];
    if constexpr (FIXED) eval_proj13(pj, dx, dy, dz, pv);
    else eval_proj<NI>(pj, dx, dy, dz, pv);
    z64 ph = zmake(1.0, 0.0);
    if (St<T>::cplx) ph = phs[wx + 8] * phs[16 + wy + 8] * phs[32 + wz + 8];
    // rows of the band group for this atom: staged (LDS) or global
    auto apply = [&](auto Xa, auto XSa, int ld) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b0 + b >= nb) continue;
        const auto Xb = Xa + static_cast<int64_t>(b) * ld;
        A sum = St<A>::zero();
#pragma unroll
        for (int i = 0; i < NI; ++i)
          if (FIXED || i < ni) {
            const T xv = Xb[i];
            sum = sum + St<A>::scale(pv[i], St<T>::widen(xv));
          }
        acc[b] = acc[b] + St<A>::phase(sum, ph);
        if constexpr (S2) {
          // the overlap's add-back from the same projector values
          const auto XSb = XSa + static_cast<int64_t>(b) * ld;
          A sumS = St<A>::zero();
#pragma unroll
          for (int i = 0; i < NI; ++i)
            if (FIXED || i < ni) {
              const T xv = XSb[i];
              sumS = sumS + St<A>::scale(pv[i], St<T>::widen(xv));
            }
          accS[b] = accS[b] + St<A>::phase(sumS, ph);
        }
      }
    };
    if constexpr (SLOT) {
      if (sl >= 0) {
        apply((lds_cptr<T>)(Xl + sl * stride), (lds_cptr<T>)(S2 ? XSl + sl * stride : Xl), ldl);
        return;
      }
    }
    if constexpr (XG)
      apply((glb_cptr<T>)(Xs + a * stride), (glb_cptr<T>)(S2 ? XSs + a * stride : Xs), ldx);
    else
      apply(Xs + a * stride, S2 ? XSs + a * stride : Xs, ldx);
  };
  const int cnt = static_cast<int>(static_cast<unsigned>(pi.w) >> 24);
  const int first = pi.w & 0xFFFFFF;
  const int c3 = cnt < 3 ? cnt : 3;
  for (int j = 0; j < c3; ++j) entry(j == 0 ? pi.x : (j == 1 ? pi.y : pi.z));
  for (int j = 3; j < cnt; ++j) {
    int code = ab.pm_code[first + j];
    asm volatile("" : "+v"(code));
    entry(code);
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

// Stencil arithmetic type: FP64 for the FP64 path; the precision form's
// stencil runs in FP32 (the add-back is summed in FP64 and rounded once).
template <typename T> struct SAcc { using type = typename St<T>::Acc; };
template <> struct SAcc<float> { using type = float; };
template <> struct SAcc<z32> { using type = z32; };
__device__ inline float s_widen(float a) { return a; }
__device__ inline z32 s_widen(z32 a) { return a; }
__device__ inline double s_widen(double a) { return a; }
__device__ inline z64 s_widen(z64 a) { return a; }
__device__ inline float s_scale(double c, float a) { return static_cast<float>(c) * a; }
__device__ inline z32 s_scale(double c, z32 a) {
  const float f = static_cast<float>(c);
  return z32{f * a.x, f * a.y};
}
__device__ inline double s_scale(double c, double a) { return c * a; }
__device__ inline z64 s_scale(double c, z64 a) { return c * a; }
__device__ inline double s_acc(float a) { return a; }
__device__ inline z64 s_acc(z32 a) { return z64{a.x, a.y}; }
__device__ inline double s_acc(double a) { return a; }
__device__ inline z64 s_acc(z64 a) { return a; }

// One band group over one x segment of one tile. SOUT: S~psi = psi +
// sum q^a (Delta S P)^a is formed in the same pass (the projector values
// and psi at the point are shared) and stored to outS.
//
// Lanes without a point of the tile (ragged tiles) or a halo cell load from
// a clamped in-bounds offset and write to a spare LDS cell, and bands past
// nb load band nb - 1, so loads and LDS writes need no branches; only the
// global stores are masked. The 13-projector parameters are staged in LDS
// (read where an entry is evaluated) to keep scalar registers free.
template <typename T, bool BLOCH, bool ADD, bool XLDS, int NI, int NB, bool SOUT, int PPL>
__global__ __launch_bounds__(PT_THREADS) void k_plane(const T *__restrict__ psi,
                                                      T *__restrict__ out,
                                                      T *__restrict__ outS,
                                                      const double *__restrict__ v,
                                                      PlaneGeom G, AddArgs ab, int nb) {
  constexpr int PF = PT_PF;
  constexpr int HR = PF + 1;  // load rings: planes x+3 .. x+3+PF (owned), x .. x+PF (halo)
  constexpr int HPL = PPL;    // halo cells per lane
  using A = typename St<T>::Acc;
  using SA = typename SAcc<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n0 = G.n0, n1 = G.n1, n2 = G.n2;
  const int plane = n1 * n2;
  const int t = threadIdx.x;
  // Workgroups are dealt to the 8 XCDs round-robin by id. All tiles of one
  // (band group, x segment) column get the same id residue, so the halo
  // rows they read from each other come from the same XCD's L2.
  const int ncols = G.ngroups * G.nseg;
  int tile, col;
  if (ncols >= 8) {
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    tile = jj % G.tiles;
    col = (jj / G.tiles) * 8 + xcd;
  } else {
    tile = blockIdx.x % G.tiles;
    col = blockIdx.x / G.tiles;
  }
  if (col >= ncols) return;  // whole workgroup: no barrier is reached
  const int grp = col % G.ngroups, seg = col / G.ngroups;
  const int b0 = grp * NB;
  const int64_t bstride = static_cast<int64_t>(n0) * plane;
  const int x0 = seg * G.xseg;
  const int x1 = min(n0, x0 + G.xseg);

  // LDS: two plane buffers [2][NB][cells + 1] (the last cell of each band
  // buffer is the spare), then the add-back staging
  const int cells = (G.TY + 6) * G.LS + 1;
  const int spare = cells - 1;
  T *lbuf = reinterpret_cast<T *>(smem);
  unsigned char *after = smem + ((2 * NB * cells * sizeof(T) + 15) / 16) * 16;
  const T *Xs = static_cast<const T *>(ab.X) + static_cast<int64_t>(b0) * ab.np;
  const T *XSs = SOUT && ADD ? static_cast<const T *>(ab.XS) + static_cast<int64_t>(b0) * ab.np
                             : nullptr;
  const z64 *phs = nullptr;
  Proj13 *pjl = nullptr;
  if (ADD) {
    if (NI == 13) {
      pjl = reinterpret_cast<Proj13 *>(after);
      if (t == 0) *pjl = load_proj13(*ab.pj);
      after += (sizeof(Proj13) + 15) / 16 * 16;
    }
    if (St<T>::cplx) {
      phs = stage_phases(ab, reinterpret_cast<z64 *>(after));
      after += 48 * sizeof(z64);
    }
  }
  const int ni = NI == 13 ? 13 : ab.pj->ni;

  // tile geometry; TYe x TZe points of the tile lie inside the grid
  const int ty = tile / G.tiles_z, tz = tile - (tile / G.tiles_z) * G.tiles_z;
  const int y0 = ty * G.TY, z0 = tz * G.TZ;
  const int TYe = min(G.TY, n1 - y0), TZe = min(G.TZ, n2 - z0);
  const int LS = G.LS;

  // XLDS: the atoms whose spheres (any periodic image) reach the tile's y-z
  // footprint get LDS slots (the first ab.cap of them, in any order: a slot
  // only says where a row is kept); their positions and X rows of this band
  // group are staged, and the add-back reads the others from global memory
  int *slot = nullptr;
  const double *lpos = nullptr;
  const T *Xl = nullptr, *XSl = nullptr;
  int ldl = 0;
  if (ADD && XLDS) {
    slot = reinterpret_cast<int *>(after);
    int *list = slot + ab.natoms;
    int *count = list + ab.cap;
    double *lp = reinterpret_cast<double *>(
        after + ((sizeof(int) * (ab.natoms + ab.cap + 1) + 15) / 16) * 16);
    T *xl = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(lp) +
                                  ((3 * sizeof(double) * ab.cap + 15) / 16) * 16);
    if (t == 0) *count = 0;
    __syncthreads();
    const double h1 = ab.pj->h[1], h2 = ab.pj->h[2];
    const double L1 = n1 * h1, L2 = n2 * h2;
    const double ya = y0 * h1, wy = (TYe - 1) * h1, za = z0 * h2, wz = (TZe - 1) * h2;
    const double reach = ab.rcmax * (1.0 + 1e-12);
    for (int a = t; a < ab.natoms; a += PT_THREADS) {
      // periodic distance from the atom to the footprint, per axis
      double dy = ab.pos[3 * a + 1] - ya, dz = ab.pos[3 * a + 2] - za;
      dy -= floor(dy / L1) * L1;
      dz -= floor(dz / L2) * L2;
      const double ey = dy <= wy ? 0.0 : fmin(dy - wy, L1 - dy);
      const double ez = dz <= wz ? 0.0 : fmin(dz - wz, L2 - dz);
      int sl = -1;
      if (ey <= reach && ez <= reach) {
        const int k = atomicAdd(count, 1);
        if (k < ab.cap) {
          sl = k;
          list[k] = a;
        }
      }
      slot[a] = sl;
    }
    __syncthreads();
    const int nl = min(*count, ab.cap);
    ldl = nl * ni;
    for (int e = t; e < 3 * nl; e += PT_THREADS) lp[e] = ab.pos[3 * list[e / 3] + e % 3];
    const int rows = min(NB, nb - b0);
    const T *Xg = static_cast<const T *>(ab.X) + static_cast<int64_t>(b0) * ab.np;
    const T *XSg = SOUT ? static_cast<const T *>(ab.XS) + static_cast<int64_t>(b0) * ab.np
                        : nullptr;
    for (int e = t; e < rows * ldl; e += PT_THREADS) {
      const int b = e / ldl, r = e - b * ldl, k = r / ni, i = r - k * ni;
      const int64_t src = static_cast<int64_t>(b) * ab.np + list[k] * ni + i;
      xl[e] = Xg[src];
      if (SOUT) xl[NB * ldl + e] = XSg[src];
    }
    lpos = lp;
    Xl = xl;
    XSl = xl + NB * ldl;
  }

  // owned points p = t + k * 512 of the tile, row-major over TYe x TZe
  bool own[PPL];
  int goff[PPL], lc[PPL], lw[PPL], py[PPL], pz[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int p = t + k * PT_THREADS;
    own[k] = p < TYe * TZe;
    const int yy = own[k] ? p / TZe : 0;
    const int zz = own[k] ? p - yy * TZe : 0;
    py[k] = y0 + yy;
    pz[k] = z0 + zz;
    goff[k] = py[k] * n2 + pz[k];
    lc[k] = (yy + 3) * LS + zz + 3;
    lw[k] = own[k] ? lc[k] : spare;
  }
  // halo cells h = t + k * 512: three full rows above and below the tile,
  // three cells left and right of every tile row; each maps to a folded
  // in-plane position whose wrap across the y and z faces gives its phase
  const int W = TZe + 6;
  const int nh = 6 * W + 6 * TYe;
  int hoff[HPL], hl[HPL];
  bool hzero[HPL];  // zero boundary, real kernels: the cell lies past a face
  z64 hph[HPL];
#pragma unroll
  for (int k = 0; k < HPL; ++k) {
    const int h = t + k * PT_THREADS;
    int r = 0, c = 0;
    if (h < 3 * W) {
      r = h / W;
      c = h - r * W;
    } else if (h < 3 * W + 6 * TYe) {
      const int q = h - 3 * W;
      r = 3 + q / 6;
      const int m = q - (q / 6) * 6;
      c = m < 3 ? m : TZe + m;
    } else if (h < nh) {
      const int q = h - 3 * W - 6 * TYe;
      r = TYe + 3 + q / W;
      c = q - (q / W) * W;
    }
    const int yg = y0 + r - 3, zg = z0 + c - 3;
    const int wy = fold_count(yg, n1), wz = fold_count(zg, n2);
    hoff[k] = (yg - wy * n1) * n2 + (zg - wz * n2);
    hph[k] = BLOCH ? G.phy[clamp3(wy) + 3] * G.phz[clamp3(wz) + 3] : zmake(1.0, 0.0);
    hzero[k] = !BLOCH && G.zbc && (wy != 0 || wz != 0);
    hl[k] = h < nh ? r * LS + c : spare;
  }

  // band rows: bands past nb read the last band (their results are not stored)
  int64_t brow[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) brow[b] = static_cast<int64_t>(min(b0 + b, nb - 1)) * bstride;

  // owned values of plane xp (any integer: folded), as loaded; the x Bloch
  // phase of the fold is applied where a value enters the window, so a
  // prefetched load is not waited for before its plane is reached
  auto load_own = [&](T (&dst)[NB][PPL], int xp) {
    const int wx = fold_count(xp, n0);
    const int64_t off = static_cast<int64_t>(xp - wx * n0) * plane;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int k = 0; k < PPL; ++k) dst[b][k] = psi[brow[b] + off + goff[k]];
  };
  auto phase_own = [&](T (&dst)[NB][PPL], const T (&src)[NB][PPL], int xp) {
    if constexpr (BLOCH) {
      const z64 ph = G.phx[clamp3(fold_count(xp, n0)) + 3];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < PPL; ++k)
          dst[b][k] = St<T>::narrow(St<A>::phase(St<T>::widen(src[b][k]), ph));
    } else {
      // zero boundary: a plane past a face is zero (uniform over the
      // workgroup: one scalar test per plane)
      const bool past = G.zbc && (xp < 0 || xp >= n0);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < PPL; ++k) dst[b][k] = past ? T{} : src[b][k];
    }
  };
  // halo values of plane xp (inside the grid), as loaded (phases at the
  // LDS write); with them the potential and, for the add-back, the entry
  // summaries of the owned points of plane xp
  auto load_halo = [&](T (&dst)[NB][HPL], double (&vd)[PPL], int4 (&pd)[PPL], int xp) {
    const int64_t off = static_cast<int64_t>(xp) * plane;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int k = 0; k < HPL; ++k) dst[b][k] = psi[brow[b] + off + hoff[k]];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      vd[k] = v[off + goff[k]];
      if (ADD) pd[k] = ab.pinfo[off + goff[k]];
    }
  };

  T q[7][NB][PPL];    // planes x-3 .. x+3 of the owned points at step x
  T pq[HR][NB][PPL];  // owned loads in flight: slot (p - x0) mod HR holds plane p + 3
  T hq[HR][NB][HPL];  // halo loads in flight: slot (p - x0) mod HR holds plane p
  double vq[HR][PPL]; // potential of plane p, same slots
  int4 iq[HR][PPL];   // entry summaries of plane p (add-back), same slots
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    load_own(pq[0], x0 - 3 + s);
    phase_own(q[s + 1], pq[0], x0 - 3 + s);
  }
#pragma unroll
  for (int s = 0; s < HR - 1; ++s) {
    load_own(pq[s], x0 + 3 + s);
    load_halo(hq[s], vq[s], iq[s], min(x0 + s, n0 - 1));
  }
  if (ADD) __syncthreads();  // staged add-back operands

  for (int xb = x0; xb < x1; xb += HR) {
#pragma unroll
    for (int k = 0; k < HR; ++k) {
      const int x = xb + k;
      if (x >= x1) break;  // uniform over the workgroup
      // shift the window: plane x+3 arrives from the ring (its load was
      // issued PF steps ago); then the loads for PF steps from now
#pragma unroll
      for (int s = 0; s < 6; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int j = 0; j < PPL; ++j) q[s][b][j] = q[s + 1][b][j];
      phase_own(q[6], pq[k], x + 3);
      // issued on every step (past the segment end they read planes that
      // are never used, clamped into the grid): a load that only some
      // paths issue makes the compiler wait for every load in flight
      load_own(pq[(k + PF) % HR], x + 3 + PF);
      load_halo(hq[(k + PF) % HR], vq[(k + PF) % HR], iq[(k + PF) % HR], min(x + PF, n0 - 1));
      // plane x into LDS buffer (x - x0) & 1
      T *L = lbuf + ((x - x0) & 1) * NB * cells;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int j = 0; j < PPL; ++j) L[b * cells + lw[j]] = q[3][b][j];
#pragma unroll
        for (int j = 0; j < HPL; ++j)
          L[b * cells + hl[j]] =
              BLOCH ? St<T>::narrow(St<A>::phase(St<T>::widen(hq[k][b][j]), hph[j]))
                    : (hzero[j] ? T{} : hq[k][b][j]);
      }
      // one barrier per plane: the buffer written next step was last read
      // before every lane arrived here
      __syncthreads();
      const int64_t xoff = static_cast<int64_t>(x) * plane;
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const int64_t g = xoff + goff[j];
        A acc[NB], accS[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[b] = St<A>::zero();
          accS[b] = St<A>::zero();
        }
        if (ADD) {
          int4 pi = iq[k][j];
          pi.w = own[j] ? pi.w : 0;  // a select, not a branch (see the loads)
          if constexpr (NI == 13)
            addback_group<T, NI, NB, SOUT, Proj13, XLDS, true>(ab, *pjl, pi, x, py[j], pz[j], ab.pos,
                                                         phs, Xs, XSs, ab.np, ni, b0, nb, acc,
                                                         accS, slot, lpos, Xl, XSl, ldl);
          else
            addback_group<T, NI, NB, SOUT, ProjDev, XLDS, true>(ab, *ab.pj, pi, x, py[j], pz[j],
                                                          ab.pos, phs, Xs, XSs, ab.np, ni, b0, nb,
                                                          acc, accS, slot, lpos, Xl, XSl, ldl);
        }
        const double cv = G.c0 + vq[k][j];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const T *Lb = L + b * cells + lc[j];
          const SA ctr = s_widen(q[3][b][j]);
          SA r;
          if constexpr (St<T>::single) {
            // single precision: the kinetic part as sum_d c_d ((u_+d - u) +
            // (u_-d - u)) (the weights of each axis sum to zero), so the
            // neighbour differences of a smooth function are exact and the
            // cancellation of the weighted sum does not cost FP32 digits
            r = s_scale(cv - G.c0, ctr);
#pragma unroll
            for (int d = 1; d <= 3; ++d) {
              const SA xs = (s_widen(q[3 + d][b][j]) - ctr) + (s_widen(q[3 - d][b][j]) - ctr);
              const SA ys = (s_widen(Lb[d * LS]) - ctr) + (s_widen(Lb[-d * LS]) - ctr);
              const SA zs = (s_widen(Lb[d]) - ctr) + (s_widen(Lb[-d]) - ctr);
              r = r + s_scale(G.cx[d - 1], xs);
              r = r + s_scale(G.cy[d - 1], ys);
              r = r + s_scale(G.cz[d - 1], zs);
            }
          } else {
            r = s_scale(cv, ctr);
#pragma unroll
            for (int d = 1; d <= 3; ++d) {
              const SA xs = s_widen(q[3 + d][b][j]) + s_widen(q[3 - d][b][j]);
              const SA ys = s_widen(Lb[d * LS]) + s_widen(Lb[-d * LS]);
              const SA zs = s_widen(Lb[d]) + s_widen(Lb[-d]);
              r = r + s_scale(G.cx[d - 1], xs);
              r = r + s_scale(G.cy[d - 1], ys);
              r = r + s_scale(G.cz[d - 1], zs);
            }
          }
          if (own[j] && b0 + b < nb) {
            const int64_t o = (b0 + b) * bstride + g;
            out[o] = St<T>::narrow(s_acc(r) + acc[b]);
            if (SOUT) outS[o] = St<T>::narrow(St<T>::widen(q[3][b][j]) + accS[b]);
          }
        }
      }
    }
  }
}

// S~psi: one lane per grid point, NB bands per workgroup; a workgroup walks
// AS_CHUNKS consecutive runs of 256 points, so the atom positions and phases
// it stages in LDS serve all of them
constexpr int AS_CHUNKS = 8;

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
  using A = typename St<T>::Acc;
  for (int c = 0; c < AS_CHUNKS; ++c) {
    const int64_t g = (static_cast<int64_t>(blockIdx.x) * AS_CHUNKS + c) * 256 + threadIdx.x;
    if (g >= ng) return;  // no barrier follows
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
}

// Non-local add-back as a pass of its own over the covered grid points (the
// points some projector sphere reaches), used for large blocks: the stencil
// kernel then runs without atoms (H~psi = (T + v) psi, S~psi = psi) at the
// occupancy and instruction count of the atom-free case, and here one lane
// per covered point adds sum_entries q (Delta H P) and q (Delta S P) to NB
// bands, the projector values of an entry evaluated once for the NB bands.
// Covered points are listed in increasing order, so a wavefront's lanes
// mostly touch consecutive points. A workgroup walks AB_CHUNKS runs of 256
// covered points: it first marks the atoms their entries name, gives the
// first ab.cap of them LDS slots and stages their positions and X rows of
// the band group there (the add-back reads the others from global memory),
// then adds. Its staged phases and slots serve all of its points.
constexpr int AB_CHUNKS = 2;
constexpr size_t AB_LDS = 60 * 1024;     // LDS of one add-back workgroup
constexpr size_t XLDS_MAX = 24 * 1024;  // k_plane: staged X rows of the atoms reaching a tile
constexpr int SLOT_ATOMS_MAX = 4096;     // atoms with a slot index in LDS

template <typename T, int NI, int NB, bool S2>
__global__ __launch_bounds__(256) void k_addback(T *__restrict__ out, T *__restrict__ outS,
                                                 const int32_t *__restrict__ cov, int64_t ncov,
                                                 int64_t ng, int nb, AddArgs ab) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  const int b0 = blockIdx.y * NB;
  const z64 *phs = nullptr;
  unsigned char *after = smem;
  if (St<T>::cplx) {
    phs = stage_phases(ab, reinterpret_cast<z64 *>(smem));
    after = smem + 48 * sizeof(z64);
  }
  const bool pos_lds = ab.natoms <= POS_LDS_MAX;
  const double *pos = stage_pos(ab, pos_lds ? reinterpret_cast<double *>(after) : nullptr,
                                ab.natoms);
  if (pos_lds) after += ((3 * sizeof(double) * ab.natoms + 15) / 16) * 16;
  // slots: slot[natoms], list[cap], count, then positions and X rows
  int *slot = reinterpret_cast<int *>(after);
  int *list = slot + ab.natoms;
  int *count = list + ab.cap;
  double *lp = reinterpret_cast<double *>(
      after + ((sizeof(int) * (ab.natoms + ab.cap + 1) + 15) / 16) * 16);
  T *xl = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(lp) +
                                ((3 * sizeof(double) * ab.cap + 15) / 16) * 16);
  if (t == 0) *count = 0;
  for (int a = t; a < ab.natoms; a += 256) slot[a] = -1;
  __syncthreads();
  const int64_t cbase = static_cast<int64_t>(blockIdx.x) * AB_CHUNKS * 256;
  // mark the atoms named by the entries of this workgroup's points (every
  // writer stores the same value)
  for (int c = 0; c < AB_CHUNKS; ++c) {
    const int64_t ci = cbase + c * 256 + t;
    if (ci >= ncov) break;
    const int4 pi = ab.pinfo[cov[ci]];
    const int cnt = static_cast<int>(static_cast<unsigned>(pi.w) >> 24);
    const int first = pi.w & 0xFFFFFF;
    for (int j = 0; j < cnt; ++j) {
      const int code = j == 0 ? pi.x : (j == 1 ? pi.y : (j == 2 ? pi.z : ab.pm_code[first + j]));
      slot[code >> 12] = -2;
    }
  }
  __syncthreads();
  for (int a = t; a < ab.natoms; a += 256) {
    if (slot[a] != -2) continue;
    const int k = atomicAdd(count, 1);
    slot[a] = k < ab.cap ? k : -1;
    if (k < ab.cap) list[k] = a;
  }
  __syncthreads();
  const int nl = min(*count, ab.cap);
  const int ni = NI == 13 ? 13 : ab.pj->ni;
  const int ldl = nl * ni;
  for (int e = t; e < 3 * nl; e += 256) lp[e] = ab.pos[3 * list[e / 3] + e % 3];
  const int rows = min(NB, nb - b0);
  const T *Xg = static_cast<const T *>(ab.X) + static_cast<int64_t>(b0) * ab.np;
  const T *XSg = S2 ? static_cast<const T *>(ab.XS) + static_cast<int64_t>(b0) * ab.np : nullptr;
  for (int e = t; e < rows * ldl; e += 256) {
    const int b = e / ldl, r = e - b * ldl, k = r / ni, i = r - k * ni;
    const int64_t src = static_cast<int64_t>(b) * ab.np + list[k] * ni + i;
    xl[e] = Xg[src];
    if (S2) xl[NB * ldl + e] = XSg[src];
  }
  __syncthreads();
  typename PJSel<NI>::type pj = PJSel<NI>::get(ab.pj);
  const T *Xs = Xg;
  const T *XSs = S2 ? XSg : Xg;
  using A = typename St<T>::Acc;
  const int n1 = pj.n[1], n2 = pj.n[2];
  const int plane = n1 * n2;
  for (int c = 0; c < AB_CHUNKS; ++c) {
    const int64_t ci = cbase + c * 256 + t;
    if (ci >= ncov) return;  // no barrier follows
    const int64_t g = cov[ci];
    const int ix = static_cast<int>(g / plane);
    const int r = static_cast<int>(g - static_cast<int64_t>(ix) * plane);
    const int iy = r / n2, iz = r - iy * n2;
    A acc[NB], accS[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[b] = St<A>::zero();
      accS[b] = St<A>::zero();
    }
    addback_group<T, NI, NB, S2, typename PJSel<NI>::type, true, true>(
        ab, pj, ab.pinfo[g], ix, iy, iz, pos, phs, Xs, XSs, ab.np, ni, b0, nb, acc, accS, slot,
        lp, xl, S2 ? xl + NB * ldl : xl, ldl);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b0 + b < nb) {
        const int64_t idx = static_cast<int64_t>(b0 + b) * ng + g;
        out[idx] = St<T>::narrow(St<T>::widen(out[idx]) + acc[b]);
        if (S2) outS[idx] = St<T>::narrow(St<T>::widen(outS[idx]) + accS[b]);
      }
  }
}

// 6th-order central second-difference weights (h^2 d^2/dx^2)
constexpr double kW[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};

// points per lane of the stencil: the tuned value, else one
int stencil_ppl(const gpaw_sys *s) { return s->tune.st_ppl == 2 ? 2 : 1; }

// Tiles of the y-z plane that fit the lanes and the LDS buffer, cheapest
// estimated cost per plane first. Each tile-plane costs one step of the
// workgroup (a fixed amount of work however full the tile is) plus its halo
// loads; z columns are split evenly.
std::vector<std::pair<int, int>> tile_candidates(int n1, int n2, int ppl, size_t keep) {
  const int TILE = PT_THREADS * ppl;
  std::vector<std::pair<double, std::pair<int, int>>> all;
  for (int tz = 1; tz <= std::min(n2, TILE); ++tz) {
    const int tzt = (n2 + tz - 1) / tz;
    if ((n2 + tzt - 1) / tzt != tz) continue;
    for (int ty = 1; ty <= std::min(n1, TILE / tz); ++ty) {
      if ((ty + 6) * (tz + 6) > PT_CELLS || 6 * (tz + 6) + 6 * ty > TILE) continue;
      const int tyt = (n1 + ty - 1) / ty;
      if (ty < n1 && (n1 + tyt - 1) / tyt != ty) continue;  // even rows too
      const double tiles = static_cast<double>(tyt) * tzt;
      const double halo = tiles * (6.0 * (tz + 6) + 6.0 * ty);
      all.push_back({tiles * TILE + 2.0 * halo, {ty, tz}});
    }
  }
  std::sort(all.begin(), all.end());
  std::vector<std::pair<int, int>> out;
  for (size_t i = 0; i < all.size() && out.size() < keep; ++i) out.push_back(all[i].second);
  return out;
}

PlaneGeom make_geom(const gpaw_sys *s, int ngroups, int ppl) {
  PlaneGeom G;
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
      // zero boundary: a neighbour past a face is zero (factor 0)
      ph[c][3 + w] = s->zbc ? zmake(0.0, 0.0) : pw;
      ph[c][3 - w] = s->zbc ? zmake(0.0, 0.0) : zconj(pw);
    }
  }
  G.zbc = s->zbc;
  const int TILE = PT_THREADS * ppl;
  const auto best = tile_candidates(s->n[1], s->n[2], ppl, 1);
  int TY = best[0].first, TZ = best[0].second;
  if (s->tune.st_ty > 0 && s->tune.st_tz > 0 &&
      (s->tune.st_ty + 6) * (s->tune.st_tz + 6) <= PT_CELLS &&
      s->tune.st_ty * s->tune.st_tz <= TILE &&
      6 * (s->tune.st_tz + 6) + 6 * s->tune.st_ty <= TILE) {
    TY = std::min(s->tune.st_ty, s->n[1]);
    TZ = std::min(s->tune.st_tz, s->n[2]);
  }
  G.TY = TY;
  G.TZ = TZ;
  G.LS = TZ + 6;
  G.tiles_z = (s->n[2] + TZ - 1) / TZ;
  G.tiles = ((s->n[1] + TY - 1) / TY) * G.tiles_z;
  // x segments: enough workgroups for ~8 per CU, segments of at least 12
  // planes (each segment first reads the 6 planes around its start)
  const int64_t wgs = static_cast<int64_t>(G.tiles) * ngroups;
  int nseg = static_cast<int>((2048 + wgs - 1) / wgs);
  nseg = std::max(1, std::min(nseg, std::max(1, s->n[0] / 12)));
  if (s->tune.st_nseg > 0) nseg = std::min(s->tune.st_nseg, s->n[0]);
  G.xseg = (s->n[0] + nseg - 1) / nseg;
  G.ngroups = ngroups;
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
  ab.rcmax = 0.0;
  for (int c = 0; c < s->proj.nchan; ++c)
    ab.rcmax = std::max(ab.rcmax, 1.0 / std::sqrt(s->proj.rc2inv[c]));
  ab.cap = 0;
  return ab;
}

// Bands per lane of the separate add-back
template <typename T> struct AddbackNB { static constexpr int value = St<T>::cplx ? 8 : 16; };

template <typename T, int NI>
int addback_t(const gpaw_sys *s, int nb, const void *X, const void *XS, void *out, void *outS,
              hipStream_t st) {
  constexpr int NB = AddbackNB<T>::value;
  AddArgs ab = make_add(s, X, XS);
  const int64_t ncov = s->tab.ncov;
  if (ncov == 0) return GPAW_OK;
  dim3 grid(static_cast<unsigned>((ncov + 256 * AB_CHUNKS - 1) / (256 * AB_CHUNKS)),
            (nb + NB - 1) / NB);
  // phases, positions and the slot table first; the rest of AB_LDS holds
  // as many atoms' positions and X rows as fit (at least one)
  const size_t row = static_cast<size_t>(NB) * s->ni * sizeof(T) * (outS ? 2 : 1);
  const size_t fixed = (St<T>::cplx ? 48 * sizeof(z64) : 0) +
                       (s->natoms <= POS_LDS_MAX ? (3 * sizeof(double) * s->natoms + 15) / 16 * 16
                                                 : 0) +
                       (sizeof(int) * (s->natoms + 1) + 15) / 16 * 16 + 16;
  const size_t per_atom = row + 3 * sizeof(double) + sizeof(int);
  const size_t fit = fixed < AB_LDS ? (AB_LDS - fixed) / per_atom : 0;
  ab.cap = static_cast<int>(std::max<size_t>(1, std::min<size_t>(s->natoms, fit)));
  const size_t lds = (St<T>::cplx ? 48 * sizeof(z64) : 0) +
                     (s->natoms <= POS_LDS_MAX ? (3 * sizeof(double) * s->natoms + 15) / 16 * 16
                                               : 0) +
                     (sizeof(int) * (s->natoms + ab.cap + 1) + 15) / 16 * 16 +
                     (3 * sizeof(double) * ab.cap + 15) / 16 * 16 + row * ab.cap;
  if (lds > 64 * 1024) return fail(GPAW_ESHAPE, "add-back: LDS layout exceeds 64 KiB");
  T *po = static_cast<T *>(out);
  T *pso = static_cast<T *>(outS);
  if (outS)
    k_addback<T, NI, NB, true><<<grid, 256, lds, st>>>(po, pso, s->tab.cov, ncov, s->ng, nb, ab);
  else
    k_addback<T, NI, NB, false><<<grid, 256, lds, st>>>(po, pso, s->tab.cov, ncov, s->ng, nb, ab);
  return GPAW_OK;
}

// The add-back runs as its own pass for blocks of at least 2^24
// band-points (below that the fused kernel is cheaper than a second launch)
inline bool separate_addback(const gpaw_sys *s, int nb) {
  return s->tab.ncov > 0 && s->natoms <= SLOT_ATOMS_MAX &&
         static_cast<int64_t>(nb) * s->ng >= (int64_t{1} << 24);
}


template <typename T, bool BLOCH, int NB, int NI, int PPL>
int plane_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
            hipStream_t st, const void *XS = nullptr, void *outS = nullptr) {
  if (X && separate_addback(s, nb)) {
    const int rc = plane_t<T, BLOCH, NB, NI, PPL>(s, psi, nb, nullptr, out, st, nullptr, outS);
    if (rc != GPAW_OK) return rc;
    return addback_t<T, NI>(s, nb, X, XS, out, outS, st);
  }
  const int ngroups = (nb + NB - 1) / NB;
  const PlaneGeom G = make_geom(s, ngroups, PPL);
  AddArgs ab = make_add(s, X, XS);
  const bool sout = outS != nullptr;
  const size_t tile =
      (2 * static_cast<size_t>(NB) * ((G.TY + 6) * G.LS + 1) * sizeof(T) + 15) / 16 * 16 +
      (X && NI == 13 ? (sizeof(Proj13) + 15) / 16 * 16 : 0);
  const size_t phb = (X && St<T>::cplx) ? 48 * sizeof(z64) : 0;
  // LDS slots for the positions and X rows of the atoms that reach a tile
  // (the rest are read from global memory)
  const size_t row = static_cast<size_t>(NB) * s->ni * sizeof(T) * (sout ? 2 : 1);
  const bool slots = X && s->natoms <= SLOT_ATOMS_MAX;
  const int cap =
      slots && row ? static_cast<int>(std::min<size_t>(s->natoms, XLDS_MAX / row)) : 0;
  const bool xlds = cap > 0;
  ab.cap = cap;
  const size_t xbytes = xlds ? (sizeof(int) * (s->natoms + cap + 1) + 15) / 16 * 16 +
                                   (3 * sizeof(double) * cap + 15) / 16 * 16 + row * cap
                             : 0;
  const size_t lds = tile + phb + xbytes;
  const int64_t cols = static_cast<int64_t>(G.ngroups) * G.nseg;
  const int64_t blocks = (cols >= 8 ? (cols + 7) / 8 * 8 : cols) * G.tiles;
  if (blocks > 0x7FFFFFFF) return fail(GPAW_ESHAPE, "stencil grid too large");
  const unsigned grid = static_cast<unsigned>(blocks);
  const T *ps = static_cast<const T *>(psi);
  T *po = static_cast<T *>(out);
  T *pso = static_cast<T *>(outS);
  auto go = [&](auto kern) -> int {
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [&] {
      attr = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    if (attr != hipSuccess) return hip_fail(attr, "hipFuncSetAttribute(k_plane)");
    kern<<<grid, PT_THREADS, lds, st>>>(ps, po, pso, s->v, G, ab, nb);
    return GPAW_OK;
  };
  auto pick = [&](auto sflag) -> int {
    constexpr bool SO = decltype(sflag)::value;
    if (!X) return go(&k_plane<T, BLOCH, false, false, NI, NB, SO, PPL>);
    if (xlds) return go(&k_plane<T, BLOCH, true, true, NI, NB, SO, PPL>);
    return go(&k_plane<T, BLOCH, true, false, NI, NB, SO, PPL>);
  };
  return sout ? pick(std::true_type{}) : pick(std::false_type{});
}

template <typename T, int NB, int NI>
int apply_S_t(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
              hipStream_t st) {
  // large blocks: S~psi = psi (a device copy), then the add-back pass over
  // the covered points with the Delta S P rows (the same sums as below)
  if (X && separate_addback(s, nb)) {
    GFD_HIP(hipMemcpyAsync(out, psi, static_cast<size_t>(nb) * s->ng * sizeof(T),
                           hipMemcpyDeviceToDevice, st));
    return addback_t<T, NI>(s, nb, X, nullptr, out, nullptr, st);
  }
  const AddArgs ab = make_add(s, X);
  dim3 grid(static_cast<unsigned>((s->ng + 256 * AS_CHUNKS - 1) / (256 * AS_CHUNKS)),
            (nb + NB - 1) / NB);
  const size_t xbytes = static_cast<size_t>(NB) * s->np * sizeof(T);
  const bool xlds = X && xbytes <= 32 * 1024;
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

// per-dtype launchers (stencil_<dtype>.hip)
int launch_stencil_f64(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                       hipStream_t st, const void *XS, void *outS);
int launch_stencil_c128(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                        hipStream_t st, const void *XS, void *outS);
int launch_stencil_f32(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                       hipStream_t st, const void *XS, void *outS);
int launch_stencil_c64(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                       hipStream_t st, const void *XS, void *outS);

}  // namespace gfd
