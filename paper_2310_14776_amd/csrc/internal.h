// Internal declarations of the gfx950 FD-PAW library: the system object,
// error plumbing, complex helpers and the kernel launchers each .hip file
// provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "gpaw_fd.h"

namespace gfd {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t err, const char *what);

#define GFD_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::gfd::hip_fail(e_, #call); \
  } while (0)

// ---------------------------------------------------------------- complex
struct z64 {
  double x, y;
};

__host__ __device__ inline z64 zmake(double a, double b) { return z64{a, b}; }
__host__ __device__ inline z64 operator+(z64 a, z64 b) { return z64{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline z64 operator-(z64 a, z64 b) { return z64{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline z64 operator*(z64 a, z64 b) {
  return z64{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline z64 operator*(double s, z64 a) { return z64{s * a.x, s * a.y}; }
__host__ __device__ inline z64 zconj(z64 a) { return z64{a.x, -a.y}; }

struct z32 {
  float x, y;
};
__host__ __device__ inline z32 operator+(z32 a, z32 b) { return z32{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline z32 operator-(z32 a, z32 b) { return z32{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline z32 operator*(z32 a, z32 b) {
  return z32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Scalar traits: one kernel body serves real and complex grids in double
// precision and, for the precision form, in single precision. Acc is the
// type partial sums are kept in (always double precision).
template <typename T> struct St;
template <> struct St<double> {
  using Acc = double;
  static constexpr bool cplx = false;
  static constexpr bool single = false;
  __host__ __device__ static double zero() { return 0.0; }
  __host__ __device__ static double conj(double a) { return a; }
  // a * b where b is a Bloch phase (identity for real systems)
  __host__ __device__ static double phase(double a, z64) { return a; }
  __host__ __device__ static double mul(double a, double b) { return a * b; }
  __host__ __device__ static double scale(double s, double a) { return s * a; }
  __host__ __device__ static double widen(double a) { return a; }
  __host__ __device__ static double narrow(double a) { return a; }
};
template <> struct St<z64> {
  using Acc = z64;
  static constexpr bool cplx = true;
  static constexpr bool single = false;
  __host__ __device__ static z64 zero() { return z64{0.0, 0.0}; }
  __host__ __device__ static z64 conj(z64 a) { return zconj(a); }
  __host__ __device__ static z64 phase(z64 a, z64 p) { return a * p; }
  __host__ __device__ static z64 mul(z64 a, z64 b) { return a * b; }
  __host__ __device__ static z64 scale(double s, z64 a) { return s * a; }
  __host__ __device__ static z64 widen(z64 a) { return a; }
  __host__ __device__ static z64 narrow(z64 a) { return a; }
};
template <> struct St<float> {
  using Acc = double;
  static constexpr bool cplx = false;
  static constexpr bool single = true;
  __host__ __device__ static float zero() { return 0.0f; }
  __host__ __device__ static float conj(float a) { return a; }
  __host__ __device__ static float phase(float a, z64) { return a; }
  __host__ __device__ static float mul(float a, float b) { return a * b; }
  __host__ __device__ static float scale(double s, float a) { return static_cast<float>(s) * a; }
  __host__ __device__ static double widen(float a) { return a; }
  __host__ __device__ static float narrow(double a) { return static_cast<float>(a); }
};
template <> struct St<z32> {
  using Acc = z64;
  static constexpr bool cplx = true;
  static constexpr bool single = true;
  __host__ __device__ static z32 zero() { return z32{0.0f, 0.0f}; }
  __host__ __device__ static z32 conj(z32 a) { return z32{a.x, -a.y}; }
  __host__ __device__ static z32 phase(z32 a, z64 p) {
    return a * z32{static_cast<float>(p.x), static_cast<float>(p.y)};
  }
  __host__ __device__ static z32 mul(z32 a, z32 b) { return a * b; }
  __host__ __device__ static z32 scale(double s, z32 a) {
    const float f = static_cast<float>(s);
    return z32{f * a.x, f * a.y};
  }
  __host__ __device__ static z64 widen(z32 a) { return z64{a.x, a.y}; }
  __host__ __device__ static z32 narrow(z64 a) {
    return z32{static_cast<float>(a.x), static_cast<float>(a.y)};
  }
};

// ---------------------------------------------------------------- projectors
// Parameters of the projector functions, passed by value to the kernels
// (device evaluation in proj.h).
constexpr int PROJ_MAX_CHAN = 8;
constexpr int PROJ_MAX_NI = 32;

struct ProjDev {
  int nchan, ni;
  int std13;                       // channel l sequence is (0, 0, 1, 1, 2)
  int same_sigma[PROJ_MAX_CHAN];   // std13: 0/1 = shares channel 0/1's sigma, -1 = own
  int l[PROJ_MAX_CHAN];
  double norm[PROJ_MAX_CHAN];
  double rc2inv[PROJ_MAX_CHAN];    // 1 / rc^2
  double a2[PROJ_MAX_CHAN];        // 1 / (2 sigma^2)
  signed char ch[PROJ_MAX_NI];     // channel of projector i
  signed char ym[PROJ_MAX_NI];     // harmonic slot (0..8) of projector i
  int n[3];
  double h[3];
  z64 ph[3][16];                   // exp(-2 pi i k_c w), w = -8..7
};

// ---------------------------------------------------------------- system
// Projector geometry. An entry is one (grid point, atom, periodic image)
// triple with the image's sphere covering the point; projector values are
// recomputed from it on the device. Two orders of the same entries:
// atom-major (projection gather) and point-major (add-back, where each grid
// point sums over the entries that reach it).
struct Tables {
  int64_t nent = 0;            // entries
  int64_t ncov = 0;            // distinct covered grid points
  int32_t *a_start = nullptr;  // [natoms+1] atom-major entry ranges
  int32_t *e_g = nullptr;      // [nent] folded grid index (atom-major)
  short4 *e_xyz = nullptr;     // [nent] unwrapped grid indices + image code (atom-major)
  int4 *pinfo = nullptr;       // [Ng] {codes of the point's first three
                               //       entries, count << 24 | index of the first}
  int32_t *pm_code = nullptr;  // [nent] atom << 12 | image code (point-major)
  int32_t *cov = nullptr;      // [ncov] covered grid points in increasing order
  double *pos = nullptr;       // [natoms][3] atom positions
  ProjDev *proj = nullptr;     // device copy of the projector parameters
};

struct Workspace {
  void *P = nullptr;       // [max_bands][Np] projections when the caller gives none
  void *X = nullptr;       // [max_bands][Np] Delta.P
  void *XS = nullptr;      // [max_bands][Np] Delta S.P (H~ and S~ in one pass)
  double *part = nullptr;  // subspace split-K partial sums
  size_t part_elems = 0;
  void *split = nullptr;   // BF16 planes of C for the split rotation
  double *eig = nullptr;   // dense eigensolver scratch
  size_t eig_elems = 0;
  int32_t *info = nullptr; // device status word for synchronous diag
  int32_t *flag = nullptr; // device word: the near-identity rotation may use one product
  void *mat = nullptr;     // [2][max_bands][max_bands] subspace-sized scratch
};

}  // namespace gfd

namespace gfd {
// Launch shapes of one system (0 = the built-in heuristic). The batched
// form's autotuner sets them per system; every choice computes the same
// result up to the order of floating-point sums.
struct Tune {
  int st_ty = 0;    // stencil tile rows (y) and columns (z): st_ty x st_tz points of
  int st_tz = 0;    //   the y-z plane per workgroup (both set, or the built-in tile)
  int st_nseg = 0;  // x segments of the stencil grid (>= 1)
  int st_ppl = 0;   // stencil points per lane: 1 or 2 (0 = 1)
  int sub_wgs = 0;  // target workgroup count of the split-K subspace product (<= 1024)
  int rot_rb = 0;   // 16-row tiles per rotation workgroup: real 4 or 8, complex 2 or 4
  int prj_nbg = 0;  // bands per projection workgroup: real 2, 4 or 8, complex 1 or 2
};
}  // namespace gfd

struct gpaw_sys {
  int device = 0;
  int32_t n[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  double k[3] = {0, 0, 0};
  double dV = 0;
  int32_t dtype = GPAW_F64;
  gfd::z64 phase[3];       // exp(2 pi i k_c)
  int32_t natoms = 0, ni = 0, np = 0;
  int64_t ng = 0;
  int32_t max_bands = 0;
  int32_t zbc = 0;  // zero boundary (finite system)
  void *td = nullptr;       // time-propagation workspace (allocated on first use)
  void *td_host = nullptr;  // pinned residual norms of the time propagation
  size_t td_bytes = 0;
  gfd::Tables tab;
  gfd::ProjDev proj;                    // projector parameters (host copy)
  double *dH = nullptr, *dS = nullptr;  // device [natoms][ni][ni]
  double *v = nullptr;                  // device [Ng]
  gfd::Workspace ws;
  gfd::Tune tune;
};

namespace gfd {

size_t elem_size(int32_t dtype);
size_t mat_elem_size(int32_t dtype);
bool is_complex(int32_t dtype);

// Host construction of the projector geometry (tables.hip): the tables are
// built and checked on the host first (no device call, so a bad geometry is
// rejected before anything is allocated), then uploaded.
struct HostTables {
  std::vector<int32_t> a_start, e_g, pm_code, cov;
  std::vector<short4> e_xyz;
  std::vector<int4> pinfo;
  std::vector<double> pos;
};
int build_tables_host(const gpaw_sys_desc *d, gpaw_sys *s, HostTables &ht);
int upload_tables(gpaw_sys *s, const HostTables &ht);

// Strided copy global -> LDS by nthr threads: eight loads in flight per
// thread before the stores, so a round costs one memory latency.
template <typename T>
__device__ inline void copy_rounds(T *dst, const T *src, int count, int tid, int nthr) {
  for (int base = 0; base < count; base += 8 * nthr) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * nthr + tid;
      v[u] = idx < count ? src[idx] : T{};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * nthr + tid;
      if (idx < count) dst[idx] = v[u];
    }
  }
}

// ---------------------------------------------------------------- launchers
// Each returns GPAW_OK or an error code with the message set.
int launch_project(const gpaw_sys *s, const void *psi, int nb, void *P, hipStream_t st);
int launch_dmat(const gpaw_sys *s, const double *D, const void *P, int nb, void *X,
                hipStream_t st);
// X = Delta H . P and XS = Delta S . P in one launch
int launch_dmat2(const gpaw_sys *s, const void *P, int nb, void *X, void *XS, hipStream_t st);
// outS (optional): S~psi formed in the same pass, XS = Delta S.P (null
// without projectors)
int launch_stencil(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st, const void *XS = nullptr, void *outS = nullptr);
// Davidson corrections out = -(Hpsi - eps Spsi) / max(t0 + v - eps, t0/2)
int launch_precond(const gpaw_sys *s, const void *Hpsi, const void *Spsi, const double *eps,
                   int nb, void *out, hipStream_t st);
// pseudo density n_out [Ng] (may be null) and atomic density matrices D_out
// [natoms][ni][ni] in the matrix dtype (may be null; needs P)
int launch_density(const gpaw_sys *s, const void *psi, int nb, const double *f, const void *P,
                   double *n_out, void *D_out, hipStream_t st);
// (rows, columns) of the cheapest stencil tiles of the system's y-z plane
std::vector<std::pair<int, int>> stencil_tiles(const gpaw_sys *s, int keep);
int launch_apply_S(const gpaw_sys *s, const void *psi, int nb, const void *X, void *out,
                   hipStream_t st);
// part/part_elems: the split-K partial sums go to this buffer of doubles
// instead of the system's workspace (the split count is capped to fit;
// GPAW_ESHAPE when even one split does not)
int launch_subspace(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                    int nb, void *H, void *S, hipStream_t st, double *part = nullptr,
                    size_t part_elems = 0);
// acc[i] += a[i] for n doubles (fixed order, one lane per element)
int launch_add_mat(const double *a, double *acc, int64_t n, hipStream_t st);
// Small subspace eigensolves (nb up to the one-workgroup limit) of several
// systems of one scalar type in one chain of launches (eigh.hip). The job
// table lives in device memory of at least eig_job_bytes() per item: filled
// by eigh_batched_prepare (a synchronous copy, outside any stream capture),
// read by the launches of launch_eigh_batched, which may be captured.
struct EigBatchItem {
  const gpaw_sys *s;
  const void *H, *S;
  int nb;
  double *eps;
  void *C;
  int32_t *info;
};
int eig_small_max(bool cplx);
size_t eig_job_bytes();
int eigh_batched_prepare(const EigBatchItem *items, int count, void *jobs);
int launch_eigh_batched(const EigBatchItem *items, int count, bool cplx, const void *jobs,
                        hipStream_t st);
size_t subspace_part_elems(const gpaw_sys *s, int nb);
// Split-K planning (gemm.hip). A product whose K range is cut into ns
// pieces launches units workgroups per piece (8 or more pieces are launched
// in whole groups of 8, one per XCD), slots of them resident at a time. The
// count returned minimises the modelled time: whole rounds of resident
// workgroups, each doing 1/ns of a tile's work (tile_s: one tile over the
// whole K range with every slot busy), plus the partial sums' traffic per
// piece (part_s); at most max_split, and at least min_k of K per piece.
int64_t balanced_splits(int64_t units, int64_t slots, double tile_s, double part_s,
                        int64_t max_split, int64_t k, int64_t min_k);
// Workgroups of a kernel resident on the whole device at once.
int64_t resident_slots(const void *kern, int threads, size_t lds);
// upper: C is upper triangular; near_id: C is close to the identity (the
// single-precision form then rotates by C - I, see the split kernels)
// nout >= 0: only the first nout output rows (C is still nb x nb; its first
// nout columns), FP64 and complex128 only
int launch_rotate(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                  void *dst, hipStream_t st, bool upper = false, bool near_id = false,
                  int nout = -1);
// precision form (gemm_split.hip)
size_t split_part_elems(int nb, bool cplx);
size_t split_c_bytes(int nb, bool cplx);
int launch_subspace_split(const gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                          int nb, void *H, void *S, hipStream_t st, double *part,
                          size_t part_elems);
int launch_rotate_split(const gpaw_sys *s, const void *C, const void *src, int nb, int64_t cols,
                        void *dst, hipStream_t st, bool upper = false, bool near_id = false);
size_t eig_ws_elems(int nmax, bool cplx);
int launch_eigh(const gpaw_sys *s, const void *H, const void *S, int nb, double *eps, void *C,
                int32_t *info, hipStream_t st);
int launch_chol_inv(const gpaw_sys *s, const void *S, int nb, void *Cout, int32_t *info,
                    hipStream_t st);

}  // namespace gfd
