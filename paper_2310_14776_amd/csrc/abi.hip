// C ABI entry points: argument checks, system construction and dispatch of
// the device kernels. No arithmetic of the method happens here.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace gfd {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t err, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(err);
  return err == hipErrorOutOfMemory ? GPAW_ENOMEM : GPAW_EHIP;
}

size_t elem_size(int32_t dtype) {
  switch (dtype) {
    case GPAW_C128: return 16;
    case GPAW_F32: return 4;
    case GPAW_C64: return 8;
    default: return 8;
  }
}

// element size of the subspace matrices (double or complex double)
size_t mat_elem_size(int32_t dtype) {
  return (dtype == GPAW_C128 || dtype == GPAW_C64) ? 16 : 8;
}

bool is_complex(int32_t dtype) { return dtype == GPAW_C128 || dtype == GPAW_C64; }

namespace {

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + nb && pb < pa + na;
}

int check_sys(const gpaw_sys *s) {
  if (!s) return fail(GPAW_EINVAL, "system is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != s->device)
    return fail(GPAW_EINVAL, "current HIP device differs from the system's device");
  return GPAW_OK;
}

int check_nb(const gpaw_sys *s, int32_t nb) {
  if (nb < 1 || nb > s->max_bands)
    return fail(GPAW_ESHAPE, "nb=" + std::to_string(nb) + " outside [1, max_bands=" +
                                 std::to_string(s->max_bands) + "]");
  return GPAW_OK;
}

int after_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return GPAW_OK;
}

// Partial-sum scratch of gpaw_subspace_matrices_noalloc: a file-scope device
// array (each GPU the library runs on holds its own copy for the life of the
// process). Host code never uses its name as an address: the device address
// comes from hipGetSymbolAddress, once per device, and is kept per device.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(8) << 20;  // 64 MiB
__device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[MAX_DEVICES] = {};

// device address of scratch on the current device (set up on first use)
int scratch_address(double **out) {
  int dev = -1;
  GFD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(GPAW_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(GPAW_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_addr[dev];
  return GPAW_OK;
}

void free_sys(gpaw_sys *s) {
  if (!s) return;
  void *bufs[] = {s->tab.a_start, s->tab.e_g, s->tab.e_xyz, s->tab.pinfo, s->tab.pm_code,
                  s->tab.pos,     s->dH,      s->dS,        s->v,          s->ws.P,
                  s->ws.X,        s->ws.part, s->ws.eig,    s->ws.info,    s->tab.proj,
                  s->ws.split,    s->ws.mat,  s->ws.XS,     s->ws.flag,    s->tab.cov};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  if (s->td) (void)hipFree(s->td);
  if (s->td_host) (void)hipHostFree(s->td_host);
  delete s;
}

template <typename T>
int dev_alloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return GPAW_OK;
  GFD_HIP(hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)));
  return GPAW_OK;
}

}  // namespace
}  // namespace gfd

using namespace gfd;

extern "C" {

const char *gpaw_last_error(void) { return g_last_error.c_str(); }

int gpaw_version(void) { return GPAW_FD_VERSION; }

int gpaw_sys_create(const gpaw_sys_desc *d, gpaw_sys **out) {
  if (!d || !out) return fail(GPAW_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  int64_t ng = 1;
  for (int c = 0; c < 3; ++c) {
    if (d->n[c] < 1) return fail(GPAW_EINVAL, "grid sizes must be >= 1");
    if (!(d->h[c] > 0.0) || !std::isfinite(d->h[c]))
      return fail(GPAW_EINVAL, "grid spacings must be finite and > 0");
    if (!std::isfinite(d->k[c])) return fail(GPAW_EINVAL, "k must be finite");
    ng *= d->n[c];
  }
  if (ng > (int64_t(1) << 31) - 1) return fail(GPAW_EINVAL, "grid has more than 2^31-1 points");
  if (d->dtype < GPAW_F64 || d->dtype > GPAW_C64) return fail(GPAW_EDTYPE, "unknown dtype");
  if (!is_complex(d->dtype) && (d->k[0] != 0.0 || d->k[1] != 0.0 || d->k[2] != 0.0))
    return fail(GPAW_EDTYPE, "a real system needs k = 0; use a complex dtype");
  if (d->natoms < 0) return fail(GPAW_EINVAL, "natoms must be >= 0");
  if (!d->v) return fail(GPAW_EINVAL, "v must not be NULL");
  if (d->max_bands < 1) return fail(GPAW_EINVAL, "max_bands must be >= 1");
  if (d->boundary != 0 && d->boundary != 1)
    return fail(GPAW_EINVAL, "boundary must be 0 (periodic / Bloch) or 1 (zero)");
  if (d->boundary == 1 && (d->k[0] != 0.0 || d->k[1] != 0.0 || d->k[2] != 0.0))
    return fail(GPAW_EINVAL, "a zero-boundary system has no Bloch vector: k must be 0");
  int ni = 0;
  if (d->natoms > 0) {
    if (!d->pos || !d->dH || !d->dS || !d->chan || d->nchan < 1)
      return fail(GPAW_EINVAL, "atoms need pos, dH, dS and at least one channel");
    for (int c = 0; c < d->nchan; ++c) {
      const gpaw_channel &ch = d->chan[c];
      if (ch.l < 0 || ch.l > 2) return fail(GPAW_EINVAL, "channel l must be 0, 1 or 2");
      if (!(ch.sigma > 0.0) || !(ch.rc > 0.0) || !std::isfinite(ch.sigma) || !std::isfinite(ch.rc))
        return fail(GPAW_EINVAL, "channel sigma and rc must be finite and > 0");
      ni += 2 * ch.l + 1;
    }
    if (ni > 32) return fail(GPAW_EINVAL, "at most 32 projectors per atom");
    for (int a = 0; a < 3 * d->natoms; ++a)
      if (!std::isfinite(d->pos[a])) return fail(GPAW_EINVAL, "atom positions must be finite");
  }
  gpaw_sys *s = new gpaw_sys();
  for (int c = 0; c < 3; ++c) {
    s->n[c] = d->n[c];
    s->h[c] = d->h[c];
    s->k[c] = d->k[c];
    const double arg = 2.0 * 3.14159265358979323846 * d->k[c];
    s->phase[c] = zmake(std::cos(arg), std::sin(arg));
  }
  s->dV = d->h[0] * d->h[1] * d->h[2];
  s->zbc = d->boundary;
  s->dtype = d->dtype;
  s->natoms = d->natoms;
  s->ni = d->natoms > 0 ? ni : 0;
  s->np = s->natoms * s->ni;
  s->ng = ng;
  s->max_bands = d->max_bands;

  int rc = GPAW_OK;
  const size_t es = elem_size(s->dtype);
  // the projector geometry is built and checked on the host before the
  // first device call
  HostTables ht;
  if (s->natoms > 0 && (rc = build_tables_host(d, s, ht)) != GPAW_OK) {
    delete s;
    return rc;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete s;
    return fail(GPAW_EHIP, "hipGetDevice failed: no usable HIP device");
  }
  s->device = dev;
  do {
    if (s->natoms > 0) {
      if ((rc = upload_tables(s, ht)) != GPAW_OK) break;
      const size_t nd = static_cast<size_t>(s->natoms) * s->ni * s->ni;
      if ((rc = dev_alloc(&s->dH, nd)) != GPAW_OK) break;
      if ((rc = dev_alloc(&s->dS, nd)) != GPAW_OK) break;
      if (hipMemcpy(s->dH, d->dH, nd * 8, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(s->dS, d->dS, nd * 8, hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(GPAW_EHIP, "upload of Delta H / Delta S failed");
        break;
      }
      const size_t pbytes = static_cast<size_t>(s->max_bands) * s->np * es;
      if ((rc = dev_alloc(reinterpret_cast<char **>(&s->ws.P), pbytes)) != GPAW_OK) break;
      if ((rc = dev_alloc(reinterpret_cast<char **>(&s->ws.X), pbytes)) != GPAW_OK) break;
      if ((rc = dev_alloc(reinterpret_cast<char **>(&s->ws.XS), pbytes)) != GPAW_OK) break;
    }
    if ((rc = dev_alloc(&s->v, static_cast<size_t>(ng))) != GPAW_OK) break;
    if (hipMemcpy(s->v, d->v, ng * 8, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(GPAW_EHIP, "upload of v failed");
      break;
    }
    s->ws.part_elems = subspace_part_elems(s, s->max_bands);
    if ((rc = dev_alloc(&s->ws.part, s->ws.part_elems)) != GPAW_OK) break;
    s->ws.eig_elems = eig_ws_elems(s->max_bands, is_complex(s->dtype));
    if ((rc = dev_alloc(&s->ws.eig, s->ws.eig_elems)) != GPAW_OK) break;
    if ((rc = dev_alloc(&s->ws.info, 1)) != GPAW_OK) break;
    if ((rc = dev_alloc(&s->ws.flag, 1)) != GPAW_OK) break;
    if ((rc = dev_alloc(reinterpret_cast<char **>(&s->ws.mat),
                        2 * static_cast<size_t>(s->max_bands) * s->max_bands *
                            mat_elem_size(s->dtype))) != GPAW_OK)
      break;
    if (s->dtype == GPAW_F32 || s->dtype == GPAW_C64)
      if ((rc = dev_alloc(reinterpret_cast<char **>(&s->ws.split),
                          split_c_bytes(s->max_bands, s->dtype == GPAW_C64))) != GPAW_OK)
        break;
  } while (false);
  if (rc != GPAW_OK) {
    free_sys(s);
    return rc;
  }
  *out = s;
  return GPAW_OK;
}

void gpaw_sys_destroy(gpaw_sys *s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_sys(s);
}

int gpaw_sys_info(const gpaw_sys *s, int64_t *info) {
  if (!s || !info) return fail(GPAW_EINVAL, "system and info must not be NULL");
  info[0] = s->ng;
  info[1] = s->np;
  info[2] = s->ni;
  info[3] = s->natoms;
  info[4] = s->tab.nent;
  info[5] = s->tab.ncov;
  info[6] = s->max_bands;
  info[7] = s->dtype;
  return GPAW_OK;
}

int gpaw_project(gpaw_sys *s, const void *psi, int32_t nb, void *P, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi) return fail(GPAW_EINVAL, "psi must not be NULL");
  if (s->np == 0) return GPAW_OK;
  if (!P) return fail(GPAW_EINVAL, "P must not be NULL");
  const size_t es = elem_size(s->dtype);
  if (overlaps(P, nb * s->np * es, psi, nb * s->ng * es))
    return fail(GPAW_EALIAS, "P overlaps psi");
  if ((rc = launch_project(s, psi, nb, P, static_cast<hipStream_t>(stream))) != GPAW_OK) return rc;
  return after_launch("gpaw_project");
}

namespace {

int apply(gpaw_sys *s, const void *psi, int32_t nb, const void *P, void *out, void *stream,
          bool hamiltonian) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi || !out) return fail(GPAW_EINVAL, "psi and output must not be NULL");
  const size_t es = elem_size(s->dtype);
  const size_t bytes = static_cast<size_t>(nb) * s->ng * es;
  if (overlaps(out, bytes, psi, bytes)) return fail(GPAW_EALIAS, "output overlaps psi");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void *X = nullptr;
  if (s->np > 0) {
    const size_t pbytes = static_cast<size_t>(nb) * s->np * es;
    if (P && overlaps(out, bytes, P, pbytes)) return fail(GPAW_EALIAS, "output overlaps P");
    if (!P) {
      if ((rc = launch_project(s, psi, nb, s->ws.P, st)) != GPAW_OK) return rc;
      P = s->ws.P;
    }
    if ((rc = launch_dmat(s, hamiltonian ? s->dH : s->dS, P, nb, s->ws.X, st)) != GPAW_OK)
      return rc;
    X = s->ws.X;
  }
  rc = hamiltonian ? launch_stencil(s, psi, nb, X, out, st) : launch_apply_S(s, psi, nb, X, out, st);
  if (rc != GPAW_OK) return rc;
  return after_launch(hamiltonian ? "gpaw_fd_apply_H" : "gpaw_fd_apply_S");
}

}  // namespace

int gpaw_fd_apply_H(gpaw_sys *s, const void *psi, int32_t nb, const void *P, void *Hpsi,
                    void *stream) {
  return apply(s, psi, nb, P, Hpsi, stream, true);
}

int gpaw_fd_apply_S(gpaw_sys *s, const void *psi, int32_t nb, const void *P, void *Spsi,
                    void *stream) {
  return apply(s, psi, nb, P, Spsi, stream, false);
}

int gpaw_fd_apply_HS(gpaw_sys *s, const void *psi, int32_t nb, const void *P, void *Hpsi,
                     void *Spsi, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi || !Hpsi || !Spsi) return fail(GPAW_EINVAL, "psi, Hpsi and Spsi must not be NULL");
  const size_t es = elem_size(s->dtype);
  const size_t bytes = static_cast<size_t>(nb) * s->ng * es;
  if (overlaps(Hpsi, bytes, psi, bytes) || overlaps(Spsi, bytes, psi, bytes) ||
      overlaps(Hpsi, bytes, Spsi, bytes))
    return fail(GPAW_EALIAS, "Hpsi, Spsi and psi must not overlap");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void *X = nullptr, *XS = nullptr;
  if (s->np > 0) {
    const size_t pbytes = static_cast<size_t>(nb) * s->np * es;
    if (P && (overlaps(Hpsi, bytes, P, pbytes) || overlaps(Spsi, bytes, P, pbytes)))
      return fail(GPAW_EALIAS, "an output overlaps P");
    if (!P) {
      if ((rc = launch_project(s, psi, nb, s->ws.P, st)) != GPAW_OK) return rc;
      P = s->ws.P;
    }
    if ((rc = launch_dmat2(s, P, nb, s->ws.X, s->ws.XS, st)) != GPAW_OK) return rc;
    X = s->ws.X;
    XS = s->ws.XS;
  }
  if ((rc = launch_stencil(s, psi, nb, X, Hpsi, st, XS, Spsi)) != GPAW_OK) return rc;
  return after_launch("gpaw_fd_apply_HS");
}

int gpaw_subspace_matrices(gpaw_sys *s, const void *psi, const void *Hpsi, const void *Spsi,
                           int32_t nb, void *H, void *S, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi || !Hpsi || !H) return fail(GPAW_EINVAL, "psi, Hpsi and H_nn must not be NULL");
  if (Spsi && !S) return fail(GPAW_EINVAL, "S_nn must not be NULL when Spsi is given");
  const size_t mbytes = static_cast<size_t>(nb) * nb * mat_elem_size(s->dtype);
  if (Spsi && overlaps(H, mbytes, S, mbytes)) return fail(GPAW_EALIAS, "H_nn overlaps S_nn");
  if ((rc = launch_subspace(s, psi, Hpsi, Spsi, nb, H, Spsi ? S : nullptr,
                            static_cast<hipStream_t>(stream))) != GPAW_OK)
    return rc;
  return after_launch("gpaw_subspace_matrices");
}

int gpaw_subspace_matrices_noalloc(gpaw_sys *s, const void *psi, const void *Hpsi,
                                   const void *Spsi, int32_t nb, void *H, void *S, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi || !Hpsi || !H) return fail(GPAW_EINVAL, "psi, Hpsi and H_nn must not be NULL");
  if (Spsi && !S) return fail(GPAW_EINVAL, "S_nn must not be NULL when Spsi is given");
  const size_t mbytes = static_cast<size_t>(nb) * nb * mat_elem_size(s->dtype);
  if (Spsi && overlaps(H, mbytes, S, mbytes)) return fail(GPAW_EALIAS, "H_nn overlaps S_nn");
  // one split-K slice of partial sums must fit the scratch array
  const size_t per_split =
      static_cast<size_t>(Spsi ? 2 : 1) * nb * nb * (is_complex(s->dtype) ? 2 : 1);
  if (per_split > NOALLOC_SCRATCH_DOUBLES)
    return fail(GPAW_ESHAPE, "gpaw_subspace_matrices_noalloc: nb=" + std::to_string(nb) +
                                 " needs " + std::to_string(per_split * 8) +
                                 " bytes of partial sums, above the " +
                                 std::to_string(NOALLOC_SCRATCH_DOUBLES * 8) + "-byte scratch");
  double *part = nullptr;
  if ((rc = scratch_address(&part)) != GPAW_OK) return rc;
  if ((rc = launch_subspace(s, psi, Hpsi, Spsi, nb, H, Spsi ? S : nullptr,
                            static_cast<hipStream_t>(stream), part, NOALLOC_SCRATCH_DOUBLES)) !=
      GPAW_OK)
    return rc;
  return after_launch("gpaw_subspace_matrices_noalloc");
}

int gpaw_density(gpaw_sys *s, const void *psi, int32_t nb, const double *f, const void *P,
                 double *n_out, void *D_out, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi || !f) return fail(GPAW_EINVAL, "psi and f must not be NULL");
  if (!n_out && !D_out) return fail(GPAW_EINVAL, "one of n_out and D_nn must be given");
  const size_t es = elem_size(s->dtype);
  const size_t bytes = static_cast<size_t>(nb) * s->ng * es;
  const size_t dbytes =
      static_cast<size_t>(s->natoms) * s->ni * s->ni * mat_elem_size(s->dtype);
  if (n_out && (overlaps(n_out, s->ng * 8, psi, bytes) || overlaps(n_out, s->ng * 8, f, nb * 8)))
    return fail(GPAW_EALIAS, "n_out overlaps an input");
  if (D_out && dbytes && (overlaps(D_out, dbytes, f, nb * 8) ||
                          (n_out && overlaps(D_out, dbytes, n_out, s->ng * 8))))
    return fail(GPAW_EALIAS, "D_out overlaps another buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (D_out && s->np > 0 && !P) {
    if ((rc = launch_project(s, psi, nb, s->ws.P, st)) != GPAW_OK) return rc;
    P = s->ws.P;
  }
  if ((rc = launch_density(s, psi, nb, f, P, n_out, D_out, st)) != GPAW_OK) return rc;
  return after_launch("gpaw_density");
}

int gpaw_subspace_diag(gpaw_sys *s, const void *H, const void *S, int32_t nb, double *eps,
                       void *C, int32_t *info, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (nb > 1024) return fail(GPAW_ESHAPE, "gpaw_subspace_diag supports nb <= 1024");
  if (!H || !S || !eps || !C) return fail(GPAW_EINVAL, "H_nn, S_nn, eps and C_nn must not be NULL");
  const size_t mbytes = static_cast<size_t>(nb) * nb * mat_elem_size(s->dtype);
  if (overlaps(C, mbytes, H, mbytes) || overlaps(C, mbytes, S, mbytes) ||
      overlaps(eps, nb * 8, C, mbytes) || overlaps(eps, nb * 8, H, mbytes) ||
      overlaps(eps, nb * 8, S, mbytes))
    return fail(GPAW_EALIAS, "outputs of gpaw_subspace_diag overlap its inputs");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t *dinfo = info ? info : s->ws.info;
  if ((rc = launch_eigh(s, H, S, nb, eps, C, dinfo, st)) != GPAW_OK) return rc;
  if ((rc = after_launch("gpaw_subspace_diag")) != GPAW_OK) return rc;
  if (info) return GPAW_OK;
  int32_t h_info = 0;
  GFD_HIP(hipMemcpyAsync(&h_info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  GFD_HIP(hipStreamSynchronize(st));
  if (h_info > 0)
    return fail(GPAW_ENOTPD, "S_nm is not positive definite (leading minor " +
                                 std::to_string(h_info) + ")");
  if (h_info < 0) return fail(GPAW_ENOCONV, "eigenvector orthogonalisation did not settle");
  return GPAW_OK;
}

int gpaw_davidson_correction(gpaw_sys *s, const void *Hpsi, const void *Spsi, const double *eps,
                              int32_t nb, void *out, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!Hpsi || !Spsi || !eps || !out)
    return fail(GPAW_EINVAL, "Hpsi, Spsi, eps and out must not be NULL");
  const size_t bytes = static_cast<size_t>(nb) * s->ng * elem_size(s->dtype);
  if (overlaps(out, bytes, Hpsi, bytes) || overlaps(out, bytes, Spsi, bytes))
    return fail(GPAW_EALIAS, "out overlaps Hpsi or Spsi");
  if ((rc = launch_precond(s, Hpsi, Spsi, eps, nb, out, static_cast<hipStream_t>(stream))) !=
      GPAW_OK)
    return rc;
  return after_launch("gpaw_davidson_correction");
}

int gpaw_davidson_step(gpaw_sys *s, int32_t nb, void *x, void *Hx, void *Sx, void *Px,
                       const double *eps, void *H2, void *S2, void *C2, double *eps2,
                       void *psi_out, void *P_out, int32_t *info, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if (s->dtype != GPAW_F64 && s->dtype != GPAW_C128)
    return fail(GPAW_EDTYPE, "gpaw_davidson_step runs on FP64 and complex128 systems");
  if (nb < 1 || 2 * nb > s->max_bands || 2 * nb > 1024)
    return fail(GPAW_ESHAPE, "gpaw_davidson_step needs 1 <= nb, 2 nb <= max_bands and <= 1024");
  if (!x || !Hx || !Sx || !eps || !H2 || !S2 || !C2 || !eps2 || !psi_out)
    return fail(GPAW_EINVAL, "x, Hx, Sx, eps, H2, S2, C2, eps2 and psi_out must not be NULL");
  if (s->np > 0 && (!Px || !P_out))
    return fail(GPAW_EINVAL, "Px and P_out must be given when the system has atoms");
  const size_t es = elem_size(s->dtype);
  const size_t row = static_cast<size_t>(s->ng) * es, prow = static_cast<size_t>(s->np) * es;
  const size_t xbytes = 2 * nb * row, obytes = nb * row;
  const size_t m2 = static_cast<size_t>(2 * nb) * (2 * nb) * mat_elem_size(s->dtype);
  if (overlaps(x, xbytes, Hx, xbytes) || overlaps(x, xbytes, Sx, xbytes) ||
      overlaps(Hx, xbytes, Sx, xbytes) || overlaps(psi_out, obytes, x, xbytes) ||
      overlaps(H2, m2, S2, m2) || overlaps(C2, m2, H2, m2) || overlaps(C2, m2, S2, m2) ||
      overlaps(eps2, 16 * nb, C2, m2))
    return fail(GPAW_EALIAS, "buffers of gpaw_davidson_step overlap");
  if (s->np > 0 && overlaps(P_out, nb * prow, Px, 2 * nb * prow))
    return fail(GPAW_EALIAS, "P_out overlaps Px");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *xd = static_cast<char *>(x) + nb * row;
  char *Hd = static_cast<char *>(Hx) + nb * row;
  char *Sd = static_cast<char *>(Sx) + nb * row;
  // corrections of the first nb rows into the last nb rows of x
  if ((rc = launch_precond(s, Hx, Sx, eps, nb, xd, st)) != GPAW_OK) return rc;
  // H~ and S~ of the corrections (their projections into the rows of Px)
  const void *X = nullptr, *XS = nullptr;
  if (s->np > 0) {
    char *Pd = static_cast<char *>(Px) + nb * prow;
    if ((rc = launch_project(s, xd, nb, Pd, st)) != GPAW_OK) return rc;
    if ((rc = launch_dmat2(s, Pd, nb, s->ws.X, s->ws.XS, st)) != GPAW_OK) return rc;
    X = s->ws.X;
    XS = s->ws.XS;
  }
  if ((rc = launch_stencil(s, xd, nb, X, Hd, st, XS, Sd)) != GPAW_OK) return rc;
  // Rayleigh-Ritz on the 2 nb block
  if ((rc = launch_subspace(s, x, Hx, Sx, 2 * nb, H2, S2, st)) != GPAW_OK) return rc;
  int32_t *dinfo = info ? info : s->ws.info;
  if ((rc = launch_eigh(s, H2, S2, 2 * nb, eps2, C2, dinfo, st)) != GPAW_OK) return rc;
  if ((rc = launch_rotate(s, C2, x, 2 * nb, s->ng, psi_out, st, false, false, nb)) != GPAW_OK)
    return rc;
  if (s->np > 0)
    if ((rc = launch_rotate(s, C2, Px, 2 * nb, s->np, P_out, st, false, false, nb)) != GPAW_OK)
      return rc;
  if ((rc = after_launch("gpaw_davidson_step")) != GPAW_OK) return rc;
  if (info) return GPAW_OK;
  int32_t h_info = 0;
  GFD_HIP(hipMemcpyAsync(&h_info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  GFD_HIP(hipStreamSynchronize(st));
  if (h_info > 0)
    return fail(GPAW_ENOTPD, "the extended overlap matrix is not positive definite (leading "
                             "minor " + std::to_string(h_info) + ")");
  if (h_info < 0) return fail(GPAW_ENOCONV, "eigenvector orthogonalisation did not settle");
  return GPAW_OK;
}

int gpaw_orthonormalize(gpaw_sys *s, const void *psi, const void *Spsi, int32_t nb,
                        void *psi_out, const void *P, void *P_out, int32_t *info, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (nb > 1024) return fail(GPAW_ESHAPE, "gpaw_orthonormalize supports nb <= 1024");
  if (!psi || !psi_out) return fail(GPAW_EINVAL, "psi and psi_out must not be NULL");
  if ((P == nullptr) != (P_out == nullptr))
    return fail(GPAW_EINVAL, "P and P_out must be both NULL or both set");
  if (!Spsi && !P && s->np > 0)
    return fail(GPAW_EINVAL, "without Spsi the projections P of psi are needed");
  const size_t es = elem_size(s->dtype);
  const size_t bytes = static_cast<size_t>(nb) * s->ng * es;
  const size_t pbytes = static_cast<size_t>(nb) * s->np * es;
  if (overlaps(psi_out, bytes, psi, bytes) || (Spsi && overlaps(psi_out, bytes, Spsi, bytes)))
    return fail(GPAW_EALIAS, "psi_out overlaps psi or Spsi");
  if (P && s->np > 0 && (overlaps(P_out, pbytes, P, pbytes) || overlaps(P_out, pbytes, psi_out, bytes)))
    return fail(GPAW_EALIAS, "P_out overlaps P or psi_out");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t mbytes = static_cast<size_t>(nb) * nb * mat_elem_size(s->dtype);
  char *Sm = static_cast<char *>(s->ws.mat);
  char *Cm = Sm + mbytes;
  int32_t *dinfo = info ? info : s->ws.info;
  if (Spsi) {
    if ((rc = launch_subspace(s, psi, Spsi, nullptr, nb, Sm, nullptr, st)) != GPAW_OK) return rc;
  } else {
    // S' = dV psi^H psi + P^H (Delta S P): the Gram matrix of the block, then
    // the projector term as a product over the Np projector columns (a view
    // of the system with Np "grid points" and unit volume element), added
    if ((rc = launch_subspace(s, psi, psi, nullptr, nb, Sm, nullptr, st)) != GPAW_OK) return rc;
    if (s->np > 0) {
      if ((rc = launch_dmat(s, s->dS, P, nb, s->ws.X, st)) != GPAW_OK) return rc;
      gpaw_sys pv = *s;
      pv.ng = s->np;
      pv.dV = 1.0;
      if ((rc = launch_subspace(&pv, P, s->ws.X, nullptr, nb, Cm, nullptr, st)) != GPAW_OK)
        return rc;
      const int64_t nel = static_cast<int64_t>(nb) * nb * (is_complex(s->dtype) ? 2 : 1);
      if ((rc = launch_add_mat(reinterpret_cast<const double *>(Cm), reinterpret_cast<double *>(Sm),
                               nel, st)) != GPAW_OK)
        return rc;
    }
  }
  if ((rc = launch_chol_inv(s, Sm, nb, Cm, dinfo, st)) != GPAW_OK) return rc;
  // L^-H is upper triangular (the rotations skip the zero half) and, for a
  // nearly orthonormal block, close to the identity
  if ((rc = launch_rotate(s, Cm, psi, nb, s->ng, psi_out, st, true, true)) != GPAW_OK) return rc;
  if (P && s->np > 0)
    if ((rc = launch_rotate(s, Cm, P, nb, s->np, P_out, st, true, true)) != GPAW_OK) return rc;
  if ((rc = after_launch("gpaw_orthonormalize")) != GPAW_OK) return rc;
  if (info) return GPAW_OK;
  int32_t h_info = 0;
  GFD_HIP(hipMemcpyAsync(&h_info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  GFD_HIP(hipStreamSynchronize(st));
  if (h_info > 0)
    return fail(GPAW_ENOTPD, "overlap of the block is not positive definite (leading minor " +
                                 std::to_string(h_info) + ")");
  return GPAW_OK;
}

int gpaw_rotate(gpaw_sys *s, const void *psi, const void *C, int32_t nb, void *psi_out,
                const void *P, void *P_out, void *stream) {
  int rc;
  if ((rc = check_sys(s)) != GPAW_OK) return rc;
  if ((rc = check_nb(s, nb)) != GPAW_OK) return rc;
  if (!psi || !C || !psi_out) return fail(GPAW_EINVAL, "psi, C_nn and psi_out must not be NULL");
  if ((P == nullptr) != (P_out == nullptr))
    return fail(GPAW_EINVAL, "P and P_out must be both NULL or both set");
  const size_t es = elem_size(s->dtype);
  const size_t bytes = static_cast<size_t>(nb) * s->ng * es;
  const size_t pbytes = static_cast<size_t>(nb) * s->np * es;
  if (overlaps(psi_out, bytes, psi, bytes)) return fail(GPAW_EALIAS, "psi_out overlaps psi");
  if (overlaps(psi_out, bytes, C, static_cast<size_t>(nb) * nb * mat_elem_size(s->dtype)))
    return fail(GPAW_EALIAS, "psi_out overlaps C_nn");
  if (P && s->np > 0 && (overlaps(P_out, pbytes, P, pbytes) || overlaps(P_out, pbytes, psi_out, bytes)))
    return fail(GPAW_EALIAS, "P_out overlaps P or psi_out");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = launch_rotate(s, C, psi, nb, s->ng, psi_out, st)) != GPAW_OK) return rc;
  if (P && s->np > 0)
    if ((rc = launch_rotate(s, C, P, nb, s->np, P_out, st)) != GPAW_OK) return rc;
  return after_launch("gpaw_rotate");
}

}  // extern "C"
