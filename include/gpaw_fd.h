/*
 * gpaw_fd.h -- C ABI of the MI355X (gfx950) library for one block step of the
 * real-space (finite-difference) PAW eigensolver.
 *
 * Method (GPAW review, arXiv:2310.14776):
 *   H~ = -1/2 nabla^2 + v~(r) + sum_a sum_ii' |p~^a_i> Delta H^a_ii' <p~^a_i'|
 *   S~ = 1 + sum_a sum_ii' |p~^a_i> Delta S^a_ii' <p~^a_i'|
 * (Sec. "Projector augmented-wave method", Eq. (dh) and the overlap operator
 * beside it), the kinetic operator represented on a uniform Cartesian grid
 * (Sec. "Wave-function representations"), and the subspace diagonalisation
 * that opens every SCF step (Sec. "Solving the Kohn-Sham equation", step 1),
 * with Cholesky decomposition and diagonalisation as dense linear algebra
 * (Sec. "Parallelization"). Arrays cross the boundary as plain pointers to
 * contiguous memory, as GPAW's C hot spots receive NumPy buffers
 * (Sec. "Developer's perspective").
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid: orthorhombic cell of n[0] x n[1] x n[2] points with spacing h[c]
 *   (bohr); point (i,j,l) sits at (i h0, j h1, l h2); axis 2 is contiguous.
 *   Ng = n0*n1*n2, dV = h0*h1*h2; integrals are dV times grid sums.
 * Boundary: Bloch, psi(r + L_c e_c) = exp(2 pi i k_c) psi(r), k in reduced
 *   units; k = 0 is the periodic (real) case. A system created with
 *   boundary = 1 is finite instead: every value outside the grid is zero
 *   (for the stencil's reach of three points too) and projector spheres do
 *   not wrap (Sec. "Solving the Kohn-Sham equation": for 0-D systems the
 *   potential vanishes on the cell boundary; the time propagation of
 *   Sec. "Real-time TDDFT" needs such boundaries).
 * Kinetic operator: per axis the 6th-order central second difference,
 *   weights (1/90, -3/20, 3/2, -49/18, 3/2, -3/20, 1/90)/h_c^2 (19-point star).
 * Projectors: every atom carries the same channel list; channel (l, sigma, rc)
 *   gives 2l+1 functions N r^l exp(-r^2/2sigma^2) (1-(r/rc)^2)^2 Y_lm(r^) for
 *   r < rc, N = [Gamma(l+3/2) sigma^(2l+3)/2]^(-1/2), m = -l..l, real
 *   harmonics ordered (y,z,x) for l=1 and (xy,yz,3z^2-r^2,xz,x^2-y^2) for l=2.
 *   ni = sum(2l+1) projectors per atom, Np = natoms*ni, index a*ni + i.
 *   Grid values sum all periodic images R with exp(i k.R).
 * Layouts (row-major, C order):
 *   psi, Hpsi, Spsi, psi_out : [nb][n0][n1][n2]  of the system dtype
 *   P, P_out                 : [nb][Np]          of the system dtype
 *   H_nn, S_nn, C_nn         : [nb][nb]          double (GPAW_F64, GPAW_F32) or
 *                                                interleaved complex double
 *                                                (GPAW_C128, GPAW_C64)
 *   eps                      : [nb]              double
 * Complex data are interleaved (re, im).
 * Memory: pointers named *_dev, and every array argument of the compute calls,
 *   are device pointers owned by the caller; the library never frees them.
 *   The library owns the gpaw_sys object: its projector tables, potential,
 *   correction matrices and workspace (sized by max_bands at creation).
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Compute calls only enqueue work and return; gpaw_subspace_diag with a
 *   NULL info pointer is the one call that waits for its stream.
 * Concurrency: calls on one gpaw_sys share its workspace; calls that overlap
 *   in time on one system (two streams, two host threads) race.
 * Errors: every int-returning call returns GPAW_OK (0) or a negative code;
 *   gpaw_last_error() gives a message for the calling host thread's last
 *   failure. A rejected call has enqueued nothing.
 */
#ifndef GPAW_FD_H
#define GPAW_FD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPAW_FD_VERSION 1

#if defined(__GNUC__)
#define GPAW_API __attribute__((visibility("default")))
#else
#define GPAW_API
#endif

enum gpaw_status {
  GPAW_OK = 0,
  GPAW_EINVAL = -1,       /* NULL pointer, bad size, bad channel, bad k  */
  GPAW_EDTYPE = -2,       /* dtype not supported by this call            */
  GPAW_ESHAPE = -3,       /* nb outside [1, max_bands] or above a limit  */
  GPAW_EALIAS = -4,       /* output overlaps an input that it must not   */
  GPAW_EHIP = -5,         /* HIP runtime or launch failure               */
  GPAW_ENOTPD = -6,       /* S_nm is not positive definite               */
  GPAW_ENOMEM = -7,       /* device or host allocation failed            */
  GPAW_ENOCONV = -8,      /* eigenvector orthogonalisation did not settle */
  GPAW_ENONFINITE = -9    /* a non-finite value where a finite one is due */
};

/* Storage/arithmetic type of the wave functions. GPAW_F32 and GPAW_C64 are
 * the precision form: single-precision stencil and projector add-back,
 * projections accumulated in double, subspace matrices and rotations as
 * split-BF16 products on the matrix cores (FP32 accumulators promoted to
 * FP64), and the Cholesky and eigensolve in FP64. */
typedef enum { GPAW_F64 = 0, GPAW_C128 = 1, GPAW_F32 = 2, GPAW_C64 = 3 } gpaw_dtype;

typedef struct {
  int32_t l;       /* 0, 1 or 2 */
  double sigma;    /* Gaussian width (bohr), > 0 */
  double rc;       /* cut-off radius (bohr), > 0 */
} gpaw_channel;

typedef struct {
  int32_t n[3];             /* grid points per axis, each >= 1 */
  double h[3];              /* grid spacing per axis (bohr), > 0 */
  double k[3];              /* Bloch vector, reduced units */
  int32_t dtype;            /* gpaw_dtype of psi; GPAW_F64 and GPAW_F32 need k = 0 */
  int32_t natoms;           /* >= 0 */
  const double *pos;        /* host [natoms][3] cartesian positions (bohr) */
  int32_t nchan;            /* >= 1 when natoms > 0 */
  const gpaw_channel *chan; /* host [nchan], same for every atom */
  const double *dH;         /* host [natoms][ni][ni], Delta H^a (real symmetric) */
  const double *dS;         /* host [natoms][ni][ni], Delta S^a (real symmetric) */
  const double *v;          /* host [n0][n1][n2], local potential v~ (Ha) */
  int32_t max_bands;        /* largest nb any call will pass, >= 1 */
  int32_t boundary;         /* 0: periodic / Bloch (above); 1: zero boundary,
                               a finite system (values vanish outside the
                               n0 x n1 x n2 points, no periodic images; k = 0) */
} gpaw_sys_desc;

typedef struct gpaw_sys gpaw_sys;

/* Build one system on the current HIP device: evaluates the projector
 * functions on the grid spheres (host), uploads tables, potential and
 * corrections, and allocates workspace. Synchronous. On success *out owns
 * the object; release it with gpaw_sys_destroy. */
GPAW_API int gpaw_sys_create(const gpaw_sys_desc *desc, gpaw_sys **out);

/* Free everything the system owns (waits for the device first). NULL is a
 * no-op. */
GPAW_API void gpaw_sys_destroy(gpaw_sys *sys);

/* Sizes of a built system, written to host info[0..7]:
 * Ng, Np, ni, natoms, sphere entries, covered grid points, max_bands, dtype. */
GPAW_API int gpaw_sys_info(const gpaw_sys *sys, int64_t *info);

/* Projections P[n][a*ni+i] = <p~^a_i | psi_n> = dV sum_r conj(q^a_i(r)) psi_n(r)
 * (the projector overlaps of Eq. (dh); the same quantity the paper's GPU
 * section stores beside psi~_n). psi [nb][Ng] -> P [nb][Np]. */
GPAW_API int gpaw_project(gpaw_sys *sys, const void *psi, int32_t nb, void *P, void *stream);

/* Hpsi = H~ psi for each band (Eq. (dh)): kinetic stencil, local potential
 * and non-local add-back sum_a q^a (Delta H^a P^a). P is the projection of
 * this psi block ([nb][Np]) or NULL, in which case the call computes it into
 * workspace. Hpsi must not overlap psi (the stencil reads neighbours). */
GPAW_API int gpaw_fd_apply_H(gpaw_sys *sys, const void *psi, int32_t nb, const void *P,
                    void *Hpsi, void *stream);

/* Spsi = S~ psi = psi + sum_a q^a (Delta S^a P^a) (overlap operator beside
 * Eq. (dh)). P as for gpaw_fd_apply_H. Spsi must not overlap psi. */
GPAW_API int gpaw_fd_apply_S(gpaw_sys *sys, const void *psi, int32_t nb, const void *P,
                    void *Spsi, void *stream);

/* Hpsi = H~ psi and Spsi = S~ psi in one pass over psi (Eq. (dh) and the
 * overlap beside it): the same results as gpaw_fd_apply_H and
 * gpaw_fd_apply_S, with the projector values at each grid point evaluated
 * once for both add-backs. P as for gpaw_fd_apply_H. Hpsi, Spsi and psi
 * must not overlap one another (GPAW_EALIAS). */
GPAW_API int gpaw_fd_apply_HS(gpaw_sys *sys, const void *psi, int32_t nb, const void *P,
                     void *Hpsi, void *Spsi, void *stream);

/* Subspace matrices of SCF step (1) (Sec. "Solving the Kohn-Sham equation"):
 * H_nm = dV sum_r conj(psi_n(r)) Hpsi_m(r), S_nm likewise with Spsi, both
 * [nb][nb], summed in a fixed order (bitwise reproducible). H_nm and S_nm
 * are Hermitian for the operators of Eq. (dh), and the call relies on it:
 * it forms the 64 x 64 (real) / 32 x 32 (complex) tiles on and above the
 * diagonal (diagonal tiles in full) and writes the conjugates of the formed
 * tiles below them. It is not a general product of two unrelated blocks.
 * Spsi may be NULL: then only H_nn is formed and S_nn is ignored. */
GPAW_API int gpaw_subspace_matrices(gpaw_sys *sys, const void *psi, const void *Hpsi,
                           const void *Spsi, int32_t nb, void *H_nn, void *S_nn,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as gpaw_subspace_matrices, with the split-K partial sums in a
 * static device array of the library (64 MiB per GPU, held until the
 * process ends) instead of the system's workspace; the call allocates
 * nothing. nb must satisfy nmat * nb^2 * (2 if complex else 1) * 8 bytes
 * <= 64 MiB (nmat = 2 with Spsi, 1 without), else GPAW_ESHAPE. Every call
 * on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must not be issued. */
GPAW_API int gpaw_subspace_matrices_noalloc(gpaw_sys *sys, const void *psi, const void *Hpsi,
                                           const void *Spsi, int32_t nb, void *H_nn,
                                           void *S_nn, void *stream);

/* Generalised Hermitian eigenproblem of the subspace (Cholesky of S_nm and
 * diagonalisation, Sec. "Parallelization"), all in double precision on the
 * device: symmetrise X <- (X + X^H)/2, S = L L^H, eigen-decompose
 * L^-1 H L^-H, C = L^-H U. Output: eps ascending [nb], C_nn [nb][nb] with
 * column j the j-th eigenvector (C^H S C = I, C^H H C = diag eps).
 * H_nn and S_nn are not modified. nb <= 1024 (blocks up to 128 real / 96
 * complex are factorised inside one workgroup's LDS, larger ones through
 * global memory).
 * info: device int32 or NULL. Non-NULL: the call is asynchronous and the
 * device writes 0 on success, j > 0 when the leading j x j minor of S_nm is
 * not positive definite, or -1 when orthogonalisation did not settle.
 * NULL: the call waits for the stream and returns GPAW_ENOTPD / GPAW_ENOCONV. */
GPAW_API int gpaw_subspace_diag(gpaw_sys *sys, const void *H_nn, const void *S_nn, int32_t nb,
                       double *eps, void *C_nn, int32_t *info, void *stream);

/* Densities of SCF steps (3)-(4) (Sec. "Solving the Kohn-Sham equation"):
 * the pseudo density n~(r) = sum_n f_n |psi~_n(r)|^2 into n_out (device
 * [Ng] FP64, real), and the atomic density matrices of
 * Eq. (atomicdensitymatrix), D^a_ii' = sum_n f_n <psi~_n|p~^a_i>
 * <p~^a_i'|psi~_n> = sum_n f_n conj(P[n][a ni + i]) P[n][a ni + i'], into
 * D_nn (device [natoms][ni][ni], FP64 for real systems, complex128 for
 * complex ones, also in the precision form). f: device [nb] FP64
 * occupation numbers. P: the block's projections ([nb][Np], the block's
 * dtype) or NULL, in which case they are computed into workspace when D_nn
 * is requested. Either output may be NULL (not both). Sums run over bands
 * in a fixed order, in FP64. Enqueues on `stream`. */
GPAW_API int gpaw_density(gpaw_sys *sys, const void *psi, int32_t nb, const double *f,
                          const void *P, double *n_out, void *D_nn, void *stream);

/* Rotation of SCF step (1): psi_out_n = sum_m C_mn psi_m (psi_out = C^T psi),
 * and, when P and P_out are both non-NULL, P_out = C^T P (the projections of
 * the rotated block). psi_out must not overlap psi, nor P_out P. */
GPAW_API int gpaw_rotate(gpaw_sys *sys, const void *psi, const void *C_nn, int32_t nb,
                void *psi_out, const void *P, void *P_out, void *stream);

/* Davidson corrections (SCF step (2), Sec. "Solving the Kohn-Sham
 * equation"; the iterative Davidson eigensolver named in Sec.
 * "Parallelization"; the paper gives no formulas, this is the textbook
 * block Davidson update with a diagonal preconditioner):
 *   out_n(r) = -(Hpsi_n - eps_n Spsi_n)(r) / max(t0 + v(r) - eps_n, t0/2),
 * t0 = (1/2)(49/18) sum_c 1/h_c^2 (the diagonal of the FD kinetic
 * operator). Hpsi, Spsi, out: [nb][Ng] in the system dtype; eps: device
 * [nb] FP64. out must not overlap Hpsi or Spsi. Enqueues on `stream`. */
GPAW_API int gpaw_davidson_correction(gpaw_sys *sys, const void *Hpsi, const void *Spsi,
                                      const double *eps, int32_t nb, void *out, void *stream);

/* One block Davidson step (FP64 and complex128 systems): from Ritz vectors
 * psi (rows 0..nb-1 of x, with H~psi, S~psi in rows 0..nb-1 of Hx, Sx,
 * their projections in rows 0..nb-1 of Px, and Ritz values eps, e.g. the
 * output of one subspace step), the corrections of
 * gpaw_davidson_correction are written to rows nb..2nb-1 of x, their
 * projections, H~ and S~ to rows nb..2nb-1 of Px, Hx, Sx; then the
 * Rayleigh-Ritz step on the 2nb block: H2, S2 ([2nb][2nb] subspace
 * matrices), eps2 ([2nb] ascending) and C2 ([2nb][2nb], C2^H S2 C2 = I),
 * and psi_out_n = sum_m C2_mn x_m, P_out_n = sum_m C2_mn Px_m for n < nb
 * (the lowest nb Ritz vectors). Needs 2 nb <= max_bands and 2 nb <= 1024.
 * x, Hx, Sx: [2nb][Ng]; Px, P_out: [2nb][Np], [nb][Np] (NULL without
 * atoms); psi_out: [nb][Ng]. info as for gpaw_subspace_diag. No Ritz value
 * rises in a step (the new span contains the old block). */
GPAW_API int gpaw_davidson_step(gpaw_sys *sys, int32_t nb, void *x, void *Hx, void *Sx, void *Px,
                                const double *eps, void *H2, void *S2, void *C2, double *eps2,
                                void *psi_out, void *P_out, int32_t *info, void *stream);

/* Orthonormality correction of a rotated block: S' = dV psi^H Spsi (Spsi =
 * S~ psi, e.g. the rotated S~psi, since S~ is linear), S' = L L^H in FP64 on
 * the device, psi_out = psi L^-H in band space (psi_out_n =
 * sum_m (L^-H)_mn psi_m), so that psi_out^H S~ psi_out = I; P_out likewise
 * from P when both are non-NULL. Cholesky-based re-orthonormalisation (the
 * paper lists Cholesky decomposition among the subspace dense linear algebra,
 * Sec. "Parallelization"). Spsi may be NULL when P holds the projections of
 * psi (or the system has no atoms): then S' = dV psi^H psi + P^H Delta S P,
 * the same matrix by Eq. (dh) (S~ = 1 + sum_a p~ Delta S p~^H, so psi^H of
 * the non-local part is conj(P) Delta S P), formed without S~psi. info: as
 * for gpaw_subspace_diag (j > 0 when the leading j x j minor of S' is not
 * positive definite). nb <= 1024. */
GPAW_API int gpaw_orthonormalize(gpaw_sys *sys, const void *psi, const void *Spsi, int32_t nb,
                                 void *psi_out, const void *P, void *P_out, int32_t *info,
                                 void *stream);

/* ------------------------------------------------------------ batched form
 * Many independent systems (uneven grids and band counts, real and Bloch)
 * stepped by one HIP graph launch: for every system the chain
 * gpaw_project -> apply H~ -> apply S~ -> gpaw_subspace_matrices ->
 * gpaw_subspace_diag -> gpaw_rotate, with the same kernels and results as
 * those calls. Independent systems or k-points are the method's natural
 * unit of parallel work (Sec. "Parallelization"); the chains are recorded on
 * up to 16 concurrent graph branches so that small systems overlap. */
typedef struct gpaw_batch gpaw_batch;

typedef struct {
  const void *psi;   /* device [nb][Ng] block of this system (system dtype) */
  int32_t nb;        /* bands, 1 <= nb <= the system's max_bands */
  void *psi_out;     /* device [nb][Ng] rotated block (must not overlap psi) */
  double *eps;       /* device [nb] Ritz values, ascending */
  void *P_out;       /* device [nb][Np] rotated projections, or NULL */
  void *H_nn;        /* device [nb][nb] subspace H, or NULL (batch workspace) */
  void *S_nn;        /* device [nb][nb] subspace S, or NULL (batch workspace) */
  void *C_nn;        /* device [nb][nb] eigenvectors, or NULL (batch workspace) */
} gpaw_batch_io;

/* Batch over nsys existing systems (host array of handles, all on the
 * current device, each at most once). The batch allocates per-system
 * intermediates (P, H~psi, S~psi, H, S, C at max_bands) and its own streams;
 * it does not own the systems, which must outlive it. */
GPAW_API int gpaw_batch_create(gpaw_sys *const *systems, int32_t nsys, gpaw_batch **out);

/* Waits for the device, then frees the batch (not its systems). NULL is a no-op. */
GPAW_API void gpaw_batch_destroy(gpaw_batch *b);

/* One step of every system. io: host array [nsys]; info: device int32
 * [nsys], written per system as gpaw_subspace_diag's info. The first call,
 * and any call whose io contents or info pointer differ from the previous
 * call's, synchronises `stream` and records the graph (the graph holds the
 * buffer addresses); otherwise the call only enqueues one graph launch on
 * `stream`. Calls of one batch must not overlap (they share its workspace
 * and the systems' workspaces). */
GPAW_API int gpaw_batch_step(gpaw_batch *b, const gpaw_batch_io *io, int32_t *info, void *stream);

/* Autotuner (synchronous, runs on the batch's own stream and overwrites the
 * io outputs): times the launch-shape choices of every system (points per
 * lane, y-z tile and x segments of the stencil, split-K width of the subspace product,
 * row tiles of the rotation, bands per projection workgroup) and then the
 * number of graph branches (1..16), keeps the fastest of each and records
 * the graph for io. Results change only in the order of floating-point sums. */
GPAW_API int gpaw_batch_tune(gpaw_batch *b, const gpaw_batch_io *io, int32_t *info);

/* Chosen shapes: out[0] = graph branches, then per system 7 values
 * (stencil points per lane, stencil tile rows, stencil tile columns,
 * stencil x segments, subspace workgroup target (0: split count balanced
 * over the resident workgroups), rotation row tiles,
 * projection bands per workgroup; 0 = built-in choice). out holds
 * 1 + 7 nsys int32 (host). */
GPAW_API int gpaw_batch_tuning(const gpaw_batch *b, int32_t *out);

/* Sets the launch shapes in the layout gpaw_batch_tuning returns (in holds
 * 1 + 7 nsys int32, host; in[0] = graph branches 0..16, 0 = default), for
 * a caller that kept an earlier autotuner result (a tuning cache) instead of
 * running the autotuner again. Values are checked as the autotuner would
 * choose them (points per lane 0/1/2; tile sides both 0 or both positive;
 * x segments 0..n0; subspace workgroups 0..1024; rotation row tiles complex
 * 2/4, real 4/8; projection bands complex 1/2, real 2/4/8; 0 = built-in),
 * single-precision systems accept only 0s; on any bad value GPAW_EINVAL and
 * nothing changes. The recorded graph is dropped; the next step records
 * again. Results change only in the order of floating-point sums. */
GPAW_API int gpaw_batch_set_tuning(gpaw_batch *b, const int32_t *in);

/* Message for the calling host thread's last non-zero return ("" if none). */
GPAW_API const char *gpaw_last_error(void);

/* GPAW_FD_VERSION of the built library. */
GPAW_API int gpaw_version(void);

/* ------------------------------------------------------------------------
 * Real-time propagation (Sec. "Real-time TDDFT", Eq. (td_ks)):
 * i S~ d psi~_n / dt = H~ psi~_n with S~ fixed; FD propagation needs the
 * finite (boundary = 1) systems above, and k = 0 in any case. complex128
 * wave functions only (GPAW_EDTYPE otherwise). Allocates, on first use, a
 * workspace of 5 x max_bands x Ng complex values kept until the system is
 * destroyed (GPAW_ENOMEM when that fails).
 * ------------------------------------------------------------------------ */

/* psi_n <- exp(-i kappa . r) psi_n at r = (i h0, j h1, l h2): the delta kick
 * of strength |kappa| (kappa: host [3], 1/bohr) on the pseudo wave
 * functions. Enqueues only. */
GPAW_API int gpaw_td_kick(gpaw_sys *sys, void *psi, int32_t nb, const double *kappa,
                          void *stream);

/* d[c] = sum_n f_n dV sum_r r_c |psi_n(r)|^2 (device f [nb], device d [3]):
 * the dipole of the pseudo density, summed in a fixed order. Enqueues only. */
GPAW_API int gpaw_td_dipole(gpaw_sys *sys, const void *psi, int32_t nb, const double *f,
                            double *d, void *stream);

/* One Crank-Nicolson step, in place: (S~ + i dt/2 H~) psi(t + dt) =
 * (S~ - i dt/2 H~) psi(t) with H~ held fixed over the step, solved per band
 * by conjugate orthogonal CG (M is complex symmetric for k = 0) from
 * psi(t), until every band's ||r|| <= tol ||rhs|| or max_iter iterations.
 * Synchronous: reads the residual norms after each iteration. iters /
 * rel_residual (host, optional): iterations run and the largest relative
 * residual. GPAW_ENOCONV when tol was not reached (psi then holds the last
 * iterate), GPAW_ENONFINITE for a non-finite residual, GPAW_EINVAL for
 * k != 0. */
GPAW_API int gpaw_td_propagate(gpaw_sys *sys, void *psi, int32_t nb, double dt, double tol,
                               int32_t max_iter, int32_t *iters, double *rel_residual,
                               void *stream);

/* ------------------------------------------------------------------------
 * Poisson equation of a finite system (Sec. "Solving the Kohn-Sham
 * equation": iterative multigrid Poisson solvers with Jacobi smoothing; for
 * finite systems the potential vanishes on the cell boundary) and the grid
 * transfers between uniform grids it uses (interpolation is one of the C
 * hot spots, Sec. "Developer's perspective").
 *
 * Zero-boundary grid: n[c] interior points per axis at x = i h_c,
 * i = 1..n[c]; values vanish at i <= 0 and i >= n[c] + 1 (also for the
 * stencil's reach of three points). Arrays are real FP64 [n0][n1][n2],
 * device memory owned by the caller. The discrete operator is the 19-point
 * 6th-order Laplacian of the kinetic term (weights above).
 * ------------------------------------------------------------------------ */
typedef struct gpaw_poisson gpaw_poisson;

/* Multigrid hierarchy for an n0 x n1 x n2 zero-boundary grid of spacing h
 * (host arrays of 3). Levels halve while every axis is odd and >= 3
 * (N = 2m + 1 -> m; coarse point j on fine point 2j + 1, 0-based); the
 * library allocates each level's right-hand side and scratch (about 2.3 x
 * the fine grid in total). GPAW_ESHAPE for grids above 2^31 points,
 * GPAW_ENOMEM when the device allocations fail. */
GPAW_API int gpaw_poisson_create(const int32_t *n, const double *h, gpaw_poisson **out);
GPAW_API void gpaw_poisson_destroy(gpaw_poisson *p);
/* Number of levels (1 = the grid does not coarsen). */
GPAW_API int gpaw_poisson_levels(const gpaw_poisson *p, int32_t *levels);

/* Solves nabla^2 phi = -4 pi rho. phi is the initial guess on entry and the
 * solution on return; V-cycles (two weighted-Jacobi sweeps, omega = 0.8,
 * before and after each coarse correction; the coarsest level smoothed with
 * 20 x its largest axis sweeps) run until ||f - A phi|| <= tol ||f||
 * (f = -4 pi rho, 2-norms) or max_cycles. Synchronous: waits for `stream`
 * after every cycle to read the residual. cycles / rel_residual (host,
 * optional) receive the count and the final relative residual. rho and phi
 * must not alias (GPAW_EALIAS); GPAW_ENONFINITE when the residual is not
 * finite. Calls on one hierarchy must not overlap (shared scratch). */
GPAW_API int gpaw_poisson_solve(gpaw_poisson *p, const double *rho, double *phi, double tol,
                                int32_t max_cycles, int32_t *cycles, double *rel_residual,
                                void *stream);

/* out = nabla^2 f on the zero-boundary grid (n, h host arrays of 3). */
GPAW_API int gpaw_laplacian_zero(const int32_t *n, const double *h, const double *f,
                                 double *out, void *stream);

/* Full-weighting restriction fine (nf) -> coarse ((nf - 1) / 2 per axis):
 * coarse[j] = sum_d prod_c w(d_c) fine[2j + 1 + d], w = (1/4, 1/2, 1/4).
 * Every axis of nf odd and >= 3 (GPAW_ESHAPE otherwise). */
GPAW_API int gpaw_grid_restrict(const int32_t *nf, const double *fine, double *coarse,
                                void *stream);
/* Trilinear interpolation coarse ((nf - 1) / 2) -> fine (nf): weight 1 on
 * the coarse point, 1/2 beside it, zero past the faces; accumulate != 0
 * adds into fine instead of overwriting it. Same shape rule. */
GPAW_API int gpaw_grid_interpolate(const int32_t *nf, const double *coarse, double *fine,
                                   int32_t accumulate, void *stream);

/* Measurement probes (they compute nothing of the method): the ceilings the
 * roofline fractions are also stated against, timed by the caller.
 * gpaw_probe_copy: dst = src over `bytes` (a multiple of 16; both device
 * buffers 16-byte aligned, not overlapping), 16-byte loads and stores
 * (moves 2 x bytes through HBM). gpaw_probe_mfma: `workgroups` x 4
 * wavefronts, each running `iters` rounds of 8 independent matrix-core
 * products: kind 0 = FP64 v_mfma_f64_16x16x4 (2048 flops each), kind 1 =
 * BF16 v_mfma_f32_16x16x32 (16384 flops each); writes one value per lane to
 * out (workgroups x 256 doubles for kind 0, floats for kind 1). Both only
 * enqueue on `stream`. */
GPAW_API int gpaw_probe_copy(const void *src, void *dst, int64_t bytes, void *stream);
GPAW_API int gpaw_probe_mfma(int32_t kind, void *out, int32_t workgroups, int32_t iters,
                             void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GPAW_FD_H */
