"""Multigrid Poisson solver for finite (zero-boundary) systems (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper: the Hartree potential of the FD mode comes from a Poisson solver,
either a direct (Fourier / Fourier-sine) one or an iterative multigrid one
with Jacobi or Gauss-Seidel smoothing; for 0-, 1- and 2-dimensional systems
the potential is taken to vanish on the cell boundary (Sec. "Solving the
Kohn-Sham equation"). Interpolating from one uniform grid to another is one
of the C hot spots (Sec. "Developer's perspective").

Readings (the paper fixes neither the discretisation nor the cycle):
  * nabla^2 phi = -4 pi rho in atomic units;
  * zero boundary: the N interior points of an axis sit at x_i = i h,
    i = 1..N; phi vanishes at i <= 0 and i >= N + 1, so the stencil's
    reach past the faces sees zeros (zero extension);
  * the operator is the 19-point 6th-order Laplacian of the kinetic term;
  * multigrid on vertex-centred grids: N = 2 m + 1 coarsens to m points,
    coarse point j on fine point 2 j; restriction by full weighting
    (weights 1/4, 1/2, 1/4 per axis), interpolation trilinear (weights
    1/2 at odd fine points, 1 at even ones, zero past the faces);
  * smoother: weighted Jacobi, phi <- phi + omega (f - A phi) / diag(A),
    omega = 0.8; V-cycle with nu1 sweeps before and nu2 after the coarse
    correction; the coarsest grid (an axis that is even or below 3 points)
    is smoothed with many sweeps;
  * the result the solver converges to is the solution of the discrete
    system, which solve_direct computes exactly (the operator is a sum of
    three one-axis operators, diagonalised axis by axis; solve_sparse is
    the same solution by a sparse direct solve, for small grids).
"""
import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from .stencil import WEIGHTS

OMEGA = 0.8


def _shift_zero(f, axis, d):
    """g[i] = f[i + d] along axis, zero where i + d leaves the grid."""
    g = np.zeros_like(f)
    n = f.shape[axis]
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if d > 0:
        src[axis] = slice(d, n)
        dst[axis] = slice(0, n - d)
    else:
        src[axis] = slice(0, n + d)
        dst[axis] = slice(-d, n)
    if n > abs(d):
        g[tuple(dst)] = f[tuple(src)]
    return g


def laplacian_zero(f, h):
    """nabla^2 f with zero extension past the faces (last three axes)."""
    f = np.asarray(f, dtype=float)
    out = np.zeros_like(f)
    for c in range(3):
        axis = f.ndim - 3 + c
        acc = WEIGHTS[0] * f
        for d in (1, 2, 3):
            acc = acc + WEIGHTS[d] * (_shift_zero(f, axis, d) + _shift_zero(f, axis, -d))
        out += acc / (h[c] * h[c])
    return out


def diagonal(h):
    """The diagonal entry of the discrete Laplacian."""
    return sum(WEIGHTS[0] / (hc * hc) for hc in h)


def laplacian_matrix(n, h):
    """The discrete Laplacian as a sparse matrix over the C-ordered grid."""
    mats = []
    for c in range(3):
        diags = [WEIGHTS[0] * np.ones(n[c])]
        offs = [0]
        for d in (1, 2, 3):
            if d < n[c]:
                diags += [WEIGHTS[d] * np.ones(n[c] - d)] * 2
                offs += [d, -d]
        mats.append(scipy.sparse.diags(diags, offs, shape=(n[c], n[c])) / (h[c] * h[c]))
    eye = [scipy.sparse.identity(n[c]) for c in range(3)]
    A = scipy.sparse.kron(scipy.sparse.kron(mats[0], eye[1]), eye[2])
    A = A + scipy.sparse.kron(scipy.sparse.kron(eye[0], mats[1]), eye[2])
    A = A + scipy.sparse.kron(scipy.sparse.kron(eye[0], eye[1]), mats[2])
    return A.tocsc()


def _axis_matrix(m, hc):
    """The 1-D zero-extension second difference on m points, dense."""
    A = np.zeros((m, m))
    for i in range(m):
        A[i, i] = WEIGHTS[0]
        for d in (1, 2, 3):
            if i + d < m:
                A[i, i + d] = A[i + d, i] = WEIGHTS[d]
    return A / (hc * hc)


def solve_direct(rho, h):
    """phi with nabla^2 phi = -4 pi rho, zero boundary. The operator is the
    sum of three commuting one-axis operators, so it is diagonalised by the
    eigenvectors of each axis: phi = Q (Q^T f / (l0 + l1 + l2))."""
    f = -4.0 * np.pi * np.asarray(rho, dtype=float)
    lam, Q = [], []
    for c in range(3):
        w, v = np.linalg.eigh(_axis_matrix(f.shape[c], h[c]))
        lam.append(w)
        Q.append(v)
    g = np.einsum("ia,jb,kc,ijk->abc", Q[0], Q[1], Q[2], f, optimize=True)
    g /= lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :]
    return np.einsum("ia,jb,kc,abc->ijk", Q[0], Q[1], Q[2], g, optimize=True)


def solve_sparse(rho, h):
    """The same solution by a sparse direct solve (small grids only)."""
    rho = np.asarray(rho, dtype=float)
    A = laplacian_matrix(rho.shape, h)
    phi = scipy.sparse.linalg.spsolve(A, -4.0 * np.pi * rho.ravel())
    return phi.reshape(rho.shape)


def residual(phi, f, h):
    """r = f - A phi."""
    return f - laplacian_zero(phi, h)


def jacobi(phi, f, h, sweeps=1, omega=OMEGA):
    """Weighted Jacobi sweeps on A phi = f."""
    dinv = omega / diagonal(h)
    for _ in range(sweeps):
        phi = phi + dinv * residual(phi, f, h)
    return phi


def coarse_shape(n):
    """Coarse grid of n, or None when an axis cannot be coarsened."""
    if any(m % 2 == 0 or m < 3 for m in n):
        return None
    return tuple((m - 1) // 2 for m in n)


def _weights_1d(n_fine):
    """R[j][i] of full weighting along one axis (coarse j = 0..m-1 sits on
    fine index 2 j + 1 in 0-based interior numbering)."""
    m = (n_fine - 1) // 2
    R = np.zeros((m, n_fine))
    for j in range(m):
        i = 2 * j + 1
        R[j, i - 1] = 0.25
        R[j, i] = 0.5
        R[j, i + 1] = 0.25
    return R


def restrict(f):
    """Full weighting of a fine grid function (odd sizes) onto the coarse grid."""
    f = np.asarray(f, dtype=float)
    out = f
    for c in range(3):
        R = _weights_1d(f.shape[c])
        out = np.moveaxis(np.tensordot(R, np.moveaxis(out, c, 0), axes=(1, 0)), 0, c)
    return out


def interpolate(g, n_fine):
    """Trilinear interpolation of a coarse grid function onto the fine grid."""
    g = np.asarray(g, dtype=float)
    out = g
    for c in range(3):
        P = 2.0 * _weights_1d(n_fine[c]).T  # fine x coarse
        out = np.moveaxis(np.tensordot(P, np.moveaxis(out, c, 0), axes=(1, 0)), 0, c)
    return out


def vcycle(phi, f, h, nu1=2, nu2=2, coarse_sweeps=None):
    """One V-cycle on A phi = f (recursion down to the coarsest grid)."""
    nc = coarse_shape(phi.shape)
    if nc is None:
        sweeps = coarse_sweeps if coarse_sweeps is not None else 20 * max(phi.shape)
        return jacobi(phi, f, h, sweeps)
    phi = jacobi(phi, f, h, nu1)
    r = residual(phi, f, h)
    hc = tuple(2.0 * x for x in h)
    e = vcycle(np.zeros(nc), restrict(r), hc, nu1, nu2, coarse_sweeps)
    phi = phi + interpolate(e, phi.shape)
    return jacobi(phi, f, h, nu2)


def solve_multigrid(rho, h, tol=1e-12, max_cycles=100):
    """V-cycles from phi = 0 until ||f - A phi|| <= tol ||f||; returns
    (phi, cycles, relative residuals after each cycle)."""
    f = -4.0 * np.pi * np.asarray(rho, dtype=float)
    phi = np.zeros_like(f)
    fn = np.linalg.norm(f)
    hist = []
    for it in range(max_cycles):
        phi = vcycle(phi, f, h)
        hist.append(np.linalg.norm(residual(phi, f, h)) / fn)
        if hist[-1] <= tol:
            return phi, it + 1, hist
    return phi, max_cycles, hist
