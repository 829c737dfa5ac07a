"""Pins of the Poisson oracle (zero-boundary multigrid, Sec. "Solving the
Kohn-Sham equation", Poisson solvers and boundary conditions).

* the discrete Laplacian against the analytic Laplacian of a compactly
  supported smooth bump, converging at 6th order;
* the direct solution of nabla^2 phi = -4 pi rho against a manufactured
  solution (the bump and its analytic Laplacian), 6th order, plus the
  Gauss-law value at the centre of a Gaussian charge far from the walls;
* restriction and interpolation: the 3-D adjoint identity
  8 <R f, g> = <f, P g>, the trilinear hat of a coarse delta, and exact
  interpolation of a function linear along each axis inside the box;
* the Jacobi smoother's fixed point is the direct solution; the V-cycle
  contracts the residual by a factor below 0.45 per cycle and converges to
  the direct solution.
"""
import numpy as np
import pytest
from scipy.special import erf

from oracle import poisson as P


def _bump(n, h, center, R, p=10):
    """(1 - r^2/R^2)^p for r < R, its analytic Laplacian."""
    x = [np.arange(1, n[c] + 1) * h[c] - center[c] for c in range(3)]
    X, Y, Z = np.meshgrid(*x, indexing="ij")
    s = (X * X + Y * Y + Z * Z) / (R * R)
    inside = s < 1.0
    t = np.where(inside, 1.0 - s, 0.0)
    f = t ** p
    r2 = s * R * R
    lap = np.where(inside, -6.0 * p / R**2 * t ** (p - 1)
                   + 4.0 * p * (p - 1) * r2 / R**4 * t ** (p - 2), 0.0)
    return f, lap


def _grid(N, L):
    h = L / (N + 1)
    return (N, N, N), (h, h, h)


def test_laplacian_sixth_order():
    L, R = 4.0, 1.7
    errs = []
    for N in (15, 31, 63):
        n, h = _grid(N, L)
        f, lap = _bump(n, h, (L / 2,) * 3, R)
        errs.append(np.abs(P.laplacian_zero(f, h) - lap).max() / np.abs(lap).max())
    # h halves twice: the error falls by about 2^6 each time
    assert 30.0 < errs[1] / errs[2] < 100.0
    assert errs[2] < 1e-5


def test_laplacian_matrix_matches_operator():
    rng = np.random.default_rng(3)
    n, h = (5, 7, 4), (0.3, 0.2, 0.25)
    f = rng.standard_normal(n)
    A = P.laplacian_matrix(n, h)
    assert np.allclose((A @ f.ravel()).reshape(n), P.laplacian_zero(f, h), rtol=0, atol=1e-12)
    # the separable eigen-solve and a sparse direct solve agree
    rho = rng.standard_normal(n)
    a, b = P.solve_direct(rho, h), P.solve_sparse(rho, h)
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    # symmetric negative definite
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() < 1e-12
    assert np.linalg.eigvalsh(Ad).max() < 0.0


def test_direct_solution_manufactured():
    L, R = 4.0, 1.7
    errs = []
    for N in (31, 63):
        n, h = _grid(N, L)
        phi, lap = _bump(n, h, (L / 2,) * 3, R)
        rho = -lap / (4.0 * np.pi)
        errs.append(np.abs(P.solve_direct(rho, h) - phi).max())
    assert errs[1] < 2e-4
    assert 30.0 < errs[0] / errs[1] < 100.0


def test_direct_solution_gauss_law():
    # Gaussian charge Q of width s in a box much larger than s: the
    # free-space potential is Q erf(r / (sqrt 2 s)) / r; with the walls at
    # distance d the zero boundary lowers it by about Q / d (the potential of
    # the charge's images), so the centre value lies between the free-space
    # value minus 2 Q / d and the free-space value
    N, L, s, Q = 31, 12.0, 0.6, 1.0
    n, h = _grid(N, L)
    x = np.arange(1, N + 1) * h[0] - L / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r2 = X * X + Y * Y + Z * Z
    rho = Q * np.exp(-r2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    phi = P.solve_direct(rho, h)
    c = N // 2
    free = Q * np.sqrt(2.0 / np.pi) / s  # limit r -> 0 of Q erf(r/(sqrt2 s))/r
    assert free - 2.0 * Q / (L / 2) < phi[c, c, c] < free
    # away from the walls the profile follows the free-space shape up to a
    # nearly constant offset
    r = np.abs(x[c + 1:c + 6])
    prof = phi[c + 1:c + 6, c, c]
    freep = Q * erf(r / (np.sqrt(2) * s)) / r
    off = prof - freep
    assert np.ptp(off) < 0.2 * abs(off.mean()) + 1e-3


def test_restrict_interpolate_adjoint_and_closed_forms():
    rng = np.random.default_rng(5)
    nf = (7, 9, 5)
    nc = P.coarse_shape(nf)
    assert nc == (3, 4, 2)
    f = rng.standard_normal(nf)
    g = rng.standard_normal(nc)
    lhs = 8.0 * np.sum(P.restrict(f) * g)
    rhs = np.sum(f * P.interpolate(g, nf))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))
    # a coarse delta interpolates to the trilinear hat prod (1 - |d|/2)
    d = np.zeros(nc)
    d[1, 2, 0] = 1.0
    hat = P.interpolate(d, nf)
    cen = (3, 5, 1)  # fine index of coarse (1, 2, 0)
    for idx in np.ndindex(*nf):
        w = 1.0
        for c in range(3):
            off = abs(idx[c] - cen[c])
            w *= 1.0 - off / 2.0 if off <= 1 else 0.0
        assert hat[idx] == pytest.approx(w, abs=1e-15)
    # a function linear along each axis is reproduced at the fine points
    # whose interpolation stencil stays inside (odd 0-based index or
    # strictly interior even index)
    a = rng.standard_normal(4)
    xc = [2 * (np.arange(nc[c]) + 1) for c in range(3)]
    G = a[0] + a[1] * xc[0][:, None, None] + a[2] * xc[1][None, :, None] + a[3] * xc[2][None, None, :]
    F = P.interpolate(G, nf)
    xf = [np.arange(nf[c]) + 1 for c in range(3)]
    lin = a[0] + a[1] * xf[0][:, None, None] + a[2] * xf[1][None, :, None] + a[3] * xf[2][None, None, :]
    inner = np.ix_(range(1, nf[0] - 1), range(1, nf[1] - 1), range(1, nf[2] - 1))
    assert np.abs(F[inner] - lin[inner]).max() < 1e-12
    # full weighting of a constant is the constant away from the faces
    assert np.allclose(P.restrict(np.ones(nf)), 1.0)


def test_jacobi_fixed_point_is_direct_solution():
    rng = np.random.default_rng(7)
    n, h = (5, 5, 5), (0.3, 0.3, 0.3)
    rho = rng.standard_normal(n)
    ref = P.solve_direct(rho, h)
    phi = P.jacobi(np.zeros(n), -4 * np.pi * rho, h, sweeps=3000)
    assert np.abs(phi - ref).max() < 1e-10 * np.abs(ref).max()


def test_vcycle_converges_to_direct_solution():
    rng = np.random.default_rng(11)
    n, h = _grid(31, 6.4)
    rho = rng.standard_normal(n)
    ref = P.solve_direct(rho, h)
    phi, cycles, hist = P.solve_multigrid(rho, h, tol=1e-12, max_cycles=60)
    rates = np.array(hist[1:]) / np.array(hist[:-1])
    assert rates.max() < 0.45
    assert cycles < 45
    assert np.abs(phi - ref).max() < 1e-9 * np.abs(ref).max()
