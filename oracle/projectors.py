"""Projector functions and their periodic-image sums on the grid (oracle).

Paper: the PAW Hamiltonian and overlap carry the projectors p~^a_i
(Sec. "Projector augmented-wave method", Eq. (dh)); real projectors come from
setup files (Sec. "PAW data sets and pseudopotentials"), which this oracle
replaces by synthetic channels.

Readings:
  * channel (l, sigma, rc): p(r) = N r^l exp(-r^2/(2 sigma^2)) chi(r/rc) Y_lm(r^),
    chi(x) = (1 - x^2)^2 for x < 1 and 0 beyond, N = [Gamma(l+3/2) sigma^(2l+3)/2]^(-1/2)
    (unit norm of the untruncated function); m runs -l..l, channels in order;
  * real harmonics with the Condon-Shortley convention folded in:
    l=1 -> (y, z, x); l=2 -> (xy, yz, 3z^2-r^2, xz, x^2-y^2);
  * grid value q^a_i(r) = sum_R exp(i k.R) p_i(r - R_a - R) over every lattice
    vector R with |r - R_a - R| < rc, for r on the cell's grid points.
    Then <p|psi> = dV sum_r conj(q) psi and the add-back is q (Delta P).
"""
from math import gamma, pi, sqrt, ceil

import numpy as np


def radial_norm(l, sigma):
    return (gamma(l + 1.5) * sigma ** (2 * l + 3) / 2.0) ** -0.5


def solid_harmonics(l, x, y, z):
    """r^l Y_lm for m = -l..l as a list of arrays (real harmonics)."""
    if l == 0:
        return [np.full_like(x, 0.5 / sqrt(pi))]
    if l == 1:
        c = sqrt(3.0 / (4.0 * pi))
        return [c * y, c * z, c * x]
    if l == 2:
        c2 = 0.5 * sqrt(15.0 / pi)
        c20 = 0.25 * sqrt(5.0 / pi)
        c22 = 0.25 * sqrt(15.0 / pi)
        r2 = x * x + y * y + z * z
        return [c2 * x * y, c2 * y * z, c20 * (3.0 * z * z - r2), c2 * x * z,
                c22 * (x * x - y * y)]
    raise ValueError("only l <= 2 is defined")


def projector_values(channels, x, y, z):
    """[ni, npts] values of every projector at displacements (x, y, z)."""
    r = np.sqrt(x * x + y * y + z * z)
    rows = []
    for (l, sigma, rc) in channels:
        s = r / rc
        chi = np.where(s < 1.0, (1.0 - s * s) ** 2, 0.0)
        radial = radial_norm(l, sigma) * np.exp(-r * r / (2.0 * sigma * sigma)) * chi
        for ylm in solid_harmonics(l, x, y, z):
            rows.append(radial * ylm)
    return np.array(rows)


def projector_matrix(n, h, k, pos, channels):
    """Q[a*ni + i, g]: q^a_i at every grid point g (C order over n)."""
    n = tuple(n)
    ni = sum(2 * l + 1 for (l, _, _) in channels)
    rmax = max(rc for (_, _, rc) in channels)
    cplx = any(kc != 0.0 for kc in k)
    L = np.array([n[c] * h[c] for c in range(3)])
    X, Y, Z = np.meshgrid(*[np.arange(n[c]) * h[c] for c in range(3)], indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    Q = np.zeros((pos.shape[0] * ni, X.size), dtype=complex if cplx else float)
    M = [int(ceil(rmax / L[c])) + 1 for c in range(3)]
    for a in range(pos.shape[0]):
        for m0 in range(-M[0], M[0] + 1):
            for m1 in range(-M[1], M[1] + 1):
                for m2 in range(-M[2], M[2] + 1):
                    R = np.array([m0, m1, m2]) * L
                    dx = X - pos[a, 0] - R[0]
                    dy = Y - pos[a, 1] - R[1]
                    dz = Z - pos[a, 2] - R[2]
                    inside = dx * dx + dy * dy + dz * dz < rmax * rmax
                    if not inside.any():
                        continue
                    vals = projector_values(channels, dx[inside], dy[inside], dz[inside])
                    if cplx:
                        vals = vals * np.exp(2j * np.pi * (k[0] * m0 + k[1] * m1 + k[2] * m2))
                    Q[a * ni:(a + 1) * ni, inside] += vals
    return Q


def projector_matrix_sparse(n, h, k, pos, channels):
    """Same matrix as projector_matrix, stored sparse (CSR): for each atom and
    lattice image only the grid points in the box around the sphere are
    visited, so that large grids fit in memory."""
    from scipy.sparse import coo_matrix
    n = tuple(n)
    ni = sum(2 * l + 1 for (l, _, _) in channels)
    rmax = max(rc for (_, _, rc) in channels)
    cplx = any(kc != 0.0 for kc in k)
    L = np.array([n[c] * h[c] for c in range(3)])
    M = [int(ceil(rmax / L[c])) + 1 for c in range(3)]
    rows, cols, vals = [], [], []
    for a in range(pos.shape[0]):
        for m0 in range(-M[0], M[0] + 1):
            for m1 in range(-M[1], M[1] + 1):
                for m2 in range(-M[2], M[2] + 1):
                    m = (m0, m1, m2)
                    centre = [pos[a, c] + m[c] * L[c] for c in range(3)]
                    axes = []
                    for c in range(3):
                        lo = max(0, int(np.floor((centre[c] - rmax) / h[c])))
                        hi = min(n[c] - 1, int(np.ceil((centre[c] + rmax) / h[c])))
                        axes.append(np.arange(lo, hi + 1))
                    if any(len(ax) == 0 for ax in axes):
                        continue
                    I, J, K = np.meshgrid(*axes, indexing="ij")
                    dx = I.ravel() * h[0] - centre[0]
                    dy = J.ravel() * h[1] - centre[1]
                    dz = K.ravel() * h[2] - centre[2]
                    inside = dx * dx + dy * dy + dz * dz < rmax * rmax
                    if not inside.any():
                        continue
                    g = ((I.ravel() * n[1] + J.ravel()) * n[2] + K.ravel())[inside]
                    v = projector_values(channels, dx[inside], dy[inside], dz[inside])
                    if cplx:
                        v = v * np.exp(2j * np.pi * (k[0] * m0 + k[1] * m1 + k[2] * m2))
                    for i in range(ni):
                        rows.append(np.full(g.size, a * ni + i))
                        cols.append(g)
                        vals.append(v[i])
    npj = pos.shape[0] * ni
    ng = n[0] * n[1] * n[2]
    dtype = complex if cplx else float
    if not rows:
        return coo_matrix((npj, ng), dtype=dtype).tocsr()
    Q = coo_matrix((np.concatenate(vals).astype(dtype),
                    (np.concatenate(rows), np.concatenate(cols))), shape=(npj, ng))
    return Q.tocsr()  # duplicates (a sphere meeting its own image) are summed
