"""Finite-system operators and real-time propagation (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper: the time-dependent Kohn-Sham equation in the PAW formalism,
i S~ d psi~_n / dt = (H~ + v(t)) psi~_n with S~ independent of time
(Sec. "Real-time TDDFT", Eq. (td_ks)), propagated forward from the ground
state; the FD implementation needs non-periodic boundaries; standard
perturbations include the delta kick v(t) = x delta(t), after which the
recorded dipole moment gives the absorption spectrum.

Readings (the paper names neither the propagator nor the kick's PAW form):
  * finite system: the operators of Eq. (dh) with every value outside the
    n0 x n1 x n2 points zero (the 6th-order stencil sees zeros past the
    faces, as in the zero-boundary Poisson problem) and projector spheres
    cut at the faces (no periodic images); grid point (i, j, l) at
    (i h0, j h1, l h2), i = 0..n0-1;
  * propagator: Crank-Nicolson over one step dt with the Hamiltonian held
    fixed, (S~ + i dt/2 H~) psi(t + dt) = (S~ - i dt/2 H~) psi(t) (a Cayley
    transform, so psi^H S~ psi is conserved); the density update between
    steps (which needs the XC and Hartree parts) is outside this path;
  * kick of strength kappa along a vector: psi~ -> exp(-i kappa . r) psi~ on
    the grid (the pseudo wave function only; the atomic corrections of the
    dipole operator are not applied);
  * dipole: d = sum_n f_n dV sum_r r |psi~_n(r)|^2 (the pseudo density's
    dipole).
"""
import numpy as np

from .poisson import laplacian_zero
from .projectors import projector_values
from .paw import block_diag_atoms


def projector_matrix_zero(n, h, pos, channels, sparse=False):
    """Q[a*ni + i, g] of a finite system: each sphere's own values, no
    images, points outside the grid dropped (sparse: CSR, visiting only the
    box around each sphere)."""
    n = tuple(n)
    ni = sum(2 * l + 1 for (l, _, _) in channels)
    rmax = max(rc for (_, _, rc) in channels)
    if sparse:
        from scipy.sparse import coo_matrix
        rows, cols, vals = [], [], []
        for a in range(pos.shape[0]):
            axes = []
            for c in range(3):
                lo = max(0, int(np.floor((pos[a, c] - rmax) / h[c])))
                hi = min(n[c] - 1, int(np.ceil((pos[a, c] + rmax) / h[c])))
                axes.append(np.arange(lo, hi + 1))
            if any(len(ax) == 0 for ax in axes):
                continue
            I, J, K = np.meshgrid(*axes, indexing="ij")
            dx = I.ravel() * h[0] - pos[a, 0]
            dy = J.ravel() * h[1] - pos[a, 1]
            dz = K.ravel() * h[2] - pos[a, 2]
            inside = dx * dx + dy * dy + dz * dz < rmax * rmax
            g = ((I.ravel() * n[1] + J.ravel()) * n[2] + K.ravel())[inside]
            v = projector_values(channels, dx[inside], dy[inside], dz[inside])
            for i in range(ni):
                rows.append(np.full(g.size, a * ni + i))
                cols.append(g)
                vals.append(v[i])
        shape = (pos.shape[0] * ni, int(np.prod(n)))
        if not rows:
            return coo_matrix(shape).tocsr()
        return coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=shape).tocsr()
    X, Y, Z = np.meshgrid(*[np.arange(n[c]) * h[c] for c in range(3)], indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    Q = np.zeros((pos.shape[0] * ni, X.size))
    for a in range(pos.shape[0]):
        dx, dy, dz = X - pos[a, 0], Y - pos[a, 1], Z - pos[a, 2]
        inside = dx * dx + dy * dy + dz * dz < rmax * rmax
        if inside.any():
            Q[a * ni:(a + 1) * ni, inside] = projector_values(channels, dx[inside], dy[inside],
                                                              dz[inside])
    return Q


class FiniteOps:
    """H~ and S~ of a finite (zero-boundary, k = 0) system on [nb, Ng] blocks."""

    def __init__(self, n, h, v, pos, channels, dH, dS, sparse=False):
        self.n, self.h = tuple(n), tuple(h)
        self.v = np.asarray(v, dtype=float).ravel()
        self.Q = projector_matrix_zero(n, h, np.asarray(pos).reshape(-1, 3), channels, sparse) \
            if len(pos) else np.zeros((0, int(np.prod(n))))
        self.DH = block_diag_atoms(np.asarray(dH))
        self.DS = block_diag_atoms(np.asarray(dS))
        self.dV = float(np.prod(h))

    @classmethod
    def from_system(cls, s, sparse=False):
        return cls(s.n, s.h, s.v, s.pos, s.channels, s.dH, s.dS, sparse)

    def project(self, psi):
        return self.dV * (self.Q @ psi.T).T

    def _addback(self, X):
        """sum_ai Q[ai, g] X[n, ai] for each band n."""
        return (self.Q.T @ X.T).T

    def apply_H(self, psi, P=None):
        nb = psi.shape[0]
        out = -0.5 * laplacian_zero(psi.real.reshape((nb,) + self.n), self.h).reshape(nb, -1)
        if np.iscomplexobj(psi):
            out = out + 1j * (-0.5) * laplacian_zero(psi.imag.reshape((nb,) + self.n),
                                                      self.h).reshape(nb, -1)
        out = out + self.v[None, :] * psi
        if self.Q.shape[0]:
            P = self.project(psi) if P is None else P
            out = out + self._addback(P @ self.DH.T)
        return out

    def apply_S(self, psi, P=None):
        out = np.array(psi, dtype=np.result_type(psi.dtype, 1.0), copy=True)
        if self.Q.shape[0]:
            P = self.project(psi) if P is None else P
            out = out + self._addback(P @ self.DS.T)
        return out

    def dense(self):
        """Dense H~ and S~ (Ng x Ng), column g = the operator on the unit
        vector at g (small grids)."""
        ng = int(np.prod(self.n))
        eye = np.eye(ng)
        return self.apply_H(eye).T, self.apply_S(eye).T


def cn_step(ops, psi, dt, H=None, S=None):
    """One Crank-Nicolson step of every band (rows of psi), solved directly."""
    if H is None:
        H, S = ops.dense()
    tau = 0.5 * dt
    A = S + 1j * tau * H
    B = S - 1j * tau * H
    return np.linalg.solve(A, B @ psi.T).T


def kick(psi, n, h, kappa):
    """psi -> exp(-i kappa . r) psi, r = (i h0, j h1, l h2)."""
    x = [np.arange(n[c]) * h[c] for c in range(3)]
    ph = np.exp(-1j * (kappa[0] * x[0][:, None, None] + kappa[1] * x[1][None, :, None]
                       + kappa[2] * x[2][None, None, :])).ravel()
    return psi * ph[None, :]


def dipole(psi, f, n, h):
    """d_c = sum_n f_n dV sum_r r_c |psi_n(r)|^2."""
    dV = float(np.prod(h))
    dens = (np.asarray(f)[:, None] * np.abs(psi) ** 2).sum(axis=0).reshape(n)
    out = np.zeros(3)
    for c in range(3):
        x = np.arange(n[c]) * h[c]
        shape = [1, 1, 1]
        shape[c] = n[c]
        out[c] = dV * np.sum(dens * x.reshape(shape))
    return out
