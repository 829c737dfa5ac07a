"""One full block eigensolver step on a synthetic system (oracle).

Order follows the paper's SCF step (1), Sec. "Solving the Kohn-Sham
equation": projections, H~Psi and S~Psi (Eq. (dh)), subspace matrices,
generalised eigensolve, rotation of the block and of its projections.
"""
from dataclasses import dataclass

import numpy as np

from .projectors import projector_matrix, projector_matrix_sparse
from .paw import project, apply_H, apply_S
from .subspace import subspace_matrices, diagonalize, rotate


@dataclass
class Operators:
    """Grid, projector matrix and PAW corrections of one system."""
    n: tuple
    h: tuple
    k: tuple
    v: np.ndarray
    Q: np.ndarray
    dH: np.ndarray
    dS: np.ndarray

    @property
    def dV(self):
        return float(self.h[0] * self.h[1] * self.h[2])

    @classmethod
    def from_system(cls, s, sparse=False, k=None):
        """sparse: store the projector matrix as CSR (large grids). k: the
        Bloch vector when s carries no block to infer it from."""
        build = projector_matrix_sparse if sparse else projector_matrix
        kk = tuple(s.k) if k is None else tuple(k)
        Q = build(s.n, s.h, kk, s.pos, s.channels)
        return cls(n=tuple(s.n), h=tuple(s.h), k=kk, v=s.v, Q=Q, dH=s.dH, dS=s.dS)

    def project(self, psi):
        return project(self.Q, psi, self.dV)

    def apply_H(self, psi, P=None):
        return apply_H(psi, self.n, self.h, self.k, self.v, self.Q, self.dH, self.dV, P)

    def apply_S(self, psi, P=None):
        return apply_S(psi, self.Q, self.dS, self.dV, P)


def fd_step(system, ops=None):
    ops = ops or Operators.from_system(system)
    psi = system.psi.reshape(system.nb, -1)
    P = ops.project(psi)
    Hpsi = ops.apply_H(psi, P)
    Spsi = ops.apply_S(psi, P)
    H, S = subspace_matrices(psi, Hpsi, Spsi, ops.dV)
    eps, C = diagonalize(H, S)
    return dict(P=P, Hpsi=Hpsi, Spsi=Spsi, H=H, S=S, eps=eps, C=C,
                psi_rot=rotate(psi, C), P_rot=rotate(P, C), ops=ops)
