"""PAW operators H~ and S~ applied to a block (oracle).

Paper, Sec. "Projector augmented-wave method", Eq. (dh) and the overlap
operator beside it:
    H~ = -1/2 nabla^2 + v~ + sum_a sum_ii' |p~^a_i> Delta H^a_ii' <p~^a_i'|
    S~ = 1 + sum_a sum_ii' |p~^a_i> Delta S^a_ii' <p~^a_i'|
with the projections <p~^a_i|psi_n> (the quantity the paper's GPU section
lists beside psi~_n, and whose products form D^a in Eq. (atomicdensitymatrix)).
Integrals are sums over grid points times dV (Sec. "Developer's
perspective", the egg-box remark).

Arrays: psi is [nb, Ng] (C-order grid flattened), Q is [Np, Ng] with
Np = natoms*ni, P is [nb, Np].
"""
import numpy as np
from scipy.linalg import block_diag

from .stencil import kinetic


def block_diag_atoms(D):
    """[natoms][ni][ni] -> [Np][Np] block-diagonal matrix."""
    if D.shape[0] == 0:
        return np.zeros((0, 0))
    return block_diag(*list(D))


def project(Q, psi, dV):
    """P[n, ai] = dV sum_g conj(Q[ai, g]) psi[n, g]."""
    return dV * (psi @ Q.conj().T)


def addback(Q, P, D):
    """sum_ai Q[ai, g] sum_aj D[ai, aj] P[n, aj] for each band n."""
    X = P @ block_diag_atoms(D).T
    return X @ Q


def apply_H(psi, grid_shape, h, k, v, Q, dH, dV, P=None):
    nb = psi.shape[0]
    if P is None:
        P = project(Q, psi, dV)
    loc = kinetic(psi.reshape((nb,) + tuple(grid_shape)), h, k).reshape(nb, -1)
    loc = loc + v.reshape(1, -1) * psi
    if Q.shape[0]:
        loc = loc + addback(Q, P, dH)
    return loc


def apply_S(psi, Q, dS, dV, P=None):
    if P is None:
        P = project(Q, psi, dV)
    out = psi.astype(np.result_type(psi.dtype, Q.dtype, 1.0), copy=True)
    if Q.shape[0]:
        out = out + addback(Q, P, dS)
    return out
