"""Subspace (Rayleigh-Ritz) step (oracle).

Paper, Sec. "Solving the Kohn-Sham equation": each SCF step starts by
diagonalising the Hamiltonian in the subspace of the current wave functions;
Sec. "Parallelization": the band and domain ranks cooperate on the matrix
elements of H and S, and Cholesky plus diagonalisation are dense linear
algebra.

Definitions:
    H_nm = dV sum_g conj(psi_n(g)) (H~ psi_m)(g),  S_nm likewise with S~psi;
    symmetrise X <- (X + X^H)/2;  solve H C = S C diag(eps), C^H S C = I,
    eps ascending;  rotated block psi'_n = sum_m C_mn psi_m  (Psi' = C^T Psi).

Orthonormality correction (a reading: the paper lists Cholesky decomposition
among the subspace dense linear algebra but states no re-orthonormalisation
step): S' = dV Psi^H (S~Psi), S' = L L^H, psi''_n = sum_m (L^-H)_mn psi_m, so
that Psi''^H S~ Psi'' = I and psi''_n lies in the span of psi_0..psi_n (the
Gram-Schmidt result in the S~ inner product).
"""
import numpy as np
import scipy.linalg


def subspace_matrices(psi, Hpsi, Spsi, dV):
    H = dV * (psi.conj() @ Hpsi.T)
    S = dV * (psi.conj() @ Spsi.T)
    return H, S


def hermiticity_defect(X):
    return np.linalg.norm(X - X.conj().T) / np.linalg.norm(X)


def diagonalize(H, S):
    Hs = 0.5 * (H + H.conj().T)
    Ss = 0.5 * (S + S.conj().T)
    eps, C = scipy.linalg.eigh(Hs, Ss)
    return eps, C


def rotate(psi, C):
    return C.T @ psi


def orthonormalize(psi, Spsi, dV):
    """Cholesky re-orthonormalisation of a block: Psi'' = (L^-H)^T Psi with
    S' = dV Psi^H (S~ Psi) = L L^H (symmetrised first)."""
    S1 = dV * (psi.conj() @ Spsi.T)
    S1 = 0.5 * (S1 + S1.conj().T)
    L = np.linalg.cholesky(S1)
    Linv = scipy.linalg.solve_triangular(L, np.eye(L.shape[0]), lower=True)
    return Linv.conj().T.T @ psi
