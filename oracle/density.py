"""Pseudo density and atomic density matrices of a block (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper, Sec. "Projector augmented-wave method": the atomic density matrices of
Eq. (atomicdensitymatrix),
    D^a_ii' = sum_n f_n <psi~_n|p~^a_i> <p~^a_i'|psi~_n>,
and the smooth (pseudo) density that the same section pairs with them,
    n~(r) = sum_n f_n |psi~_n(r)|^2
(the pseudo-density counterpart of Eq. (allelectrondensity) without
compensation charges, which belong to the Poisson step). With the
projections P[n, ai] = <p~^a_i|psi~_n> (oracle.project), <psi~_n|p~^a_i> is
conj(P[n, ai]). Steps (3)-(4) of the SCF loop (Sec. "Solving the Kohn-Sham
equation") consume both. f_n are occupation numbers (any reals here).

Arrays: psi [nb, Ng], P [nb, natoms*ni], f [nb]; n~ [Ng] (real);
D [natoms, ni, ni] (complex for complex blocks).
"""
import numpy as np


def pseudo_density(psi, f):
    """n~[g] = sum_n f[n] |psi[n, g]|^2 (real, float64)."""
    psi = np.asarray(psi)
    f = np.asarray(f, dtype=np.float64)
    return (f[:, None] * (psi.real ** 2 + psi.imag ** 2 if np.iscomplexobj(psi)
                          else psi ** 2)).sum(axis=0)


def atomic_density_matrices(P, f, natoms, ni):
    """D[a, i, j] = sum_n f[n] conj(P[n, a ni + i]) P[n, a ni + j]."""
    P = np.asarray(P)
    f = np.asarray(f, dtype=np.float64)
    nb = P.shape[0]
    Pa = P.reshape(nb, natoms, ni)
    return np.einsum("n,nai,naj->aij", f, Pa.conj(), Pa)


def paw_norm(n_tilde, D, dS, dV):
    """Expectation value of S~ summed with the occupations, by the paper's
    <O> = sum_n <psi~_n|O~|psi~_n> + sum_a sum_ii' D^a_ii' Delta O^a_i'i
    with O = 1: dV sum_g n~[g] + sum_a tr(D^a Delta S^a)."""
    corr = sum(np.trace(D[a] @ dS[a]) for a in range(D.shape[0]))
    return dV * float(n_tilde.sum()) + float(np.real(corr))
