"""One block Davidson step around the subspace step (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper, Sec. "Solving the Kohn-Sham equation": step (2) of the SCF loop takes
the wave functions through "one or more steps" of the iterative eigensolver;
Sec. "Parallelization" names the iterative Davidson and RMM-DIIS methods of
the FD mode, whose subspace diagonalisations are the dense linear algebra of
step (1). The paper states neither the correction vectors nor a
preconditioner; the reading taken here (the textbook block Davidson update):

  given Ritz vectors psi_n with Ritz values eps_n (the subspace step's
  output),
    residuals       R_n = H~ psi_n - eps_n S~ psi_n                (Eq. (dh))
    corrections     d_n(r) = -R_n(r) / p_n(r),
                    p_n(r) = max(t0 + v(r) - eps_n, t0 / 2),
                    t0 = (1/2) (49/18) sum_c 1/h_c^2, the diagonal of the FD
                    kinetic operator (a diagonal, Jacobi-type preconditioner
                    of the local part of H~ - eps S~, kept positive);
    Rayleigh-Ritz   on span{psi_1..psi_nb, d_1..d_nb} (2 nb vectors): the
                    subspace matrices of the extended block, the generalised
                    eigenproblem, the lowest nb eigenpairs;
    update          psi'_n = sum_m C_mn x_m over the extended block x, for
                    n < nb (C: the lowest nb eigenvectors).
The span contains the old block, so by the min-max principle no Ritz value
rises; iterated, the step converges to the lowest nb eigenpairs of (H~, S~).
"""
import numpy as np

from .subspace import subspace_matrices, diagonalize

KIN_DIAG_WEIGHT = 49.0 / 18.0  # |w_0| of the 1-D 6th-order second difference


def kinetic_diagonal(h):
    """t0 = -1/2 sum_c w_0 / h_c^2 with w_0 = -49/18."""
    return 0.5 * KIN_DIAG_WEIGHT * sum(1.0 / (hc * hc) for hc in h)


def precondition(R, eps, v, h):
    """d_n(r) = -R_n(r) / max(t0 + v(r) - eps_n, t0 / 2)."""
    t0 = kinetic_diagonal(h)
    p = np.maximum(t0 + v.reshape(1, -1) - np.asarray(eps).reshape(-1, 1), 0.5 * t0)
    return -R / p


def davidson_step(ops, psi, eps, Hpsi=None, Spsi=None):
    """One step from Ritz vectors psi [nb, Ng] with Ritz values eps.
    Returns (eps', psi', residual norms dV sum |R_n|^2 before the step)."""
    nb = psi.shape[0]
    if Hpsi is None:
        Hpsi = ops.apply_H(psi)
    if Spsi is None:
        Spsi = ops.apply_S(psi)
    R = Hpsi - np.asarray(eps).reshape(-1, 1) * Spsi
    d = precondition(R, eps, ops.v.ravel(), ops.h)
    x = np.concatenate([psi, d.astype(psi.dtype)], axis=0)
    H2, S2 = subspace_matrices(x, np.concatenate([Hpsi, ops.apply_H(d)]),
                               np.concatenate([Spsi, ops.apply_S(d)]), ops.dV)
    e2, C2 = diagonalize(H2, S2)
    psi_new = C2[:, :nb].T @ x
    rnorm = ops.dV * np.sum(np.abs(R) ** 2, axis=1)
    return e2[:nb], psi_new, rnorm
