"""Pins of the oracle's block Davidson step (a reading: the paper names the
iterative Davidson eigensolver of SCF step (2) but gives no formulas).

  * the preconditioner's t0 is the diagonal of the FD kinetic operator,
    assembled element by element (tests/brute.py);
  * no Ritz value rises in a step (min-max: the new span contains the old);
  * no Ritz value falls below the exact eigenvalue (Cauchy interlacing);
  * iterated from a smooth block on a dense 6^3 system (real and Bloch), the
    Ritz values below the widest spectral gap inside the block converge to
    the eigenvalues of the dense (H~, S~) (LAPACK on the brute-force
    matrices) to 1e-11 relative, and their residuals fall by orders of
    magnitude. (The rate is set by the gap at the block's edge relative to
    the spectral width: with a diagonal preconditioner the step is a
    preconditioned block steepest descent.)
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth

from . import brute
from .test_oracle_step import _dense_ops


def test_t0_is_the_kinetic_diagonal():
    n, h = (7, 8, 9), (0.25, 0.21, 0.18)
    T = brute.dense_kinetic(n, h, (0.0, 0.0, 0.0))
    assert np.allclose(np.diag(T).real, oracle.kinetic_diagonal(h), rtol=1e-14, atol=0)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)], ids=["real", "bloch"])
def test_davidson_converges_to_the_dense_spectrum(k):
    s = synth.make_system(n=(6, 6, 6), h=0.45, nb=10, natoms=2, rc=1.3, seed=21, k=k,
                          bands="smooth")
    H, S = _dense_ops(s)
    exact_all = scipy.linalg.eigh(H, S, eigvals_only=True)
    exact = exact_all[:s.nb]
    scale = np.abs(exact_all).max()
    ncv = int(np.argmax(np.diff(exact)[: s.nb - 1])) + 1   # below the widest gap
    ops = oracle.Operators.from_system(s)
    r = oracle.fd_step(s, ops)
    eps, psi = r["eps"], r["psi_rot"]
    first = None
    for it in range(200):
        e_new, psi, rn = oracle.davidson_step(ops, psi, eps)
        first = rn[:ncv].max() if first is None else first
        assert np.all(e_new <= eps + 1e-12 * scale)          # no Ritz value rises
        assert np.all(e_new >= exact - 1e-12 * scale)        # interlacing
        eps = e_new
        if np.abs(eps[:ncv] - exact[:ncv]).max() < 1e-11 * scale:
            break
    assert np.abs(eps[:ncv] - exact[:ncv]).max() < 1e-11 * scale, it
    R = ops.apply_H(psi) - eps[:, None] * ops.apply_S(psi)
    last = (ops.dV * np.sum(np.abs(R[:ncv]) ** 2, axis=1)).max()
    assert last < 1e-8 * first
