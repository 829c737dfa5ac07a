"""Pins of the finite-system operators and the real-time propagation oracle
(Sec. "Real-time TDDFT", Eq. (td_ks); zero boundary of finite systems,
Sec. "Solving the Kohn-Sham equation").

* the zero-boundary kinetic operator equals the periodic one on a function
  supported away from the faces;
* the finite projector matrix equals the periodic construction's values in
  the first octant of a cell twice as large (no image reaches it);
* H~ is symmetric and S~ symmetric positive definite;
* Crank-Nicolson: psi^H S~ psi is conserved; an eigenvector of (H~, S~)
  picks up exactly the Cayley factor (1 - i tau eps) / (1 + i tau eps);
  a step forward and one backward return the start; the one-step error
  against exp(-i dt S~^-1 H~) falls as dt^3;
* the kick leaves |psi| unchanged and the dipole of a Gaussian is its
  centre times its norm.
"""
import numpy as np
import scipy.linalg

import synth
from oracle import tddft as T
from oracle.projectors import projector_matrix
from oracle.stencil import kinetic


def _system(seed=2, natoms=2):
    s = synth.make_system(n=(8, 9, 7), h=0.4, nb=3, natoms=natoms, rc=1.2, seed=seed)
    s.meta["boundary"] = "zero"
    return s


def test_zero_kinetic_equals_periodic_away_from_faces():
    n, h = (16, 14, 15), (0.3, 0.3, 0.3)
    rng = np.random.default_rng(1)
    f = np.zeros(n)
    f[5:11, 4:10, 5:10] = rng.standard_normal((6, 6, 5))
    ops = T.FiniteOps(n, h, np.zeros(n), np.zeros((0, 3)), [], np.zeros((0, 1, 1)),
                      np.zeros((0, 1, 1)))
    a = ops.apply_H(f.reshape(1, -1)).reshape(n)
    b = kinetic(f, h)
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_finite_projectors_equal_unwrapped_periodic_values():
    s = _system()
    # an atom near a face: its sphere is cut there
    pos = np.array([[0.3, 1.5, 1.2], [1.6, 3.3, 2.6]])
    Q = T.projector_matrix_zero(s.n, s.h, pos, s.channels)
    n2 = tuple(2 * m for m in s.n)
    # shift by one cell length so that no image of the doubled cell reaches
    # the first octant from the far side
    L = np.array([s.n[c] * s.h[c] for c in range(3)])
    Qp = projector_matrix(n2, s.h, (0.0, 0.0, 0.0), pos + L, s.channels)
    Qp = Qp.reshape(Qp.shape[0], *n2)[:, s.n[0]:, s.n[1]:, s.n[2]:].reshape(Qp.shape[0], -1)
    assert np.abs(Q - Qp).max() < 1e-14
    assert np.count_nonzero(Q) > 0


def test_finite_operators_symmetric():
    s = _system()
    ops = T.FiniteOps.from_system(s)
    H, S = ops.dense()
    assert np.abs(H - H.T).max() < 1e-10 * np.abs(H).max()
    assert np.abs(S - S.T).max() < 1e-12
    assert np.linalg.eigvalsh(S).min() > 0.0


def test_crank_nicolson_pins():
    s = _system()
    ops = T.FiniteOps.from_system(s)
    H, S = ops.dense()
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((3, H.shape[0])) + 1j * rng.standard_normal((3, H.shape[0]))
    dt = 0.05
    out = T.cn_step(ops, psi, dt, H, S)
    n0 = np.einsum("ng,gh,nh->n", psi.conj(), S, psi).real
    n1 = np.einsum("ng,gh,nh->n", out.conj(), S, out).real
    assert np.abs(n1 - n0).max() < 1e-12 * n0.max()
    # eigenvectors: the Cayley factor
    eps, C = scipy.linalg.eigh(H, S)
    tau = dt / 2
    for j in (0, 7, H.shape[0] - 1):
        phi = C[:, j][None, :].astype(complex)
        got = T.cn_step(ops, phi, dt, H, S)
        fac = (1 - 1j * tau * eps[j]) / (1 + 1j * tau * eps[j])
        assert np.abs(got - fac * phi).max() < 1e-10 * np.abs(phi).max()
    # forward then backward
    back = T.cn_step(ops, out, -dt, H, S)
    assert np.abs(back - psi).max() < 1e-10 * np.abs(psi).max()
    # third-order local error against the exact propagator (smooth start:
    # the lowest eigenvectors)
    Ssi = np.linalg.solve(S, H)
    start = (C[:, :4] @ rng.standard_normal(4))[None, :].astype(complex)
    errs = []
    for d in (0.02, 0.01):
        exact = (scipy.linalg.expm(-1j * d * Ssi) @ start.T).T
        errs.append(np.abs(T.cn_step(ops, start, d, H, S) - exact).max())
    assert 6.0 < errs[0] / errs[1] < 10.0


def test_kick_and_dipole():
    n, h = (12, 13, 11), (0.3, 0.3, 0.3)
    x = [np.arange(n[c]) * h[c] for c in range(3)]
    c = (1.7, 1.9, 1.5)
    g = np.exp(-((x[0][:, None, None] - c[0]) ** 2 + (x[1][None, :, None] - c[1]) ** 2
                 + (x[2][None, None, :] - c[2]) ** 2) / (2 * 0.5 ** 2)).ravel()[None, :]
    kicked = T.kick(g.astype(complex), n, h, (0.3, -0.2, 0.1))
    assert np.abs(np.abs(kicked) - g).max() < 1e-15
    d = T.dipole(kicked, [2.0], n, h)
    norm = 2.0 * np.prod(h) * np.sum(g ** 2)
    assert np.allclose(d, np.array(c) * norm, rtol=1e-6)


def test_sparse_projectors_match_dense():
    s = _system(seed=9, natoms=3)
    a = T.FiniteOps.from_system(s)
    b = T.FiniteOps.from_system(s, sparse=True)
    psi = s.psi.reshape(s.nb, -1)
    assert np.abs(a.apply_H(psi) - b.apply_H(psi)).max() < 1e-12
    assert np.abs(a.apply_S(psi) - b.apply_S(psi)).max() < 1e-12
