"""Pins of the oracle's full step: dense operators, spectra and invariants.

Paper: Eq. (dh) and the overlap operator (Sec. "Projector augmented-wave
method"); subspace diagonalisation as SCF step (1) (Sec. "Solving the
Kohn-Sham equation"). The dense matrices below are assembled element by
element (tests/brute.py), independently of the oracle's vectorised code.
"""
import numpy as np
import pytest

import oracle
import synth

from . import brute


def _dense_ops(s):
    n, h, k = s.n, s.h, s.k
    dV = h[0] * h[1] * h[2]
    T = brute.dense_kinetic(n, h, k)
    Q = brute.projector_matrix(n, h, k, s.pos, s.channels)
    DH = oracle.block_diag_atoms(s.dH)
    DS = oracle.block_diag_atoms(s.dS)
    H = T + np.diag(s.v.ravel()) + dV * Q.T @ DH @ Q.conj()
    S = np.eye(T.shape[0]) + dV * Q.T @ DS @ Q.conj()
    return H, S


def _small(k=(0.0, 0.0, 0.0), nb=6, seed=21):
    # 8^3 grid, cell 2.0 bohr < 2 rc: spheres overlap their own images
    return synth.make_system(n=(8, 8, 8), h=0.25, nb=nb, natoms=2, rc=1.1, seed=seed, k=k)


@pytest.fixture(scope="module", params=[(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)], ids=["real", "bloch"])
def dense_case(request):
    s = _small(k=request.param)
    H, S = _dense_ops(s)
    return s, H, S


def test_dense_matrices_are_hermitian(dense_case):
    _, H, S = dense_case
    assert np.abs(H - H.conj().T).max() < 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(S).min() > 0.5


def test_apply_matches_dense_operator(dense_case):
    s, H, S = dense_case
    ops = oracle.Operators.from_system(s)
    psi = s.psi.reshape(s.nb, -1)
    assert np.abs(ops.apply_H(psi) - psi @ H.T).max() < 1e-12 * np.abs(psi @ H.T).max()
    assert np.abs(ops.apply_S(psi) - psi @ S.T).max() < 1e-13 * np.abs(psi @ S.T).max()


def _dense_spectrum(H, S):
    w, U = np.linalg.eigh(S)
    Sih = (U / np.sqrt(w)) @ U.conj().T
    return np.linalg.eigvalsh(Sih @ H @ Sih)


def test_full_block_reproduces_dense_spectrum(dense_case):
    s0, H, S = dense_case
    s = synth.make_system(n=s0.n, h=s0.h, nb=512, natoms=2, rc=1.1, seed=21, k=s0.k)
    r = oracle.fd_step(s)
    lam = _dense_spectrum(H, S)
    assert np.abs(r["eps"] - lam).max() < 1e-8 * np.abs(lam).max()


def test_partial_block_interlaces(dense_case):
    s, H, S = dense_case
    lam = _dense_spectrum(H, S)
    r = oracle.fd_step(s)
    # Ritz values from a subspace bound the exact eigenvalues from above
    assert np.all(r["eps"] >= lam[:s.nb] - 1e-10 * np.abs(lam).max())


def _plane_wave_block(n, h, k, nb):
    L = [n[c] * h[c] for c in range(3)]
    r = np.meshgrid(*[np.arange(n[c]) * h[c] for c in range(3)], indexing="ij")
    Gs = [np.array(g) for g in np.ndindex(5, 5, 5)]
    Gs = [g - 2 for g in Gs]

    def sym(G):
        q = [2 * np.pi * (k[c] + G[c]) / L[c] for c in range(3)]
        return -0.5 * sum(oracle.symbol_1d(q[c] * h[c]) / h[c] ** 2 for c in range(3)), q
    Gs.sort(key=lambda G: sym(G)[0])
    out, vals = [], []
    for G in Gs[:nb]:
        e, q = sym(G)
        out.append(np.exp(1j * sum(q[c] * r[c] for c in range(3))))
        vals.append(e)
    return np.array(out), np.array(vals)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)])
def test_free_electron_eigenvalues(k):
    """No atoms, v = 0: Ritz values of a block of plane waves are the symbol."""
    n, h = (12, 10, 14), (0.2, 0.22, 0.18)
    psi, vals = _plane_wave_block(n, h, k, 19)
    rng = np.random.default_rng(0)
    mix = rng.standard_normal((19, 19)) + 1j * rng.standard_normal((19, 19))
    psi = (mix @ psi.reshape(19, -1)).reshape(psi.shape)   # hide the basis
    s = synth.make_system(n=n, h=h, nb=19, natoms=0, rc=2.0, seed=0, k=k, complex_psi=True)
    s.v = np.zeros(n)
    s.psi = psi
    r = oracle.fd_step(s)
    assert np.abs(r["eps"] - np.sort(vals)).max() < 1e-11 * np.abs(vals).max()


def test_free_electron_overlap_is_diagonal():
    n, h, k = (10, 10, 10), (0.2, 0.2, 0.2), (0.25, 0.0, 0.5)
    psi, _ = _plane_wave_block(n, h, k, 7)
    ops = oracle.Operators(n=n, h=h, k=k, v=np.zeros(n), Q=np.zeros((0, 1000)),
                           dH=np.zeros((0, 13, 13)), dS=np.zeros((0, 13, 13)))
    p = psi.reshape(7, -1)
    H, S = oracle.subspace_matrices(p, ops.apply_H(p), ops.apply_S(p), ops.dV)
    assert np.abs(S - 1000 * ops.dV * np.eye(7)).max() < 1e-12


@pytest.mark.parametrize("name", ["A", "B"])
def test_config_matrices_hermitian_and_pd(name):
    s = synth.config_system(name)
    r = oracle.fd_step(s)
    assert oracle.hermiticity_defect(r["H"]) <= 1e-14
    assert oracle.hermiticity_defect(r["S"]) <= 1e-14
    np.linalg.cholesky(0.5 * (r["S"] + r["S"].T))
    assert np.all(np.diff(r["eps"]) >= 0)


def test_shift_by_multiple_of_overlap():
    """H~ + c S~ (v += c, Delta H += c Delta S) shifts every eigenvalue by c."""
    s = synth.config_system("A")
    r0 = oracle.fd_step(s)
    c = 0.731
    s.v = s.v + c
    s.dH = s.dH + c * s.dS
    r1 = oracle.fd_step(s)
    assert np.abs(r1["eps"] - r0["eps"] - c).max() < 1e-12 * np.abs(r0["eps"]).max()


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)])
def test_rotated_block_is_orthonormal_and_diagonal(k):
    s = synth.make_system(n=(16, 14, 18), h=0.2, nb=12, natoms=3, rc=1.8, seed=5, k=k)
    r = oracle.fd_step(s)
    ops = r["ops"]
    p = r["psi_rot"]
    H1, S1 = oracle.subspace_matrices(p, ops.apply_H(p), ops.apply_S(p), ops.dV)
    assert np.abs(S1 - np.eye(s.nb)).max() < 1e-12
    assert np.abs(H1 - np.diag(r["eps"])).max() < 1e-12 * np.abs(r["eps"]).max()
    # rotated projections are the projections of the rotated block
    assert np.abs(r["P_rot"] - ops.project(p)).max() < 1e-12 * np.abs(r["P_rot"]).max()


def _gram_schmidt_S(psi, ops):
    """Classical Gram-Schmidt in the S~ inner product, one band at a time
    (pure Python loop over bands; S~ applied by the oracle operator)."""
    out = []
    for n in range(psi.shape[0]):
        v = psi[n].astype(complex if np.iscomplexobj(psi) else float)
        for u in out:
            v = v - ops.dV * np.vdot(u, ops.apply_S(v[None])[0]) * u
        nrm = np.sqrt(ops.dV * np.vdot(v, ops.apply_S(v[None])[0]).real)
        out.append(v / nrm)
    return np.array(out)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)])
def test_orthonormalize_is_gram_schmidt_in_the_overlap(k):
    """The Cholesky correction equals Gram-Schmidt in the S~ inner product
    (both give the unique S~-orthonormal block whose band n lies in the span
    of bands 0..n with a positive coefficient on band n)."""
    s = synth.make_system(n=(10, 12, 9), h=0.22, nb=7, natoms=2, rc=1.5, seed=77, k=k)
    ops = oracle.Operators.from_system(s)
    psi = s.psi.reshape(s.nb, -1)
    got = oracle.orthonormalize(psi, ops.apply_S(psi), ops.dV)
    want = _gram_schmidt_S(psi, ops)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    S1 = oracle.subspace_matrices(got, ops.apply_H(got), ops.apply_S(got), ops.dV)[1]
    assert np.abs(S1 - np.eye(s.nb)).max() <= 1e-12
