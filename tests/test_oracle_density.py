"""Pins of the oracle's pseudo density and atomic density matrices.

Paper: Eq. (atomicdensitymatrix) and the expectation-value formula after it,
<O> = sum_n <psi~_n|O~|psi~_n> + sum_a sum_ii' D^a_ii' Delta O^a_i'i
(Sec. "Projector augmented-wave method"). The pins tie n~ and D to operators
pinned elsewhere (S~, H~ and the add-back of Eq. (dh)) rather than to
their own formulas:
  * charge: with S~-orthonormal Ritz vectors, dV sum n~ + sum tr(D dS) =
    sum f (the expectation value of S~ with O = 1);
  * energy: dV sum v n~ + sum f <psi|T|psi> + sum D_ii' dH_ii' = sum f eps
    (Ritz vectors diagonalise H~);
  * index order: for a complex Hermitian per-atom matrix dO, the non-local
    operator sum |p_i> dO_ii' <p_i'| (the oracle's add-back) has the
    expectation sum_ii' D_ii' dO_ii', which tells D from its transpose;
  * a normalised plane wave gives the constant density |c|^2.
Occupations are non-uniform throughout, so a dropped f fails.
"""
import numpy as np
import pytest

import oracle
import synth


def _ritz(k, seed=31, nb=7):
    s = synth.make_system(n=(12, 10, 14), h=0.22, nb=nb, natoms=3, rc=1.3, seed=seed, k=k)
    ops = oracle.Operators.from_system(s)
    r = oracle.fd_step(s, ops)
    f = np.linspace(2.0, 0.25, nb)
    return s, ops, r, f


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)], ids=["real", "bloch"])
def test_charge_of_orthonormal_ritz_vectors(k):
    s, ops, r, f = _ritz(k)
    psi, P = r["psi_rot"], r["P_rot"]
    n = oracle.pseudo_density(psi, f)
    D = oracle.atomic_density_matrices(P, f, s.natoms, 13)
    total = oracle.paw_norm(n, D, s.dS, ops.dV)
    assert abs(total - f.sum()) <= 1e-12 * f.sum()
    # the PAW correction matters: the pseudo charge alone misses it
    assert abs(ops.dV * n.sum() - f.sum()) > 1e-6


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)], ids=["real", "bloch"])
def test_energy_of_ritz_vectors(k):
    s, ops, r, f = _ritz(k)
    psi, P, eps = r["psi_rot"], r["P_rot"], r["eps"]
    n = oracle.pseudo_density(psi, f)
    D = oracle.atomic_density_matrices(P, f, s.natoms, 13)
    grid = psi.reshape((psi.shape[0],) + tuple(s.n))
    Tpsi = oracle.kinetic(grid, s.h, s.k).reshape(psi.shape[0], -1)
    kin = ops.dV * np.real(np.sum(f[:, None] * psi.conj() * Tpsi))
    loc = ops.dV * float(np.sum(s.v.ravel() * n))
    nl = float(np.real(sum(np.sum(D[a] * s.dH[a]) for a in range(s.natoms))))
    assert abs(kin + loc + nl - float(f @ eps)) <= 1e-11 * float(np.abs(f) @ np.abs(eps))


def test_index_order_against_the_addback():
    s, ops, r, f = _ritz((0.25, 0.0, 0.5), seed=33)
    psi, P = r["psi_rot"], r["P_rot"]
    rng = np.random.default_rng(5)
    A = rng.standard_normal((s.natoms, 13, 13)) + 1j * rng.standard_normal((s.natoms, 13, 13))
    dO = A + np.conj(np.transpose(A, (0, 2, 1)))  # complex Hermitian
    Opsi = oracle.addback(ops.Q, P, dO)
    grid_side = ops.dV * np.sum(f[:, None] * psi.conj() * Opsi)
    D = oracle.atomic_density_matrices(P, f, s.natoms, 13)
    from_D = sum(np.sum(D[a] * dO[a]) for a in range(s.natoms))
    assert abs(grid_side - from_D) <= 1e-12 * abs(grid_side)
    # the transpose (conjugate) of D gives a different value here
    wrong = sum(np.sum(D[a].T * dO[a]) for a in range(s.natoms))
    assert abs(wrong - from_D) > 1e-3 * abs(from_D)
    # D is Hermitian and positive semidefinite for positive occupations
    for a in range(s.natoms):
        assert np.abs(D[a] - D[a].conj().T).max() <= 1e-14 * np.abs(D[a]).max()
        assert np.linalg.eigvalsh(D[a]).min() >= -1e-13 * np.abs(D[a]).max()


def test_plane_wave_density_is_constant():
    n, h = (6, 8, 10), (0.3, 0.25, 0.2)
    r = np.meshgrid(*[np.arange(n[c]) * h[c] for c in range(3)], indexing="ij")
    G = [2 * np.pi * 2 / (n[0] * h[0]), 2 * np.pi * 1 / (n[1] * h[1]), -2 * np.pi * 3 / (n[2] * h[2])]
    c = 0.7 - 0.2j
    psi = (c * np.exp(1j * sum(G[i] * r[i] for i in range(3)))).reshape(1, -1)
    dens = oracle.pseudo_density(psi, [1.5])
    assert np.allclose(dens, 1.5 * abs(c) ** 2, rtol=1e-14, atol=0)
