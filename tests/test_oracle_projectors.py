"""Pins of the oracle's projector functions and projections.

The projector shapes are a synthetic stand-in for PAW setup data (Sec. "PAW
data sets and pseudopotentials"); they are pinned by 1-D quadrature of the
radial norm, by SciPy's spherical harmonics, and the image-summed grid
matrix by a scalar brute-force loop. The projection/add-back pair is pinned
by the adjoint identity, translation invariance and the Bloch phase of a
lattice translation.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle
import synth

from . import brute


def test_radial_norm_quadrature():
    for l in (0, 1, 2):
        for sigma in (0.4, 0.6667, 1.1):
            N = oracle.radial_norm(l, sigma)
            val, _ = scipy.integrate.quad(
                lambda r: (N * r**l * math.exp(-r * r / (2 * sigma * sigma)))**2 * r * r,
                0, np.inf, epsabs=1e-13, epsrel=1e-13)
            assert abs(val - 1.0) < 1e-10


def test_solid_harmonics_match_scipy():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((3, 50))
    r = np.linalg.norm(v, axis=0)
    x, y, z = v
    theta = np.arccos(z / r)
    phi = np.arctan2(y, x)
    for l in (0, 1, 2):
        got = oracle.solid_harmonics(l, x, y, z)
        for idx, m in enumerate(range(-l, l + 1)):
            want = brute.real_ylm_scipy(l, m, theta, phi) * r**l
            assert np.allclose(got[idx], want, rtol=1e-13, atol=1e-14), (l, m)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)])
def test_projector_matrix_brute_force(k):
    # cell lengths below 2 rc: each sphere meets its own periodic images
    n = (5, 6, 4)
    h = (0.3, 0.25, 0.35)
    channels = synth.standard_channels(1.0)
    pos = np.array([[0.1, 0.7, 0.5], [1.2, 0.05, 1.3]])
    Q = oracle.projector_matrix(n, h, k, pos, channels)
    B = brute.projector_matrix(n, h, k, pos, channels)
    assert np.abs(Q - B).max() < 1e-12 * np.abs(B).max()
    if k == (0.0, 0.0, 0.0):
        assert Q.dtype == np.float64


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5), (0.1, 0.37, 0.8)])
def test_sparse_projector_matrix_brute_force(k):
    # the box-restricted sparse build against the element-by-element brute force,
    # on a cell where spheres meet their own images and one where they do not
    for n, h, rc in (((5, 6, 4), (0.3, 0.25, 0.35), 1.0), ((14, 12, 16), (0.2, 0.21, 0.19), 1.1)):
        channels = synth.standard_channels(rc)
        pos = np.array([[0.1, 0.7, 0.5], [1.2, 0.05, 1.3], [2.6, 2.4, 0.02]])
        Q = oracle.projector_matrix_sparse(n, h, k, pos, channels).toarray()
        B = brute.projector_matrix(n, h, k, pos, channels)
        assert np.abs(Q - B).max() < 1e-12 * np.abs(B).max()


def test_sparse_operators_match_dense():
    s = synth.make_system(n=(12, 10, 14), h=0.22, nb=3, natoms=3, rc=1.5, seed=9,
                          k=(0.25, 0.1, 0.5))
    d = oracle.Operators.from_system(s)
    sp = oracle.Operators.from_system(s, sparse=True)
    psi = s.psi.reshape(s.nb, -1)
    for f in ("project", "apply_H", "apply_S"):
        a, b = getattr(d, f)(psi), getattr(sp, f)(psi)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), f


def _system(k=(0.0, 0.0, 0.0), seed=7):
    return synth.make_system(n=(12, 10, 14), h=0.22, nb=4, natoms=3, rc=1.5, seed=seed, k=k)


def test_translation_by_grid_step_leaves_projections():
    s = _system()
    for c in range(3):
        ops = oracle.Operators.from_system(s)
        P0 = ops.project(s.psi.reshape(s.nb, -1))
        pos = s.pos.copy()
        pos[:, c] += s.h[c]
        Q1 = oracle.projector_matrix(s.n, s.h, s.k, pos, s.channels)
        psi1 = np.roll(s.psi, 1, axis=1 + c).reshape(s.nb, -1)
        P1 = oracle.project(Q1, psi1, ops.dV)
        assert np.abs(P1 - P0).max() < 1e-12 * np.abs(P0).max()


def test_lattice_translation_phase():
    k = (0.25, 0.1, 0.5)
    s = _system(k=k)
    ops = oracle.Operators.from_system(s)
    P0 = ops.project(s.psi.reshape(s.nb, -1))
    for c in range(3):
        pos = s.pos.copy()
        pos[:, c] += s.n[c] * s.h[c]
        Q1 = oracle.projector_matrix(s.n, s.h, s.k, pos, s.channels)
        P1 = oracle.project(Q1, s.psi.reshape(s.nb, -1), ops.dV)
        assert np.abs(P1 - np.exp(2j * np.pi * k[c]) * P0).max() < 1e-12 * np.abs(P0).max()


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.3, 0.7, 0.1)])
def test_addback_is_adjoint_of_projection(k):
    s = _system(k=k)
    ops = oracle.Operators.from_system(s)
    rng = np.random.default_rng(2)
    phi = s.psi.reshape(s.nb, -1)
    Np = ops.Q.shape[0]
    X = rng.standard_normal((s.nb, Np)) + 1j * rng.standard_normal((s.nb, Np))
    eye = np.broadcast_to(np.eye(s.ni), (s.natoms, s.ni, s.ni))
    lhs = ops.dV * np.sum(phi.conj() * oracle.addback(ops.Q, X, eye), axis=1)
    rhs = np.sum(X * ops.project(phi).conj(), axis=1)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=0)


def test_ncpp_limit_overlap_is_identity():
    """Delta S = 0 (norm-conserving limit, Sec. PAW data sets) gives S~ = 1."""
    s = _system(k=(0.2, 0.0, 0.0))
    ops = oracle.Operators.from_system(s)
    ops.dS = np.zeros_like(s.dS)
    psi = s.psi.reshape(s.nb, -1)
    assert np.array_equal(ops.apply_S(psi), psi)
