"""Pins of the oracle's kinetic operator against closed forms and brute force.

The paper fixes no stencil (FD representation, Sec. "Wave-function
representations"); the reading is the 6th-order central second difference
with a Bloch boundary. These tests pin the weights by their moment
conditions, the assembled operator by its plane-wave symbol and by h^6
convergence on a smooth function, and the roll/phase code by a dense matrix
built element by element.
"""
import math

import numpy as np
import pytest

import oracle

from . import brute

pytestmark = pytest.mark.filterwarnings("ignore")


def test_weight_moments_sixth_order():
    w = oracle.WEIGHTS
    d = np.arange(-3, 4)
    wd = np.array([w[abs(i)] for i in d])
    # exact on 1, x^2, x^4, x^6 (odd moments vanish by symmetry): sum w d^2 = 2
    assert abs(wd.sum()) < 1e-14
    assert abs((wd * d**2).sum() - 2.0) < 1e-14
    assert abs((wd * d**4).sum()) < 1e-13
    assert abs((wd * d**6).sum()) < 1e-12
    # first surviving error moment: sum w d^8 / 8! gives the theta^8/560 term
    assert abs((wd * d**8).sum() / math.factorial(8) - 1.0 / 560.0) < 1e-15


def test_symbol_taylor():
    for th in (0.05, 0.1, 0.2):
        lam = oracle.symbol_1d(th)
        assert abs((lam + th**2) / th**8 - 1.0 / 560.0) < 5e-3 * (1.0 / 560.0) + 1e-3 * th**2


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5), (0.1, 0.37, 0.8)])
def test_plane_wave_symbol(k):
    n = (10, 12, 9)
    h = (0.2, 0.25, 0.3)
    L = [n[c] * h[c] for c in range(3)]
    r = np.meshgrid(*[np.arange(n[c]) * h[c] for c in range(3)], indexing="ij")
    rng = np.random.default_rng(5)
    for _ in range(4):
        G = rng.integers(-4, 5, 3)
        q = [2 * np.pi * (k[c] + G[c]) / L[c] for c in range(3)]
        psi = np.exp(1j * sum(q[c] * r[c] for c in range(3)))
        expect = -0.5 * sum(oracle.symbol_1d(q[c] * h[c]) / h[c]**2 for c in range(3))
        got = oracle.kinetic(psi, h, k)
        assert np.allclose(got, expect * psi, rtol=0, atol=1e-11 * abs(expect) + 1e-12)


def test_real_path_matches_complex_path():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((2, 7, 6, 8))
    h = (0.3, 0.2, 0.25)
    a = oracle.kinetic(f, h)
    b = oracle.kinetic(f.astype(complex), h)
    assert a.dtype == np.float64
    assert np.abs(a - b.real).max() <= 1e-14 * np.abs(a).max() and not b.imag.any()


def test_sixth_order_convergence():
    """-1/2 lap of sin(2 pi x/L) cos(4 pi y/L) sin(2 pi z/L): error falls ~2^6."""
    errs = []
    for N in (12, 24):
        L = 3.0
        h = (L / N,) * 3
        x = np.arange(N) * h[0]
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        a = 2 * np.pi / L
        f = np.sin(a * X) * np.cos(2 * a * Y) * np.sin(a * Z)
        exact = 0.5 * (a * a + 4 * a * a + a * a) * f
        errs.append(np.abs(oracle.kinetic(f, h) - exact).max())
    assert 50.0 < errs[0] / errs[1] < 80.0


@pytest.mark.parametrize("n,k", [((5, 6, 7), (0.0, 0.0, 0.0)),
                                 ((5, 6, 7), (0.25, 0.0, 0.5)),
                                 ((2, 4, 3), (0.3, 0.6, 0.9))])
def test_dense_brute_force(n, k):
    h = (0.31, 0.22, 0.27)
    T = brute.dense_kinetic(n, h, k)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    got = oracle.kinetic(psi, h, k).reshape(3, -1)
    want = psi.reshape(3, -1) @ T.T
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
