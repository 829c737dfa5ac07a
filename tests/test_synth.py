"""Checks of the seeded input generators (no method arithmetic lives there).

The smooth-band blocks must satisfy the Bloch condition of the FD grid: a
block built as exp(i k.r) times a periodic band-limited function has a
kinetic energy equal to the spectral sum over its plane-wave content of the
stencil's symbol at G + k. A wrong sign or scale of k in the generator would
break the equality, as would any mismatch with the Bloch boundary the kinetic
operator uses.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore")


def _spectral_kinetic(psi, n, h, k):
    """<psi|T|psi> from the plane-wave content of exp(-i k.r) psi."""
    L = [n[c] * h[c] for c in range(3)]
    x = [np.arange(n[c]) * h[c] for c in range(3)]
    kr = sum((2 * np.pi * k[c] / L[c]) * x[c].reshape([-1 if d == c else 1 for d in range(3)])
             for c in range(3))
    u = psi * np.exp(-1j * kr)
    c = np.fft.fftn(u) / np.prod(n)
    lam = 0.0
    for ax in range(3):
        theta = (2 * np.pi * np.fft.fftfreq(n[ax]) + 2 * np.pi * k[ax] / n[ax])
        sym = -0.5 * oracle.symbol_1d(theta) / h[ax] ** 2
        lam = lam + sym.reshape([-1 if d == ax else 1 for d in range(3)])
    return np.sum(np.abs(c) ** 2 * lam) * np.prod(n)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5), (0.1, 0.37, 0.2)])
def test_smooth_bands_satisfy_bloch_condition(k):
    n, h = (12, 10, 14), (0.2, 0.22, 0.18)
    s = synth.make_system(n=n, h=h, nb=3, natoms=0, rc=2.0, seed=7, k=k, bands="smooth",
                          complex_psi=any(k))
    for psi in s.psi:
        direct = np.vdot(psi, oracle.kinetic(psi, s.h, s.k)).real
        spectral = _spectral_kinetic(psi, n, s.h, s.k)
        assert abs(direct - spectral) <= 1e-10 * abs(spectral)


def test_smooth_bands_scale_and_ritz_range():
    s = synth.make_system(n=(20, 20, 20), h=0.2, nb=8, natoms=2, rc=2.0, seed=3, bands="smooth")
    assert np.isrealobj(s.psi)
    for b in s.psi:
        assert abs(np.sqrt(np.mean(b ** 2)) - 1 / np.sqrt(3)) < 1e-12
    ref = oracle.fd_step(s)
    assert ref["eps"].max() < 10.0 and ref["eps"].min() > -10.0


@pytest.mark.parametrize("k,bands", [((0.0, 0.0, 0.0), "noise"), ((0.25, 0.0, 0.5), "noise"),
                                     ((0.25, 0.0, 0.5), "smooth")])
def test_bands_regenerate_alone_and_lazily(k, bands):
    """Every band comes from its own stream: the materialised block, a lazy
    block's band ranges and single bands regenerated out of order agree
    exactly, whatever the thread count."""
    cfg = dict(n=(9, 8, 10), h=0.2, nb=7, natoms=2, rc=1.0, seed=11, k=k, bands=bands)
    full = synth.make_system(**cfg)
    lazy = synth.make_system(lazy=True, **cfg)
    assert lazy.psi is None and lazy.nb == 7 and lazy.is_complex == full.is_complex
    assert np.array_equal(lazy.bands(0, 7, threads=1), full.psi)
    assert np.array_equal(lazy.bands(2, 5, threads=3), full.psi[2:5])
    assert np.array_equal(lazy.band_list([6, 0, 3]), full.psi[[6, 0, 3]])
    # positions, corrections and potential do not depend on how bands are made
    assert np.array_equal(lazy.pos, full.pos) and np.array_equal(lazy.dH, full.dH)
    assert np.array_equal(lazy.v, full.v)


def test_noise_bands_are_uniform_and_independent():
    s = synth.make_system(n=(16, 16, 16), h=0.2, nb=4, natoms=0, rc=1.0, seed=5,
                          k=(0.25, 0.0, 0.0))
    x = s.psi.reshape(4, -1)
    for part in (x.real, x.imag):
        assert part.min() >= -1.0 and part.max() < 1.0
        assert abs(part.mean()) < 0.02 and abs(part.var() - 1.0 / 3.0) < 0.01
    c = np.corrcoef(np.vstack([x.real, x.imag]))
    assert np.abs(c - np.eye(8)).max() < 0.07  # ~4.5 sigma for 4096 samples
