"""Seeded synthetic systems shaped like the paper's FD-mode workloads.

Recipe (one system):
  * orthorhombic periodic cell of n = (N0, N1, N2) points, spacing h (bohr),
    grid points at r = (i h0, j h1, k h2);
  * Bloch vector k in reduced units (k = 0 gives a real problem);
  * atom sites: fractional U[0,1)^3 times the cell lengths;
  * one Gaussian well per atom for the local potential,
    v(r) = depth * sum_a sum_R exp(-|r - R_a - R|^2 / (2 width^2)),
    periodic images truncated at 8 widths;
  * per atom 13 projectors: channels (l, sigma) = (0, rc/3), (0, rc/5),
    (1, rc/3), (1, rc/5), (2, rc/3), each a Gaussian times r^l with a smooth
    cut-off at rc (the functions themselves are evaluated by the consumers);
  * Delta H^a = (A + A^T)/2 and Delta S^a = s (B + B^T)/2 with A, B drawn
    U[-1,1]^{13x13} per atom (s = 0.1);
  * the block of wave functions: U[-1,1) per grid value (real), or
    independent U[-1,1) real and imaginary parts (complex).

Draw order from numpy.random.default_rng(seed): positions, Delta H,
Delta S. Band b of the block comes from its own stream,
numpy.random.default_rng([seed, 1, b]) for noise bands and
default_rng([seed, 2, b]) for smooth bands, so any band can be regenerated
alone (the oracle checks sampled bands of blocks too large to hold twice)
and a large block can be generated in parallel and streamed to a device.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import concurrent.futures
import math
import os

import numpy as np


def standard_channels(rc: float):
    """The 13-projector channel set: (l, sigma, rc) triples, channel-major."""
    return [(0, rc / 3.0, rc), (0, rc / 5.0, rc), (1, rc / 3.0, rc),
            (1, rc / 5.0, rc), (2, rc / 3.0, rc)]


@dataclass
class System:
    n: tuple            # grid points per axis (N0, N1, N2); axis 2 is contiguous
    h: tuple            # grid spacing per axis (bohr)
    k: tuple            # Bloch vector, reduced units
    pos: np.ndarray     # [natoms][3] cartesian bohr
    channels: list      # [(l, sigma, rc)]
    dH: np.ndarray      # [natoms][ni][ni] real symmetric
    dS: np.ndarray      # [natoms][ni][ni] real symmetric
    v: np.ndarray       # [N0][N1][N2] float64
    psi: np.ndarray     # [nb][N0][N1][N2] float64 or complex128, or None (lazy)
    name: str = ""
    meta: dict = field(default_factory=dict)
    nbands: int = 0     # band count of a lazy block (psi None)
    complex_psi: bool = False

    @property
    def natoms(self):
        return self.pos.shape[0]

    @property
    def nb(self):
        return self.psi.shape[0] if self.psi is not None else self.nbands

    def bands(self, lo, hi, threads=None):
        """Bands lo..hi-1 of the block as [hi-lo][N0][N1][N2] (generated from
        their own streams when the block is lazy)."""
        if self.psi is not None:
            return self.psi[lo:hi]
        return _gen_bands(self, range(lo, hi), threads)

    def band_list(self, idx, threads=None):
        """The bands with the given indices, [len(idx)][N0][N1][N2]."""
        if self.psi is not None:
            return self.psi[list(idx)]
        return _gen_bands(self, list(idx), threads)

    @property
    def ni(self):
        return sum(2 * l + 1 for (l, _, _) in self.channels)

    @property
    def ng(self):
        return int(np.prod(self.n))

    @property
    def cell(self):
        return tuple(self.n[c] * self.h[c] for c in range(3))

    @property
    def is_complex(self):
        return np.iscomplexobj(self.psi) if self.psi is not None else self.complex_psi


def gaussian_potential(n, h, pos, depth=-2.0, width=1.0):
    """Sum of periodic Gaussian wells, one per atom (an input field)."""
    L = [n[c] * h[c] for c in range(3)]
    axes = [np.arange(n[c]) * h[c] for c in range(3)]
    v = np.zeros(n)
    reach = 8.0 * width
    for a in range(pos.shape[0]):
        parts = []
        for c in range(3):
            m = int(math.ceil(reach / L[c])) + 1
            d = axes[c][:, None] - pos[a, c] - L[c] * np.arange(-m, m + 1)[None, :]
            g = np.exp(-d * d / (2.0 * width * width))
            g[np.abs(d) > reach] = 0.0
            parts.append(g.sum(axis=1))
        # the Gaussian factorises over axes, and so does its image sum
        v += parts[0][:, None, None] * parts[1][None, :, None] * parts[2][None, None, :]
    return depth * v


def noise_band(seed, b, n, complex_psi):
    """Band b of a noise block: U[-1, 1) per grid value, complex values with
    independent real and imaginary parts, from default_rng([seed, 1, b])."""
    ng = int(np.prod(n))
    rng = np.random.default_rng([seed, 1, b])
    out = np.empty(2 * ng if complex_psi else ng)
    rng.random(out=out)
    out *= 2.0
    out -= 1.0
    return (out.view(np.complex128) if complex_psi else out).reshape(n)


def smooth_band(seed, b, n, h, k, complex_psi, g0=2.0):
    """Band b of a band-limited block: plane-wave coefficients drawn from a
    standard normal (default_rng([seed, 2, b])), damped by
    exp(-|G + k|^2 / (2 g0^2)) (g0 in 1/bohr), then the Bloch factor
    exp(i k.r) applied so that psi(r + L_c e_c) equals exp(2 pi i k_c) psi(r).
    Real blocks (k = 0) take the real part. The band is scaled to an RMS of
    1/sqrt(3) per component, that of U[-1, 1]. The Rayleigh quotients of such
    bands lie in the 1-10 Ha range."""
    L = [n[c] * h[c] for c in range(3)]
    G = [2.0 * np.pi * np.fft.fftfreq(n[c], d=h[c]) + 2.0 * np.pi * k[c] / L[c] for c in range(3)]
    G2 = G[0][:, None, None] ** 2 + G[1][None, :, None] ** 2 + G[2][None, None, :] ** 2
    env = np.exp(-G2 / (2.0 * g0 * g0))
    rng = np.random.default_rng([seed, 2, b])
    c = rng.standard_normal(tuple(n)) + 1j * rng.standard_normal(tuple(n))
    psi = np.fft.ifftn(c * env)
    if complex_psi:
        x = [np.arange(n[c]) * h[c] for c in range(3)]
        kr = (2.0 * np.pi * k[0] / L[0]) * x[0][:, None, None] \
            + (2.0 * np.pi * k[1] / L[1]) * x[1][None, :, None] \
            + (2.0 * np.pi * k[2] / L[2]) * x[2][None, None, :]
        psi = psi * np.exp(1j * kr)
        rms = np.sqrt(np.mean(np.abs(psi) ** 2) / 2.0)
    else:
        psi = psi.real
        rms = np.sqrt(np.mean(psi ** 2))
    return psi * (1.0 / (np.sqrt(3.0) * rms))


def _one_band(s, b):
    seed = s.meta["seed"]
    if s.meta.get("bands", "noise") == "smooth":
        return smooth_band(seed, b, s.n, s.h, s.k, s.is_complex)
    return noise_band(seed, b, s.n, s.is_complex)


def _gen_bands(s, idx, threads=None):
    idx = list(idx)
    out = np.empty((len(idx),) + tuple(s.n), dtype=np.complex128 if s.is_complex else np.float64)
    if not idx:
        return out
    threads = threads or min(16, len(os.sched_getaffinity(0)))

    def fill(i):
        out[i] = _one_band(s, idx[i])
    with concurrent.futures.ThreadPoolExecutor(max(1, min(threads, len(idx)))) as ex:
        list(ex.map(fill, range(len(idx))))
    return out


def make_system(n, h, nb, natoms, rc, seed, k=(0.0, 0.0, 0.0), complex_psi=None,
                ds_scale=0.1, depth=-2.0, width=1.0, name="", bands="noise", lazy=False):
    """One seeded system. lazy: do not hold the block (psi is None); its
    bands are generated on request by System.bands / System.band_list."""
    n = tuple(int(x) for x in n)
    h = (float(h),) * 3 if np.isscalar(h) else tuple(float(x) for x in h)
    k = tuple(float(x) for x in k)
    if complex_psi is None:
        complex_psi = any(x != 0.0 for x in k)
    rng = np.random.default_rng(seed)
    L = np.array([n[c] * h[c] for c in range(3)])
    pos = rng.random((natoms, 3)) * L[None, :]
    channels = standard_channels(rc)
    ni = sum(2 * l + 1 for (l, _, _) in channels)
    A = rng.uniform(-1.0, 1.0, (natoms, ni, ni))
    dH = 0.5 * (A + A.transpose(0, 2, 1))
    B = rng.uniform(-1.0, 1.0, (natoms, ni, ni))
    dS = ds_scale * 0.5 * (B + B.transpose(0, 2, 1))
    if bands not in ("noise", "smooth"):
        raise ValueError("bands must be 'noise' or 'smooth'")
    v = gaussian_potential(n, h, pos, depth, width)
    s = System(n=n, h=h, k=k, pos=pos, channels=channels, dH=dH, dS=dS, v=v,
               psi=None, name=name, nbands=int(nb), complex_psi=bool(complex_psi),
               meta=dict(seed=seed, rc=rc, ds_scale=ds_scale, depth=depth, width=width,
                         bands=bands))
    if not lazy:
        s.psi = s.bands(0, nb)
    return s


# The five workloads: small real case, the single-GPU FP64 case, the precision
# form, the complex Bloch case and the batched form (grid spacing 0.2 bohr and
# rc = 2.0 bohr where the workload does not state them).
CONFIGS = {
    "A": dict(n=(24, 24, 24), h=0.2, nb=16, natoms=4, rc=2.0, seed=0),
    "B": dict(n=(48, 48, 48), h=0.18, nb=128, natoms=16, rc=2.2, seed=1),
    "C": dict(n=(96, 96, 96), h=0.2, nb=512, natoms=64, rc=2.0, seed=2),
    "D": dict(n=(120, 120, 160), h=0.2, nb=1024, natoms=128, rc=2.0, seed=3,
              k=(0.25, 0.0, 0.5)),
}


def config_system(name, nb=None, lazy=False):
    """The named workload; nb overrides the band count (for bounded samples);
    lazy leaves the block to be generated band by band."""
    cfg = dict(CONFIGS[name])
    if nb is not None:
        cfg["nb"] = nb
    return make_system(name=name, lazy=lazy, **cfg)


def batched_systems(count=64, seed=4):
    """Uneven independent systems: grids 16..48 per axis, 8..96 bands,
    2..16 atoms, half of them complex with k ~ U[0, 0.5)^3."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = tuple(int(x) for x in rng.integers(16, 49, 3))
        nb = int(rng.integers(8, 97))
        natoms = int(rng.integers(2, 17))
        cplx = bool(s % 2)
        k = tuple(rng.uniform(0.0, 0.5, 3)) if cplx else (0.0, 0.0, 0.0)
        sub_seed = int(rng.integers(0, 2**31 - 1))
        out.append(dict(n=n, h=0.2, nb=nb, natoms=natoms, rc=2.0, seed=sub_seed,
                        k=k, complex_psi=cplx))
    return out


def ragged_cases():
    """Small shapes that exercise tile tails, odd sizes, self-overlapping
    spheres, no atoms and a single band."""
    return [
        dict(n=(13, 17, 11), h=(0.21, 0.19, 0.23), nb=5, natoms=3, rc=1.6, seed=11),
        dict(n=(16, 16, 16), h=0.2, nb=1, natoms=2, rc=2.0, seed=12),
        dict(n=(10, 9, 12), h=0.2, nb=7, natoms=0, rc=2.0, seed=13),
        dict(n=(20, 18, 66), h=0.2, nb=33, natoms=5, rc=2.0, seed=14),
    ]
