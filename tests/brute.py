"""Element-by-element constructions used to pin the oracle (tests only).

These rebuild the kinetic matrix and the projector matrix with scalar loops
and SciPy's spherical harmonics, so that they share no vectorised code path
with the oracle they check.
"""
import itertools
import math

import numpy as np
import scipy.special

import oracle


def dense_1d(N, h, phase):
    D = np.zeros((N, N), dtype=complex)
    for i in range(N):
        for d in range(-3, 4):
            j = i + d
            wraps = math.floor(j / N)
            D[i, j - wraps * N] += oracle.WEIGHTS[abs(d)] * phase**wraps / h**2
    return D


def dense_kinetic(n, h, k):
    Ds = [dense_1d(n[c], h[c], np.exp(2j * np.pi * k[c])) for c in range(3)]
    I = [np.eye(n[c]) for c in range(3)]
    lap = (np.kron(np.kron(Ds[0], I[1]), I[2]) + np.kron(np.kron(I[0], Ds[1]), I[2])
           + np.kron(np.kron(I[0], I[1]), Ds[2]))
    return -0.5 * lap


def real_ylm_scipy(l, m, theta, phi):
    def Y(mm):
        if hasattr(scipy.special, "sph_harm_y"):
            return scipy.special.sph_harm_y(l, mm, theta, phi)
        return scipy.special.sph_harm(mm, l, phi, theta)
    if m == 0:
        return Y(0).real
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Y(m).real
    return math.sqrt(2) * (-1) ** m * Y(-m).imag


def projector_matrix(n, h, k, pos, channels):
    ni = sum(2 * l + 1 for (l, _, _) in channels)
    L = [n[c] * h[c] for c in range(3)]
    rmax = max(c[2] for c in channels)
    M = [int(math.ceil(rmax / L[c])) + 1 for c in range(3)]
    Q = np.zeros((len(pos) * ni, n[0] * n[1] * n[2]), dtype=complex)
    images = list(itertools.product(*[range(-M[c], M[c] + 1) for c in range(3)]))
    for a, R0 in enumerate(pos):
        for g, (i, j, kk) in enumerate(itertools.product(range(n[0]), range(n[1]), range(n[2]))):
            r = (i * h[0], j * h[1], kk * h[2])
            for m in images:
                d = [r[c] - R0[c] - m[c] * L[c] for c in range(3)]
                dist = math.sqrt(d[0]**2 + d[1]**2 + d[2]**2)
                if dist >= rmax:
                    continue
                arg = 2 * math.pi * sum(k[c] * m[c] for c in range(3))
                phase = complex(math.cos(arg), math.sin(arg))
                theta = math.acos(d[2] / dist) if dist > 0 else 0.0
                phi = math.atan2(d[1], d[0])
                row = 0
                for (l, sigma, rc) in channels:
                    s = dist / rc
                    chi = (1 - s * s) ** 2 if s < 1 else 0.0
                    rad = (oracle.radial_norm(l, sigma) * dist**l
                           * math.exp(-dist * dist / (2 * sigma * sigma)) * chi)
                    for mm in range(-l, l + 1):
                        Q[a * ni + row, g] += phase * rad * real_ylm_scipy(l, mm, theta, phi)
                        row += 1
    return Q
