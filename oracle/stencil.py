"""Kinetic operator -1/2 nabla^2 on a uniform periodic/Bloch grid (oracle).

Paper: the FD mode represents the kinetic energy operator on a uniform
Cartesian grid (Sec. "Wave-function representations"); applying an FD
stencil is one of the C hot spots (Sec. "Developer's perspective").

Readings (the paper states neither order nor coefficients nor boundary):
  * per axis the 6th-order central second difference with weights
    (1/90, -3/20, 3/2, -49/18, 3/2, -3/20, 1/90)/h^2 (19-point star in 3-D);
  * Bloch boundary psi(r + L_c e_c) = exp(2 pi i k_c) psi(r), k reduced;
    a neighbour fetched past the upper face carries exp(+2 pi i k_c), past
    the lower face exp(-2 pi i k_c).
"""
import numpy as np

# w_0, w_1, w_2, w_3 of d^2/dx^2 * h^2 (6th order, symmetric)
WEIGHTS = (-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0)


def symbol_1d(theta):
    """h^2 times the eigenvalue of the 1-D difference operator on exp(i theta j)."""
    theta = np.asarray(theta, dtype=float)
    return WEIGHTS[0] + 2.0 * sum(WEIGHTS[d] * np.cos(d * theta) for d in (1, 2, 3))


def _shifted(f, axis, d, phase):
    """g(r) = f(r + d h e_axis) for a Bloch field stored on one cell."""
    n = f.shape[axis]
    g = np.roll(f, -d, axis=axis)           # g[i] = f[(i + d) mod n]
    if phase != 1.0:
        wraps = (np.arange(n) + d) // n      # number of faces crossed (signed)
        ph = np.asarray(phase, dtype=complex) ** wraps
        shape = [1] * f.ndim
        shape[axis] = n
        g = g * ph.reshape(shape)
    return g


def laplacian(f, h, k=(0.0, 0.0, 0.0)):
    """nabla^2 f on the last three axes of f (leading axes are bands)."""
    f = np.asarray(f)
    cplx = np.iscomplexobj(f) or any(kc != 0.0 for kc in k)
    f = f.astype(complex if cplx else float)
    out = np.zeros_like(f)
    for c in range(3):
        axis = f.ndim - 3 + c
        phase = np.exp(2j * np.pi * k[c]) if k[c] != 0.0 else 1.0
        acc = WEIGHTS[0] * f
        for d in (1, 2, 3):
            acc = acc + WEIGHTS[d] * (_shifted(f, axis, d, phase) + _shifted(f, axis, -d, phase))
        out += acc / (h[c] * h[c])
    return out


def kinetic(f, h, k=(0.0, 0.0, 0.0)):
    return -0.5 * laplacian(f, h, k)
