"""Degenerate and clustered spectra through the device eigensolver.

* Free electrons (v = 0, no atoms): every grid plane wave is an eigenvector of
  the FD kinetic operator, with the closed-form eigenvalue
  -1/2 sum_c symbol(q_c h_c) / h_c^2 (the 1-D stencil symbol, pinned in the
  oracle's tests). On a cubic grid whole shells of plane waves (the orbits of
  the cube's symmetry group) share one value, so the subspace problem of a
  block of plane waves, hidden by a random unitary mixing, has exactly
  degenerate eigenvalues. Real blocks use cos/sin pairs. The full step runs
  on the GPU, on both eigensolver paths (one-workgroup LDS path and the
  global-memory path above 128 real / 96 complex bands).
* Wilkinson's W21+ (tridiagonal, diagonal |10 - i|, off-diagonal 1), whose
  largest eigenvalues come in pairs closer than 1e-13 relative, and direct
  sums of copies of it (every eigenvalue repeated), rotated by a random
  orthogonal/unitary matrix, with S = I, against LAPACK (SciPy).
Tolerance: the FP64 path's 1e-12 (eigenvalues relative to max|eps|;
C^H S C = I and C^H H C = diag(eps) element-wise; spectral projectors of
each degenerate cluster norm-wise).
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import oracle
import synth
import paper_2310_14776_amd as gfd

from .gpu_util import say, to_dev, host, rel

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


def _free_electron_value(q, h):
    return -0.5 * sum(oracle.symbol_1d(q[c] * h[c]) / h[c] ** 2 for c in range(3))


def _plane_wave_block(n, h, k, nb, real, gmax=4):
    """nb lowest plane waves exp(i (G + k).r) (complex) or cos/sin pairs
    (real, k = 0), with their closed-form eigenvalues."""
    L = [n[c] * h[c] for c in range(3)]
    r = np.meshgrid(*[np.arange(n[c]) * h[c] for c in range(3)], indexing="ij")
    Gs = [np.array(g) - gmax for g in np.ndindex(2 * gmax + 1, 2 * gmax + 1, 2 * gmax + 1)]
    if real:
        # one of +-G (first non-zero component positive), G = 0 once
        Gs = [G for G in Gs if not np.any(G) or G[np.flatnonzero(G)[0]] > 0]
    qs = [[2 * np.pi * (k[c] + G[c]) / L[c] for c in range(3)] for G in Gs]
    vals = [_free_electron_value(q, h) for q in qs]
    order = np.argsort(vals, kind="stable")
    funcs, evs = [], []
    for i in order:
        q, e = qs[i], vals[i]
        phase = sum(q[c] * r[c] for c in range(3))
        if not real:
            funcs.append(np.exp(1j * phase))
            evs.append(e)
        elif not np.any(q):
            funcs.append(np.ones(n))
            evs.append(e)
        else:
            funcs += [np.cos(phase), np.sin(phase)]
            evs += [e, e]
        if len(funcs) >= nb:
            break
    return np.array(funcs[:nb]), np.array(evs[:nb])


def _random_unitary(m, cplx, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, m))
    if cplx:
        A = A + 1j * rng.standard_normal((m, m))
    Q, R = np.linalg.qr(A)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def _clusters(vals, tol):
    out, start = [], 0
    for i in range(1, len(vals) + 1):
        if i == len(vals) or vals[i] - vals[i - 1] > tol:
            if i - start > 1:
                out.append((start, i))
            start = i
    return out


FREE = {
    # name: (k, nb, real); cubic 12^3 grid, h = 0.2
    "real_nb100": ((0.0, 0.0, 0.0), 100, True),
    "real_nb200": ((0.0, 0.0, 0.0), 200, True),
    "complex_nb81": ((0.0, 0.0, 0.0), 81, False),
    "complex_nb123": ((0.0, 0.0, 0.0), 123, False),
    "bloch_nb90": ((0.25, 0.0, 0.5), 90, False),
    "bloch_nb140": ((0.25, 0.0, 0.5), 140, False),
}


@pytest.mark.parametrize("name", list(FREE))
def test_free_electron_shells(name):
    k, nb, real = FREE[name]
    n, h = (12, 12, 12), (0.2, 0.2, 0.2)
    funcs, vals = _plane_wave_block(n, h, k, nb, real)
    mix = _random_unitary(nb, not real, seed=nb)
    psi_h = mix @ funcs.reshape(nb, -1)   # hide the basis
    s = synth.make_system(n=n, h=h, nb=nb, natoms=0, rc=2.0, seed=0, k=k,
                          complex_psi=not real)
    s.v = np.zeros(n)
    s.psi = psi_h.reshape((nb,) + n)
    cl = _clusters(np.sort(vals), 1e-9 * np.abs(vals).max())
    say(f"[degenerate] {name}: nb={nb} k={k}, {len(cl)} degenerate shells, largest "
        f"{max(b - a for a, b in cl)}")
    ref = oracle.fd_step(s)
    g = gfd.System.from_synth(s)
    out = g.step(to_dev(psi_h))
    torch.cuda.synchronize()
    eps = host(out["eps"])
    scale = np.abs(vals).max()
    err_closed = np.abs(eps - np.sort(vals)).max() / scale
    err_oracle = np.abs(eps - ref["eps"]).max() / scale
    C = host(out["C"])
    Hs = 0.5 * (ref["H"] + ref["H"].conj().T)
    Ss = 0.5 * (ref["S"] + ref["S"].conj().T)
    Ch = C.conj().T
    orth = np.abs(Ch @ Ss @ C - np.eye(nb)).max()
    diag = np.abs(Ch @ Hs @ C - np.diag(ref["eps"])).max() / scale
    # spectral projectors of every degenerate shell (the basis inside a
    # shell is arbitrary; the projector C_cl C_cl^H is not). A perturbation
    # of the matrices of relative size TOL turns the projector of a shell by
    # at most TOL max|eps| / gap (Davis-Kahan), gap = distance to the nearest
    # other eigenvalue of the block; the ratio to that bound is asserted.
    Co = ref["C"]
    sv = np.sort(vals)
    proj = 0.0
    for a, b in cl:
        gap = sv[a] - sv[a - 1] if a > 0 else np.inf
        gap = min(gap, sv[b] - sv[b - 1] if b < nb else np.inf)
        e = rel(C[:, a:b] @ C[:, a:b].conj().T, Co[:, a:b] @ Co[:, a:b].conj().T)
        proj = max(proj, e * gap / scale)
    Coh = Co.conj().T
    diag_lapack = np.abs(Coh @ Hs @ Co - np.diag(ref["eps"])).max() / scale
    D = np.abs(Ch @ Hs @ C - np.diag(ref["eps"]))
    i, j = np.unravel_index(np.argmax(D), D.shape)
    same = any(a <= i < b and a <= j < b for a, b in cl)
    say(f"  eps vs closed form {err_closed:.1e}, vs oracle {err_oracle:.1e}, "
        f"C^H S C - I {orth:.1e}, C^H H C - diag {diag:.1e} (LAPACK's C: {diag_lapack:.1e}; "
        f"largest at ({i},{j}), {'inside' if same else 'outside'} a shell), "
        f"shell projectors x gap/max|eps| {proj:.1e}")
    assert err_closed <= TOL and err_oracle <= TOL
    assert orth <= TOL and diag <= TOL
    assert proj <= TOL
    assert rel(host(out["psi_rot"]), oracle.rotate(psi_h, C)) <= TOL
    g.close()


def _wilkinson(m=21):
    half = (m - 1) // 2
    return np.diag(np.abs(np.arange(m) - half).astype(float)) + np.eye(m, k=1) + np.eye(m, k=-1)


@pytest.mark.parametrize("copies,cplx", [(1, False), (1, True), (4, False), (4, True),
                                         (7, False), (5, True)])
def test_wilkinson_clusters_against_lapack(copies, cplx):
    W = scipy.linalg.block_diag(*([_wilkinson()] * copies))
    n = W.shape[0]
    Q = _random_unitary(n, cplx, seed=100 + n)
    H = Q @ W @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    S = np.eye(n, dtype=H.dtype)
    say(f"[wilkinson] {copies} x W21+ (n={n}) complex={cplx}")
    g = gfd.System(n=(4, 4, 4), h=0.2, k=(0.25, 0.0, 0.0) if cplx else (0, 0, 0),
                   pos=np.zeros((0, 3)), channels=[], dH=np.zeros(0), dS=np.zeros(0),
                   v=np.zeros(64), max_bands=n, complex_=cplx)
    eps, C = g.subspace_diag(to_dev(H), to_dev(S))
    torch.cuda.synchronize()
    want = scipy.linalg.eigh(H, eigvals_only=True)
    scale = np.abs(want).max()
    Cd = host(C)
    d_eps = np.abs(host(eps) - want).max() / scale
    orth = np.abs(Cd.conj().T @ Cd - np.eye(n)).max()
    diag = np.abs(Cd.conj().T @ H @ Cd - np.diag(want)).max() / scale
    say(f"  eps {d_eps:.1e}, C^H C - I {orth:.1e}, C^H H C - diag {diag:.1e}")
    assert d_eps <= TOL and orth <= TOL and diag <= TOL
    g.close()
