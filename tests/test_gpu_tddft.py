"""Finite (zero-boundary) systems and real-time propagation on the GPU, through
the C ABI, against the oracle (Sec. "Real-time TDDFT", Eq. (td_ks); zero
boundaries of finite systems, Sec. "Solving the Kohn-Sham equation").

* P, H~psi and S~psi of zero-boundary systems (atoms whose spheres are cut
  by the faces, ragged grids, no atoms; FP64, complex128 with k = 0 and the
  FP32 precision form) element by element against the oracle's finite
  operators, and the whole eigensolver step on such a system;
* the delta kick, one to three Crank-Nicolson steps and the dipole against
  the oracle's dense Crank-Nicolson solve (complex128, 1e-11);
* at sizes the dense solve cannot reach: S~-norm conservation of every band
  and the residual of the Crank-Nicolson equation, both evaluated with the
  oracle's (sparse) operators on the GPU's result; a 95 x 95 x 127 box with
  32 atoms among them;
* error paths.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import tddft as T
import paper_2310_14776_amd as gfd

from .gpu_util import say, to_dev, host, rel

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


def _finite(**kw):
    s = synth.make_system(**kw)
    s.meta["boundary"] = "zero"
    return s


CASES = {
    "ragged_f64": dict(n=(13, 17, 11), h=(0.21, 0.19, 0.23), nb=5, natoms=3, rc=1.6, seed=21),
    "faces_c128": dict(n=(20, 18, 24), h=0.2, nb=6, natoms=5, rc=2.0, seed=22,
                       complex_psi=True),
    "no_atoms_f64": dict(n=(9, 10, 8), h=0.2, nb=3, natoms=0, rc=2.0, seed=23),
    "wide_c128": dict(n=(33, 30, 70), h=0.2, nb=4, natoms=6, rc=2.0, seed=24, complex_psi=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_zero_boundary_operators(name):
    s = _finite(**CASES[name])
    ops = T.FiniteOps.from_system(s)
    psi = s.psi.reshape(s.nb, -1)
    g = gfd.System.from_synth(s)
    assert g.boundary == "zero"
    out = g.step(to_dev(psi))
    torch.cuda.synchronize()
    Pref = ops.project(psi)
    Href = ops.apply_H(psi, Pref)
    Sref = ops.apply_S(psi, Pref)
    if s.natoms:
        assert rel(host(out["P"]), Pref) <= TOL
    for key, ref in (("Hpsi", Href), ("Spsi", Sref)):
        got = host(out[key])
        assert np.abs(got - ref).max() <= TOL * np.abs(ref).max(), key
    H, S = oracle.subspace_matrices(psi, Href, Sref, ops.dV)
    eps, _ = oracle.diagonalize(H, S)
    assert rel(host(out["H"]), H) <= TOL and rel(host(out["S"]), S) <= TOL
    assert np.abs(host(out["eps"]) - eps).max() <= TOL * np.abs(eps).max()
    g.close()


def test_zero_boundary_precision_form():
    s = _finite(**CASES["ragged_f64"])
    s.psi = s.psi.astype(np.float32).astype(np.float64)
    ops = T.FiniteOps.from_system(s)
    psi = s.psi.reshape(s.nb, -1)
    g = gfd.System.from_synth(s, precision="single")
    Hp, Sp = g.apply_HS(to_dev(psi.astype(np.float32)), None)
    torch.cuda.synchronize()
    assert rel(host(Hp), ops.apply_H(psi)) <= 1e-6
    assert rel(host(Sp), ops.apply_S(psi)) <= 1e-6
    g.close()


def test_kick_propagate_dipole_against_dense_oracle():
    s = _finite(n=(8, 9, 7), h=0.4, nb=3, natoms=2, rc=1.2, seed=31, complex_psi=True)
    ops = T.FiniteOps.from_system(s)
    H, S = ops.dense()
    psi = s.psi.reshape(s.nb, -1)
    f = np.array([2.0, 1.0, 0.5])
    kappa = (0.2, -0.1, 0.3)
    g = gfd.System.from_synth(s)
    x = to_dev(psi)
    g.td_kick(x, kappa)
    ref = T.kick(psi, s.n, s.h, kappa)
    assert np.abs(host(x) - ref).max() <= TOL * np.abs(ref).max()
    d = host(g.td_dipole(x, torch.tensor(f)))
    assert np.abs(d - T.dipole(ref, f, s.n, s.h)).max() <= TOL * np.abs(d).max()
    dt = 0.05
    for step in range(3):
        it, res = g.td_propagate(x, dt, tol=1e-13, max_iter=400)
        ref = T.cn_step(ops, ref, dt, H, S)
        err = np.abs(host(x) - ref).max() / np.abs(ref).max()
        say(f"[tddft] step {step}: COCG iterations {it}, residual {res:.1e}, error {err:.1e}")
        assert err <= 1e-11
    d = host(g.td_dipole(x, torch.tensor(f)))
    assert np.abs(d - T.dipole(ref, f, s.n, s.h)).max() <= 1e-11 * np.abs(d).max()
    g.close()


def _cn_checks(s, nb_check, steps, dt, sparse):
    ops = T.FiniteOps.from_system(s, sparse=sparse)
    g = gfd.System.from_synth(s)
    psi0 = s.psi.reshape(s.nb, -1)
    x = to_dev(psi0)
    prev = psi0
    for step in range(steps):
        it, res = g.td_propagate(x, dt, tol=1e-12, max_iter=500)
        cur = host(x)
        say(f"[tddft] n={s.n} nb={s.nb} step {step}: COCG iterations {it}, residual {res:.1e}")
        assert res <= 1e-12
        b = prev[:nb_check]
        xc = cur[:nb_check]
        Sb, Hb = ops.apply_S(b), ops.apply_H(b)
        Sx, Hx = ops.apply_S(xc), ops.apply_H(xc)
        tau = 0.5 * dt
        lhs = Sx + 1j * tau * Hx
        rhs = Sb - 1j * tau * Hb
        r = np.linalg.norm(lhs - rhs, axis=1) / np.linalg.norm(rhs, axis=1)
        n0 = np.einsum("ng,ng->n", b.conj(), Sb).real
        n1 = np.einsum("ng,ng->n", xc.conj(), Sx).real
        say(f"  CN equation residual {r.max():.1e}, S-norm change {np.abs(n1 - n0).max() / n0.max():.1e}")
        assert r.max() <= 1e-11
        assert np.abs(n1 - n0).max() <= 1e-11 * n0.max()
        prev = cur
    g.close()


def test_cn_conservation_24cubed():
    s = _finite(n=(24, 24, 24), h=0.2, nb=8, natoms=4, rc=2.0, seed=41, complex_psi=True,
                bands="smooth")
    _cn_checks(s, nb_check=8, steps=3, dt=0.1, sparse=False)


@pytest.mark.timeout(900)
def test_cn_large_box():
    s = _finite(n=(95, 95, 127), h=0.2, nb=8, natoms=32, rc=2.0, seed=42, complex_psi=True,
                bands="smooth")
    _cn_checks(s, nb_check=3, steps=1, dt=0.05, sparse=True)


def test_td_error_paths():
    s = _finite(n=(8, 8, 8), h=0.3, nb=2, natoms=1, rc=1.0, seed=51)
    g = gfd.System.from_synth(s)  # real FP64: no propagation
    x = to_dev(s.psi.reshape(2, -1))
    with pytest.raises(gfd.GpawError) as e:
        g.td_propagate(x, 0.1)
    assert e.value.status == "GPAW_EDTYPE"
    g.close()
    sb = synth.make_system(n=(8, 8, 8), h=0.3, nb=2, natoms=1, rc=1.0, seed=52, k=(0.25, 0, 0))
    gb = gfd.System.from_synth(sb)
    xb = to_dev(sb.psi.reshape(2, -1))
    with pytest.raises(gfd.GpawError) as e:
        gb.td_propagate(xb, 0.1)
    assert e.value.status == "GPAW_EINVAL"
    gb.close()
    with pytest.raises(gfd.GpawError) as e:
        gfd.System.from_synth(sb, boundary="zero")
    assert e.value.status == "GPAW_EINVAL"
    sc = _finite(n=(8, 8, 8), h=0.3, nb=2, natoms=1, rc=1.0, seed=53, complex_psi=True)
    gc = gfd.System.from_synth(sc)
    xc = to_dev(sc.psi.reshape(2, -1))
    with pytest.raises(gfd.GpawError) as e:
        gc.td_propagate(xc, 0.1, tol=1e-30, max_iter=2)
    assert e.value.status == "GPAW_ENOCONV"
    gc.close()
