"""Block Davidson step on the GPU against the oracle (a reading of SCF step
(2): the paper names the iterative Davidson eigensolver but gives no
formulas; see oracle/davidson.py).

For each case the oracle's subspace step supplies Ritz vectors; the device
step is compared stage by stage with the oracle on the same input:
corrections, their projections, H~ and S~ of the corrections, the 2nb x 2nb
subspace matrices, the eigenvalues (against LAPACK on the oracle's
matrices) and the new block (the oracle rotating by the device's C). Three
steps are chained on the device, each checked against one oracle step from
the device's previous output, with non-increasing Ritz values. Tolerance:
the FP64 path's 1e-12 relative.
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

CASES = {
    "real": dict(n=(24, 22, 20), h=0.2, nb=16, natoms=4, rc=2.0, seed=71, bands="smooth"),
    "bloch": dict(n=(18, 20, 16), h=0.2, nb=12, natoms=3, rc=1.8, seed=72, k=(0.25, 0.0, 0.5),
                  bands="smooth"),
    "noatoms_ragged": dict(n=(13, 17, 11), h=(0.21, 0.19, 0.23), nb=9, natoms=0, rc=1.4,
                           seed=73),
    "large_real": dict(n=(20, 18, 22), h=0.2, nb=80, natoms=3, rc=1.6, seed=74, bands="smooth"),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


@pytest.mark.parametrize("name", list(CASES))
def test_davidson_steps_against_oracle(name):
    s = synth.make_system(**CASES[name])
    say(f"[davidson] {name} n={s.n} nb={s.nb} natoms={s.natoms} k={s.k}")
    ops = oracle.Operators.from_system(s)
    r = oracle.fd_step(s, ops)
    psi, eps = r["psi_rot"], r["eps"]
    nb, ng, npj = s.nb, s.ng, ops.Q.shape[0]
    g = gfd.System.from_synth(s, max_bands=2 * nb)
    dt = g.dtype
    for step in range(3):
        P = ops.project(psi)
        Hpsi, Spsi = ops.apply_H(psi, P), ops.apply_S(psi, P)
        x = torch.zeros((2 * nb, ng), dtype=dt, device="cuda")
        Hx, Sx = torch.zeros_like(x), torch.zeros_like(x)
        x[:nb] = to_dev(psi)
        Hx[:nb] = to_dev(Hpsi)
        Sx[:nb] = to_dev(Spsi)
        Px = torch.zeros((2 * nb, npj), dtype=dt, device="cuda")
        if npj:
            Px[:nb] = to_dev(P)
        out = g.davidson_step(x, Hx, Sx, Px, to_dev(eps))
        torch.cuda.synchronize()
        # the oracle on the same input
        R = Hpsi - eps[:, None] * Spsi
        d = oracle.precondition(R, eps, s.v.ravel(), s.h)
        xe = np.concatenate([psi, d])
        He = np.concatenate([Hpsi, ops.apply_H(d)])
        Se = np.concatenate([Spsi, ops.apply_S(d)])
        H2, S2 = oracle.subspace_matrices(xe, He, Se, ops.dV)
        want = scipy.linalg.eigh(0.5 * (H2 + H2.conj().T), 0.5 * (S2 + S2.conj().T),
                                 eigvals_only=True)
        C2 = host(out["C2"])
        errs = {"d": rel(host(x[nb:]), d), "Hd": rel(host(Hx[nb:]), He[nb:]),
                "Sd": rel(host(Sx[nb:]), Se[nb:]),
                "H2": rel(host(out["H2"]), H2), "S2": rel(host(out["S2"]), S2),
                "eps2": np.abs(host(out["eps2"]) - want).max() / np.abs(want).max(),
                "psi": rel(host(out["psi"]), C2[:, :nb].T @ xe)}
        if npj:
            errs["Pd"] = rel(host(Px[nb:]), ops.project(d))
            errs["P"] = rel(host(out["P"]), C2[:, :nb].T @ np.concatenate([P, ops.project(d)]))
        e_new = host(out["eps"])
        say(f"  step {step}: " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()) +
            f"; max eps change {np.max(e_new - eps):.2e}")
        for k, v in errs.items():
            assert v <= TOL, (k, v)
        # no Ritz value rises
        assert np.all(e_new <= eps + 1e-12 * np.abs(eps).max())
        psi, eps = host(out["psi"]), e_new
    g.close()


def test_davidson_error_paths():
    s = synth.make_system(**CASES["real"])
    g = gfd.System.from_synth(s)  # max_bands = nb: no room for 2 nb
    nb = s.nb
    x = torch.zeros((2 * nb, s.ng), dtype=torch.float64, device="cuda")
    Px = torch.zeros((2 * nb, g.np), dtype=torch.float64, device="cuda")
    eps = torch.zeros(nb, dtype=torch.float64, device="cuda")
    with pytest.raises(gfd.GpawError) as e:
        g.davidson_step(x, x.clone(), x.clone(), Px, eps)
    assert e.value.status == "GPAW_ESHAPE"
    g.close()
    gs = gfd.System.from_synth(s, max_bands=2 * nb, precision="single")
    xs = x.float()
    with pytest.raises(gfd.GpawError) as e:
        gs.davidson_step(xs, xs.clone(), xs.clone(), Px.float(), eps)
    assert e.value.status == "GPAW_EDTYPE"
    gs.close()
