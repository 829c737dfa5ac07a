"""Pseudo density and atomic density matrices on the GPU against the oracle.

Paper: Eq. (atomicdensitymatrix) and the pseudo density of the PAW section.
Cases: real and Bloch blocks with atoms, a ragged grid, no atoms, one band,
the precision form (single-precision block, FP64 sums), and the 96^3
512-band workload sampled (whole density against the oracle's band sums,
computed chunk by chunk). Occupations are non-uniform. Tolerance: the FP64
path's 1e-12 relative (norm-wise for n~, per atom for D). The precision
form is compared against the oracle on the same rounded block: n~ to 1e-12
(its sums run in FP64 over the stored values), D to 2e-7, since the
precision form's projections P are stored in single precision (relative
rounding 6e-8 per element).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2310_14776_amd as gfd

from .gpu_util import say, to_dev, host, rel

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = {
    "real": dict(n=(24, 22, 20), h=0.2, nb=40, natoms=4, rc=2.0, seed=61),
    "bloch": dict(n=(18, 20, 16), h=0.2, nb=33, natoms=3, rc=1.8, seed=62, k=(0.25, 0.0, 0.5)),
    "ragged": dict(n=(13, 17, 11), h=(0.21, 0.19, 0.23), nb=9, natoms=2, rc=1.4, seed=63),
    "noatoms": dict(n=(16, 16, 16), h=0.2, nb=12, natoms=0, rc=2.0, seed=64),
    "one_band": dict(n=(16, 18, 20), h=0.2, nb=1, natoms=2, rc=1.8, seed=65),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


def _check(s, g, psi_host, f, precision):
    tol_D = TOL if precision == "double" else 2e-7
    ops = oracle.Operators.from_system(s)
    P = ops.project(psi_host)
    n_ref = oracle.pseudo_density(psi_host, f)
    D_ref = oracle.atomic_density_matrices(P, f, s.natoms, 13) if s.natoms else None
    psi = to_dev(psi_host).to(g.dtype)
    fd = to_dev(f)
    n_dev, D_dev = g.density(psi, fd)
    # with caller projections too
    Pd = g.project(psi)
    n2, D2 = g.density(psi, fd, P=Pd)
    torch.cuda.synchronize()
    en = rel(host(n_dev), n_ref)
    say(f"  n~ {en:.1e}" + (f", D {max(rel(host(D_dev)[a], D_ref[a]) for a in range(s.natoms)):.1e}"
                            if s.natoms else ""))
    assert en <= TOL and rel(host(n2), n_ref) <= TOL
    if s.natoms:
        for a in range(s.natoms):
            assert rel(host(D_dev)[a], D_ref[a]) <= tol_D
            assert rel(host(D2)[a], D_ref[a]) <= tol_D


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["double", "single"])
def test_density_against_oracle(name, precision):
    s = synth.make_system(**CASES[name])
    say(f"[density] {name} {precision} n={s.n} nb={s.nb} natoms={s.natoms}")
    psi = s.psi.reshape(s.nb, -1)
    if precision == "single":
        psi = psi.astype(np.complex64 if s.is_complex else np.float32).astype(psi.dtype)
    f = np.linspace(2.0, 0.1, s.nb)
    g = gfd.System.from_synth(s, precision=precision)
    _check(s, g, psi, f, precision)
    g.close()


def test_density_96cubed_512_bands():
    s = synth.config_system("C", lazy=True)
    say(f"[density] C n={s.n} nb={s.nb}: streaming the block")
    g = gfd.System.from_synth(s)
    psi = synth.block_to_device(s, "cuda", dtype=g.dtype)
    f = np.linspace(2.0, 0.0, s.nb)
    n_dev, D_dev = g.density(psi, to_dev(f))
    torch.cuda.synchronize()
    del psi
    ops = oracle.Operators.from_system(s, sparse=True)
    n_ref = np.zeros(s.ng)
    D_ref = np.zeros((s.natoms, 13, 13))
    for lo in range(0, s.nb, 64):
        x = s.bands(lo, min(s.nb, lo + 64)).reshape(-1, s.ng)
        n_ref += oracle.pseudo_density(x, f[lo:lo + 64])
        D_ref += oracle.atomic_density_matrices(ops.project(x), f[lo:lo + 64], s.natoms, 13)
    en = rel(host(n_dev), n_ref)
    eD = max(rel(host(D_dev)[a], D_ref[a]) for a in range(s.natoms))
    say(f"  n~ {en:.1e}, D {eD:.1e}")
    assert en <= TOL and eD <= TOL
    g.close()


def test_density_error_paths():
    s = synth.make_system(**CASES["real"])
    g = gfd.System.from_synth(s)
    psi = to_dev(s.psi.reshape(s.nb, -1))
    with pytest.raises(ValueError):
        g.density(psi, torch.ones(3, dtype=torch.float64, device="cuda"))
    f = torch.ones(s.nb, dtype=torch.float64, device="cuda")
    n = torch.empty(s.ng, dtype=torch.float64, device="cuda")
    with pytest.raises(gfd.GpawError) as e:
        g.density(psi, f, n_out=psi.view(-1)[: s.ng])  # n~ written over psi
    assert e.value.status == "GPAW_EALIAS"
    g.close()
