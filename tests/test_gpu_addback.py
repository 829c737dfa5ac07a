"""The non-local add-back of Eq. (dh) as a pass of its own (blocks of at
least 2^24 band-points run the stencil without atoms, then add
sum q (Delta H P) and q (Delta S P) at the covered points), through the
C ABI, element by element against the oracle:

* periodic real, Bloch complex and finite (zero-boundary) systems, 1e-12 of
  the largest value (the FP64 sums are the fused kernel's, in the same order);
* H~psi from the one-pass call equals the H-only call bit for bit, and
  S~psi equals the S-only call (its own one-lane-per-point kernel) to
  1e-15;
* the single-precision form against the oracle on the same rounded block,
  within the 1e-6 of the largest value that bounds its grid arrays (FP32
  stencil sums and storage; H~psi is rounded once more here, after the
  stencil and after the add-back).
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

# 26^3 x 1000 bands = 17.6e6 >= 2^24 band-points
CASES = {
    "real": dict(n=(26, 26, 26), h=0.2, nb=1000, natoms=6, rc=2.0, seed=61),
    "bloch": dict(n=(26, 26, 26), h=0.2, nb=1000, natoms=6, rc=2.0, seed=62,
                  k=(0.25, 0.0, 0.5)),
    "finite": dict(n=(27, 25, 26), h=0.2, nb=1000, natoms=7, rc=2.0, seed=63,
                   complex_psi=True),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


def _system(name):
    s = synth.make_system(name=name, **CASES[name])
    assert s.nb * int(np.prod(s.n)) >= 1 << 24
    if name == "finite":
        s.meta["boundary"] = "zero"
        return s, T.FiniteOps.from_system(s)
    return s, oracle.Operators.from_system(s)


@pytest.mark.parametrize("name", list(CASES))
def test_separate_addback_against_oracle(name):
    s, ops = _system(name)
    say(f"[addback] case={name} n={s.n} nb={s.nb} natoms={s.natoms}")
    psi_h = s.psi.reshape(s.nb, -1)
    g = gfd.System.from_synth(s)
    psi = to_dev(psi_h)
    P = g.project(psi)
    Hf, Sf = g.apply_HS(psi, P)
    Hs = g.apply_H(psi, P)
    Ss = g.apply_S(psi, P)
    torch.cuda.synchronize()
    Pref = ops.project(psi_h)
    assert rel(host(P), Pref) <= TOL
    Href = ops.apply_H(psi_h, Pref)
    Sref = ops.apply_S(psi_h, Pref)
    for got, ref, what in ((Hf, Href, "H"), (Sf, Sref, "S")):
        err = np.abs(host(got) - ref).max() / np.abs(ref).max()
        say(f"  {what}: max err {err:.2e}")
        assert err <= TOL, what
    assert torch.equal(Hf, Hs)
    assert rel(host(Sf), host(Ss)) <= 1e-15
    g.close()


def test_separate_addback_precision_form():
    s, ops = _system("bloch")
    psi_h = s.psi.reshape(s.nb, -1).astype(np.complex64).astype(np.complex128)
    say("[addback] precision form, case=bloch")
    g = gfd.System.from_synth(s, precision="single")
    psi = to_dev(psi_h.astype(np.complex64))
    P = g.project(psi)
    Hf, Sf = g.apply_HS(psi, P)
    torch.cuda.synchronize()
    # the reference takes the device's own projections (their FP32 rounding
    # is the projection's business, tested elsewhere)
    Pd = host(P).astype(np.complex128)
    Href = ops.apply_H(psi_h, Pd)
    Sref = ops.apply_S(psi_h, Pd)
    for got, ref, what in ((Hf, Href, "H"), (Sf, Sref, "S")):
        err = np.abs(host(got).astype(np.complex128) - ref).max() / np.abs(ref).max()
        say(f"  {what}: max err {err:.2e}")
        assert err <= 1e-6, what
    g.close()
