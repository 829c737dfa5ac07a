"""gpaw_subspace_matrices_noalloc against gpaw_subspace_matrices.

The no-allocation entry point keeps its split-K partial sums in the
library's static device array (split count capped to fit it) instead of the
system's workspace; its results must equal the ordinary call's to the FP64
path's 1e-12 (norm-wise relative; the sums run in a different order) and,
for the single-precision form, to 1e-7. Two calls in a row on each system,
the second with fewer bands (the array keeps the first call's contents), the
oracle as a third witness, and the size limit as an error path.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2310_14776_amd as gfd

from .gpu_util import say, to_dev, host, rel

pytestmark = pytest.mark.gpu

CASES = {
    "real": (dict(n=(24, 22, 20), h=0.2, nb=96, natoms=4, rc=2.0, seed=91), "double", 1e-12),
    "bloch": (dict(n=(18, 20, 16), h=0.2, nb=80, natoms=3, rc=1.8, seed=92, k=(0.25, 0.0, 0.5)),
              "double", 1e-12),
    "large_real": (dict(n=(20, 18, 22), h=0.2, nb=300, natoms=3, rc=1.6, seed=93), "double", 1e-12),
    "single": (dict(n=(24, 22, 20), h=0.2, nb=96, natoms=4, rc=2.0, seed=94), "single", 1e-7),
    "single_bloch": (dict(n=(18, 20, 16), h=0.2, nb=64, natoms=3, rc=1.8, seed=95,
                          k=(0.25, 0.0, 0.5)), "single", 1e-7),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


@pytest.mark.parametrize("name", list(CASES))
def test_noalloc_matches_subspace_matrices(name):
    cfg, precision, tol = CASES[name]
    s = synth.make_system(**cfg)
    say(f"[noalloc] {name} n={s.n} nb={s.nb} {precision}")
    g = gfd.System.from_synth(s, precision=precision)
    psi_full = to_dev(s.psi.reshape(s.nb, -1)).to(g.dtype)
    for nb in (s.nb, s.nb // 2 + 3):  # second call smaller
        psi = psi_full[:nb].contiguous()
        P = g.project(psi)
        Hpsi, Spsi = g.apply_HS(psi, P)
        H0, S0 = g.subspace_matrices(psi, Hpsi, Spsi)
        H1 = torch.full_like(H0, float("nan"))
        S1 = torch.full_like(S0, float("nan"))
        g.subspace_matrices_noalloc(psi, Hpsi, Spsi, H1, S1)
        # H only (Spsi NULL): S_nn untouched
        H2 = torch.full_like(H0, float("nan"))
        S2 = torch.full_like(S0, 7.0)
        g.subspace_matrices_noalloc(psi, Hpsi, None, H2, S2)
        torch.cuda.synchronize()
        x = psi.double() if not s.is_complex else psi.to(torch.complex128)
        Href, Sref = oracle.subspace_matrices(host(x), host(Hpsi).astype(host(x).dtype),
                                              host(Spsi).astype(host(x).dtype), float(np.prod(s.h)))
        eH, eS = rel(host(H1), host(H0)), rel(host(S1), host(S0))
        eH2 = rel(host(H2), host(H0))
        say(f"  nb={nb}: vs ordinary call H {eH:.1e} S {eS:.1e} (H only {eH2:.1e}); "
            f"vs oracle H {rel(host(H1), Href):.1e}")
        assert np.all(np.isfinite(host(H1))) and np.all(np.isfinite(host(S1)))
        assert eH <= tol and eS <= tol and eH2 <= tol
        assert np.all(host(S2) == 7.0)
        assert rel(host(H1), Href) <= tol and rel(host(S1), Sref) <= tol
    g.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    # 1500 complex bands with S: 2 * 1500^2 * 2 doubles > 64 MiB
    nb = 1500
    g = gfd.System(n=(4, 4, 4), h=0.2, k=(0.25, 0.0, 0.0), pos=np.zeros((0, 3)), channels=[],
                   dH=np.zeros(0), dS=np.zeros(0), v=np.zeros(64), max_bands=nb, complex_=True)
    psi = torch.zeros((nb, 64), dtype=torch.complex128, device="cuda")
    H = torch.empty((nb, nb), dtype=torch.complex128, device="cuda")
    S = torch.empty_like(H)
    with pytest.raises(gfd.GpawError) as e:
        g.subspace_matrices_noalloc(psi, psi.clone(), psi.clone(), H, S)
    assert e.value.status == "GPAW_ESHAPE"
    # H alone (nmat = 1) fits
    g.subspace_matrices_noalloc(psi, psi.clone(), None, H, S)
    torch.cuda.synchronize()
    assert float(torch.abs(H).max()) == 0.0
    g.close()
