"""Parity of the multigrid Poisson solver and its grid transfers (zero-
boundary grids; Sec. "Solving the Kohn-Sham equation", Poisson solvers and
boundary conditions) with the oracle, through the C ABI.

* gpaw_laplacian_zero, gpaw_grid_restrict, gpaw_grid_interpolate element by
  element against the oracle's plain definitions (1e-13 of the largest
  value: the same sums, in another order);
* gpaw_poisson_solve to a relative residual of 1e-12 against the exact
  discrete solution (oracle solve_direct): every element within 1e-10 of
  the largest |phi| (the discrete operator's condition number at these
  sizes is below 1e3, so a 1e-12 residual bounds the error well below
  that); its cycle count matches the oracle's V-cycle to within one;
* ragged shapes whose hierarchy stops early (an even axis), a grid that does
  not coarsen at all, a 119 x 119 x 159 box (the wave-function grid of the
  largest workload, made odd) and error paths.
"""
import numpy as np
import pytest
import torch

from oracle import poisson as P
import paper_2310_14776_amd as gfd

from .gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,h", [((13, 17, 11), (0.21, 0.19, 0.23)),
                                 ((33, 31, 35), (0.2, 0.2, 0.2)),
                                 ((3, 2, 5), (0.3, 0.3, 0.3))])
def test_laplacian_zero(n, h):
    rng = np.random.default_rng(sum(n))
    f = rng.standard_normal(n)
    out = _host(gfd.laplacian_zero(_dev(f), h))
    ref = P.laplacian_zero(f, h)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("nf", [(7, 9, 5), (33, 31, 35), (3, 3, 3), (65, 17, 129)])
def test_restrict_interpolate(nf):
    rng = np.random.default_rng(sum(nf))
    nc = P.coarse_shape(nf)
    f = rng.standard_normal(nf)
    g = rng.standard_normal(nc)
    r = _host(gfd.grid_restrict(_dev(f)))
    ref = P.restrict(f)
    assert np.abs(r - ref).max() <= 1e-14 * np.abs(ref).max()
    base = rng.standard_normal(nf)
    out = _dev(base)
    gfd.grid_interpolate(_dev(g), nf, out=out, accumulate=True)
    ref = base + P.interpolate(g, nf)
    assert np.abs(_host(out) - ref).max() <= 1e-14 * np.abs(ref).max()
    out = gfd.grid_interpolate(_dev(g), nf)
    ref = P.interpolate(g, nf)
    assert np.abs(_host(out) - ref).max() <= 1e-14 * np.abs(ref).max()


def _gaussians(n, h, seed, count=4):
    rng = np.random.default_rng(seed)
    L = [(n[c] + 1) * h[c] for c in range(3)]
    x = [np.arange(1, n[c] + 1) * h[c] for c in range(3)]
    rho = np.zeros(n)
    for _ in range(count):
        c = [L[i] * rng.uniform(0.3, 0.7) for i in range(3)]
        s = rng.uniform(0.4, 0.9)
        q = rng.uniform(-1.0, 1.0)
        g = [np.exp(-(x[i] - c[i]) ** 2 / (2 * s * s)) for i in range(3)]
        rho += q * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :] / (2 * np.pi * s * s) ** 1.5
    return rho


@pytest.mark.parametrize("n,h,kind", [((31, 31, 31), (0.2, 0.2, 0.2), "gauss"),
                                      ((21, 15, 9), (0.25, 0.2, 0.3), "noise"),
                                      ((63, 31, 47), (0.2, 0.22, 0.18), "gauss"),
                                      ((10, 12, 8), (0.3, 0.3, 0.3), "noise")])
def test_poisson_solve(n, h, kind):
    rho = _gaussians(n, h, sum(n)) if kind == "gauss" else \
        np.random.default_rng(sum(n)).standard_normal(n)
    ref = P.solve_direct(rho, h)
    solver = gfd.Poisson(n, h)
    levels = solver.levels
    phi, cycles, res = solver.solve(_dev(rho), tol=1e-12, max_cycles=200)
    out = _host(phi)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    _, ocycles, _ = P.solve_multigrid(rho, h, tol=1e-12, max_cycles=200)
    say(f"[poisson] n={n} levels={levels} cycles={cycles} (oracle {ocycles}) "
        f"residual={res:.2e} err={err:.2e}")
    assert res <= 1e-12
    assert err <= 1e-10
    assert abs(cycles - ocycles) <= 1
    # started from the solution, one cycle suffices
    phi2, cyc2, res2 = solver.solve(_dev(rho), phi=_dev(out), tol=1e-11)
    assert cyc2 == 1 and res2 <= 1e-11
    solver.close()


@pytest.mark.timeout(600)
def test_poisson_largest_box():
    n, h = (119, 119, 159), (0.2, 0.2, 0.2)
    rho = _gaussians(n, h, 3, count=8)
    say(f"[poisson] n={n}: oracle solve")
    ref = P.solve_direct(rho, h)
    solver = gfd.Poisson(n, h)
    phi, cycles, res = solver.solve(_dev(rho), tol=1e-12, max_cycles=300)
    out = _host(phi)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    say(f"  levels={solver.levels} cycles={cycles} residual={res:.2e} err={err:.2e}")
    assert res <= 1e-12 and err <= 1e-10
    solver.close()


def test_poisson_error_paths():
    n, h = (7, 7, 7), (0.2, 0.2, 0.2)
    solver = gfd.Poisson(n, h)
    rho = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(gfd.GpawError) as e:
        solver.solve(rho, phi=rho)
    assert e.value.status == "GPAW_EALIAS"
    with pytest.raises(gfd.GpawError) as e:
        solver.solve(rho, tol=-1.0)
    assert e.value.status == "GPAW_EINVAL"
    nan = torch.full(n, float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(gfd.GpawError) as e:
        solver.solve(nan)
    assert e.value.status == "GPAW_ENONFINITE"
    solver.close()
    with pytest.raises(gfd.GpawError) as e:
        gfd.grid_restrict(torch.zeros((8, 7, 7), dtype=torch.float64, device="cuda"))
    assert e.value.status == "GPAW_ESHAPE"
    with pytest.raises(gfd.GpawError) as e:
        gfd.Poisson((0, 4, 4), h)
    assert e.value.status == "GPAW_ESHAPE"
