"""Parity at the full workload sizes, in the launch configuration the
benchmark uses.

* 120x120x160 Bloch grid, k = (0.25, 0, 0.5), 128 atoms, 1024 bands: the
  largest single-GPU workload, in complex128 and in the complex64 precision
  form (2.36e9 elements per block, so every kernel indexes past 2^31). The
  block is generated band by band and streamed to the device; the oracle
  (sparse projector matrix) computes every projection, sampled bands of
  H~psi and S~psi, whole sampled columns of H_nm and S_nm, and sampled
  rotated bands (from the device's eigenvectors); the eigensolver is
  checked against LAPACK on the device's own matrices, and C through
  C^H S C = I and C^H H C = diag(eps).
* 96^3 real grid, 512 bands, 64 atoms: the same checks, FP64 and FP32.
* 120x120x160 Bloch grid on a 16-band block: every step against the oracle.
* 1024 bands (the largest block of that workload) on a 24^3 grid, real and
  complex: the full step against the oracle, including the global-memory
  eigensolver at its maximum size.
Tolerance: 1e-12 relative for the FP64 path; the precision form's values
are FP32 numbers, so its grid arrays are held to 1e-6 and its subspace
matrices to 1e-7 relative (the oracle runs on the same rounded inputs).
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


def _widen(x, single):
    """The block values the device holds, as FP64 (single precision: the
    rounded values)."""
    if not single:
        return x
    return x.astype(np.complex64 if np.iscomplexobj(x) else np.float32).astype(x.dtype)


def _sampled_full_step(s, precision, bands, chunk=64):
    single = precision == "single"
    tol_grid, tol_mat, tol_lin = (1e-6, 1e-7, 1e-12) if single else (TOL, TOL, TOL)
    cplx = s.is_complex
    say(f"[fullsize] {s.name} n={s.n} nb={s.nb} natoms={s.natoms} k={s.k} {precision}: "
        f"streaming the block")
    g = gfd.System.from_synth(s, precision=precision)
    psi = synth.block_to_device(s, "cuda", dtype=g.dtype)
    say("  block on the device; running the step")
    out = g.step(psi)
    torch.cuda.synchronize()
    del psi
    say("  step done; oracle on sampled bands")
    ops = oracle.Operators.from_system(s, sparse=True)
    xs = _widen(s.band_list(bands).reshape(len(bands), -1), single)
    Pref = ops.project(xs)
    Href = ops.apply_H(xs, Pref)
    Sref = ops.apply_S(xs, Pref)
    errs = {"Hpsi": rel(host(out["Hpsi"][bands]), Href),
            "Spsi": rel(host(out["Spsi"][bands]), Sref)}
    H, S, C = host(out["H"]), host(out["S"]), host(out["C"])
    eps = host(out["eps"])
    Pd = host(out["P"])
    # one pass over the whole block, regenerated chunk by chunk on the host:
    # every projection, whole columns m of H_nm = dV sum_r psi_n^* (H~psi_m),
    # and the rotated bands n = sum_m C_mn psi_m
    Hcol = np.zeros((s.nb, len(bands)), dtype=H.dtype)
    Scol = np.zeros_like(Hcol)
    rot = np.zeros((len(bands), s.ng), dtype=xs.dtype)
    Pall = np.zeros((s.nb, ops.Q.shape[0]), dtype=xs.dtype)
    for lo in range(0, s.nb, chunk):
        hi = min(s.nb, lo + chunk)
        x = _widen(s.bands(lo, hi).reshape(hi - lo, -1), single)
        Pall[lo:hi] = ops.project(x)
        Hcol[lo:hi] = ops.dV * (x.conj() @ Href.T)
        Scol[lo:hi] = ops.dV * (x.conj() @ Sref.T)
        rot += C[lo:hi, bands].T @ x
        if lo % (8 * chunk) == 0:
            say(f"  oracle pass: bands {lo}..{hi}")
    errs["P"] = rel(Pd, Pall)
    errs["H_cols"] = rel(H[:, bands], Hcol)
    errs["S_cols"] = rel(S[:, bands], Scol)
    errs["psi_rot"] = rel(host(out["psi_rot"][bands]), rot)
    errs["P_rot"] = rel(host(out["P_rot"][bands]), C[:, bands].T @ Pall)
    # the eigensolver on the device's own matrices, against LAPACK
    Hs, Ss = 0.5 * (H + H.conj().T), 0.5 * (S + S.conj().T)
    want = scipy.linalg.eigh(Hs, Ss, eigvals_only=True)
    scale = np.abs(want).max()
    errs["eps_vs_lapack"] = np.abs(eps - want).max() / scale
    Ch = C.conj().T
    errs["C_orth"] = np.abs(Ch @ Ss @ C - np.eye(s.nb)).max()
    errs["C_diag"] = np.abs(Ch @ Hs @ C - np.diag(eps)).max() / scale
    say("  errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert errs["P"] <= tol_grid and errs["Hpsi"] <= tol_grid and errs["Spsi"] <= tol_grid
    assert errs["H_cols"] <= tol_mat and errs["S_cols"] <= tol_mat
    assert errs["psi_rot"] <= tol_grid and errs["P_rot"] <= tol_grid
    assert errs["eps_vs_lapack"] <= tol_lin
    assert errs["C_orth"] <= tol_lin and errs["C_diag"] <= tol_lin
    assert np.all(np.diff(eps) >= 0)
    del out
    g.close()
    torch.cuda.empty_cache()


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("precision", ["double", "single"])
def test_bloch_120x120x160_1024_bands_sampled(precision):
    s = synth.config_system("D", lazy=True)
    _sampled_full_step(s, precision, bands=[0, 1, 511, 1023])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["double", "single"])
def test_96cubed_512_bands_sampled(precision):
    s = synth.config_system("C", lazy=True)
    _sampled_full_step(s, precision, bands=[0, 1, 257, 511])


def _full_step_against_oracle(s, sparse):
    ops = oracle.Operators.from_system(s, sparse=sparse)
    ref = oracle.fd_step(s, ops)
    g = gfd.System.from_synth(s)
    psi = to_dev(s.psi.reshape(s.nb, -1))
    out = g.step(psi)
    torch.cuda.synchronize()
    for key in ("P", "Hpsi", "Spsi", "H", "S"):
        assert rel(host(out[key]), ref[key]) <= TOL, key
    eps = host(out["eps"])
    assert np.abs(eps - ref["eps"]).max() <= TOL * np.abs(ref["eps"]).max()
    C = host(out["C"])
    Hs = 0.5 * (ref["H"] + ref["H"].conj().T)
    Ss = 0.5 * (ref["S"] + ref["S"].conj().T)
    assert np.abs(C.conj().T @ Ss @ C - np.eye(s.nb)).max() <= TOL
    assert np.abs(C.conj().T @ Hs @ C - np.diag(ref["eps"])).max() <= TOL * np.abs(ref["eps"]).max()
    assert rel(host(out["psi_rot"]), oracle.rotate(s.psi.reshape(s.nb, -1), C)) <= TOL
    assert rel(host(out["P_rot"]), oracle.rotate(ref["P"], C)) <= TOL
    g.close()


def test_bloch_120x120x160_grid_16_bands():
    s = synth.config_system("D", nb=16)
    say(f"[fullsize] n={s.n} nb={s.nb} natoms={s.natoms} k={s.k}")
    _full_step_against_oracle(s, sparse=True)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, 0.0, 0.5)])
def test_1024_bands(k):
    s = synth.make_system(n=(24, 24, 24), h=0.2, nb=1024, natoms=4, rc=2.0, seed=71, k=k)
    say(f"[fullsize] n={s.n} nb={s.nb} k={k}")
    _full_step_against_oracle(s, sparse=False)
