"""Precision form on the GPU against the FP64 oracle on the same inputs.

The block is rounded to FP32 once; the oracle then runs in FP64 on exactly
those values, so the comparison measures only the arithmetic of the precision
form: FP32 stencil and add-back, projections accumulated in double, split-BF16
subspace matrices and rotation on the matrix cores, FP64 Cholesky and
eigensolve, and the Cholesky orthonormality correction of the rotated block.
Every error is printed; the bounds asserted are the targets for this form:
eigenvalues within 1e-6 Ha, subspace matrices to 1e-7 relative (norm-wise),
the corrected block S~-orthonormal to 1e-6.
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
    "A_single": dict(synth.CONFIGS["A"]),
    "A_smooth_single": dict(synth.CONFIGS["A"], bands="smooth"),
    "medium_single": dict(n=(32, 32, 32), h=0.2, nb=96, natoms=6, rc=2.0, seed=51),
    "medium_smooth_single": dict(n=(32, 32, 32), h=0.2, nb=96, natoms=6, rc=2.0, seed=51,
                                 bands="smooth"),
    "bloch_single": dict(n=(16, 14, 18), h=0.2, nb=12, natoms=3, rc=1.8, seed=52, k=(0.25, 0.0, 0.5)),
    "bloch_smooth_single": dict(n=(16, 14, 18), h=0.2, nb=12, natoms=3, rc=1.8, seed=52,
                                k=(0.25, 0.0, 0.5), bands="smooth"),
    "large_single_nb192": dict(n=(20, 18, 22), h=0.2, nb=192, natoms=3, rc=1.6, seed=53),
}


def fp32_system(cfg):
    s = synth.make_system(**cfg)
    if s.is_complex:
        s.psi = s.psi.astype(np.complex64).astype(np.complex128)
    else:
        s.psi = s.psi.astype(np.float32).astype(np.float64)
    return s


@pytest.mark.parametrize("name", list(CASES))
def test_precision_form_against_fp64_oracle(name):
    s = fp32_system(CASES[name])
    say(f"[precision] case={name} n={s.n} nb={s.nb} natoms={s.natoms} complex={s.is_complex}")
    ref = oracle.fd_step(s)
    ops = ref["ops"]
    g = gfd.System.from_synth(s, precision="single")
    assert g.dtype in (torch.float32, torch.complex64)
    psi = to_dev(s.psi.reshape(s.nb, -1).astype(np.complex64 if s.is_complex else np.float32))
    out = g.step(psi)
    # S~ on the stored rotated block (projections: the rotated P), then the
    # Cholesky correction, as the precision form's step does
    Spsi_rot = g.apply_S(out["psi_rot"], out["P_rot"] if s.natoms else None)
    psi_fin, _ = g.orthonormalize(out["psi_rot"], Spsi_rot)
    torch.cuda.synchronize()
    errs = {
        "P": rel(host(out["P"]), ref["P"]) if s.natoms else 0.0,
        "Hpsi": rel(host(out["Hpsi"]), ref["Hpsi"]),
        "Spsi": rel(host(out["Spsi"]), ref["Spsi"]),
        "H": rel(host(out["H"]), ref["H"]),
        "S": rel(host(out["S"]), ref["S"]),
    }
    eps = host(out["eps"])
    d_eps = np.abs(eps - ref["eps"])
    errs["eps_max_abs"] = d_eps.max()
    C = host(out["C"])
    Hs = 0.5 * (ref["H"] + ref["H"].conj().T)
    Ss = 0.5 * (ref["S"] + ref["S"].conj().T)
    errs["C_orth"] = np.abs(C.conj().T @ Ss @ C - np.eye(s.nb)).max()
    pf = host(psi_fin).astype(np.complex128 if s.is_complex else np.float64)
    H1, S1 = oracle.subspace_matrices(pf, ops.apply_H(pf), ops.apply_S(pf), ops.dV)
    errs["final_S_minus_I"] = np.abs(S1 - np.eye(s.nb)).max()
    errs["final_rayleigh_vs_eps"] = np.abs(np.diag(H1).real - ref["eps"]).max()
    say("  errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    say("  per-eigenvalue |d eps| (Ha): " + " ".join(f"{x:.1e}" for x in d_eps))
    assert errs["H"] <= 1e-7 and errs["S"] <= 1e-7
    assert errs["eps_max_abs"] <= 1e-6
    assert errs["final_S_minus_I"] <= 1e-6
    # Rayleigh quotients of the corrected block as stored (single precision):
    # the storage rounding enters to first order through the residual
    # (H~ - eps S~) psi'', which is of the size of |eps| for noise bands, so
    # the bound is 1e-6 Ha or 2e-8 |eps|, whichever is larger
    assert errs["final_rayleigh_vs_eps"] <= max(1e-6, 2e-8 * np.abs(ref["eps"]).max())
    g.close()


def _round(x, cplx):
    return x.astype(np.complex64 if cplx else np.float32)


@pytest.mark.parametrize("precision", ["double", "single"])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("start", ["rotated", "raw"])
def test_orthonormalize_against_oracle(precision, cplx, start):
    """gpaw_orthonormalize on oracle-made inputs against the oracle's
    Cholesky correction of the same values: psi'' = (L^-H)^T psi with
    S' = dV psi^H S~psi = L L^H. 'rotated' starts from the oracle's rotated
    block (S' close to I: the single-precision form then takes its
    one-product path), 'raw' from the noise block itself (S' far from I).
    Bounds: 1e-12 relative in FP64; in single precision the inputs are the
    rounded values and the bound is FP32 resolution (1e-6 relative)."""
    cfg = dict(n=(16, 14, 18), h=0.2, nb=24, natoms=3, rc=1.8, seed=54)
    if cplx:
        cfg["k"] = (0.25, 0.0, 0.5)
    s = synth.make_system(**cfg)
    say(f"[orthonormalize-oracle] precision={precision} complex={cplx} start={start}")
    ref = oracle.fd_step(s)
    ops = ref["ops"]
    x = ref["psi_rot"] if start == "rotated" else s.psi.reshape(s.nb, -1)
    Sx = ops.apply_S(x)
    single = precision == "single"
    if single:
        # the oracle sees exactly the rounded values the GPU gets
        x = _round(x, cplx).astype(np.complex128 if cplx else np.float64)
        Sx = _round(Sx, cplx).astype(np.complex128 if cplx else np.float64)
    want = oracle.orthonormalize(x, Sx, ops.dV)
    g = gfd.System.from_synth(s, precision=precision)
    up = (lambda a: to_dev(_round(a, cplx))) if single else to_dev
    got, _ = g.orthonormalize(up(x), up(Sx))
    torch.cuda.synchronize()
    err = rel(host(got).astype(want.dtype), want)
    say(f"  ||psi'' - oracle|| / ||oracle|| = {err:.2e}")
    assert err <= (1e-6 if single else 1e-12)
    g.close()


@pytest.mark.parametrize("cplx", [False, True])
def test_orthonormalize_far_from_orthonormal(cplx):
    """The single-precision correction on a block far from S~-orthonormal:
    L^-H is then far from I, so the rotation takes all six split products;
    the result must be S~-orthonormal at FP32 resolution (FP64 oracle)."""
    cfg = dict(n=(16, 14, 18), h=0.2, nb=24, natoms=3, rc=1.8, seed=51)
    if cplx:
        cfg["k"] = (0.25, 0.0, 0.5)
    s = fp32_system(cfg)
    say(f"[orthonormalize] far case complex={cplx}")
    ops = oracle.Operators.from_system(s)
    g = gfd.System.from_synth(s, precision="single")
    psi = to_dev(s.psi.reshape(s.nb, -1).astype(np.complex64 if cplx else np.float32))
    Spsi = g.apply_S(psi)
    fin, _ = g.orthonormalize(psi, Spsi)
    torch.cuda.synchronize()
    pf = host(fin).astype(np.complex128 if cplx else np.float64)
    S1 = oracle.subspace_matrices(pf, ops.apply_H(pf), ops.apply_S(pf), ops.dV)[1]
    dev = np.abs(S1 - np.eye(s.nb)).max()
    say(f"  max |S' - I| = {dev:.2e}")
    assert dev <= 1e-5
    g.close()


@pytest.mark.parametrize("nb", [150, 1024])
@pytest.mark.parametrize("cplx", [False, True])
def test_orthonormalize_one_product_ragged(cplx, nb):
    """The one-product correction (L^-H = I + E, max |E| <= 2^-21) at a
    ragged band count (150: a partial row chunk and a partial 32-wide K
    step) and at the largest one the column-panel kernel takes (1024), on a
    grid whose 3315 columns are no multiple of the 32 or 64 columns a
    workgroup owns. The block is an S~-orthonormal one (oracle) mixed by
    I + P with |P| ~ 1e-7, so that E is a few 1e-7 and the correction moves
    the block by about 1e-6 relative: the device result must match the
    oracle's Cholesky correction of the same FP32 values to FP32 resolution
    and to a quarter of the size of the correction itself (a dropped or
    mis-signed product term misses by the whole term)."""
    cfg = dict(n=(15, 13, 17), h=0.2, nb=nb, natoms=3, rc=1.8, seed=57)
    if cplx:
        cfg["k"] = (0.25, 0.0, 0.5)
    s = synth.make_system(**cfg)
    say(f"[orthonormalize] one-product case complex={cplx} nb={nb}")
    ops = oracle.Operators.from_system(s)
    raw = s.psi.reshape(s.nb, -1)
    x0 = oracle.orthonormalize(raw, ops.apply_S(raw), ops.dV)
    rng = np.random.default_rng(5)
    P = rng.uniform(-1, 1, (nb, nb)) * 1.2e-7
    if cplx:
        P = P + 1j * rng.uniform(-1, 1, (nb, nb)) * 1.2e-7
    x = _round(x0 + P @ x0, cplx).astype(x0.dtype)
    Sx = _round(ops.apply_S(x), cplx).astype(x0.dtype)
    # precondition: the case is the one-product one, with a margin for the
    # device's own rounding of S'
    S1 = ops.dV * (x.conj() @ Sx.T)
    S1 = 0.5 * (S1 + S1.conj().T)
    Linv = np.linalg.inv(np.linalg.cholesky(S1))
    offid = np.abs(Linv.conj().T - np.eye(nb)).max()
    assert offid <= 0.8 * 2.0 ** -21, offid
    want = oracle.orthonormalize(x, Sx, ops.dV)
    corr = rel(x, want)
    g = gfd.System.from_synth(s, precision="single")
    got, _ = g.orthonormalize(to_dev(_round(x, cplx)), to_dev(_round(Sx, cplx)))
    torch.cuda.synchronize()
    err = rel(host(got).astype(want.dtype), want)
    say(f"  max|E| = {offid:.2e}, correction {corr:.2e}, ||psi'' - oracle|| / ||oracle|| = {err:.2e}")
    assert err <= 1e-6 and err <= 0.25 * corr
    g.close()


@pytest.mark.parametrize("precision", ["double", "single"])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("start", ["rotated", "raw"])
def test_orthonormalize_from_projections(precision, cplx, start):
    """gpaw_orthonormalize without S~psi: S' = dV psi^H psi + P^H Delta S P
    from the block and its projections (Eq. (dh): the non-local part of
    S~ seen from psi is conj(P) Delta S P) against the oracle's correction
    through S~psi on the same values, with the same bounds as the S~psi form
    (1e-12 relative in FP64, FP32 resolution in single precision; the
    projections are rounded too, which moves S' by about 1e-8). The rotated
    projections P_out must be the projections of the corrected block. Without
    S~psi the call needs P: GPAW_EINVAL otherwise."""
    cfg = dict(n=(16, 14, 18), h=0.2, nb=24, natoms=3, rc=1.8, seed=54)
    if cplx:
        cfg["k"] = (0.25, 0.0, 0.5)
    s = synth.make_system(**cfg)
    say(f"[orthonormalize-P] precision={precision} complex={cplx} start={start}")
    ref = oracle.fd_step(s)
    ops = ref["ops"]
    x = ref["psi_rot"] if start == "rotated" else s.psi.reshape(s.nb, -1)
    single = precision == "single"
    if single:
        x = _round(x, cplx).astype(np.complex128 if cplx else np.float64)
    Px = ops.project(x)
    want = oracle.orthonormalize(x, ops.apply_S(x, Px), ops.dV)
    g = gfd.System.from_synth(s, precision=precision)
    up = (lambda a: to_dev(_round(a, cplx))) if single else to_dev
    got, Pgot = g.orthonormalize(up(x), None, P=up(Px))
    torch.cuda.synchronize()
    err = rel(host(got).astype(want.dtype), want)
    perr = rel(host(Pgot).astype(want.dtype), ops.project(want))
    say(f"  ||psi'' - oracle|| / ||oracle|| = {err:.2e}, projections {perr:.2e}")
    tol = 1e-6 if single else 1e-12
    assert err <= tol and perr <= tol
    with pytest.raises(gfd.GpawError) as e:
        g.orthonormalize(up(x), None)
    assert e.value.status == "GPAW_EINVAL"
    g.close()
