"""Batched form on the GPU: many uneven systems through one graph launch.

Every system of a small mixed batch (real and Bloch, uneven grids and band
counts, one above the one-workgroup eigensolver limit, one without atoms) is
checked against the FP64 oracle to the single-system bar (1e-12 relative),
through the same gauge-free quantities as the single-system parity tests.
The graph is replayed several times with eager work in between, every replay
checked; after the autotuner has changed the launch shapes the results are
checked again. At the 64-system workload (grids 16..48 per axis, 8..96 bands,
2..16 atoms, half complex) a sample of systems spanning the size range is
checked against the oracle, and the rest through the invariants of their own
subspace matrices.
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

SMALL = [
    dict(n=(16, 16, 16), h=0.2, nb=8, natoms=2, rc=2.0, seed=61),
    dict(n=(18, 14, 20), h=0.2, nb=5, natoms=3, rc=1.8, seed=62, k=(0.1, 0.2, 0.3)),
    dict(n=(20, 20, 17), h=0.2, nb=24, natoms=4, rc=2.0, seed=63),
    dict(n=(16, 21, 16), h=0.2, nb=12, natoms=2, rc=2.0, seed=64, k=(0.25, 0.0, 0.5)),
    dict(n=(13, 17, 11), h=(0.21, 0.19, 0.23), nb=3, natoms=0, rc=2.0, seed=65),
    dict(n=(24, 16, 16), h=0.2, nb=40, natoms=5, rc=1.6, seed=66, k=(0.4, 0.1, 0.0)),
    dict(n=(16, 18, 20), h=0.2, nb=140, natoms=2, rc=1.6, seed=67),
    dict(n=(17, 16, 18), h=0.2, nb=1, natoms=1, rc=2.0, seed=68),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gfd.load()


class Run:
    """Systems, device buffers and a batch for a list of synthetic systems."""

    def __init__(self, systems):
        self.s = systems
        self.g = [gfd.System.from_synth(s) for s in systems]
        self.psi = [to_dev(s.psi.reshape(s.nb, -1)) for s in systems]
        self.out = [torch.empty_like(p) for p in self.psi]
        self.eps = [torch.empty(s.nb, dtype=torch.float64, device="cuda") for s in systems]
        self.P = [torch.empty((s.nb, g.np), dtype=g.dtype, device="cuda") for s, g in
                  zip(systems, self.g)]
        self.H = [torch.empty((s.nb, s.nb), dtype=g.mat_dtype, device="cuda") for s, g in
                  zip(systems, self.g)]
        self.S = [torch.empty_like(h) for h in self.H]
        self.C = [torch.empty_like(h) for h in self.H]
        self.info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
        self.batch = gfd.Batch(self.g)
        self.io = self.batch.io(self.psi, self.out, self.eps, self.P, self.H, self.S, self.C)

    def step(self):
        self.batch.step(self.io, self.info)
        torch.cuda.synchronize()
        assert host(self.info).tolist() == [0] * len(self.s)

    def close(self):
        self.batch.close()
        for g in self.g:
            g.close()


def check_against_oracle(r, i, ref=None):
    s = r.s[i]
    ops = oracle.Operators.from_system(s)
    ref = ref or oracle.fd_step(s, ops)
    H, S, eps, C = host(r.H[i]), host(r.S[i]), host(r.eps[i]), host(r.C[i])
    assert rel(H, ref["H"]) <= TOL
    assert rel(S, ref["S"]) <= TOL
    assert np.abs(eps - ref["eps"]).max() <= TOL * np.abs(ref["eps"]).max()
    Hs = 0.5 * (ref["H"] + ref["H"].conj().T)
    Ss = 0.5 * (ref["S"] + ref["S"].conj().T)
    assert np.abs(C.conj().T @ Ss @ C - np.eye(s.nb)).max() <= TOL
    assert rel(host(r.out[i]), oracle.rotate(s.psi.reshape(s.nb, -1), C)) <= TOL
    if s.natoms:
        assert rel(host(r.P[i]), oracle.rotate(ref["P"], C)) <= TOL
    return ref


def test_batch_small_mixed_against_oracle():
    systems = [synth.make_system(name=f"small{i}", **c) for i, c in enumerate(SMALL)]
    say(f"[batch] small mixed batch of {len(systems)}")
    r = Run(systems)
    r.step()
    refs = [check_against_oracle(r, i) for i in range(len(systems))]
    first = [host(x).copy() for x in r.out]
    # replays with eager work in between: every replay equals the first
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (junk * 2.0).sum().item()
        r.step()
        for i in range(len(systems)):
            assert np.array_equal(host(r.out[i]), first[i]), (rep, i)
    # the autotuner changes launch shapes only: results stay within the bar
    r.batch.tune(r.io, r.info)
    torch.cuda.synchronize()
    nbr, shapes = r.batch.tuning()
    say(f"  tuned branches={nbr} shapes={shapes}")
    assert 1 <= nbr <= 16
    r.step()
    for i in range(len(systems)):
        check_against_oracle(r, i, refs[i])
    r.close()


def test_batch_rerecords_when_buffers_change():
    systems = [synth.make_system(name=f"small{i}", **c) for i, c in enumerate(SMALL[:3])]
    say("[batch] re-record on new output buffers")
    r = Run(systems)
    r.step()
    a = [host(x).copy() for x in r.out]
    r.out = [torch.full_like(x, float("nan")) for x in r.out]
    r.io = r.batch.io(r.psi, r.out, r.eps, r.P, r.H, r.S, r.C)
    r.step()
    for i in range(len(systems)):
        assert np.array_equal(host(r.out[i]), a[i])
    r.close()


def test_batch_error_paths():
    systems = [synth.make_system(name=f"small{i}", **c) for i, c in enumerate(SMALL[:2])]
    say("[batch] error paths")
    r = Run(systems)
    bad = r.batch.io(r.psi, r.psi, r.eps)  # psi_out aliases psi
    with pytest.raises(gfd.GpawError) as e:
        r.batch.step(bad, r.info)
    assert e.value.status == "GPAW_EALIAS"
    io = r.batch.io(r.psi, r.out, r.eps)
    io[1].nb = systems[1].nb + 1
    with pytest.raises(gfd.GpawError) as e:
        r.batch.step(io, r.info)
    assert e.value.status == "GPAW_ESHAPE"
    with pytest.raises(gfd.GpawError):
        gfd.Batch([r.g[0], r.g[0]])
    r.close()


def test_batch_full_workload_sampled():
    cfgs = synth.batched_systems()
    systems = [synth.make_system(name=f"E{i}", **c) for i, c in enumerate(cfgs)]
    say(f"[batch] full workload: {len(systems)} systems")
    r = Run(systems)
    r.batch.tune(r.io, r.info)
    r.step()
    size = [s.ng * s.nb for s in systems]
    real = [i for i, s in enumerate(systems) if not s.is_complex]
    cplx = [i for i, s in enumerate(systems) if s.is_complex]
    sample = {min(real, key=size.__getitem__), max(real, key=size.__getitem__),
              min(cplx, key=size.__getitem__), max(cplx, key=size.__getitem__)}
    for i in sorted(sample):
        say(f"  oracle check system {i}: n={systems[i].n} nb={systems[i].nb} "
            f"complex={systems[i].is_complex}")
        check_against_oracle(r, i)
    # every system: C is S-orthonormal and diagonalises H (its own matrices)
    for i, s in enumerate(systems):
        H, S, C, eps = host(r.H[i]), host(r.S[i]), host(r.C[i]), host(r.eps[i])
        Hs, Ss = 0.5 * (H + H.conj().T), 0.5 * (S + S.conj().T)
        assert np.all(np.diff(eps) >= 0)
        assert np.abs(C.conj().T @ Ss @ C - np.eye(s.nb)).max() <= 1e-12
        assert np.abs(C.conj().T @ Hs @ C - np.diag(eps)).max() <= 1e-12 * np.abs(eps).max()
    r.close()


def test_batch_mixed_precision():
    """Single-precision systems (FP32 and complex64 storage, split-BF16
    products) in one batch with FP64 and complex128 ones: the FP64 systems
    meet the 1e-12 bar, the single-precision ones the precision form's
    (eigenvalues within 1e-6 Ha of the oracle on the same rounded inputs, or
    2e-8 of the largest |eps| where that is larger: FP32 storage of H~psi
    resolves 6e-8 of a value, and these noise bands reach ~100 Ha; H and S
    within 1e-7 relative) and equal their own per-system step; the autotuner
    leaves the single-precision shapes fixed and the results hold."""
    cfgs = [SMALL[0], SMALL[1], SMALL[2], SMALL[3], SMALL[5]]
    prec = ["double", "single", "single", "double", "single"]
    systems = []
    for i, (c, p) in enumerate(zip(cfgs, prec)):
        s = synth.make_system(name=f"mixed{i}", **c)
        if p == "single":
            s.psi = s.psi.astype(np.complex64 if s.is_complex else np.float32).astype(s.psi.dtype)
        systems.append(s)
    say(f"[batch] mixed precision batch: {prec}")
    gs = [gfd.System.from_synth(s, precision=p) for s, p in zip(systems, prec)]
    psi = []
    for s, g in zip(systems, gs):
        x = s.psi.reshape(s.nb, -1)
        psi.append(to_dev(x).to(g.dtype))
    out = [torch.empty_like(p) for p in psi]
    eps = [torch.empty(s.nb, dtype=torch.float64, device="cuda") for s in systems]
    P = [torch.empty((s.nb, g.np), dtype=g.dtype, device="cuda") for s, g in zip(systems, gs)]
    H = [torch.empty((s.nb, s.nb), dtype=g.mat_dtype, device="cuda") for s, g in zip(systems, gs)]
    S = [torch.empty_like(h) for h in H]
    C = [torch.empty_like(h) for h in H]
    info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    batch = gfd.Batch(gs)
    io = batch.io(psi, out, eps, P, H, S, C)
    refs = [oracle.fd_step(s) for s in systems]

    def check():
        torch.cuda.synchronize()
        assert host(info).tolist() == [0] * len(systems)
        for i, (s, p, ref) in enumerate(zip(systems, prec, refs)):
            e = host(eps[i])
            if p == "double":
                assert rel(host(H[i]), ref["H"]) <= TOL and rel(host(S[i]), ref["S"]) <= TOL
                assert np.abs(e - ref["eps"]).max() <= TOL * np.abs(ref["eps"]).max()
            else:
                assert rel(host(H[i]), ref["H"]) <= 1e-7 and rel(host(S[i]), ref["S"]) <= 1e-7
                err = np.abs(e - ref["eps"]).max()
                bound = max(1e-6, 2e-8 * np.abs(ref["eps"]).max())
                say(f"  system {i} ({'complex64' if s.is_complex else 'FP32'}): max |d eps| "
                    f"{err:.2e} Ha (bound {bound:.1e}, max |eps| {np.abs(ref['eps']).max():.1f})")
                assert err <= bound

    batch.step(io, info)
    check()
    # the single-precision systems equal their own per-system step
    for i, p in enumerate(prec):
        if p == "single":
            own = gs[i].step(psi[i])
            torch.cuda.synchronize()
            assert np.array_equal(host(own["eps"]), host(eps[i])), i
            assert np.array_equal(host(own["psi_rot"]), host(out[i])), i
    batch.tune(io, info)
    torch.cuda.synchronize()
    nbr, shapes = batch.tuning()
    say(f"  tuned branches={nbr} shapes={shapes}")
    for i, p in enumerate(prec):
        if p == "single":
            assert all(v == 0 for v in shapes[i].values()), i
    batch.step(io, info)
    check()
    batch.close()
    for g in gs:
        g.close()


def test_batch_tuning_cache(tmp_path):
    """Autotuned shapes saved to a file and applied to a new batch of the
    same systems give that batch the same shapes and the same results, bit
    for bit, without running the autotuner; a file made for other systems is
    refused, and so are shapes the autotuner would never choose."""
    systems = [synth.make_system(name=f"small{i}", **c) for i, c in enumerate(SMALL[:4])]
    say("[batch] tuning cache")
    r = Run(systems)
    r.batch.tune(r.io, r.info)
    r.step()
    path = str(tmp_path / "tuning.json")
    r.batch.save_tuning(path)
    tuned = r.batch.tuning()
    ref = [host(x).copy() for x in r.out]
    ref_eps = [host(x).copy() for x in r.eps]
    r.close()
    r2 = Run(systems)
    assert r2.batch.load_tuning(path)
    assert r2.batch.tuning() == tuned
    r2.step()
    for i in range(len(systems)):
        assert np.array_equal(host(r2.out[i]), ref[i]), i
        assert np.array_equal(host(r2.eps[i]), ref_eps[i]), i
    # a different set of systems: the file does not apply
    r3 = Run(systems[:3])
    before = r3.batch.tuning()
    assert not r3.batch.load_tuning(path)
    assert r3.batch.tuning() == before
    # values outside the autotuner's choices are rejected, nothing changes
    bad = [dict(s) for s in tuned[1][:3]]
    bad[1]["rotate_rb"] = 3
    with pytest.raises(gfd.GpawError) as e:
        r3.batch.set_tuning(4, bad)
    assert e.value.status == "GPAW_EINVAL"
    assert r3.batch.tuning() == before
    r3.step()
    r3.close()
    r2.close()
