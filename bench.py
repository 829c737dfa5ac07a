#!/usr/bin/env python3
"""Benchmark: one FD-PAW block eigensolver step per iteration on one MI355X.

Step = projections, H~psi and S~psi (one pass), subspace matrices H_nm and
S_nm, FP64 Cholesky + generalised eigensolve, rotation of the block and of
its projections. Default workload: the largest single-GPU case, a Bloch
120x120x160 grid (h = 0.2 bohr, k = (0.25, 0, 0.5)), 1024 bands, 128 atoms
with 13 projectors each, complex128. Seeded synthetic inputs, already
resident in HBM when the timed region starts.

Prints one JSON line: throughput (band*gridpoints/s), per-part times, the
roofline of the dominant kernel, the precision form (complex64 storage,
split-BF16 matrix-core products, FP64 eigensolve, Cholesky orthonormality
correction) and the batched form beside the FP64 step, the 48^3 and 96^3
real workloads as extra lines, the paths beside the step (density, Davidson
correction, zero-boundary multigrid Poisson, Crank-Nicolson propagation),
and the CPU oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="D", choices=["A", "B", "C", "D"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision-form and batched-form measurements")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form measurement (profiler runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workload lines (48^3 and 96^3 real)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in launch shapes (skip the autotuner; for profiler runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, run a plain 256 MiB device copy three times "
                         "(reference kernel for hardware byte counters)")
    return ap.parse_args()


# kernels behind each timed call, and the sources they are built from
PART_KERNELS = {
    "project": (["k_project"], ["csrc/nonlocal.hip", "csrc/proj.h"]),
    # H~psi and S~psi: Delta H.P and Delta S.P (one launch), then the stencil (with the
    # add-back fused, or for large blocks followed by the add-back pass)
    "apply_HS": (["k_dmat2", "k_plane", "k_addback"],
                 ["csrc/stencil.hip", "csrc/stencil_impl.h", "csrc/stencil_f64.hip",
                  "csrc/stencil_c128.hip", "csrc/nonlocal.hip", "csrc/proj.h"]),
    # (k_subspace matches the narrow- and wide-block kernels)
    "subspace": (["k_subspace", "k_subspace_reduce"], ["csrc/gemm.hip", "csrc/tile_order.h"]),
    # the block and its projections
    "rotate": (["k_rotate", "k_rot_small"], ["csrc/gemm.hip", "csrc/tile_order.h"]),
}


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(ROOT, "paper_2310_14776_amd")
    for f in files:
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(part, workload_tag):
    """HBM bytes per launch of a part from the committed counter summary, or
    None when there is none or the kernels' sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{part}_{workload_tag}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    try:
        if fields.get("source_sha256") != source_hash(PART_KERNELS[part][1]):
            return None
        return int(float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def timed(fn, stream, steps, warmup):
    """Mean milliseconds of fn() over `steps` calls (HIP events on `stream`)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def say(*msg):
    print(*msg, file=sys.stderr, flush=True)


def workload_label(s):
    kind = (f"Bloch k=({s.k[0]:g},{s.k[1]:g},{s.k[2]:g})" if s.is_complex else "periodic")
    return (f"FD-PAW block step, {kind} {s.n[0]}x{s.n[1]}x{s.n[2]} grid h={s.h[0]:g} bohr, "
            f"{s.nb} bands, {s.natoms} atoms x 13 projectors")


class Step:
    """Buffers and the call sequence of one block step on one system."""

    def __init__(self, g, psi, stream):
        import torch
        self.g, self.psi, self.stream = g, psi, stream
        nb, dev = psi.shape[0], psi.device
        self.nb = nb
        self.P = torch.empty((nb, g.np), dtype=g.dtype, device=dev)
        self.Hpsi = torch.empty_like(psi)
        self.Spsi = torch.empty_like(psi)
        self.H = torch.empty((nb, nb), dtype=g.mat_dtype, device=dev)
        self.S = torch.empty_like(self.H)
        self.C = torch.empty_like(self.H)
        self.eps = torch.empty(nb, dtype=torch.float64, device=dev)
        self.psi_rot = torch.empty_like(psi)
        self.P_rot = torch.empty_like(self.P)
        self.info = torch.zeros(1, dtype=torch.int32, device=dev)
        self.single = g.precision == "single"
        if self.single:
            self.psi_fin = torch.empty_like(psi)
            self.P_fin = torch.empty_like(self.P)

    def parts(self):
        g, st = self.g, self.stream
        out = [
            ("project", lambda: g.project(self.psi, out=self.P, stream=st)),
            ("apply_HS", lambda: g.apply_HS(self.psi, self.P, Hpsi=self.Hpsi, Spsi=self.Spsi,
                                            stream=st)),
            ("subspace", lambda: g.subspace_matrices(self.psi, self.Hpsi, self.Spsi, H=self.H,
                                                     S=self.S, stream=st)),
            ("diag", lambda: g.subspace_diag(self.H, self.S, eps=self.eps, C=self.C,
                                             info=self.info, stream=st)),
            ("rotate", lambda: g.rotate(self.psi, self.C, out=self.psi_rot, P=self.P,
                                        P_out=self.P_rot, stream=st)),
        ]
        if self.single:
            # the Cholesky orthonormality correction of the stored rotated
            # block, its overlap formed from the block and its (rotated)
            # projections: S' = dV psi'^H psi' + P'^H Delta S P'
            out.append(("orthonormalize", lambda: g.orthonormalize(
                self.psi_rot, None, out=self.psi_fin, P=self.P_rot, P_out=self.P_fin,
                info=self.info, stream=st)))
        return out

    def run(self):
        for _, fn in self.parts():
            fn()

    def check(self):
        if int(self.info.item()) != 0:
            raise RuntimeError(f"eigensolver status {int(self.info.item())}")


def time_parts(step, steps, warmup):
    """Whole-step time (HIP events around the timed steps on the launch
    stream) and per-part mean times (events around each call)."""
    import torch
    parts = step.parts()
    for _ in range(warmup):
        step.run()
    torch.cuda.synchronize()
    ev = {name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(steps)] for name, _ in parts}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(step.stream)
    for k in range(steps):
        for name, fn in parts:
            a, b = ev[name][k]
            a.record(step.stream)
            fn()
            b.record(step.stream)
    stop.record(step.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    step.check()
    ms_step = start.elapsed_time(stop) / steps
    part_ms = {name: float(np.mean([a.elapsed_time(b) for a, b in ev[name]])) for name, _ in parts}
    return ms_step, part_ms, wall


def tune(g, psi, stream):
    """Launch shapes from the library's autotuner (kept in the system; every
    choice computes the same results)."""
    import torch
    import paper_2310_14776_amd as gfd
    out = torch.empty_like(psi)
    eps = torch.empty(psi.shape[0], dtype=torch.float64, device=psi.device)
    info = torch.zeros(1, dtype=torch.int32, device=psi.device)
    tb = gfd.Batch([g])
    tb.tune(tb.io([psi], [out], [eps]), info)
    t = tb.tuning()[1][0]
    tb.close()
    torch.cuda.synchronize()
    return t


def measured_peaks(dev, stream):
    """Achievable ceilings of this device from the library's probes: a 16-byte
    copy over 2 x 4 GiB buffers (HBM bytes moved = 2 x size) and matrix-core
    loops of independent FP64 and BF16 products (8 workgroups per CU)."""
    import torch
    import paper_2310_14776_amd as gfd
    nbytes = 4 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    copy_ms = timed(lambda: gfd.probe_copy(a, b, stream=stream), stream, 10, 2)
    del a, b
    wgs, out = 2048, {}
    for kind, name, flops, iters, dt in ((0, "fp64_mfma_TFLOPs", 2048, 4000, torch.float64),
                                         (1, "bf16_mfma_TFLOPs", 16384, 4000, torch.float32)):
        buf = torch.empty(wgs * 256, dtype=dt, device=dev)
        ms = timed(lambda: gfd.probe_mfma(kind, buf, wgs, iters, stream=stream), stream, 5, 1)
        out[name] = round(wgs * 4 * iters * 8 * flops / (ms * 1e-3) / 1e12, 1)
    out["hbm_copy_GBs"] = round(2 * nbytes / (copy_ms * 1e-3) / 1e9, 1)
    return out


def part_costs(s, info, es):
    """Algorithmic bytes and flops per launch of each part (es = bytes per
    element of the block). A complex-by-complex product costs three real
    products (the contractions use the three-multiplication form), a real
    projector value times a complex value two."""
    nb, ng, npj, ni = s.nb, s.ng, info["np"], info["ni"]
    ent = info["entries"]
    cf = 3 if s.is_complex else 1
    cp = 2 if s.is_complex else 1
    return {
        # gather psi at every sphere entry, read the entry table once, write P
        "project": dict(bytes=ent * nb * es + ent * 12 + nb * npj * es,
                        flops=2 * ent * ni * nb * cp),
        # read psi, write H~psi and S~psi, read v and the add-back tables once
        "apply_HS": dict(bytes=3 * nb * ng * es + ng * 8 + ng * 16 + ent * 4, flops=0),
        # read psi, H~psi, S~psi; two Hermitian nb x nb products over Ng, of
        # which the nb (nb + 1) / 2 entries on and above the diagonal are
        # needed (2 flops per multiply-add)
        "subspace": dict(bytes=3 * nb * ng * es, flops=2 * nb * (nb + 1) * ng * cf),
        "diag": dict(bytes=0, flops=0),
        # read psi, write psi'; nb x nb times nb x (Ng + Np)
        "rotate": dict(bytes=2 * nb * (ng + npj) * es, flops=2 * nb * nb * (ng + npj) * cf),
    }


def roofline(part_ms, costs, tag, peaks=None):
    """Roofline object of the costliest part with a bandwidth or matrix-core
    bound (FP64 MFMA for the contractions, HBM otherwise); with measured
    ceilings, also the fraction of those."""
    dom = max((n for n in part_ms if n in costs and (costs[n]["bytes"] or costs[n]["flops"])),
              key=part_ms.get)
    c = costs[dom]
    t = part_ms[dom] * 1e-3
    intensity = c["flops"] / c["bytes"] if c["bytes"] else float("inf")
    ridge = FP64_MFMA_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if c["flops"] and intensity >= ridge:
        achieved = c["flops"] / t / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4)}
    else:
        achieved = c["bytes"] / t / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof["kernel"] = " + ".join(PART_KERNELS[dom][0])
    roof["traffic"] = measured_traffic(dom, tag)
    if peaks:
        mp = peaks["fp64_mfma_TFLOPs"] if roof["bound"] == "mfma" else peaks["hbm_copy_GBs"]
        roof["measured_peak"] = mp
        roof["frac_of_measured"] = round(roof["achieved"] / mp, 4)
    return roof


def part_rows(part_ms, costs):
    rows = {}
    for name, ms in part_ms.items():
        c = costs.get(name, dict(bytes=0, flops=0))
        t = ms * 1e-3
        rows[name] = dict(ms=round(ms, 4),
                          GBs=round(c["bytes"] / t / 1e9, 1) if c["bytes"] else None,
                          TFLOPs=round(c["flops"] / t / 1e12, 2) if c["flops"] else None)
    return rows


def run_config(name, steps, warmup, dev, stream, single_inputs=False, do_tune=True, peaks=None):
    """FP64 step of one workload. Returns (result dict, system, step)."""
    import torch
    import synth
    import paper_2310_14776_amd as gfd
    s = synth.config_system(name, lazy=True)
    say(f"[bench] {name}: {workload_label(s)}; generating and uploading the block")
    g = gfd.System.from_synth(s)
    if single_inputs:
        # values rounded to single precision (widened exactly on the device),
        # so that the precision form later sees the same inputs
        low = synth.block_to_device(s, dev, dtype=torch.complex64 if s.is_complex
                                    else torch.float32)
        psi = low.to(g.dtype)
    else:
        low = None
        psi = synth.block_to_device(s, dev, dtype=g.dtype)
    es = psi.element_size()
    if do_tune:
        say(f"[bench] {name}: autotuning the launch shapes")
    tuning = tune(g, psi, stream) if do_tune else "heuristic"
    step = Step(g, psi, stream)
    say(f"[bench] {name}: timing {steps} steps")
    ms, part_ms, wall = time_parts(step, steps, warmup)
    costs = part_costs(s, g.info, es)
    res = dict(ms_per_step=ms, value=s.nb * s.ng / (ms * 1e-3), wall_s=wall,
               workload=workload_label(s), dtype="c128" if s.is_complex else "f64",
               parts=part_rows(part_ms, costs), launch_tuning=tuning,
               roofline=roofline(part_ms, costs, f"{s.n[0]}x{s.n[1]}x{s.n[2]}_nb{s.nb}", peaks))
    return res, s, step, low


def precision_form(s, low, fp64_step, fp64_ms, steps, warmup, dev, stream):
    """The precision form on the same (rounded) block as the FP64 step:
    single-precision storage, split-BF16 products, FP64 eigensolve, Cholesky
    orthonormality correction of the stored rotated block."""
    import torch
    import paper_2310_14776_amd as gfd
    g = gfd.System.from_synth(s, precision="single")
    step = Step(g, low, stream)
    say(f"[bench] precision form: timing {steps} steps")
    ms, part_ms, _ = time_parts(step, steps, warmup)
    e64 = fp64_step.eps.cpu().numpy()
    e32 = step.eps.cpu().numpy()
    rel = lambda a, b: float(torch.linalg.norm(a.to(b.dtype) - b) / torch.linalg.norm(b))
    res = {
        "workload": workload_label(s) + f", {'complex64' if s.is_complex else 'FP32'} storage",
        "ms_per_step": round(ms, 3), "value": s.nb * s.ng / (ms * 1e-3),
        "fp64_ms_per_step": round(fp64_ms, 3),
        "speedup_vs_fp64": round(fp64_ms / ms, 3),
        "parts_ms": {k: round(v, 4) for k, v in part_ms.items()},
        "max_abs_d_eps_Ha": float(np.abs(e32 - e64).max()),
        "max_abs_eps_Ha": float(np.abs(e64).max()),
        "H_rel": rel(step.H, fp64_step.H), "S_rel": rel(step.S, fp64_step.S),
        "error_reference": "the FP64 step on the same rounded inputs (both paths are "
                           "parity-tested against the oracle; this is their difference)",
    }
    g.close()
    return res


def batched_form(steps, warmup, dev, stream):
    """64 uneven systems (grids 16..48 per axis, 8..96 bands, 2..16 atoms, half
    complex): one tuned graph launch vs the same systems as per-system calls."""
    import torch
    import synth
    import paper_2310_14776_amd as gfd
    systems = [synth.make_system(**c) for c in synth.batched_systems()]
    gs = [gfd.System.from_synth(s) for s in systems]
    psi = [torch.from_numpy(s.psi.reshape(s.nb, -1)).to(dev) for s in systems]
    for s in systems:
        s.psi = None
    outb = [torch.empty_like(p) for p in psi]
    eps = [torch.empty(p.shape[0], dtype=torch.float64, device=dev) for p in psi]
    Pb = [torch.empty((p.shape[0], g.np), dtype=g.dtype, device=dev) for p, g in zip(psi, gs)]
    info = torch.zeros(len(gs), dtype=torch.int32, device=dev)
    batch = gfd.Batch(gs)
    io = batch.io(psi, outb, eps, Pb)
    t0 = time.perf_counter()
    batch.tune(io, info)
    tune_s = time.perf_counter() - t0
    nbr, _ = batch.tuning()
    graph_ms = timed(lambda: batch.step(io, info, stream=stream), stream, steps, warmup)
    if int(info.abs().sum().item()) != 0:
        raise RuntimeError("batched form: eigensolver status")
    work = [Step(g, p, stream) for g, p in zip(gs, psi)]

    def eager():
        for w in work:
            for name, fn in w.parts():
                fn()
    eager_ms = timed(eager, stream, max(1, steps // 2), 1)
    work_units = sum(int(p.shape[0]) * int(p.shape[1]) for p in psi)
    res = {
        "workload": f"{len(gs)} independent systems, grids 16..48 per axis, 8..96 bands, "
                    f"2..16 atoms, {sum(g.dtype == torch.complex128 for g in gs)} complex",
        "graph_ms_per_step": round(graph_ms, 3),
        "per_system_calls_ms_per_step": round(eager_ms, 3),
        "speedup": round(eager_ms / graph_ms, 3),
        "value": work_units / (graph_ms * 1e-3),
        "unit": "band*gridpoints/s",
        "graph_branches": nbr,
        "tune_seconds": round(tune_s, 1),
        "note": "per-system calls use the tuned launch shapes too",
    }
    batch.close()
    for g in gs:
        g.close()
    return res


def other_paths(dev, stream):
    """The rows beside the step, each on a workload of its own: density and
    atomic density matrices and the Davidson correction at 96^3 / 512 bands
    (FP64), the zero-boundary multigrid Poisson solve on a 119x119x159 box,
    and one Crank-Nicolson step of 16 complex bands in a finite 95x95x127
    box with 32 atoms."""
    import torch
    import synth
    import paper_2310_14776_amd as gfd
    out = {}
    s = synth.config_system("C", lazy=True)
    say(f"[bench] density / Davidson correction: {workload_label(s)}")
    g = gfd.System.from_synth(s)
    psi = synth.block_to_device(s, dev, dtype=g.dtype)
    P = g.project(psi)
    f = torch.full((s.nb,), 2.0, dtype=torch.float64, device=dev)
    n_out = torch.empty(s.ng, dtype=torch.float64, device=dev)
    D = torch.empty((s.natoms, g.ni, g.ni), dtype=g.mat_dtype, device=dev)
    ms = timed(lambda: g.density(psi, f, P=P, n_out=n_out, D=D, stream=stream), stream, 5, 1)
    byt = s.nb * s.ng * psi.element_size() + s.ng * 8
    out["density"] = {"workload": workload_label(s), "ms": round(ms, 3),
                      "GBs": round(byt / (ms * 1e-3) / 1e9, 1),
                      "frac_hbm": round(byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
    Hpsi = torch.empty_like(psi)
    Spsi = torch.empty_like(psi)
    g.apply_HS(psi, P, Hpsi=Hpsi, Spsi=Spsi, stream=stream)
    eps = torch.linspace(-1.0, 1.0, s.nb, dtype=torch.float64, device=dev)
    corr = torch.empty_like(psi)
    ms = timed(lambda: g.davidson_correction(Hpsi, Spsi, eps, out=corr, stream=stream), stream, 5, 1)
    byt = 3 * s.nb * s.ng * psi.element_size()
    out["davidson_correction"] = {"workload": workload_label(s), "ms": round(ms, 3),
                                  "GBs": round(byt / (ms * 1e-3) / 1e9, 1),
                                  "frac_hbm": round(byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
    del psi, Hpsi, Spsi, corr, P
    g.close()
    torch.cuda.empty_cache()

    n, h = (119, 119, 159), (0.2, 0.2, 0.2)
    say(f"[bench] Poisson: zero-boundary {n[0]}x{n[1]}x{n[2]} grid")
    x = [np.arange(1, n[c] + 1) * h[c] for c in range(3)]
    rng = np.random.default_rng(7)
    rho = np.zeros(n)
    for _ in range(8):
        c = [(n[i] + 1) * h[i] * rng.uniform(0.3, 0.7) for i in range(3)]
        w = rng.uniform(0.4, 0.9)
        gg = [np.exp(-(x[i] - c[i]) ** 2 / (2 * w * w)) for i in range(3)]
        rho += rng.uniform(-1, 1) * gg[0][:, None, None] * gg[1][None, :, None] * gg[2][None, None, :]
    rho_d = torch.from_numpy(rho).to(dev)
    solver = gfd.Poisson(n, h)
    phi = torch.zeros_like(rho_d)
    res = {}

    def solve():
        phi.zero_()
        res["r"] = solver.solve(rho_d, phi=phi, tol=1e-10, max_cycles=200, stream=stream)
    ms = timed(solve, stream, 3, 1)
    cycles = res["r"][1]
    ng = int(np.prod(n))
    # per V-cycle on the finest level: 4 Jacobi sweeps + 1 residual, each
    # reading two arrays and writing one (24 bytes per point)
    out["poisson"] = {"workload": f"zero-boundary {n[0]}x{n[1]}x{n[2]} grid, h=0.2 bohr, "
                                  f"{solver.levels} levels, 8 Gaussian charges",
                      "ms_per_solve": round(ms, 3), "cycles": cycles,
                      "ms_per_cycle": round(ms / cycles, 4), "rel_residual": res["r"][2],
                      "fine_level_GBs": round(5 * 24 * ng / (ms / cycles * 1e-3) / 1e9, 1)}
    solver.close()
    del rho_d, phi
    torch.cuda.empty_cache()

    s = synth.make_system(n=(95, 95, 127), h=0.2, nb=16, natoms=32, rc=2.0, seed=42,
                          complex_psi=True, bands="smooth", lazy=True)
    say("[bench] Crank-Nicolson step: finite 95x95x127 box, 16 bands, 32 atoms")
    g = gfd.System.from_synth(s, boundary="zero")
    psi = synth.block_to_device(s, dev, dtype=g.dtype)
    g.td_kick(psi, (0.01, 0.0, 0.0), stream=stream)
    it = {}

    def cn():
        it["r"] = g.td_propagate(psi, 0.05, tol=1e-10, max_iter=500, stream=stream)
    ms = timed(cn, stream, 2, 1)
    P = g.project(psi)
    Hp, Sp = torch.empty_like(psi), torch.empty_like(psi)
    ms_hs = timed(lambda: g.apply_HS(psi, P, Hpsi=Hp, Spsi=Sp, stream=stream), stream, 5, 1)
    out["tddft"] = {"workload": "finite 95x95x127 box, h=0.2 bohr, 16 complex128 bands, "
                                "32 atoms, dt=0.05 au, tol 1e-10",
                    "ms_per_step": round(ms, 3), "cocg_iterations": it["r"][0],
                    "ms_per_iteration": round(ms / max(1, it["r"][0] + 1), 3),
                    "apply_HS_ms": round(ms_hs, 3)}
    g.close()
    return out


def cpu_baseline(name, budget_s, nb_sample):
    """The oracle (sparse projector matrix) on the first nb_sample bands of
    the same system: full oracle steps, timed on this host."""
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    cores = min(threads, len(os.sched_getaffinity(0)))
    s = synth.config_system(name, nb=nb_sample)
    t0 = time.perf_counter()
    ops = oracle.Operators.from_system(s, sparse=True)
    t_setup = time.perf_counter() - t0
    reps, t_steps = 0, 0.0
    while reps == 0 or (t_steps < budget_s and reps < 50):
        t1 = time.perf_counter()
        oracle.fd_step(s, ops)
        t_steps += time.perf_counter() - t1
        reps += 1
    per_step = t_steps / reps
    return {"value": s.nb * s.ng / per_step, "unit": "band*gridpoints/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} full oracle steps on bands 0..{s.nb - 1} of the same "
                      f"{s.n[0]}x{s.n[1]}x{s.n[2]} system (sparse projector matrix, built in "
                      f"{t_setup:.1f}s, excluded), {per_step * 1e3:.0f} ms/step"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2310_14776_amd as gfd

    if not os.path.exists(gfd.library_path()):
        from paper_2310_14776_amd.build import build
        build()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    forms = not args.no_forms

    say("[bench] measured ceilings (copy and matrix-core probes)")
    peaks = measured_peaks(dev, stream)
    res, s, step, low = run_config(args.config, args.steps, args.warmup, dev, stream,
                                   single_inputs=forms, do_tune=not args.no_tune, peaks=peaks)
    out = {
        "metric": "band*gridpoints/s for H|psi>+subspace step",
        "value": res["value"],
        "unit": "band*gridpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "wall_s": res["wall_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res["dtype"],
        "data": "synthetic (seeded; values rounded to single precision so that the "
                "precision form sees the same block)" if forms else "synthetic (seeded)",
        "config": {"workload": res["workload"], "grid": list(s.n), "bands": s.nb,
                   "atoms": s.natoms, "k": list(s.k), "parallelism": "single GPU"},
        "parts": res["parts"],
        "launch_tuning": res["launch_tuning"],
        "roofline": res["roofline"],
        "measured_peaks": peaks,
    }
    fp64_ms = res["ms_per_step"]
    # the FP64 step ran on the rounded block: its eps, H and S are the error
    # reference of the precision form; its grid buffers are freed first
    for attr in ("psi", "Hpsi", "Spsi", "psi_rot"):
        setattr(step, attr, None)
    step.g.close()
    torch.cuda.empty_cache()
    if args.calib_copy:
        xa = torch.empty(32 << 20, dtype=torch.float64, device=dev)
        xb = torch.empty_like(xa)
        for _ in range(3):
            xb.copy_(xa)
        torch.cuda.synchronize()
        del xa, xb
    if forms:
        out["forms"] = {"precision": precision_form(s, low, step, fp64_ms,
                                                    max(2, min(args.steps, 10)), 1, dev, stream)}
        del low
        torch.cuda.empty_cache()
        if not args.no_batched:
            out["forms"]["batched"] = batched_form(max(3, min(args.steps, 10)), 2, dev, stream)
    del step
    torch.cuda.empty_cache()
    if not args.no_extra:
        extra = {}
        for name in ("B", "C"):
            if name == args.config:
                continue
            r, _, st, _ = run_config(name, max(5, args.steps), 2, dev, stream, peaks=peaks)
            st.g.close()
            del st
            torch.cuda.empty_cache()
            extra[name] = {k: r[k] for k in ("workload", "dtype", "ms_per_step", "value",
                                             "parts", "roofline", "launch_tuning")}
        out["extra_workloads"] = extra
        out["other_paths"] = other_paths(dev, stream)
    if not args.no_cpu:
        say("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_seconds,
                                           nb_sample=8 if s.nb >= 512 else s.nb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
