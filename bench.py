#!/usr/bin/env python3
"""Benchmark: one FD-PAW block eigensolver step per iteration on one MI355X.

Step = projections, H~psi, S~psi, subspace matrices H_nm/S_nm, FP64
Cholesky + generalised eigensolve, rotation of the block and its projections.
Workload: periodic 48^3 grid, h = 0.18 bohr, 128 bands, 16 atoms with 13
projectors each (rc = 2.2 bohr), FP64 real; seeded synthetic inputs already
resident in HBM when the timed region starts.

Prints one JSON line with the throughput (band*gridpoints/s), per-part times,
the roofline of the dominant kernel and the CPU oracle timed on this host.
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="B")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision-form and batched-form measurements")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, run a plain 256 MiB device copy three times "
                         "(reference kernel for hardware byte counters)")
    return ap.parse_args()


# kernels behind each timed call, and the sources they are built from
PART_KERNELS = {
    "project": (["k_project"], ["csrc/nonlocal.hip", "csrc/proj.h"]),
    # H~psi and S~psi in one pass: Delta H.P and Delta S.P (one launch), then the stencil
    "apply_HS": (["k_dmat2", "k_stencil"],
                 ["csrc/stencil.hip", "csrc/nonlocal.hip", "csrc/proj.h"]),
    "subspace": (["k_subspace", "k_subspace_reduce"], ["csrc/gemm.hip"]),
    # the block and its projections
    "rotate": (["k_rotate", "k_rot_small"], ["csrc/gemm.hip"]),
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


def precision_form(steps, warmup):
    """FP64 step vs the precision form (single-precision storage, split-BF16
    products, FP64 eigensolve, Cholesky orthonormality correction of the
    stored rotated block) on the same FP32-rounded 96^3, 512-band, 64-atom
    block."""
    import torch
    import synth
    import paper_2310_14776_amd as gfd
    s = synth.config_system("C")
    nb, ng = s.nb, s.ng
    psi32_h = s.psi.reshape(nb, ng).astype(np.float32)
    s.psi = None
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    out = {}
    results = {}
    tuned = {}
    for prec in ("double", "single"):
        g = gfd.System(s.n, s.h, s.k, s.pos, s.channels, s.dH, s.dS, s.v, nb, complex_=False,
                       precision=prec)
        psi = torch.from_numpy(psi32_h).to(dev)
        if prec == "double":
            psi = psi.double()
        P = torch.empty((nb, g.np), dtype=g.dtype, device=dev)
        Hpsi, Spsi, psi_rot, Spsi_rot, psi_fin = (torch.empty_like(psi) for _ in range(5))
        H = torch.empty((nb, nb), dtype=g.mat_dtype, device=dev)
        S, C = torch.empty_like(H), torch.empty_like(H)
        eps = torch.empty(nb, dtype=torch.float64, device=dev)
        P_rot, P_fin = torch.empty_like(P), torch.empty_like(P)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        # both forms run with the launch shapes the library's autotuner picks
        tb = gfd.Batch([g])
        tb.tune(tb.io([psi], [psi_rot], [eps]), info)
        t = tb.tuning()[1][0]
        # single-precision systems have fixed launch shapes (all knobs report 0)
        tuned[prec] = t if any(t.values()) else "fixed"
        tb.close()
        torch.cuda.synchronize()

        def step():
            g.project(psi, out=P, stream=stream)
            g.apply_HS(psi, P, Hpsi=Hpsi, Spsi=Spsi, stream=stream)
            g.subspace_matrices(psi, Hpsi, Spsi, H=H, S=S, stream=stream)
            g.subspace_diag(H, S, eps=eps, C=C, info=info, stream=stream)
            g.rotate(psi, C, out=psi_rot, P=P, P_out=P_rot, stream=stream)
            if prec == "single":
                # S~ applied to the stored rotated block (its projections are
                # the rotated P), then the Cholesky correction
                g.apply_S(psi_rot, P_rot, out=Spsi_rot, stream=stream)
                g.orthonormalize(psi_rot, Spsi_rot, out=psi_fin, P=P_rot, P_out=P_fin,
                                 info=info, stream=stream)
        ms = timed(step, stream, steps, warmup)
        if int(info.item()) != 0:
            raise RuntimeError(f"precision form: eigensolver status {int(info.item())}")
        results[prec] = dict(ms=ms, eps=eps.cpu().numpy(), H=H.cpu().numpy(), S=S.cpu().numpy(),
                             psi_fin=psi_fin if prec == "single" else None, g=g)
        out[prec] = dict(ms_per_step=round(ms, 3), value=nb * ng / (ms * 1e-3),
                         launch_tuning=tuned[prec])
        del Hpsi, Spsi, psi_rot, Spsi_rot, P, P_rot, P_fin
        if prec == "single":
            del psi
        torch.cuda.empty_cache()
    # overlap of the corrected single-precision block, measured with the FP64 operators
    g64 = results["double"]["g"]
    pf = results["single"]["psi_fin"].double()
    Sf = g64.apply_S(pf)
    Hf = g64.apply_H(pf)
    H1, S1 = g64.subspace_matrices(pf, Hf, Sf)
    torch.cuda.synchronize()
    e64, e32 = results["double"]["eps"], results["single"]["eps"]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    res = {
        "workload": f"periodic {s.n[0]}x{s.n[1]}x{s.n[2]} grid h={s.h[0]} bohr, {nb} bands, "
                    f"{s.natoms} atoms x 13 projectors, real, inputs rounded to FP32",
        "fp64": out["double"], "single_split_bf16": out["single"],
        "speedup": round(results["double"]["ms"] / results["single"]["ms"], 3),
        "max_abs_d_eps_Ha": float(np.abs(e32 - e64).max()),
        "max_abs_eps_Ha": float(np.abs(e64).max()),
        "H_rel": rel(results["single"]["H"], results["double"]["H"]),
        "S_rel": rel(results["single"]["S"], results["double"]["S"]),
        "final_S_minus_I": float((S1.cpu() - torch.eye(nb, dtype=torch.float64)).abs().max()),
        "error_reference": "FP64 GPU path on the same rounded inputs (parity-tested to 1e-12)",
    }
    for r in results.values():
        r["g"].close()
    return res


def batched_form(steps, warmup):
    """64 uneven systems (grids 16..48 per axis, 8..96 bands, 2..16 atoms, half
    complex): one tuned graph launch vs the same systems as per-system calls."""
    import torch
    import synth
    import paper_2310_14776_amd as gfd
    systems = [synth.make_system(**c) for c in synth.batched_systems()]
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
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
    # the same work as separate calls, one system after another on one stream
    work = []
    for g, p in zip(gs, psi):
        nb = p.shape[0]
        work.append(dict(g=g, psi=p, P=torch.empty((nb, g.np), dtype=g.dtype, device=dev),
                         Hpsi=torch.empty_like(p), Spsi=torch.empty_like(p),
                         H=torch.empty((nb, nb), dtype=g.mat_dtype, device=dev),
                         S=torch.empty((nb, nb), dtype=g.mat_dtype, device=dev),
                         C=torch.empty((nb, nb), dtype=g.mat_dtype, device=dev),
                         eps=torch.empty(nb, dtype=torch.float64, device=dev),
                         out=torch.empty_like(p),
                         Pr=torch.empty((nb, g.np), dtype=g.dtype, device=dev)))

    def eager():
        for w in work:
            g = w["g"]
            g.project(w["psi"], out=w["P"], stream=stream)
            g.apply_H(w["psi"], w["P"], out=w["Hpsi"], stream=stream)
            g.apply_S(w["psi"], w["P"], out=w["Spsi"], stream=stream)
            g.subspace_matrices(w["psi"], w["Hpsi"], w["Spsi"], H=w["H"], S=w["S"], stream=stream)
            g.subspace_diag(w["H"], w["S"], eps=w["eps"], C=w["C"], info=info, stream=stream)
            g.rotate(w["psi"], w["C"], out=w["out"], P=w["P"], P_out=w["Pr"], stream=stream)
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


def part_costs(s, info):
    """Algorithmic bytes and flops per launch of each part (FP64, 8 B)."""
    nb, ng, npj, ni = s.nb, s.ng, info["np"], info["ni"]
    ent = info["entries"]
    es = 16 if s.is_complex else 8
    return {
        # gather psi at every sphere entry, read the projector table once, write P
        "project": dict(bytes=ent * nb * es + ent * (ni * es + 4) + nb * npj * es,
                        flops=2 * ent * ni * nb),
        # read psi, write H~psi and S~psi, read v and the add-back tables once
        "apply_HS": dict(bytes=3 * nb * ng * es + ng * 8 + info["covered"] * 8
                         + ent * (ni * es + 4), flops=0),
        # read psi, H~psi, S~psi; two Hermitian nb x nb products over Ng, of
        # which the nb (nb + 1) / 2 entries on and above the diagonal are
        # needed (real FP64 flops: 2 per multiply-add, 4 times that complex)
        "subspace": dict(bytes=3 * nb * ng * es, flops=2 * nb * (nb + 1) * ng * (4 if s.is_complex else 1)),
        "diag": dict(bytes=0, flops=0),
        # read psi, write psi'; nb x nb times nb x (Ng + Np)
        "rotate": dict(bytes=2 * nb * (ng + npj) * es,
                       flops=2 * nb * nb * (ng + npj) * (4 if s.is_complex else 1)),
    }


def cpu_baseline(s, budget_s):
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    cores = min(threads, len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    ops = oracle.Operators.from_system(s)
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
            "sample": f"{reps} full oracle steps of the same {s.n[0]}x{s.n[1]}x{s.n[2]} "
                      f"{s.nb}-band system (projector matrix build {t_setup:.1f}s excluded), "
                      f"{per_step * 1e3:.0f} ms/step"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2310_14776_amd as gfd

    if not os.path.exists(gfd.library_path()):
        from paper_2310_14776_amd.build import build
        build()
    s = synth.config_system(args.config)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sysg = gfd.System.from_synth(s)
    nb, ng, npj = s.nb, s.ng, sysg.np
    dt = sysg.dtype
    psi = torch.from_numpy(s.psi.reshape(nb, ng)).to(dev)
    P = torch.empty((nb, npj), dtype=dt, device=dev)
    Hpsi = torch.empty_like(psi)
    Spsi = torch.empty_like(psi)
    H = torch.empty((nb, nb), dtype=dt, device=dev)
    S = torch.empty_like(H)
    eps = torch.empty(nb, dtype=torch.float64, device=dev)
    C = torch.empty_like(H)
    psi_rot = torch.empty_like(psi)
    P_rot = torch.empty_like(P)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    # launch shapes from the library's autotuner (kept in the system; every
    # choice computes the same results)
    tb = gfd.Batch([sysg])
    tio = tb.io([psi], [psi_rot], [eps])
    tb.tune(tio, info)
    tuning = tb.tuning()
    tb.close()
    torch.cuda.synchronize()

    parts = [
        ("project", lambda: sysg.project(psi, out=P, stream=stream)),
        ("apply_HS", lambda: sysg.apply_HS(psi, P, Hpsi=Hpsi, Spsi=Spsi, stream=stream)),
        ("subspace", lambda: sysg.subspace_matrices(psi, Hpsi, Spsi, H=H, S=S, stream=stream)),
        ("diag", lambda: sysg.subspace_diag(H, S, eps=eps, C=C, info=info, stream=stream)),
        ("rotate", lambda: sysg.rotate(psi, C, out=psi_rot, P=P, P_out=P_rot, stream=stream)),
    ]

    for _ in range(args.warmup):
        for _, fn in parts:
            fn()
    torch.cuda.synchronize()

    ev = {name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)] for name, _ in parts}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        for name, fn in parts:
            a, b = ev[name][k]
            a.record(stream)
            fn()
            b.record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    if int(info.item()) != 0:
        raise RuntimeError(f"eigensolver status {int(info.item())}")

    ms_step = start.elapsed_time(stop) / args.steps
    part_ms = {name: float(np.mean([a.elapsed_time(b) for a, b in ev[name]])) for name, _ in parts}
    value = nb * ng / (ms_step * 1e-3)

    costs = part_costs(s, sysg.info)
    rows = {}
    for name, ms in part_ms.items():
        c = costs[name]
        t = ms * 1e-3
        rows[name] = dict(ms=round(ms, 4),
                          GBs=round(c["bytes"] / t / 1e9, 1) if c["bytes"] else None,
                          TFLOPs=round(c["flops"] / t / 1e12, 2) if c["flops"] else None)
    # dominant kernel: the costliest part with a bandwidth or matrix-core roofline
    dom = max((n for n in part_ms if costs[n]["bytes"] or costs[n]["flops"]), key=part_ms.get)
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
    roof["traffic"] = measured_traffic(dom, f"{s.n[0]}x{s.n[1]}x{s.n[2]}_nb{nb}")

    out = {
        "metric": "band*gridpoints/s for H|psi>+subspace step",
        "value": value,
        "unit": "band*gridpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FD-PAW block step, periodic {s.n[0]}x{s.n[1]}x{s.n[2]} grid "
                               f"h={s.h[0]} bohr, {nb} bands, {s.natoms} atoms x 13 projectors, "
                               f"FP64 real",
                   "grid": list(s.n), "bands": nb, "atoms": s.natoms, "parallelism": "single GPU"},
        "parts": rows,
        "launch_tuning": tuning[1][0] if tuning else None,
        "roofline": roof,
    }
    sysg.close()
    del psi, Hpsi, Spsi, psi_rot, P, P_rot
    torch.cuda.empty_cache()
    if args.calib_copy:
        xa = torch.empty(32 << 20, dtype=torch.float64, device=dev)
        xb = torch.empty_like(xa)
        for _ in range(3):
            xb.copy_(xa)
        torch.cuda.synchronize()
        del xa, xb
    if not args.no_forms:
        forms_steps = max(3, min(args.steps, 10))
        out["forms"] = {"precision": precision_form(forms_steps, 2),
                        "batched": batched_form(forms_steps, 2)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
