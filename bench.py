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
    return ap.parse_args()


def part_costs(s, info):
    """Algorithmic bytes and flops per launch of each part (FP64, 8 B)."""
    nb, ng, npj, ni = s.nb, s.ng, info["np"], info["ni"]
    ent = info["entries"]
    es = 16 if s.is_complex else 8
    return {
        # gather psi at every sphere entry, read the projector table once, write P
        "project": dict(bytes=ent * nb * es + ent * (ni * es + 4) + nb * npj * es,
                        flops=2 * ent * ni * nb),
        # read psi, write H~psi, read v and the add-back tables once
        "apply_H": dict(bytes=2 * nb * ng * es + ng * 8 + info["covered"] * 8
                        + ent * (ni * es + 4), flops=0),
        "apply_S": dict(bytes=2 * nb * ng * es + info["covered"] * 8 + ent * (ni * es + 4),
                        flops=0),
        # read psi, H~psi, S~psi; two full nb x nb products over Ng
        "subspace": dict(bytes=3 * nb * ng * es, flops=2 * 2 * nb * nb * ng),
        "diag": dict(bytes=0, flops=0),
        # read psi, write psi'; nb x nb times nb x (Ng + Np)
        "rotate": dict(bytes=2 * nb * (ng + npj) * es, flops=2 * nb * nb * (ng + npj)),
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
        print("bench.py measures one GPU: this build has no multi-GPU path "
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

    parts = [
        ("project", lambda: sysg.project(psi, out=P, stream=stream)),
        ("apply_H", lambda: sysg.apply_H(psi, P, out=Hpsi, stream=stream)),
        ("apply_S", lambda: sysg.apply_S(psi, P, out=Spsi, stream=stream)),
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
    roof["kernel"] = dom
    roof["traffic"] = None

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
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    sysg.close()


if __name__ == "__main__":
    main()
