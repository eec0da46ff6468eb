#!/usr/bin/env python3
"""Benchmark of the ghost-penalty apply y = G(gamma) u on one MI355X.

Default workload: 3D Q5 on GLL nodes, 128^3 cells of [-1,1]^3 cut by a ball of
radius 0.73 (122,353 ghost faces, 396 patch DoFs per face), u ~ U[-1,1] from
seed 1, gamma_j = 0.5 h^{2j-1}/(j!)^2.  One step = one FP64 accumulating apply
(gather, normal contraction, tangential masses, expansion, scatter) over every
ghost face.  The FP32 apply is timed the same way and reported with its
normwise error against the FP64 result.

Prints ONE JSON line.  Metric: ghost-face patch DoFs per second,
faces * (2k+1)(k+1)^{d-1} / t / 1e9.  The roofline object refers to the box
kernel (the dominant kernel of an apply; the halo pass that follows it adds
the other boxes' parts at nodes shared between boxes): its algorithmic HBM
bytes per launch (read u, read and write y on the support: 24 B per support
DoF in FP64) over its average launch duration, measured with HIP events that
the library records on the apply's stream around each kernel during a second
pass of the same length (the headline step time comes from a pass without
them).  apply_roofline_frac gives the same ratio for the whole apply.  Extra
fields: the overwrite mode, and the applies captured in a HIP graph and
replayed (no launch gaps).
"""

import argparse
import hashlib
import json
import os
import platform
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(ROOT, "paper_2503_00246_amd", "csrc", "ghost_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ball3d_q5_128")
    ap.add_argument("--scatter", default="box", choices=["box", "atomic", "coloured"])
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one plain device copy of u (known bytes) to scale PMC byte counters")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--sweep", action="store_true", help="one JSON line per degree/mesh of the roofline sweep")
    ap.add_argument("--mode", default="apply", choices=["apply", "vjp", "cg", "balls", "micro", "cell", "macro"],
                    help="apply: the benchmark line; vjp: ghost_vjp on ball3d_q4_96; cg: FP64 vs mixed CG on "
                         "ball3d_q7_96; balls: the multiple-ball problem, throughput against the cut fraction; "
                         "micro: the single-face compute-bound microbenchmark, d = 2, 3 and k = 1..7; "
                         "cell: the interior-cell Laplacian and (K_inside + G) u on the workload; "
                         "macro: the macro-patch stabilisation against the derivative form, k = 3..7, and its "
                         "VJP (extra lines, not the benchmark metric)")
    ap.add_argument("--balls-k", type=int, default=3, help="degree of the multiple-ball problem")
    ap.add_argument("--balls-n", type=int, default=128, help="cells per axis of the multiple-ball problem")
    ap.add_argument("--cg-max-iter", type=int, default=5000)
    ap.add_argument("--traffic", default=TRAFFIC_FILE, help="JSON file with measured HBM bytes per launch")
    return ap.parse_args()


def timed_applies(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3 / steps  # seconds per step


def cpu_baseline(w, u_np, budget_s=10.0):
    """The oracle's apply on the same workload, repeated for about budget_s on the host cores.

    The oracle's own set-up (classification, face set, quadrature assembly of the patch matrices)
    is excluded; each repetition is one full apply (gather, dense patch matvec by BLAS, scatter-add).
    """
    from threadpoolctl import threadpool_info
    from oracle.operator import GhostOracle
    t_setup = time.perf_counter()
    o = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), centre=w.centre, radius=w.radius)
    t_setup = time.perf_counter() - t_setup
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    reps, t0 = 0, time.perf_counter()
    while True:
        o.apply(u_np)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    faces = o.n_faces()
    return {"value": round(reps * faces * w.n_p / dt / 1e9, 6), "unit": "GDoF/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} full oracle applies of {w.name} ({faces} faces each: dense per-face patch matvec "
                      f"by BLAS + scatter-add) in {dt:.1f} s (oracle set-up, timed apart: {t_setup:.1f} s); host "
                      f"{cpu_model()}, {os.cpu_count()} logical CPUs, BLAS threads {threads}"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def graph_time(fn, steps, repeats=10):
    """Seconds per apply from HIP events around a graph of `steps` captured applies: the median of
    `repeats` replays (no launch gaps between the applies)."""
    import statistics
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(steps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        g.replay()
        end.record()
        torch.cuda.synchronize()
        times.append(start.elapsed_time(end) / 1e3 / steps)
    del g
    return statistics.median(times)


def run_workload(w, args, with_cpu, penalty="derivative"):
    import numpy as np
    import torch
    from paper_2503_00246_amd.operator import GhostOperator
    from paper_2503_00246_amd.workloads import SEED_U, uniform_vector

    op = GhostOperator.from_workload(w, scatter=args.scatter, penalty=penalty)
    st = op.stats
    u_np = uniform_vector(w.n_lattice, SEED_U)
    u = torch.from_numpy(u_np).cuda()
    y = torch.zeros_like(u)

    def timed(fn):
        # the applies are timed without the library's per-kernel events (which add work of their own);
        # a second pass of the same length records them, for the box kernel's and the halo pass's times
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = timed_applies(fn, args.steps, 0)
        op.kernel_times()  # drop anything recorded before
        op.set_timing(True)
        timed_applies(fn, args.steps, 0)
        op.set_timing(False)
        kt = op.kernel_times()
        return t, kt["main_ms"] / 1e3 / kt["calls"], kt["halo_ms"] / 1e3 / kt["calls"]

    t64, box64, halo64 = timed(lambda: op.apply(u, y, accumulate=True))
    patch_dofs = st["n_faces_total"] * st["n_patch_dofs"]
    out = {"t64": t64, "box64": box64, "halo64": halo64, "gdofs64": patch_dofs / t64 / 1e9, "stats": st}
    if not args.sweep:
        t64o, _, _ = timed(lambda: op.apply(u, y, accumulate=False))
        out["t64_overwrite"] = t64o
        out["t64_graph"] = graph_time(lambda: op.apply(u, y, accumulate=True), args.steps)
    if not args.no_fp32:
        u32 = u.float()
        y32 = torch.zeros_like(u32)
        t32, box32, halo32 = timed(lambda: op.apply_f32(u32, y32, accumulate=True))
        ref = op.apply(u)
        got = op.apply_f32(u32).double()
        err = float((got - ref).abs().max() / ref.abs().max())
        out.update(t32=t32, box32=box32, halo32=halo32, gdofs32=patch_dofs / t32 / 1e9, err32=err)
    if args.calibrate:
        c = torch.empty_like(u)
        c.copy_(u)  # one plain copy: n_lattice * 8 bytes read and written
        torch.cuda.synchronize()
        out["copy_bytes"] = 8 * w.n_lattice
    if not args.sweep:
        # a plain device copy of u (read and write of the whole lattice), for the attainable HBM rate
        c = torch.empty_like(u)
        t_copy = timed_applies(lambda: c.copy_(u), 20, 3)
        out["copy_GBps"] = 2 * 8 * w.n_lattice / t_copy / 1e9
        del c
    if with_cpu:
        out["cpu"] = cpu_baseline(w, u_np)
    del u, y
    torch.cuda.empty_cache()
    return out


def run_vjp(w, args, penalty="derivative"):
    """ghost_vjp (du = G w and dgamma) timed like the apply; box-kernel bytes: u and w read on the
    support, du written on the exclusive nodes (overwrite mode)."""
    import torch
    from paper_2503_00246_amd.operator import GhostOperator
    from paper_2503_00246_amd.workloads import SEED_T, SEED_U, uniform_vector

    op = GhostOperator.from_workload(w, scatter=args.scatter, penalty=penalty)
    st = op.stats
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    wv = torch.from_numpy(uniform_vector(w.n_lattice, SEED_T)).cuda()
    du = torch.zeros_like(u)
    fn = lambda: op.vjp(u, wv, du=du, accumulate=False)
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t = timed_applies(fn, args.steps, 0)  # without the per-kernel events; a second pass records them
    op.kernel_times()
    op.set_timing(True)
    timed_applies(fn, args.steps, 0)
    op.set_timing(False)
    kt = op.kernel_times()
    box_t = kt["main_ms"] / 1e3 / kt["calls"]
    alg = 24 * st["n_support_dofs"]  # u and w read, du written on the support
    print(json.dumps({"metric": "ghost_vjp patch DoFs/s (GDoF/s), FP64", "workload": w.name, "penalty": penalty,
                      "value": round(st["n_faces_total"] * st["n_patch_dofs"] / t / 1e9, 4), "unit": "GDoF/s",
                      "ms_per_step": round(t * 1e3, 5), "steps": args.steps,
                      "box_kernel_us": round(box_t * 1e6, 2), "halo_pass_us": round(kt["halo_ms"] / kt["calls"] * 1e3, 2),
                      "roofline": {"bound": "hbm", "achieved": round(alg / box_t / 1e9, 2), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(alg / box_t / 1e9 / HBM_PEAK_GBS, 4),
                                   "bytes_per_launch": alg}}), flush=True)


def run_cg(w, args):
    """(M_h + G) x = b to a relative true residual of 1e-10: pure FP64 CG vs FP64-outer / FP32-inner CG,
    unpreconditioned and with the Jacobi preconditioner (one JSON line per preconditioner)."""
    import time as _time
    import torch
    from paper_2503_00246_amd.operator import GhostOperator
    from paper_2503_00246_amd.workloads import SEED_B, uniform_vector

    op = GhostOperator.from_workload(w, scatter=args.scatter)
    diag = op.mass_diag()
    b = torch.from_numpy(uniform_vector(w.n_lattice, SEED_B)).cuda()
    b = torch.where(diag > 0, b, torch.zeros_like(b))
    for precond in ("none", "jacobi"):
        out = {"metric": "CG on (M_h + G) x = b to 1e-10 relative true residual", "workload": w.name,
               "precond": precond, "active_dofs": int((diag > 0).sum()), "max_iter": args.cg_max_iter}
        for mode in ("fp64", "mixed"):
            op.cg(b, mode=mode, tol=1e-4, max_iter=20, precond=precond)  # warm-up: workspace, kernels
            torch.cuda.synchronize()
            t0 = _time.perf_counter()
            x, res = op.cg(b, mode=mode, tol=1e-10, max_iter=args.cg_max_iter, precond=precond)
            torch.cuda.synchronize()
            out[mode] = {"seconds": round(_time.perf_counter() - t0, 4), **res}
        out["mixed_speedup"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
        print(json.dumps(out), flush=True)


def run_cell(w, args):
    """The interior-cell Laplacian (y += K_inside u) and the operator without its cut-cell part,
    (K_inside + G) u, timed like the apply.  Metrics: cell DoFs per second (inside cells x (k+1)^d / t)
    and, for the whole operator, active DoFs per second; bytes: 24 per inside node (u read, y read and
    written) for the cell operator."""
    import torch
    from paper_2503_00246_amd.operator import GhostOperator
    from paper_2503_00246_amd.workloads import SEED_U, uniform_vector
    op = GhostOperator.from_workload(w, scatter=args.scatter)
    st = op.stats
    n_inside = st["n_active_cells"] - st["n_cut_cells"]
    cell_dofs = n_inside * (w.k + 1) ** w.d
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    out = {"metric": "interior-cell Laplacian and (K_inside + G) u", "workload": w.name, "inside_cells": n_inside,
           "inside_dofs": st["n_inside_dofs"], "active_dofs": st["n_active_dofs"], "steps": args.steps}
    for dt, key, elem in ((torch.float64, "fp64", 8), (torch.float32, "fp32", 4)):
        uu = u.to(dt)
        y = torch.zeros_like(uu)
        t_cell = timed_applies(lambda: op.cell_apply(uu, y), args.steps, args.warmup)
        if dt == torch.float64:
            t_sys = timed_applies(lambda: (op.cell_apply(uu, y), op.apply(uu, y, accumulate=True)), args.steps,
                                  args.warmup)
        else:
            t_sys = timed_applies(lambda: (op.cell_apply(uu, y), op.apply_f32(uu, y, accumulate=True)), args.steps,
                                  args.warmup)
        alg = 3 * elem * st["n_inside_dofs"]
        out[key] = {"cell_ms": round(t_cell * 1e3, 5), "cell_gdofs": round(cell_dofs / t_cell / 1e9, 3),
                    "cell_GBps": round(alg / t_cell / 1e9, 1), "cell_frac": round(alg / t_cell / 1e9 / HBM_PEAK_GBS, 4),
                    "system_ms": round(t_sys * 1e3, 5),
                    "system_active_gdofs": round(st["n_active_dofs"] / t_sys / 1e9, 3)}
        del uu, y
    print(json.dumps(out), flush=True)


def run_micro(args, blocks=2048, reps=100):
    """Single-face microbenchmark: `blocks` workgroups of faces, each face's operator applied `reps`
    times to resident values (no gather, no scatter); time per face application, flop rate against the
    vector peak of the precision, and the time relative to k = 1 (the paper's presentation)."""
    import torch
    from paper_2503_00246_amd.operator import GhostOperator
    from paper_2503_00246_amd.workloads import gamma_paper
    peak = {torch.float64: 78.6e12, torch.float32: 157.3e12}
    for d in (2, 3):
        base = {}
        for k in range(1, 8):
            h = 0.25
            op = GhostOperator(d, (8,) * d, (-1.0,) * d, h, k, gamma_paper(k, h),
                               centre=(0.011, 0.017, 0.023)[:d], radius=0.73)
            nn, tl = 2 * k + 1, (k + 1) ** (d - 1)
            nf = blocks * 8 * (64 // tl)
            flops = op.stats["flops_per_face"]
            line = {"metric": "single-face ghost-penalty application (compute-bound microbenchmark)",
                    "d": d, "k": k, "faces": nf, "reps": reps, "flops_per_face": flops}
            for dt in (torch.float64, torch.float32):
                x = torch.rand((nf, nn, tl), dtype=dt, device="cuda") * 2 - 1
                y = torch.empty_like(x)
                op.face_bench(x, y, reps=reps)
                torch.cuda.synchronize()
                start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                start.record()
                op.face_bench(x, y, reps=reps)
                end.record()
                torch.cuda.synchronize()
                t = start.elapsed_time(end) / 1e3
                per = t / (nf * reps)
                key = "fp64" if dt == torch.float64 else "fp32"
                base.setdefault(key, per)
                line[key] = {"ns_per_face": round(per * 1e9, 5), "tflops": round(flops / per / 1e12, 3),
                             "frac_of_vector_peak": round(flops / per / peak[dt], 4),
                             "relative_to_k1": round(per / base[key], 3)}
                del x, y
            print(json.dumps(line), flush=True)
            del op
            torch.cuda.empty_cache()


def run_balls(args):
    """The multiple-ball problem: one line per ball count, with the cut fraction of the active cells."""
    from paper_2503_00246_amd.workloads import multiball_workload
    args.sweep = True  # one line per workload: no overwrite or graph timings
    for nb in (1, 2, 4, 8, 16, 32, 64):
        w = multiball_workload(args.balls_k, args.balls_n, nb)
        r = run_workload(w, args, with_cpu=False)
        st = r["stats"]
        print(json.dumps({"metric": "ghost-face patch DoFs/s (GDoF/s), multiple-ball problem", "workload": w.name,
                          "balls": nb, "radius": w.radius, "active_cells": st["n_active_cells"],
                          "cut_cells": st["n_cut_cells"], "cut_fraction": st["n_cut_cells"] / max(1, st["n_active_cells"]),
                          "faces": st["n_faces_total"], "support_dofs": st["n_support_dofs"],
                          "ms64": r["t64"] * 1e3, "gdofs64": r["gdofs64"], "box_ms64": r["box64"] * 1e3,
                          "box_frac64": box_bytes(st, 8) / r["box64"] / 1e9 / HBM_PEAK_GBS,
                          "ms32": r.get("t32", 0) * 1e3, "gdofs32": r.get("gdofs32"), "err32": r.get("err32")}),
              flush=True)


def run_macro(args):
    """The macro-patch stabilisation against the derivative-jump penalty on the same meshes: one line per
    degree, both forms timed like the apply (the same box layout, bytes and faces; the macro form adds
    the k x k order coupling per tangential line)."""
    from paper_2503_00246_amd.workloads import sweep_workload
    args.sweep = True  # one line per workload: no overwrite or graph timings
    for k, n in [(3, 128), (4, 96), (5, 128), (6, 96), (7, 96)]:
        w = sweep_workload(k, n)
        line = {"metric": "ghost-face patch DoFs/s (GDoF/s), macro-patch vs derivative-jump form",
                "workload": w.name}
        for pen in ("macro", "derivative"):
            r = run_workload(w, args, with_cpu=False, penalty=pen)
            st = r["stats"]
            line[pen] = {"ms64": round(r["t64"] * 1e3, 5), "gdofs64": round(r["gdofs64"], 2),
                         "box_ms64": round(r["box64"] * 1e3, 5),
                         "box_frac64": round(box_bytes(st, 8) / r["box64"] / 1e9 / HBM_PEAK_GBS, 4),
                         "ms32": round(r.get("t32", 0) * 1e3, 5), "gdofs32": round(r.get("gdofs32", 0), 2),
                         "err32": r.get("err32")}
        line["faces"], line["n_p"] = st["n_faces_total"], st["n_patch_dofs"]
        print(json.dumps(line), flush=True)
    from paper_2503_00246_amd.workloads import WORKLOADS
    for pen in ("macro", "derivative"):
        run_vjp(WORKLOADS["ball3d_q4_96"], args, penalty=pen)


def box_bytes(st, elem):
    """Algorithmic bytes of one accumulating box-kernel launch: u on the support, and y read and written
    on the support (every support node is written to y by exactly one box, the first that touches it;
    the halo pass then adds the other boxes' parts at the shared nodes)."""
    return 3 * elem * st["n_support_dofs"]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is a "
              f"design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2503_00246_amd.workloads import WORKLOADS, sweep_workload

    if args.mode == "vjp":
        run_vjp(WORKLOADS["ball3d_q4_96" if args.workload == "ball3d_q5_128" else args.workload], args)
        return
    if args.mode == "cg":
        run_cg(WORKLOADS["ball3d_q7_96" if args.workload == "ball3d_q5_128" else args.workload], args)
        return
    if args.mode == "balls":
        run_balls(args)
        return
    if args.mode == "micro":
        run_micro(args)
        return
    if args.mode == "cell":
        run_cell(WORKLOADS[args.workload], args)
        return
    if args.mode == "macro":
        run_macro(args)
        return
    if args.sweep:
        for k, n in [(3, 128), (3, 96), (4, 96), (5, 96), (5, 128), (6, 96), (7, 96)]:
            w = sweep_workload(k, n)
            r = run_workload(w, args, with_cpu=False)
            st = r["stats"]
            print(json.dumps({"workload": w.name, "faces": st["n_faces_total"], "n_p": st["n_patch_dofs"],
                              "ms64": r["t64"] * 1e3, "box_ms64": r["box64"] * 1e3, "gdofs64": r["gdofs64"],
                              "frac64": st["bytes_fp64"] / r["t64"] / 1e9 / HBM_PEAK_GBS,
                              "box_frac64": box_bytes(st, 8) / r["box64"] / 1e9 / HBM_PEAK_GBS,
                              "ms32": r.get("t32", 0) * 1e3, "gdofs32": r.get("gdofs32"),
                              "frac32": st["bytes_fp32"] / r["t32"] / 1e9 / HBM_PEAK_GBS if "t32" in r else None,
                              "err32": r.get("err32")}), flush=True)
        return

    w = WORKLOADS[args.workload]
    r = run_workload(w, args, with_cpu=not args.no_cpu)
    st = r["stats"]
    achieved = box_bytes(st, 8) / r["box64"] / 1e9
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            rec = json.load(f).get(f"{w.name}/{args.scatter}/f64")
        # measured bytes are only valid for the kernel source they were taken with
        if rec and rec.get("kernel_sha") == kernel_hash():
            traffic = rec["bytes_per_launch"]
    line = {
        "metric": "ghost-face patch DoFs/s for G.u (GDoF/s), FP64 vs FP32 at stated error, d=3",
        "value": round(r["gdofs64"], 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["t64"] * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "d": w.d, "k": w.k, "cells_per_axis": w.n[0],
                   "faces": st["n_faces_total"], "patch_dofs_per_face": st["n_patch_dofs"],
                   "support_dofs": st["n_support_dofs"], "halo_dofs": st["n_halo_nodes"],
                   "lattice_dofs": st["n_lattice"], "scatter": args.scatter, "mode": "accumulate"},
        "roofline": {"bound": "hbm", "kernel": "box_kernel<double>", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_launch": box_bytes(st, 8),
                     "avg_launch_us": round(r["box64"] * 1e6, 2), "halo_pass_us": round(r["halo64"] * 1e6, 2)},
        "apply_roofline_frac": round(st["bytes_fp64"] / r["t64"] / 1e9 / HBM_PEAK_GBS, 4),
        # a plain device copy of the lattice vector on the same GPU: the HBM rate a streaming kernel attains
        "copy_GBps": round(r["copy_GBps"], 1),
        # faces x patch DoFs x 24 B per apply time: the traffic the per-face patches would move without
        # any reuse between overlapping patches
        "patch_traffic_GBps": round(r["gdofs64"] * 24, 1),
        "overwrite": {"ms_per_step": round(r["t64_overwrite"] * 1e3, 5),
                      "value": round(st["n_faces_total"] * st["n_patch_dofs"] / r["t64_overwrite"] / 1e9, 4)},
        "graph": {"ms_per_step": round(r["t64_graph"] * 1e3, 5),
                  "value": round(st["n_faces_total"] * st["n_patch_dofs"] / r["t64_graph"] / 1e9, 4),
                  "timing": f"median of 10 replays of a graph of {args.steps} captured applies"},
        "fp32": None if "t32" not in r else {
            "value": round(r["gdofs32"], 4), "unit": "GDoF/s", "ms_per_step": round(r["t32"] * 1e3, 5),
            "normwise_err_vs_fp64": r["err32"],
            "box_kernel_frac": round(box_bytes(st, 4) / r["box32"] / 1e9 / HBM_PEAK_GBS, 4),
            "apply_roofline_frac": round(st["bytes_fp32"] / r["t32"] / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": r.get("cpu"),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
