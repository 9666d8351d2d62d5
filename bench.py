"""Benchmark of the hex8 SIMP state-solve hot path on one GPU.

One step = one full pass of the hot path on the 768x384x384 random-field
cantilever (113,246,208 elements, 341,955,075 DOFs, 7 levels): set the density
(moduli on all levels, Jacobi diagonals, coarsest inverse), solve K u = f with
mixed-precision MGPCG to a relative binary64 residual of 1e-6, and evaluate
compliance and the adjoint sensitivity.  Inputs are resident on the GPU before
the timed region.

Prints one JSON line.  `value` is the step throughput: DOFs of the state solved
per second over the whole step.  Besides it the line reports K u throughput
(binary32 and binary64), the solve seconds of the three precisions (binary32
V-cycle and outer K p, binary32 V-cycle with binary64 K p, plain binary64) with
iterations, binary64 residuals and compliances, the roofline of the dominant
kernel and of K u (timed with HIP events on the stream they run on, inside the
bench), and, on rank 0, the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K·u GDOF/s + MGPCG solve s to 1e-6 residual, FP32-mixed vs FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0

# Kernel families the library times per launch, and their algorithmic HBM
# bytes per level-0 launch: every vector read or written once (4 or 8 B per
# DOF), the moduli once (4 or 8 B per element), the support bits once (1 B per
# node).
FAMILY_BYTES = {
    "smooth_f32": (16, 4),    # read u, f, omega/D, write u
    "smooth1_f32": (12, 4),   # the sweep on the first sweep from zero, formed from f and omega/D: read f, omega/D, write u
    "residual_f32": (12, 4),  # read u, f, write r
    "apply_f32": (8, 4),      # read u, write A u
    "apply_f64": (16, 8),     # binary64 solves; the mixed solver's K p reads a binary32 p: (12, 8), set in main()
    "smooth_f64": (32, 8),
    "smooth1_f64": (24, 8),
    "residual_f64": (24, 8),
}


def family_bytes(g, fam) -> float:
    per_dof, per_elem = FAMILY_BYTES[fam]
    return per_dof * g.n_dof + per_elem * g.n_elem + 1.0 * g.n_node


def apply_bytes(g, word) -> float:
    """Algorithmic bytes of y = K u: read u, write y, read E, read support bits."""
    return 2.0 * word * g.n_dof + word * g.n_elem + 1.0 * g.n_node


# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (each scaled by the same counter over a device copy of
# known size), keyed by workload, kernel family, kernel choice and a digest of
# the kernel source they were taken on: any change to the kernel voids them.
TRAFFIC = {
    # level-0 binary32 Jacobi sweep, 768x384x384, 2 rows x 4 waves, z-chunks 8
    # and 4 (profiles/stream_smooth_f32_L0_cantilever_768x384x384_rf_traffic.md)
    ("cantilever_768x384x384_rf", "smooth_f32", "stream", 8, 0, "dfc1f4b9e31fd384"): 6410424012.8,
    ("cantilever_768x384x384_rf", "smooth_f32", "stream", 4, 0, "dfc1f4b9e31fd384"): 6496693145.6,
}


def stream_source_digest() -> str:
    import hashlib

    p = os.path.join(ROOT, "paper_2201_12931_amd", "csrc", "stream.hip")
    with open(p, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_bytes(workload, family, choice):
    key = (workload, family, choice[0], int(choice[1]), int(choice[2]), stream_source_digest())
    return TRAFFIC.get(key)


def time_events(fn, reps, stream):
    """Mean, median and minimum milliseconds of fn() over reps, from events on stream."""
    import torch

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for k in range(reps):
        fn()
        ev[k + 1].record(stream)
    ev[-1].synchronize()
    t = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))
    return ev[0].elapsed_time(ev[-1]) / reps, t[len(t) // 2], t[0]


def copy_probe(mib, dev):
    """Three device-to-device copies of mib MiB (calibration of HBM byte counters)."""
    if not mib:
        return
    import torch

    src = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_baseline(workload_dofs: int, workload_name: str):
    """The FP64 oracle (assembled operators, assembled V-cycle, PCG to 1e-6,
    sensitivity) on a bounded sample: the 128x64x64 random-field cantilever
    with 5 levels (about 10 s on one thread).  Its DOFs per second are the
    oracle's rate; scaled per DOF to the bench workload (whose assembled matrix
    would not fit in host memory) it is labelled as extrapolated."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import fem, multigrid as mg

    nx, ny, nz, levels = 128, 64, 64, 5
    g = W.Grid(nx, ny, nz)
    rho = W.random_field_density(g, seed=1, lo=0.01)
    f = W.cantilever_line_load(g)
    mask = W.fixed_mask_face_x0(g)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        h = mg.Hierarchy(nx, ny, nz, rho, mask, levels)
        u, its, rel, _ = mg.mgpcg(h, f, rtol=1e-6)
        fem.sensitivity(nx, ny, nz, rho, u)
        c = fem.compliance(f, u)
        dt = time.perf_counter() - t0
    rate = g.n_dof / dt / 1e9
    return {
        "value": rate,
        "unit": "GDOF/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nx}x{ny}x{nz} random-field cantilever ({g.n_dof} DOFs), {levels} levels, rtol 1e-6: "
                  f"assembly + MGPCG ({its} its) + sensitivity in {dt:.2f} s (scipy sparse, one thread); "
                  f"for {workload_name} ({workload_dofs} DOFs) extrapolated per DOF: "
                  f"{workload_dofs / (rate * 1e9):.0f} s per step",
        "extrapolated": workload_dofs != g.n_dof,
        "compliance": c,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cantilever_768x384x384_rf")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "mixed32"],
                    help="solver precision of the timed step (the other forms are timed once each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ku-reps", type=int, default=20)
    ap.add_argument("--only-step", action="store_true",
                    help="time the step of --precision only (no other precisions, no K u; for profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run 3 device copies of this many MiB (calibration for HBM byte counters)")
    ap.add_argument("--coarse-cycle", default="", metavar="LEVEL:BLOCKS",
                    help="pin the cooperative coarse-cycle launch (0:0 = off) instead of the timed choice")
    ap.add_argument("--l0-choice", default="", metavar="KIND:ZCHUNK:SHAPE",
                    help="pin the level-0 binary32 kernel (KIND stream|gather) instead of the timed choice, "
                         "e.g. for counter runs whose timings are perturbed by the profiler")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2201_12931_amd import hexmg

    g, rho, f, mask, spec = W.workload(args.workload)
    levels, rtol = spec["levels"], spec["rtol"]
    print(f"bench: {args.workload} {g.nx}x{g.ny}x{g.nz}, {g.n_dof} DOFs, {levels} levels", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rho_d = torch.from_numpy(rho).to(dev)
    f_d = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    del rho, f
    u_d = torch.zeros_like(f_d)
    dc_d = torch.empty(g.n_elem, dtype=torch.float64, device=dev)
    precs = {"mixed32": hexmg.MIXED32, "mixed": hexmg.MIXED, "fp64": hexmg.FP64}

    def step(grid):
        grid.set_density(rho_d)
        code, info = grid.solve(f_d, u_d, rtol=rtol, maxit=500)
        # the solve already formed the compliance f . u (binary64, on the device)
        grid.compliance_sensitivity(f_d, u_d, dc_d, compliance=False)
        if code != 0:
            raise RuntimeError(f"solve did not converge: {info[0]}")
        return info[0]

    if args.precision == "mixed":  # K p reads the binary32 search direction
        FAMILY_BYTES["apply_f64"] = (12, 8)
    main_grid = hexmg.Grid(g.nx, g.ny, g.nz, levels, precision=precs[args.precision])
    if args.coarse_cycle:  # before the first set_density: the timed choice is then skipped
        lv, nb = (int(v) for v in args.coarse_cycle.split(":"))
        main_grid.set_coarse_cycle(hexmg.F32, lv, nb)
    main_grid.set_density(rho_d)  # first success times the kernel variants
    if args.l0_choice:
        kind, zc, shape = args.l0_choice.split(":")
        main_grid.set_kernel_choice(0, hexmg.F32, hexmg.KERNEL_STREAM if kind == "stream" else hexmg.KERNEL_GATHER,
                                    int(zc), int(shape))
    for _ in range(args.warmup):
        step(main_grid)
    torch.cuda.synchronize()
    print("bench: warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step(main_grid))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    info_main = infos[-1]
    print(f"bench: timed steps done, {ms_per_step:.2f} ms per step", file=sys.stderr, flush=True)
    if args.only_step:
        # for profiler runs: a few binary32 K u launches (public entry) and the
        # copy calibration, then the step time
        u32 = torch.randn(g.n_dof, dtype=torch.float32, device=dev)
        y32 = torch.empty_like(u32)
        for _ in range(3):
            main_grid.apply_K(u32, y32)
        del u32, y32
        copy_probe(args.copy_probe, dev)
        print(json.dumps({"metric": METRIC, "ms_per_step": ms_per_step, "steps": args.steps,
                          "config": {"workload": args.workload, "precision": args.precision}}), flush=True)
        main_grid.close()
        return

    # Kernel durations: the same steps again with the library's per-launch
    # timing on (events stamped by the level-0 dispatches themselves, on the
    # stream they run on).  It is kept out of the timed steps above because the
    # timed dispatches cost a few microseconds each.
    main_grid.profile_enable(True)
    for _ in range(args.steps):
        step(main_grid)
    torch.cuda.synchronize()
    kernel_ms = {fam: list(main_grid.profile_query(fam)) for fam in FAMILY_BYTES}
    main_grid.profile_enable(False)

    # K u throughput (level 0, the public entry: input masked on load) in both precisions
    u32 = torch.randn(g.n_dof, dtype=torch.float32, device=dev)
    y32 = torch.empty_like(u32)
    main_grid.apply_K(u32, y32)
    ms32, med32, min32 = time_events(lambda: main_grid.apply_K(u32, y32), args.ku_reps, stream)
    del y32
    u64 = u32.double()
    del u32
    y64 = torch.empty_like(u64)
    main_grid.apply_K(u64, y64)
    ms64, med64, min64 = time_events(lambda: main_grid.apply_K(u64, y64), args.ku_reps, stream)
    del u64, y64
    # per level, precision and mode (K u, sweep, residual): (kind, z-chunk, shape)
    choices = {f"L{l}": {dt: {m: main_grid.kernel_choice(l, d, i) for i, m in enumerate(("apply", "smooth", "residual"))}
                         for dt, d in (("f32", hexmg.F32), ("f64", hexmg.F64))}
               for l in range(levels)}
    choices["coarse_cycle"] = main_grid.coarse_cycle_choice(hexmg.F32)
    main_grid.close()
    del main_grid
    torch.cuda.empty_cache()

    # the other precisions of the same step, one timed step each after one untimed
    solves = {args.precision: info_main}
    step_s = {args.precision: ms_per_step * 1e-3}
    for name in ("mixed32", "mixed", "fp64"):
        if name == args.precision:
            continue
        grid = hexmg.Grid(g.nx, g.ny, g.nz, levels, precision=precs[name])
        step(grid)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        solves[name] = step(grid)
        torch.cuda.synchronize()
        step_s[name] = time.perf_counter() - ta
        grid.close()
        del grid
        torch.cuda.empty_cache()
        print(f"bench: {name} step {step_s[name] * 1e3:.1f} ms", file=sys.stderr, flush=True)

    copy_probe(args.copy_probe, dev)

    # the device copy rate on this GPU (a 1 GiB binary32 copy, read + write),
    # against which the roofline fractions are also reported
    src = torch.empty((1 << 30) // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms, _, copy_min = time_events(lambda: dst.copy_(src), 5, stream)
    copy_gbs = 2.0 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()

    # dominant kernel: the family with the largest device time over the profiled steps
    dom = max(kernel_ms, key=lambda k: kernel_ms[k][1])
    n_dom, t_dom = kernel_ms[dom]
    avg_ms = t_dom / max(n_dom, 1)
    dom_bytes = family_bytes(g, dom)
    achieved = dom_bytes / (avg_ms * 1e-3) / 1e9
    dom_choice = choices["L0"]["f32" if dom.endswith("f32") else "f64"][dom.split("_")[0]]
    c64 = solves["fp64"]["compliance"]
    out = {
        "metric": METRIC,
        "value": g.n_dof / (ms_per_step * 1e-3) / 1e9,
        "unit": "GDOF/s (state solved per second: set density + MGPCG to 1e-6 + compliance/sensitivity)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 V-cycle and K p, f64 CG" if args.precision == "mixed32"
                  else "f32 V-cycle and search direction, f64 K p arithmetic and CG"),
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": [g.nx, g.ny, g.nz],
            "elements": g.n_elem,
            "dofs": g.n_dof,
            "levels": levels,
            "rtol": rtol,
            "precision": args.precision,
            "step": "set_density + MGPCG to binary64 rtol + compliance/sensitivity",
        },
        "ku_gdofs": {"f32": g.n_dof / (ms32 * 1e-3) / 1e9, "f64": g.n_dof / (ms64 * 1e-3) / 1e9},
        "ku_ms": {"f32": ms32, "f64": ms64, "f32_median": med32, "f32_min": min32, "f64_median": med64,
                  "f64_min": min64},
        "ku_hbm_frac": {"f32": apply_bytes(g, 4) / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "f64": apply_bytes(g, 8) / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "solve_s": {k: v["ms_solve"] * 1e-3 for k, v in solves.items()},
        "step_s": step_s,
        "iterations": {k: v["iterations"] for k, v in solves.items()},
        "rel_res_true": {k: v["rel_res_true"] for k, v in solves.items()},
        "compliance": {k: v["compliance"] for k, v in solves.items()},
        "compliance_rel_diff_vs_fp64": {k: abs(v["compliance"] - c64) / abs(c64) for k, v in solves.items()},
        "kernel_ms": kernel_ms,
        "kernel_choice": choices,
        "roofline": {
            "kernel": f"{dom} level 0 (%s, z-chunk %d, shape %d)" % dom_choice,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_bytes(args.workload, dom, dom_choice),
            "avg_launch_ms": avg_ms,
            "launches": n_dom,
            "bytes_per_launch": dom_bytes,
            "timing": "per-dispatch HIP events over %d untimed repeats of the step" % args.steps,
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "roofline_ku": {
            "kernel": "K u binary32, level 0, public entry (%s, z-chunk %d, shape %d)" % choices["L0"]["f32"]["apply"],
            "bound": "hbm",
            "achieved": apply_bytes(g, 4) / (ms32 * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": apply_bytes(g, 4) / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "bytes_per_launch": apply_bytes(g, 4),
            "timing": "HIP events on the launching stream, mean of %d launches" % args.ku_reps,
            "copy_gbs": copy_gbs,
            "frac_of_copy": apply_bytes(g, 4) / (ms32 * 1e-3) / 1e9 / copy_gbs,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g.n_dof, args.workload)
    print(json.dumps(out), flush=True)
    del rho_d, f_d, u_d, dc_d
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
