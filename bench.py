"""Benchmark of the hex8 SIMP state-solve hot path on one GPU.

One step = one full pass of the hot path on the 128x64x64 random-field
cantilever (524,288 elements, 1,635,075 DOFs): set the density (moduli on all
levels, Jacobi diagonals, coarsest inverse), solve K u = f with mixed-precision
MGPCG to a relative residual of 1e-6, and evaluate compliance and the adjoint
sensitivity.  Inputs are resident on the GPU before the timed region.

Prints one JSON line.  Besides the step throughput it reports K u throughput
(binary32 and binary64), the mixed and plain-binary64 solve times, the roofline
of the dominant kernel (timed with HIP events on its own stream inside the timed
region) and, on rank 0, the CPU oracle timed on a bounded sample.
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


def smooth_bytes_per_launch(g) -> float:
    """Algorithmic HBM bytes of one level-0 Jacobi sweep in binary32:
    read u, f, omega/D and write u (4 x 4 B per DOF), read E (4 B per element),
    read the support bits (1 B per node)."""
    return 16.0 * g.n_dof + 4.0 * g.n_elem + 1.0 * g.n_node


# HBM bytes per launch of the level-0 binary32 Jacobi sweep, from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes (each scaled by the same counter over a
# device copy of known size), keyed by workload, kernel choice and a digest of
# the kernel source they were taken on: any change to the kernel voids them.
# The mean over the sweep's launches, weighted by launch count: the plain
# sweep and the last sweep of each V-cycle, which also forms r . z.
TRAFFIC = {
    # profiles/stream_smooth_f32_L0_cantilever_128x64x64_rf_traffic.md
    ("cantilever_128x64x64_rf", "stream", 4, 0, "af1a4333bf3d22e2"): 44811741.9,
    ("cantilever_128x64x64_rf", "stream", 4, 4, "af1a4333bf3d22e2"): 41935410.0,
}


def stream_source_digest() -> str:
    import hashlib

    p = os.path.join(ROOT, "paper_2201_12931_amd", "csrc", "stream.hip")
    with open(p, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_bytes(workload, choice):
    key = (workload, choice[0], int(choice[1]), int(choice[2]), stream_source_digest())
    return TRAFFIC.get(key)


def apply_bytes(g, word) -> float:
    """Algorithmic bytes of y = K u: read u, write y, read E, read support bits."""
    return 2.0 * word * g.n_dof + word * g.n_elem + 1.0 * g.n_node


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


def cpu_baseline(name: str):
    """The FP64 oracle (assembled operators, assembled V-cycle, PCG, sensitivity)
    on the 128x64x64 random-field cantilever with 5 levels -- the bench workload
    itself, a sample of the larger ones -- held to one BLAS thread so that
    ``cores`` is what it used."""
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
    return {
        "value": g.n_dof / dt / 1e9,
        "unit": "GDOF/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nx}x{ny}x{nz} random-field cantilever ({g.n_dof} DOFs), {levels} levels, rtol 1e-6: "
                  f"assembly + MGPCG ({its} its) + sensitivity in {dt:.2f} s (scipy sparse, one thread)",
        "compliance": c,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cantilever_128x64x64_rf")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ku-reps", type=int, default=20)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run 3 device copies of this many MiB (calibration for HBM byte counters)")
    ap.add_argument("--coarse-cycle", default="", metavar="LEVEL:BLOCKS",
                    help="pin the cooperative coarse-cycle launch (0:0 = off) instead of the timed choice")
    ap.add_argument("--l0-choice", default="", metavar="KIND:ZCHUNK:SHAPE",
                    help="pin the level-0 binary32 kernel (KIND stream|gather) instead of the timed choice, "
                         "e.g. for counter runs whose timings are perturbed by the profiler")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2201_12931_amd import hexmg

    g, rho, f, mask, spec = W.workload(args.workload)
    levels, rtol = spec["levels"], spec["rtol"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rho_d = torch.from_numpy(rho).to(dev)
    f_d = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    u_d = torch.zeros_like(f_d)
    dc_d = torch.empty(g.n_elem, dtype=torch.float64, device=dev)

    mixed = hexmg.Grid(g.nx, g.ny, g.nz, levels, precision=hexmg.MIXED)
    fp64 = hexmg.Grid(g.nx, g.ny, g.nz, levels, precision=hexmg.FP64)

    def step(grid):
        grid.set_density(rho_d)
        code, info = grid.solve(f_d, u_d, rtol=rtol, maxit=500)
        # the solve already formed the compliance f . u (binary64, on the device)
        grid.compliance_sensitivity(f_d, u_d, dc_d, compliance=False)
        return code, info[0], info[0]["compliance"]

    if args.coarse_cycle:  # before the first set_density: the timed choice is then skipped
        lv, nb = (int(v) for v in args.coarse_cycle.split(":"))
        for dt in (hexmg.F32, hexmg.F64):
            mixed.set_coarse_cycle(dt, lv, nb)
    mixed.set_density(rho_d)  # first success times the kernel variants
    if args.l0_choice:
        kind, zc, shape = args.l0_choice.split(":")
        mixed.set_kernel_choice(0, hexmg.F32, hexmg.KERNEL_STREAM if kind == "stream" else hexmg.KERNEL_GATHER,
                                int(zc), int(shape))
    for _ in range(args.warmup):
        step(mixed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step(mixed))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    code, info_mixed, c_mixed = infos[-1]

    # Kernel durations: the same steps again with the library's per-launch
    # timing on (events stamped by the level-0 dispatches themselves, on the
    # stream they run on).  It is kept out of the timed steps above because the
    # timed dispatches cost a few microseconds each.
    mixed.profile_enable(True)
    for _ in range(args.steps):
        step(mixed)
    torch.cuda.synchronize()
    n_smooth, ms_smooth = mixed.profile_query("smooth_f32")
    n_res, ms_res = mixed.profile_query("residual_f32")
    n_app, ms_app = mixed.profile_query("apply_f64")
    mixed.profile_enable(False)

    # plain binary64 form of the same step
    step(fp64)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    code64, info64, c64 = step(fp64)
    torch.cuda.synchronize()
    t3 = time.perf_counter()

    # K u throughput (level 0) in both precisions
    u32 = torch.randn(g.n_dof, dtype=torch.float32, device=dev)
    y32 = torch.empty_like(u32)
    u64 = u32.double()
    y64 = torch.empty_like(u64)
    mixed.apply_K(u32, y32)
    mixed.apply_K(u64, y64)
    ms32, med32, min32 = time_events(lambda: mixed.apply_K(u32, y32), args.ku_reps, stream)
    ms64, med64, min64 = time_events(lambda: mixed.apply_K(u64, y64), args.ku_reps, stream)

    if args.copy_probe:
        src = torch.empty(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    avg_smooth_ms = ms_smooth / max(n_smooth, 1)
    sb = smooth_bytes_per_launch(g)
    achieved = sb / (avg_smooth_ms * 1e-3) / 1e9
    choices = {f"L{l}": {"f32": mixed.kernel_choice(l, hexmg.F32), "f64": mixed.kernel_choice(l, hexmg.F64)}
               for l in range(levels)}
    choices["coarse_cycle"] = {"f32": mixed.coarse_cycle_choice(hexmg.F32),
                               "f64": mixed.coarse_cycle_choice(hexmg.F64)}
    out = {
        "metric": METRIC,
        "value": g.n_dof / (ms_per_step * 1e-3) / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mixed(f64 CG)",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": [g.nx, g.ny, g.nz],
            "elements": g.n_elem,
            "dofs": g.n_dof,
            "levels": levels,
            "rtol": rtol,
            "step": "set_density + mixed MGPCG to rtol + compliance/sensitivity",
        },
        "ku_gdofs": {"f32": g.n_dof / (ms32 * 1e-3) / 1e9, "f64": g.n_dof / (ms64 * 1e-3) / 1e9},
        "ku_ms": {"f32": ms32, "f64": ms64, "f32_median": med32, "f32_min": min32, "f64_median": med64,
                  "f64_min": min64},
        "ku_hbm_frac": {"f32": apply_bytes(g, 4) / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "f64": apply_bytes(g, 8) / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "solve_s": {"mixed": info_mixed["ms_solve"] * 1e-3, "fp64": info64["ms_solve"] * 1e-3},
        "step_s": {"mixed": ms_per_step * 1e-3, "fp64": t3 - t2},
        "iterations": {"mixed": info_mixed["iterations"], "fp64": info64["iterations"]},
        "rel_res_true": {"mixed": info_mixed["rel_res_true"], "fp64": info64["rel_res_true"]},
        "compliance": {"mixed": c_mixed, "fp64": c64, "rel_diff": abs(c_mixed - c64) / abs(c64)},
        "kernel_ms": {"smooth_f32": [n_smooth, ms_smooth], "residual_f32": [n_res, ms_res],
                      "apply_f64": [n_app, ms_app]},
        "kernel_choice": choices,
        "roofline": {
            "kernel": "level-0 binary32 damped Jacobi sweep (%s, z-chunk %d, shape %d)" % choices["L0"]["f32"],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_bytes(args.workload, choices["L0"]["f32"]),
            "avg_launch_ms": avg_smooth_ms,
            "bytes_per_launch": sb,
            "timing": "per-dispatch HIP events over %d untimed repeats of the step" % args.steps,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
