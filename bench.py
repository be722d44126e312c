"""Benchmark of the Hermite wave half step on one MI355X.

Workload: 128^3 periodic cells, m = 3 (64 scaled derivatives per node per
field), c = 1, cfl = 0.5, u0 = seeded sum of 8 Fourier modes (wave numbers in
[1, 8], amplitudes ~ N(0, 1)), u_t = 0. One step = one full time step (two
half steps, primal -> dual -> primal) of the whole grid. The state stays
resident in HBM; the timed region is hermite_step(K) on the torch stream.

Prints ONE JSON line (rank 0). Metric: DOF-updates/s, a DOF-update being one
scaled derivative of u or u_t produced on the other grid by one half step:
value = 2 (m+1)^3 n^3 * 2 K / seconds.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s at m=3, plain FP64 vs mixed-precision at rel L2 <= 1e-6"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6     # 256 CU x 2.4 GHz x 64 FP64 FMA lanes/clk x 2
FP64_MFMA_PEAK_TFLOPS = 78.6

# Useful FP64 flops per cell per half step of the fused formulation: the
# dense per-parity-class operators (2 flops per nonzero entry; 13,499 / 2,047 /
# 255 nonzeros for m = 3 / 2 / 1, Taylor and RK4 alike) plus the shared 2x2x2
# butterfly of the corner data (24 adds per derivative index and field).
NNZ = {1: 255, 2: 2047, 3: 13499}


def fused_flops_per_cell(m: int) -> float:
    return 2.0 * NNZ[m] + 24.0 * 2 * (m + 1) ** 3


def fused_bytes_per_cell(m: int) -> float:
    # read one two-field node of the old grid, write one of the new grid (FP64)
    return 2.0 * 2 * (m + 1) ** 3 * 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--m", type=int, default=3)
    ap.add_argument("--variant", default="fused-taylor",
                    choices=["fused-taylor", "fused-rk4", "two-taylor", "two-rk4"])
    ap.add_argument("--all-variants", action="store_true", help="also time the other three variants")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=48, help="grid of the oracle's timed sample")
    return ap.parse_args()


def variant_kwargs(v: str) -> dict:
    fused, evo = v.split("-")
    return {"fused": fused == "fused", "evolution": evo}


def time_variant(B, torch, n, m, u0, ut0, steps, warmup, variant):
    # A stream of our own (default priority): torch's current stream is the
    # null stream, which the library would replace by a private one, and the
    # timing events must sit on the stream the kernels run on.
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream), B.Solver(n, m, 0.5, 1.0, stream=stream, **variant_kwargs(variant)) as s:
        s.set_initial(u0, ut0)
        s.step(warmup)
        s.sync()
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        t0 = time.perf_counter()
        s.step(steps)
        end.record(stream)
        end.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(end)
        u = torch.empty_like(u0)
        ut = torch.empty_like(ut0)
        s.gather_device(u, ut)
        s.sync()
        t_final, nsteps, _ = s.time()
    return ms, wall, u, ut, t_final


def cpu_baseline(m: int, n_s: int) -> dict:
    """The oracle (plain FP64 C, OpenMP) on a bounded sample of the workload:
    the same data recipe and order on an n_s^3 grid, one full step."""
    from oracle import oracle as O
    from paper_1609_09841_amd import inputs as I
    O.load()
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    u0, ut0 = I.fourier_initial(n_s, m)
    u0, ut0 = u0.numpy(), ut0.numpy()
    t0 = time.perf_counter()
    O.run(n_s, m, 0.5, 1.0, u0, ut0, 1)
    sec = time.perf_counter() - t0
    dofs = 2 * (m + 1) ** 3 * n_s ** 3 * 2 * 1
    return {"value": dofs / sec, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_s}^3 cells, m={m}, 1 full step (2 half steps) of the same Fourier-mode "
                      f"workload, {sec:.2f} s on {cores} threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1609_09841_amd import binding as B
    from paper_1609_09841_amd import inputs as I
    B.load()
    n, m, K, W = args.n, args.m, args.steps, args.warmup
    torch.cuda.set_device(0)
    u0, ut0 = I.fourier_initial(n, m, device="cuda")
    torch.cuda.synchronize()
    dof_updates_per_step = 2 * (m + 1) ** 3 * n ** 3 * 2

    ms, wall, u, ut, t_final = time_variant(B, torch, n, m, u0, ut0, K, W, args.variant)
    sec = ms / 1e3
    value = dof_updates_per_step * K / sec

    # error of the final state against the exact solution (context, not timed)
    modes = I.fourier_modes()
    ue, ute = I.fourier_exact(n, m, modes, t=t_final, device="cuda")
    err_u, err_ut = I.rel_l2(u, ue), I.rel_l2(ut, ute)
    del ue, ute

    launches = 2 * K if args.variant.startswith("fused") else 4 * K
    avg_launch_s = sec / launches
    cells = n ** 3
    if args.variant.startswith("fused"):
        flops = fused_flops_per_cell(m) * cells
        achieved_tflops = flops / avg_launch_s / 1e12
        mfma = (m == 3)
        roofline = {"bound": "mfma" if mfma else "alu", "achieved": achieved_tflops,
                    "peak": FP64_MFMA_PEAK_TFLOPS if mfma else FP64_VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved_tflops / FP64_VALU_PEAK_TFLOPS, "traffic": None,
                    "kernel": "fused_mfma_kernel (FP64 MFMA 16x16x4)" if mfma else f"fused_kernel<{m + 1}> (FP64 VALU)",
                    "avg_launch_ms": avg_launch_s * 1e3,
                    "hbm_GBps_algorithmic": fused_bytes_per_cell(m) * cells / avg_launch_s / 1e9}
    else:
        roofline = None

    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded Fourier modes, u_t = 0)",
        "config": {"workload": f"wave equation, {n}^3 periodic cells, m={m}, c=1, cfl=0.5, "
                               f"{args.variant}, plain FP64", "cells_per_side": n, "m": m,
                   "variant": args.variant, "precision": "fp64", "dof_per_grid": dof_updates_per_step // 2},
        "roofline": roofline,
        "error_vs_exact": {"u": err_u, "u_t": err_ut, "t": t_final},
        "wall_s": wall,
    }
    if args.all_variants:
        others = {}
        for v in ("fused-taylor", "fused-rk4", "two-taylor", "two-rk4"):
            if v == args.variant:
                continue
            vms, _, _, _, _ = time_variant(B, torch, n, m, u0, ut0, K, W, v)
            others[v] = {"value": dof_updates_per_step * K / (vms / 1e3), "ms_per_step": vms / K}
            torch.cuda.empty_cache()
        out["variants"] = others
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
