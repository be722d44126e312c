"""Benchmark of the Hermite wave half step on one MI355X.

Workload (headline): 128^3 periodic cells, m = 3 (64 scaled derivatives per
node per field), c = 1, cfl = 0.5, u0 = seeded sum of 8 Fourier modes (wave
numbers in [1, 8], amplitudes ~ N(0, 1)), u_t = 0, plain FP64, fused kernel
with Taylor evolution. One step = one full time step (two half steps,
primal -> dual -> primal) of the whole grid. The state stays resident in HBM;
the timed region is hermite_step(K) on a torch stream, between HIP events.

Prints ONE JSON line. Metric: DOF-updates/s, a DOF-update being one scaled
derivative of u or u_t produced on the other grid by one half step:
value = 2 (m+1)^3 n^3 * 2 K / seconds.

Also reported (outside the timed region of the headline):
  * the other kernel organisations / evolutions at the same workload;
  * the mixed-precision contractions (FP32, split BF16x3) at the same
    workload: rate and error against the FP64 run after the same K steps;
  * precision study: 256^3 cells, m = 3, 200 steps, final-time rel L2 of the
    mixed paths against the plain FP64 GPU path (whose parity with the CPU
    oracle is tested separately);
  * batched point-source workload: 64 seeded shots of uneven sizes and
    orders, one Gaussian/Ricker source each, 150 steps, stepped together by
    the batch API (graph replay, autotuned launch shapes), FP32 and FP64,
    against the same shots run one after the other;
  * the paper's advection workload (Eq. 1): 150^3 cells, 200 steps, m = 1..3,
    time to solution next to the paper's (GTX 980, FP32: context only);
  * gradient of a receiver misfit (96^3, m = 3, 200 steps, point source, 32
    receivers) by the adjoint sweep, with a full-size central-difference
    check;
  * the CPU oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s at m=3, plain FP64 vs mixed-precision at rel L2 <= 1e-6"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
MEASURED_FP64_MFMA_TFLOPS = 68.9  # v_mfma_f64_4x4x4f64 (4 blocks) throughput measured on gfx950
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64, vector and matrix alike

# Useful FP64 flops per cell per half step of the fused formulation: the
# dense per-parity-class operators (2 flops per nonzero entry; 13,499 / 2,047 /
# 255 nonzeros for m = 3 / 2 / 1, Taylor and RK4 alike) plus the shared 2x2x2
# butterfly of the corner data (24 adds per derivative index and field).
NNZ = {1: 255, 2: 2047, 3: 13499}

# Source files of the m = 3 fused FP64 kernel; traffic counters taken on
# another version of these files are not reported.
MFMA_SOURCES = ["fused_mfma.hip", "fused_common.h", "mfma_order.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_fused_mfma4_128cube_m3.md")


def fused_flops_per_cell(m: int) -> float:
    return 2.0 * NNZ[m] + 24.0 * 2 * (m + 1) ** 3


def fused_bytes_per_cell(m: int) -> float:
    # read one two-field node of the old grid, write one of the new grid (FP64)
    return 2.0 * 2 * (m + 1) ** 3 * 8


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in MFMA_SOURCES:
        with open(os.path.join(ROOT, "paper_1609_09841_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the m = 3 fused FP64 kernel from the committed
    rocprofv3 summary, if it was taken on the current kernel sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^(\w+) = (\S+)$", text, re.M))
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-precision-study", action="store_true", help="skip the 256^3 precision study")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched point-source leg")
    ap.add_argument("--no-advection", action="store_true", help="skip the advection leg")
    ap.add_argument("--no-gradient", action="store_true", help="skip the adjoint-gradient leg")
    ap.add_argument("--no-slab", action="store_true", help="skip the one-slab (sharded share) leg")
    ap.add_argument("--gradient-steps", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=96, help="grid of the oracle's timed sample")
    return ap.parse_args()


def variant_kwargs(v: str) -> dict:
    fused, evo = v.split("-")
    return {"fused": fused == "fused", "evolution": evo}


def time_variant(B, torch, n, m, u0, ut0, steps, warmup, variant, precision="fp64"):
    # A stream of our own (default priority): torch's current stream is the
    # null stream, which the library would replace by a private one, and the
    # timing events must sit on the stream the kernels run on.
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream), B.Solver(n, m, 0.5, 1.0, stream=stream, precision=precision,
                                             **variant_kwargs(variant)) as s:
        s.set_initial(u0, ut0)
        s.step(warmup)
        s.set_initial(u0, ut0)   # the timed steps start from t = 0
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


def errors(I, u, ut, ru, rut) -> dict:
    """rel L2 against a reference: over all DOFs and over node values (d = 0)."""
    return {"u": I.rel_l2(u, ru), "u_t": I.rel_l2(ut, rut),
            "u_nodes": I.rel_l2(u[0, 0, 0], ru[0, 0, 0]), "u_t_nodes": I.rel_l2(ut[0, 0, 0], rut[0, 0, 0])}


def precision_study(B, torch, I, n=256, m=3, steps=200) -> dict:
    """Final-time error of the mixed paths against the plain FP64 GPU path."""
    u0, ut0 = I.fourier_initial(n, m, device="cuda")
    ms, _, ru, rut, _ = time_variant(B, torch, n, m, u0, ut0, steps, 0, "fused-taylor", "fp64")
    out = {"workload": f"{n}^3 cells, m={m}, {steps} steps, same Fourier-mode data",
           "reference": "plain FP64 fused Taylor on the GPU (parity with the CPU oracle tested at 128^3)",
           "fp64": {"ms_per_step": ms / steps}}
    for prec in ("fp32", "bf16x3"):
        pms, _, u, ut, _ = time_variant(B, torch, n, m, u0, ut0, steps, 0, "fused-taylor", prec)
        e = errors(I, u, ut, ru, rut)
        out[prec] = {"ms_per_step": pms / steps, "speedup_vs_fp64": ms / pms, "rel_l2_vs_fp64": e,
                     "meets_1e-6_all_dofs": max(e["u"], e["u_t"]) <= 1e-6,
                     "meets_1e-6_node_values": max(e["u_nodes"], e["u_t_nodes"]) <= 1e-6}
        del u, ut
    del u0, ut0, ru, rut
    torch.cuda.empty_cache()
    return out


def batch_leg(B, torch, I, steps: int = 150, warmup: int = 2, count: int = 64) -> dict:
    """The batched point-source workload: `count` seeded shots of uneven sizes
    and orders (inputs.batch_shots), zero data, one source each, stepped
    together (one graph replay per full step, autotuned launch shapes). FP32
    contractions for the m = 3 shots (m = 1, 2 shots run FP64); error stated
    against the same batch in FP64; compared with the shots run one after the
    other as single-grid contexts."""
    shots = I.batch_shots(count=count)
    dof = sum(2 * (sh["m"] + 1) ** 3 * sh["n"] ** 3 * 2 for sh in shots)      # DOF-updates per full step
    hbm = sum(2 * 32 * (sh["m"] + 1) ** 3 * sh["n"] ** 3 for sh in shots)     # algorithmic bytes per full step
    m3 = [i for i, sh in enumerate(shots) if sh["m"] == 3]
    out = {"workload": f"{count} shots, n from {{32,48,64,96}} and m from {{1,2,3}} by seed, zero data, "
                       f"Gaussian source (sigma 2h) with a Ricker wavelet (f0 = c/(8h), t0 = 1.2/f0), "
                       f"{steps} steps, cfl 0.5",
           "dof_updates_per_step": dof, "steps": steps}
    finals = {}
    for prec in ("fp64", "fp32"):
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream), B.Batch(shots, precision=prec, stream=stream) as b:
            b.step(warmup)            # graph capture and first replays
            for i in range(len(shots)):
                b.set_initial(i)      # every shot back to zero data at t = 0
            b.sync()
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            b.step(steps)
            end.record(stream)
            end.synchronize()
            ms = start.elapsed_time(end)
            tuning = {}
            for m in (1, 2, 3):
                try:
                    ch, tms = b.tuning(m)
                    tuning[f"m{m}"] = {"choice": ch, "half_step_ms": tms}
                except B.HermiteError:
                    pass
            res = {"value": dof * steps / (ms / 1e3), "unit": "DOF-updates/s", "ms_per_step": ms / steps,
                   "hbm_GBps_algorithmic": hbm * steps / (ms / 1e3) / 1e9, "autotune": tuning}
            if prec == "fp64":
                for i in m3:
                    finals[i] = b.gather(i)[:2]
            else:
                worst = {"u": 0.0, "u_t": 0.0, "u_nodes": 0.0, "u_t_nodes": 0.0}
                for i in m3:
                    u, ut, _ = b.gather(i)
                    ru, rut = finals[i]
                    e = errors(I, u, ut, ru, rut)
                    worst = {k: max(worst[k], e[k]) for k in worst}
                res["rel_l2_vs_fp64_worst_m3_shot"] = worst
        out[prec] = res
    finals.clear()
    # the same shots one after the other, each its own single-grid context
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    solvers = []
    with torch.cuda.stream(stream):
        for sh in shots:
            s = B.Solver(sh["n"], sh["m"], 0.5, 1.0, stream=stream, precision="fp32" if sh["m"] == 3 else "fp64")
            M, n = sh["m"] + 1, sh["n"]
            z = torch.zeros((M, M, M, n, n, n), dtype=torch.float64, device="cuda")
            s.set_initial(z, z)
            s.set_source(sh["source"])
            solvers.append(s)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for s in solvers:
            s.step(steps)
        end.record(stream)
        end.synchronize()
        sms = start.elapsed_time(end)
    for s in solvers:
        s.close()
    torch.cuda.empty_cache()
    out["sequential_single_contexts_fp32"] = {"value": dof * steps / (sms / 1e3), "ms_per_step": sms / steps}
    out["batch_speedup_vs_sequential"] = sms / (out["fp32"]["ms_per_step"] * steps)
    return out


# Time to solution of the paper's advection table (150^3 grid points, 200
# steps, GTX 980, FP32), seconds per order m, monolithic and two kernels:
# context only.
PAPER_ADVECTION_S = {1: 2.09, 2: 13.77, 3: 36.17}
PAPER_ADVECTION_TWO_S = {1: 2.42, 2: 13.77, 3: 37.23}


def advection_leg(B, torch, I, n: int = 150, steps: int = 200, warmup: int = 1) -> dict:
    """The paper's advection workload (Eq. 1): n^3 cells, 200 steps, m = 1..3,
    seeded Fourier-mode data, fused FP64 kernel (the exact series composed with
    interpolation into one separable operator per axis)."""
    out = {"workload": f"advection u_t = u_x1 + u_x2 + u_x3, {n}^3 periodic cells, {steps} steps, cfl 0.5, "
                       f"seeded Fourier modes, fused FP64",
           "paper_context": "GTX 980, FP32, monolithic kernel (two kernels in paper_two_kernel_time_s): " +
                            ", ".join(f"m={m} {t} s" for m, t in PAPER_ADVECTION_S.items())}
    def timed(m, u0, fused):
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream), B.Solver(n, m, 0.5, 1.0, equation="advection", fused=fused,
                                                 stream=stream) as s:
            s.set_initial(u0)
            s.step(warmup)
            s.set_initial(u0)
            s.sync()
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            s.step(steps)
            end.record(stream)
            end.synchronize()
            return start.elapsed_time(end)

    for m in (1, 2, 3):
        u0, _ = I.fourier_initial(n, m, device="cuda")
        ms = timed(m, u0, True)
        ms2 = timed(m, u0, False)
        dof = (m + 1) ** 3 * n ** 3 * 2 * steps            # one field, two half steps per step
        gbs = 16 * dof / (ms / 1e3) / 1e9                  # 8 B read + 8 B written per DOF-update
        out[f"m{m}"] = {"time_to_solution_s": ms / 1e3, "value": dof / (ms / 1e3), "unit": "DOF-updates/s",
                        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS, "kernel": f"advect_kernel<{m + 1}>"},
                        "two_kernel_time_s": ms2 / 1e3,
                        "paper_time_s": PAPER_ADVECTION_S[m], "paper_two_kernel_time_s": PAPER_ADVECTION_TWO_S[m]}
        del u0
        torch.cuda.empty_cache()
    return out


def slab_leg(B, torch, I, n: int = 128, nz: int = 16, half_steps: int = 100, warmup: int = 20) -> dict:
    """One device's share of the headline grid cut into z-slabs (n x n x nz
    cells of the n^3 grid, m = 3, fused FP64 on the matrix cores): half steps
    of the slab kernel alone, with the one-plane halo copy before each (here a
    copy of the slab's own boundary plane, the same bytes a peer copy would
    move), and with that copy on a second stream overlapping the interior
    cells (the boundary plane after it). No multi-device figure: no second
    device takes part."""
    m, M = 3, 4
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    u0, ut0 = I.fourier_initial(n, m)
    u0 = u0.numpy()[:, :, :, :nz].copy()
    ut0 = ut0.numpy()[:, :, :, :nz].copy()
    out = {"workload": f"z-slab {n} x {n} x {nz} cells of the {n}^3 m=3 grid (1/{n // nz} of it), fused FP64"}
    with B.Slab(n, nz, stream=stream) as sl:
        sl.set_initial(u0, ut0)

        def run(k, exchange, compute=True):
            nxt = B.HERMITE_SLAB_PRIMAL_HALO
            for i in range(k):
                if exchange:
                    if nxt == B.HERMITE_SLAB_PRIMAL_HALO:
                        sl.copy_plane_from(nxt, sl, B.HERMITE_SLAB_PRIMAL_FIRST)
                    else:
                        sl.copy_plane_from(nxt, sl, B.HERMITE_SLAB_DUAL_LAST)
                if compute:
                    nxt = sl.half_step()
                else:
                    nxt = B.HERMITE_SLAB_DUAL_HALO if i % 2 == 0 else B.HERMITE_SLAB_PRIMAL_HALO

        comm = torch.cuda.Stream()

        def run_overlapped(k):
            # interior cells while the halo plane is copied on a second stream,
            # then the boundary plane once the copy is in
            for _ in range(k):
                ready, done = torch.cuda.Event(), torch.cuda.Event()
                ready.record(stream)
                halo = sl.half_step_part(B.HERMITE_SLAB_INTERIOR)
                comm.wait_event(ready)
                src = B.HERMITE_SLAB_PRIMAL_FIRST if halo == B.HERMITE_SLAB_PRIMAL_HALO else B.HERMITE_SLAB_DUAL_LAST
                sl.copy_plane_from(halo, sl, src, stream=comm)
                done.record(comm)
                stream.wait_event(done)
                sl.half_step_part(B.HERMITE_SLAB_BOUNDARY)

        res = {}
        run_overlapped(warmup)
        sl.sync()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        run_overlapped(half_steps)
        end.record(stream)
        end.synchronize()
        res["overlapped"] = start.elapsed_time(end) / half_steps
        for name, exchange, compute in (("kernel_only", False, True), ("with_plane_copy", True, True),
                                        ("plane_copy_only", True, False)):
            run(warmup, exchange, compute)
            sl.sync()
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            run(half_steps, exchange, compute)
            end.record(stream)
            end.synchronize()
            res[name] = start.elapsed_time(end) / half_steps
        sl.sync()
    dof = 2 * M ** 3 * n * n * nz
    plane_bytes = 2 * M ** 3 * n * n * 8
    out.update({"ms_per_half_step": res["kernel_only"], "ms_per_half_step_with_plane_copy": res["with_plane_copy"],
                "ms_per_half_step_copy_overlapping_interior": res["overlapped"],
                "value": dof / (res["kernel_only"] / 1e3), "unit": "DOF-updates/s",
                "plane_bytes": plane_bytes, "plane_copy_ms": res["plane_copy_only"],
                "plane_copy_GBps_on_device": plane_bytes / (res["plane_copy_only"] / 1e3) / 1e9})
    return out


def gradient_leg(B, torch, I, n: int = 96, m: int = 3, steps: int = 200) -> dict:
    """The differentiation workload: n^3 cells, order m, FP64, a Ricker point
    source at the cube centre (sigma = 2h, f0 = c/(8h), t0 = 1.2/f0), 32
    receivers on the plane z = 0.75, `steps` steps; misfit 1/2 |traces - obs|^2
    against traces from a seeded perturbed initial u; gradient with respect to
    u0, u_t0 and the per-half-step source amplitudes by the library's adjoint
    sweep. Checked at full size by central differences in one direction."""
    from paper_1609_09841_amd.autograd import receiver_traces
    M = m + 1
    f0 = n / 8.0
    src = {"x": (0.5, 0.5, 0.5), "sigma": 2.0 / n, "freq": f0, "t0": 1.2 / f0, "amplitude": 1.0}
    kz = int(round(0.75 * n))
    rec = [((12 * a + 6) * n // 96, (24 * b + 12) * n // 96, kz) for a in range(8) for b in range(4)]
    u0, ut0 = I.fourier_initial(n, m, device="cuda")
    du, _ = I.fourier_initial(n, m, seed=1610, nmodes=4, kmax=4, device="cuda")
    amps = torch.ones(2 * steps, dtype=torch.float64, device="cuda")
    out = {"workload": f"{n}^3 cells, m={m}, FP64, Ricker source at the centre, 32 receivers on z=0.75, "
                       f"{steps} steps, misfit against traces from u0 + 0.1 du (seeded)"}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream), B.Solver(n, m, 0.5, 1.0, stream=stream) as s:
        s.set_receivers(rec)
        s.set_source(src)
        obs = receiver_traces(s, u0 + 0.1 * du, ut0, amps, steps).detach()
        x = [u0.clone().requires_grad_(), ut0.clone().requires_grad_(), amps.clone().requires_grad_()]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = receiver_traces(s, *x, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J = 0.5 * ((tr - obs) ** 2).sum()
        grads = torch.autograd.grad(J, x)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        d = torch.randn(u0.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
        eps = 1e-3
        with torch.no_grad():
            jp = 0.5 * ((receiver_traces(s, x[0] + eps * d, x[1], x[2], steps) - obs) ** 2).sum().item()
            jm = 0.5 * ((receiver_traces(s, x[0] - eps * d, x[1], x[2], steps) - obs) ** 2).sum().item()
        fd = (jp - jm) / (2 * eps)
        ad = (grads[0] * d).sum().item()
    dof = 2 * M ** 3 * n ** 3 * 2 * steps
    out.update({"misfit": J.item(), "forward_s": t1 - t0, "adjoint_s": t2 - t1,
                "forward_DOF_updates_per_s": dof / (t1 - t0), "adjoint_DOF_updates_per_s": dof / (t2 - t1),
                "grad_norms": {"u0": grads[0].norm().item(), "ut0": grads[1].norm().item(),
                               "amps": grads[2].norm().item()},
                "central_difference_check": {"fd": fd, "adjoint": ad, "rel_err": abs(fd - ad) / abs(ad)}})
    del u0, ut0, du, x, grads, tr, obs, d
    torch.cuda.empty_cache()
    return out


def cpu_baseline(m: int, n_s: int) -> dict:
    """The oracle (plain FP64 C, OpenMP) on a bounded sample of the workload:
    the same data recipe and order on an n_s^3 grid, one full step."""
    from oracle import oracle as O
    from paper_1609_09841_amd import inputs as I
    O.load()
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    u0, ut0 = I.fourier_initial(n_s, m)
    u0, ut0 = u0.numpy(), ut0.numpy()
    c0, t0 = time.process_time(), time.perf_counter()
    O.run(n_s, m, 0.5, 1.0, u0, ut0, 1)
    sec = time.perf_counter() - t0
    cpu = time.process_time() - c0   # summed over the process's threads
    dofs = 2 * (m + 1) ** 3 * n_s ** 3 * 2 * 1
    # a CPU quota of the container caps the cores the threads really get
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, period = fh.read().split()
            quota = None if q == "max" else float(q) / float(period)
    except (OSError, ValueError):
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    # one thread, in a child process (the OpenMP team size is fixed once the
    # oracle library is loaded): a 32^3 sample of the same recipe
    single = None
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "from oracle import oracle as O\nfrom paper_1609_09841_amd import inputs as I\n"
            "u0, ut0 = I.fourier_initial(32, %d)\nt0 = time.perf_counter()\n"
            "O.run(32, %d, 0.5, 1.0, u0.numpy(), ut0.numpy(), 1)\nprint(time.perf_counter() - t0)\n") % (ROOT, m, m)
    try:
        import subprocess
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, OMP_NUM_THREADS="1"))
        s1 = float(r.stdout.strip().splitlines()[-1])
        single = {"value": 2 * (m + 1) ** 3 * 32 ** 3 * 2 / s1, "cores": 1,
                  "sample": f"32^3 cells, m={m}, 1 full step, {s1:.2f} s on 1 thread"}
    except Exception as exc:  # reported, not fatal
        single = {"error": str(exc)}
    return {"value": dofs / sec, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_s}^3 cells, m={m}, 1 full step (2 half steps) of the same Fourier-mode "
                      f"workload, {sec:.2f} s on {cores} threads",
            "effective_parallelism": cpu / sec, "cgroup_cpu_quota": quota,
            "cpu_model": model, "single_thread": single}


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
    roofline = None
    if args.variant.startswith("fused"):
        flops = fused_flops_per_cell(m) * cells
        achieved = flops / avg_launch_s / 1e12
        gbs = fused_bytes_per_cell(m) * cells / avg_launch_s / 1e9
        common = {"avg_launch_ms": avg_launch_s * 1e3,
                  "algorithmic_bytes_per_launch": fused_bytes_per_cell(m) * cells,
                  "algorithmic_flops_per_launch": flops}
        if m == 3:
            # arithmetic intensity 14.7 flop/B, above the FP64 ridge (78.6 / 8 = 9.8)
            traffic = measured_traffic() if n == 128 else None
            roofline = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                        "kernel": "fused_mfma4_kernel (FP64 MFMA 4x4x4, two z-adjacent batches per wave)",
                        # context: the FP64 MFMA rate measured on this chip by the committed
                        # microbenchmark (profiles/mfma_throughput_gfx950.md)
                        "measured_mfma_fp64_TFLOPs": MEASURED_FP64_MFMA_TFLOPS,
                        "frac_of_measured_mfma": achieved / MEASURED_FP64_MFMA_TFLOPS,
                        "hbm_GBps_algorithmic": gbs, "hbm_frac_algorithmic": gbs / HBM_PEAK_GBS, **common}
        else:
            # m = 1, 2: 3.5 and 6.2 flop/B, below the ridge: HBM-bound
            roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                        "kernel": f"fused_valu_small_kernel<{m + 1}> (FP64 VALU)",
                        "fp64_TFLOPs": achieved, **common}

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
    if not args.no_mixed and m == 3 and args.variant == "fused-taylor":
        mixed = {}
        for prec in ("fp32", "bf16x3"):
            pms, _, pu, put, _ = time_variant(B, torch, n, m, u0, ut0, K, W, "fused-taylor", prec)
            mixed[prec] = {"value": dof_updates_per_step * K / (pms / 1e3), "ms_per_step": pms / K,
                           "speedup_vs_fp64": ms / pms, "rel_l2_vs_fp64": errors(I, pu, put, u, ut)}
            del pu, put
        out["mixed"] = mixed
    del u, ut
    torch.cuda.empty_cache()
    if not args.no_precision_study and m == 3:
        del u0, ut0
        torch.cuda.empty_cache()
        out["precision_study"] = precision_study(B, torch, I)
    if not args.no_advection:
        out["advection"] = advection_leg(B, torch, I)
    if not args.no_batch:
        out["batch"] = batch_leg(B, torch, I, steps=args.batch_steps)
    if not args.no_gradient:
        out["gradient"] = gradient_leg(B, torch, I, steps=args.gradient_steps)
    if not args.no_slab and m == 3:
        out["slab"] = slab_leg(B, torch, I, n=args.n)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
