"""Throughput of the explicit PVD phase-field step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A "step" is one explicit Euler step of the whole hot path (potentials,
mobility, conserved updates, deposition, vapour transport) over the whole
grid of the workload.  The default workload is the 1024 x 1024 FP32
production run (50,000 steps, FP64 diagnostics, seeded synthetic inputs with
the paper's dataset parameter ranges).  The state is resident in HBM before
timing starts; W untimed steps are followed by exactly K timed steps
bracketed by device synchronisation.  Prints one JSON line with GLUPS
(giga lattice-site updates per second), the roofline of the stepper kernel
(algorithmic bytes per launch over the event-timed average launch duration,
against the 8 TB/s HBM peak), a size sweep for the bandwidth claim at
working sets larger than the 256 MB Infinity Cache, and the FP64 CPU oracle
timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_LUP = {"f32": 24, "f64": 48}   # read + write c, phi, rho


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="dns_1024_f32",
                    choices=["dns_1024_f32", "dns_8192_f32", "batched_32x512_f32", "dns_small_128_f64",
                             "adjoint_256_f32"])
    ap.add_argument("--temporal-block", type=int, default=None)
    ap.add_argument("--graph-mode", type=int, default=0, help="0: replay HIP graphs of launches; 1: plain launches")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--ref-copy", action="store_true",
                    help="first run one 512 MiB device copy (reference kernel for counter scaling)")
    return ap.parse_args()


def make_params(name: str):
    from paper_2312_05410_amd import workloads

    if name == "dns_1024_f32":
        return workloads.dns_production(0), workloads.STEPS[name]
    if name == "dns_8192_f32":
        return workloads.dns_production(0, n=8192), workloads.STEPS[name]
    if name == "batched_32x512_f32":
        return workloads.batched(0), workloads.STEPS[name]
    return workloads.dns_small(0, "f64"), workloads.STEPS[name]


def time_steps(sim, steps: int, warmup: int):
    """Event-timed K steps on the stream the kernels are launched on."""
    import torch

    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    t0 = time.perf_counter()
    sim.step(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def launches_for(steps: int, K: int) -> int:
    """Number of stepper launches the library issues for `steps` steps with
    K fused sub-steps (K full launches, the remainder, and one split when
    the count is odd and a launch has two or more sub-steps)."""
    q, rem = divmod(steps, K)
    L = q + (1 if rem else 0)
    if L % 2 == 1 and (rem >= 2 or (K >= 2 and q >= 1)):
        L += 1
    return L


def kernel_name(prec: str, K: int, rows: int) -> str:
    t = "float" if prec == "f32" else "double"
    if K == 1:
        ahead = rows + 1 if rows <= 8 else 4      # load look-ahead rows of the strip-march kernel
        return f"march_kernel<{t}, {rows}, {ahead}>"
    return f"step_kernel<{t}, {K}, {rows}>"


def gpu_leg(args, p, steps, warmup, K):
    import torch

    from paper_2312_05410_amd._lib import Simulator

    if args.ref_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sim = Simulator(p, temporal_block=K, graph_mode=args.graph_mode)
    Kr, rows = sim.launch
    dt_s, wall = time_steps(sim, steps, warmup)
    m = sim.mass()
    e = sim.energy()
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(e))
    sim.close()
    cells = p.nx * p.ny * p.batch
    glups = cells * steps / dt_s / 1e9
    return dict(seconds=dt_s, wall=wall, glups=glups, launches=launches_for(steps, Kr), K=Kr, rows=rows)


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed counter summary of this
    workload, if it was taken on the current stepper sources and kernel."""
    from paper_2312_05410_amd import rocprof_summary

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("stepper_source_sha256_16") != rocprof_summary.stepper_hash() or kv.get("kernel") != kernel:
        return None
    return float(kv["hbm_bytes_per_launch"])


def sweep(K, graph_mode, sizes=(1024, 2048, 4096, 8192)):
    """GLUPS of the production model at growing sizes, in the library's
    launch shape for each size (the HBM claim needs working sets well above
    the 256 MB Infinity Cache: 8192^2 FP32 is 805 MB, 1.6 GB ping-pong)."""
    from paper_2312_05410_amd import workloads
    from paper_2312_05410_amd._lib import Simulator

    out = []
    for n in sizes:
        p = workloads.dns_production(0, n=n)
        steps = max(40, int(4e9 / (n * n)) // 2 * 2)
        sim = Simulator(p, temporal_block=K, graph_mode=graph_mode)
        Kr, rows = sim.launch
        dt_s, _ = time_steps(sim, steps, 20)
        sim.close()
        glups = n * n * steps / dt_s / 1e9
        state_mb = 3 * n * n * 4 / 1e6
        out.append(dict(n=n, steps=steps, state_MB=round(state_mb, 1), glups=round(glups, 2),
                        kernel=kernel_name("f32", Kr, rows),
                        effective_GBs=round(glups * BYTES_PER_LUP["f32"], 1),
                        frac_hbm=round(glups * BYTES_PER_LUP["f32"] / HBM_PEAK_GBS, 4)))
        print(f"# sweep {n}^2: {glups:.1f} GLUPS", file=sys.stderr, flush=True)
    return out


def cpu_leg(p, seconds: float):
    """The FP64 oracle as it stands, on the host cores, on a bounded sample
    of the same workload (first realisation, seeded initial condition)."""
    import oracle

    q = p.replace(batch=1, precision="f64", v0_per=None, c0_per=None,
                  v0=p.v0_of(0), c0=p.c0_of(0))
    s = oracle.State.seeded(q)
    t0 = time.perf_counter()
    s.step(4)
    probe = time.perf_counter() - t0
    n = max(4, int(seconds / max(probe / 4, 1e-9)))
    t0 = time.perf_counter()
    s.step(n)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=round(q.nx * q.ny * n / el / 1e9, 6), unit="GLUPS", cores=threads, kind="oracle",
                sample=f"{q.nx}x{q.ny} FP64, {n} steps of realisation 0 from its seeded initial condition "
                       f"({el:.1f} s, OpenMP over rows)")


def adjoint_leg(args):
    """Forward with checkpoints plus the reverse sweep (recompute + adjoint)
    of the adjoint workload; GLUPS counts forward steps of the whole job."""
    import torch

    from paper_2312_05410_amd import workloads
    from paper_2312_05410_amd.adjoint import final_state, l2_mismatch
    from paper_2312_05410_amd.inputs import initial_state

    p = workloads.adjoint_case(precision="f32")
    n, every = workloads.ADJOINT_STEPS, workloads.ADJOINT_EVERY
    c, phi, rho = initial_state(p)
    dev = lambda a: torch.as_tensor(a, dtype=torch.float32, device="cuda").contiguous()
    u0 = (dev(c), dev(phi), dev(rho))
    # target: the same seed with the target parameters, run by the stepper
    tp = p.replace(M_scale=workloads.ADJOINT_TARGET[0], v0=workloads.ADJOINT_TARGET[1] * p.v0)
    from paper_2312_05410_amd._lib import Simulator

    ts = Simulator(tp, tensors=[t.clone() for t in u0])
    ts.step(n)
    target = (ts.c, ts.phi, ts.rho)
    times = []
    for rep in range(2):
        Ms = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        v0 = torch.tensor(p.v0, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = l2_mismatch(final_state(Ms, v0, p, u0, n, every), target, p.h)
        L.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    el = times[-1]
    cells = p.nx * p.ny
    return {"metric": "adjoint forward+reverse time", "value": round(el * 1e3, 2), "unit": "ms",
            "n_gpus": 1, "steps": n, "warmup": 1, "higher_is_better": False, "dtype": "f32",
            "data": "synthetic (seeded)", "vs_baseline": None,
            "config": {"workload": "adjoint_256_f32", "nx": p.nx, "ny": p.ny, "checkpoint_every": every,
                       "loss": float(L), "dL_dMscale": float(Ms.grad), "dL_dv0": float(v0.grad)},
            "glups_equiv": round(cells * n / el / 1e9, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)
    if args.workload == "adjoint_256_f32":
        print(json.dumps(adjoint_leg(args)), flush=True)
        return
    import torch

    from paper_2312_05410_amd import workloads

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    p, total_steps = make_params(args.workload)
    prec = p.precision
    K = args.temporal_block if args.temporal_block is not None else workloads.BENCH_TEMPORAL_BLOCK[prec]
    steps = args.steps if args.steps is not None else total_steps
    warmup = args.warmup if args.warmup is not None else min(1000, steps)

    g = gpu_leg(args, p, steps, warmup, K)
    cells = p.nx * p.ny * p.batch
    launch_s = g["seconds"] / g["launches"]
    bytes_per_launch = BYTES_PER_LUP[prec] * cells * steps / g["launches"]
    achieved = bytes_per_launch / launch_s / 1e9
    kname = kernel_name(prec, g["K"], g["rows"])
    tb = measured_traffic(args.workload, kname)
    traffic = None if tb is None else round(tb / launch_s / 1e9, 1)
    result = {
        "metric": "phase-field GLUPS & %HBM peak",
        "value": round(g["glups"], 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": g["seconds"] * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded; parameter ranges of the paper's dataset)",
        "config": {"workload": args.workload, "nx": p.nx, "ny": p.ny, "batch": p.batch,
                   "steps_total": total_steps, "temporal_block": g["K"], "tile_rows": g["rows"],
                   "launches": g["launches"],
                   "graph_mode": args.graph_mode,
                   "seed": p.seed, "dt": None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kname,
                     "avg_launch_us": round(launch_s * 1e6, 3),
                     "bytes_per_launch": int(bytes_per_launch),
                     "traffic_bytes_per_launch": None if tb is None else int(tb)},
        "host_wall_s": round(g["wall"], 4),
    }
    if not args.no_sweep and prec == "f32":
        result["size_sweep"] = sweep(K, args.graph_mode)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_leg(p, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
