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
against the 8 TB/s HBM peak; with two fused steps per launch, or the
resident stepper's one launch per call that keeps the state on chip, the
effective rate can exceed the peak), the HBM bytes per launch from the
committed counter summary when it matches the sources, a size sweep for the bandwidth
claim at working sets larger than the 256 MB Infinity Cache, a plain device
copy rate, and the FP64 CPU oracle timed on a bounded sample on the host
cores.  Other workloads: dns_8192_f32, batched_32x512_f32, dns_small_128_f64,
the model variants (midpoint_1024_f32, interface_1024_f32), adjoint_256_f32,
unet_512_bf16 (U-Net training and inference) and blended_512_f32 (the
blended DNS + U-Net run against plain DNS at fixed error).
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
# explicit midpoint: the first stage reads the state and writes the midpoint
# (6 words per cell), the second reads the midpoint and the base state and
# writes the new state in place (9 words per cell)
MIDPOINT_WORDS = (6, 9)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="dns_1024_f32",
                    choices=["dns_1024_f32", "dns_8192_f32", "batched_32x512_f32", "dns_small_128_f64",
                             "midpoint_1024_f32", "interface_1024_f32",
                             "adjoint_256_f32", "unet_512_bf16", "blended_512_f32"])
    ap.add_argument("--temporal-block", type=int, default=None)
    ap.add_argument("--lane-cols", type=int, default=0, help="single-step kernel: grid columns per lane (0: auto)")
    ap.add_argument("--graph-mode", type=int, default=0, help="0: replay HIP graphs of launches; 1: plain launches")
    ap.add_argument("--fused", type=int, default=0,
                    help="kernel of fused launches: 1 LDS tile, 2 register march, 3 resident stepper (0: auto)")
    ap.add_argument("--tile-rows", type=int, default=0, help="rows per wave / tile height (0: auto)")
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
    if name == "midpoint_1024_f32":
        return workloads.dns_production(0).replace(integrator="midpoint"), workloads.STEPS["dns_1024_f32"]
    if name == "interface_1024_f32":
        return (workloads.dns_production(0).replace(interface_noise=workloads.INTERFACE_SIGMA),
                workloads.STEPS["dns_1024_f32"])
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


def kernel_name(prec: str, K: int, rows: int, base: bool = False, noise: bool = False, cols: int = 1,
                fused: int = 1, mid: bool = False) -> str:
    t = "float" if prec == "f32" else "double"
    if fused == 3:                                # resident stepper: one launch per call
        return f"resident_kernel<{rows}, {'true' if mid else 'false'}, {'true' if noise else 'false'}>"
    if K == 2 and fused == 2:                     # two steps in the register strip march
        return f"march_k2_kernel<{t}, {rows}, {rows + 1 if rows <= 8 else 4}, false>"
    if K == 1:
        ahead = rows + 1 if rows <= 8 else 4      # load look-ahead rows of the strip-march kernel
        b = "true" if base else "false"           # second midpoint stage: update added to a base state
        d = "true" if noise else "false"          # interface composition draws
        if cols == 2:                             # two grid columns per lane (FP32)
            return f"march2_kernel<{rows}, {ahead}, {b}, {d}>"
        return f"march_kernel<{t}, {rows}, {ahead}, {b}, {d}>"
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
    sim = Simulator(p, temporal_block=K, graph_mode=args.graph_mode, lane_cols=args.lane_cols,
                    fused_kernel=args.fused, tile_rows=args.tile_rows)
    Kr, rows = sim.launch
    cols = sim.lane_cols
    fused = sim.fused_kernel
    dt_s, wall = time_steps(sim, steps, warmup)
    m = sim.mass()
    e = sim.energy()
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(e))
    sim.close()
    cells = p.nx * p.ny * p.batch
    glups = cells * steps / dt_s / 1e9
    launches = 1 if fused == 3 and steps >= 2 else launches_for(steps, Kr)
    return dict(seconds=dt_s, wall=wall, glups=glups, launches=launches, K=Kr, rows=rows, cols=cols,
                fused=fused)


def measured_traffic(workload: str, kernel: str, steps_per_launch: int = 0):
    """HBM bytes per launch from the committed counter summary of this
    workload, if it was taken on the current stepper sources and kernel (for
    a kernel whose launch runs a whole call, the summary's bytes per step
    times the steps of this launch)."""
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
    if "hbm_bytes_per_step" in kv and steps_per_launch:
        return float(kv["hbm_bytes_per_step"]) * steps_per_launch
    return float(kv["hbm_bytes_per_launch"])


def sweep(K, graph_mode, lane_cols=0, sizes=(1024, 2048, 4096, 8192)):
    """GLUPS of the production model at growing sizes, in the library's
    launch shape for each size (the HBM claim needs working sets well above
    the 256 MB Infinity Cache: 8192^2 FP32 is 805 MB, 1.6 GB ping-pong)."""
    from paper_2312_05410_amd import workloads
    from paper_2312_05410_amd._lib import Simulator

    out = []
    for n in sizes:
        p = workloads.dns_production(0, n=n)
        steps = max(40, int(4e9 / (n * n)) // 2 * 2)
        sim = Simulator(p, temporal_block=K, graph_mode=graph_mode, lane_cols=lane_cols)
        Kr, rows = sim.launch
        cols, fused = sim.lane_cols, sim.fused_kernel
        dt_s, _ = time_steps(sim, steps, 20)
        sim.close()
        glups = n * n * steps / dt_s / 1e9
        state_mb = 3 * n * n * 4 / 1e6
        out.append(dict(n=n, steps=steps, state_MB=round(state_mb, 1), glups=round(glups, 2),
                        kernel=kernel_name("f32", Kr, rows, cols=cols, fused=fused),
                        effective_GBs=round(glups * BYTES_PER_LUP["f32"], 1),
                        # algorithmic bytes over time: with two fused steps per launch the state
                        # moves once per two updates, so this can exceed 1; it is not DRAM traffic
                        effective_frac_of_peak=round(glups * BYTES_PER_LUP["f32"] / HBM_PEAK_GBS, 4)))
        print(f"# sweep {n}^2: {glups:.1f} GLUPS", file=sys.stderr, flush=True)
    return out


def copy_bandwidth(nbytes: int = 2 << 30, reps: int = 10) -> float:
    """Device-to-device copy rate (read + write bytes per second, GB/s) of a
    plain tensor copy: the practical ceiling beside the 8 TB/s spec figure."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbs, 1)


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


MFMA_BF16_PEAK_TFLOPS = 2500.0


def unet_forward_flops(cfg) -> float:
    """Multiply-adds x 2 of one forward pass of one sample (convolutions and
    up-samplings; the normalisations and the MLP are negligible)."""
    H, W, L, w = cfg.height, cfg.width, cfg.levels, [cfg.base << l for l in range(cfg.levels)]
    P = lambda l: (H >> l) * (W >> l)
    f = 0.0
    for l in range(L):
        f += 2 * 9 * P(l) * w[l] * (w[l - 1] if l else cfg.in_ch)      # encoder blocks
    f += 2 * 9 * P(L - 1) * w[L - 1] * w[L - 1]                        # bottom block
    for l in range(L - 2, -1, -1):
        f += 2 * P(l + 1) * w[l + 1] * 4 * w[l]                         # up-sampling
        f += 2 * 9 * P(l) * w[l] * 2 * w[l]                             # decoder blocks
    f += 2 * 9 * P(0) * cfg.out_ch * w[0]                              # head
    return f


def unet_leg(args):
    """Training steps (forward, backward, Adam) at the paper's batch of 5 and
    inference at batch 1 on 512^2; the roofline is that of the largest
    convolution (the top decoder block, 64 -> 32 channels at 512^2) timed
    alone with HIP events on its stream."""
    import torch

    from paper_2312_05410_amd import unet as U

    cfg = U.UNetConfig(max_batch=5)
    net = U.UNet(cfg, seed=0)
    n = 5
    st = [torch.rand(n, cfg.height, cfg.width, device="cuda") for _ in range(3)]
    tg = [u + 1e-3 for u in st]
    jump = torch.ones(n, device="cuda")
    steps = args.steps if args.steps is not None else 100
    warmup = args.warmup if args.warmup is not None else 10
    out = net.forward(*st, jump)
    for _ in range(warmup):
        net.forward(*st, jump, out=out)
        net.backward(out, tg, want_loss=False)
        net.adam_step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        net.forward(*st, jump, out=out)
        net.backward(out, tg, want_loss=False)
        net.adam_step()
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / steps
    fwd = unet_forward_flops(cfg)
    # inference, batch 1
    one = [u[:1].contiguous() for u in st]
    o1 = net.forward(*one, jump[:1], train=False)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        net.forward(*one, jump[:1], out=o1, train=False)
    e1.record()
    torch.cuda.synchronize()
    infer_ms = e0.elapsed_time(e1) / steps
    net.close()
    # dominant convolution alone
    x1 = torch.rand(n, cfg.height, cfg.width, 32, device="cuda").to(torch.bfloat16)
    x2 = torch.rand(n, cfg.height, cfg.width, 32, device="cuda").to(torch.bfloat16)
    w = torch.rand(9, 32, 64, device="cuda") - 0.5
    wp = U.conv3x3_prepare(w, 32, 32)
    y = U.conv3x3_fwd_prepared(x1, wp, 32, x2)
    torch.cuda.synchronize()
    reps = 50
    e0.record()
    for _ in range(reps):
        U.conv3x3_fwd_prepared(x1, wp, 32, x2, out=y)
    e1.record()
    torch.cuda.synchronize()
    conv_s = e0.elapsed_time(e1) / reps / 1e3
    conv_flops = 2.0 * 9 * n * cfg.height * cfg.width * 32 * 64
    achieved = conv_flops / conv_s / 1e12
    res = {"metric": "U-Net training throughput", "value": round(n / (train_ms / 1e3), 2), "unit": "samples/s",
           "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(train_ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic (uniform random fields)",
           "config": {"workload": "unet_512_bf16", "height": cfg.height, "width": cfg.width, "batch": n,
                      "levels": cfg.levels, "base": cfg.base,
                      "forward_gflop_per_sample": round(fwd / 1e9, 2),
                      "train_tflops": round(3 * fwd * n / (train_ms / 1e3) / 1e12, 1),
                      "inference_ms_batch1": round(infer_ms, 4),
                      "inference_tflops_batch1": round(fwd / (infer_ms / 1e3) / 1e12, 1)},
           "roofline": {"bound": "mfma", "achieved": round(achieved, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                        "kernel": "conv3_lds_kernel<0, 2, 8, 32, 32, false> (conv3x3 64->32, 5 x 512^2)",
                        "avg_launch_us": round(conv_s * 1e6, 2), "flops_per_launch": conv_flops}}
    if not args.no_cpu:
        res["cpu_baseline"] = unet_cpu_leg(cfg, args.cpu_seconds)
    return res


def unet_cpu_leg(cfg, seconds):
    """The FP64 PyTorch-CPU oracle's forward pass on one 512^2 sample."""
    import numpy as np
    import torch

    from oracle import unet_oracle as uo
    from paper_2312_05410_amd import unet as U
    from paper_2312_05410_amd.unet_inputs import init_params

    params = init_params([(e[0], e[2]) for e in U.param_entries(cfg)], 0)
    net = uo.Net(cfg, params)
    st = [np.full((1, cfg.height, cfg.width), 0.5) for _ in range(3)]
    n, t0 = 0, time.perf_counter()
    with torch.no_grad():
        while True:
            net.forward(*st, np.ones(1))
            n += 1
            if time.perf_counter() - t0 > seconds:
                break
    el = time.perf_counter() - t0
    return {"value": round(n / el, 4), "unit": "samples/s (forward)", "cores": torch.get_num_threads(),
            "kind": "oracle", "sample": f"{n} FP64 forward passes of one 512^2 sample ({el:.1f} s)"}


def blended_leg(args):
    """The blended run (200 DNS steps, then one U-Net leap of 4 x 100 steps,
    repeated to 50,000 steps on 512^2; steps at 0.2 of the stability limit,
    or each DNS segment in fewer steps at 0.95 of it) against plain DNS at
    0.2 of the limit and at larger time steps.  `value`: the best blended
    configuration's time-to-solution ratio against the fastest plain DNS
    whose S2 error is at most the blended run's."""
    import numpy as np

    from paper_2312_05410_amd import surrogate as S
    from paper_2312_05410_amd import unet as U

    path = os.path.join(ROOT, "paper_2312_05410_amd", "weights", "unet_blend_512.npz")
    with np.load(path, allow_pickle=False) as z:
        params = {k: z[k] for k in z.files}
    net = U.UNet(U.UNetConfig(max_batch=1), params=params)
    r = S.compare(net, log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    net.close()
    b = r["runs"][r["best_blend"] or "blend_leap"]
    return {"metric": "blended vs DNS time-to-solution at fixed error", "value": r["speedup_fixed_error"],
            "unit": "x (DNS time / blended time)", "n_gpus": 1, "steps": r["steps"], "warmup": 0,
            "ms_per_step": round(b["ms"] / r["steps"], 6), "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "f32 (DNS) + bf16 (U-Net)",
            "data": "synthetic (seeded; U-Net trained on stepper snapshots only)",
            "config": {"workload": "blended_512_f32", "n": r["n"], "seed": r["seed"],
                       "schedule": f"{S.BLEND_DNS} DNS steps + 1 leap of {S.BLEND_JUMPS} x {S.JUMP} steps",
                       "best_blend": r["best_blend"], "speedup_same_dt": r["speedup_same_dt"],
                       "dns_ms": r["dns_ms"], "runs": r["runs"]}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)
    if args.workload == "adjoint_256_f32":
        print(json.dumps(adjoint_leg(args)), flush=True)
        return
    if args.workload == "unet_512_bf16":
        print(json.dumps(unet_leg(args)), flush=True)
        return
    if args.workload == "blended_512_f32":
        print(json.dumps(blended_leg(args)), flush=True)
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
    noise = p.interface_noise > 0
    if p.integrator == "midpoint" and g["fused"] == 3:
        # the resident stepper: one launch per call, both stages of every step
        word = BYTES_PER_LUP[prec] // 6
        bytes_per_launch = sum(MIDPOINT_WORDS) * word * cells * steps / g["launches"]
        kname = kernel_name(prec, 1, g["rows"], noise=noise, fused=3, mid=True)
    elif p.integrator == "midpoint":
        # two launches per step; the roofline is that of the pair
        word = BYTES_PER_LUP[prec] // 6
        g["launches"] = 2 * steps
        bytes_per_launch = sum(MIDPOINT_WORDS) * word * cells / 2
        kname = (kernel_name(prec, 1, g["rows"], cols=g["cols"]) + " + " +
                 kernel_name(prec, 1, g["rows"], base=True, noise=noise, cols=g["cols"]))
    else:
        bytes_per_launch = BYTES_PER_LUP[prec] * cells * steps / g["launches"]
        kname = kernel_name(prec, g["K"], g["rows"], noise=noise, cols=g["cols"], fused=g["fused"])
    launch_s = g["seconds"] / g["launches"]
    achieved = bytes_per_launch / launch_s / 1e9
    tb = measured_traffic(args.workload, kname, steps if g["fused"] == 3 and g["launches"] == 1 else 0)
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
                   "lane_cols": g["cols"], "fused_kernel": g["fused"],
                   "launches": g["launches"],
                   "graph_mode": args.graph_mode,
                   "seed": p.seed, "dt": None, "integrator": p.integrator,
                   "interface_noise": p.interface_noise},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_frac": None if traffic is None else round(traffic / HBM_PEAK_GBS, 4),
                     "kernel": kname,
                     "avg_launch_us": round(launch_s * 1e6, 3),
                     "bytes_per_launch": int(bytes_per_launch),
                     "traffic_bytes_per_launch": None if tb is None else int(tb)},
        "host_wall_s": round(g["wall"], 4),
    }
    if not args.no_sweep and prec == "f32" and args.workload == "dns_1024_f32":
        result["size_sweep"] = sweep(K, args.graph_mode, args.lane_cols)
        result["device_copy_GBs"] = copy_bandwidth()
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_leg(p, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
