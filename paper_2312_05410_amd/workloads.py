"""The standard workloads of the stepper, by name, with their sizes.

* dns_small_128_f64: 128 x 128, FP64, 1000 explicit Euler steps at 0.2 of
  the stability limit, c = 0.5 +- 0.01 seeded noise, flat film (parity case).
* dns_1024_f32: 1024 x 1024, FP32 fields with FP64 diagnostics, 50,000
  steps; deposition rate and composition drawn per seed (rate in [0.5, 2] x
  nominal, composition in [0.3, 0.7]).  The throughput workload.
* dns_8192_f32: the production model on 8192 x 8192 (805 MB of state, 1.6 GB
  with the ping-pong copy), 500 steps: the size for the HBM-bandwidth claim.
* midpoint_1024_f32 / interface_1024_f32: dns_1024_f32 with the explicit
  midpoint integrator (two launches per step), or with truncated-Gaussian
  interface composition draws (sigma 0.1) after every step.
* batched_32x512_f32: 32 independent 512 x 512 FP32 realisations with seeded
  (rate, composition) pairs, 10,000 steps each.

All inputs are synthetic and seeded (see inputs.py); the paper's dataset is
not available, these stand in for its 256^2 PVD trajectories with the
parameter ranges of its dataset description.
"""
from __future__ import annotations

from .inputs import PFParams, realisation_draws

V0_NOM = 0.5

# fused sub-steps per launch used by the throughput measurement and by the
# full-size parity tests, which run the same launch configuration: 0 means
# the library's own choice for the grid
BENCH_TEMPORAL_BLOCK = {"f32": 0, "f64": 0}


def dns_small(seed: int = 0, precision: str = "f64") -> PFParams:
    return PFParams(nx=128, ny=128, batch=1, precision=precision, seed=seed, v0=V0_NOM, c0=0.5)


def dns_production(seed: int = 0, n: int = 1024, precision: str = "f32") -> PFParams:
    v0, c0 = realisation_draws(seed, 1, V0_NOM)
    return PFParams(nx=n, ny=n, batch=1, precision=precision, seed=seed, v0=float(v0[0]), c0=float(c0[0]))


def batched(seed: int = 0, batch: int = 32, n: int = 512, precision: str = "f32") -> PFParams:
    v0, c0 = realisation_draws(seed, batch, V0_NOM)
    return PFParams(nx=n, ny=n, batch=batch, precision=precision, seed=seed, v0=V0_NOM,
                    v0_per=v0, c0_per=c0)


# Adjoint workload: 256 x 256, 2000 steps with a checkpoint every 50; the
# loss is the L2 mismatch of the final fields to a target run of the same
# seed with (M_scale, v0) = (1.1, 0.9 v0_nom); gradients in (M_scale, v0) at
# a fixed dt chosen below the stability limit of both runs (the P0 limit is
# 4.17e-3 at M_scale = 1 and 3.79e-3 at M_scale = 1.1).
ADJOINT_STEPS = 2000
ADJOINT_EVERY = 50
ADJOINT_TARGET = (1.1, 0.9)
ADJOINT_DT = 7.5e-4


def adjoint_case(seed: int = 0, precision: str = "f32") -> PFParams:
    return PFParams(nx=256, ny=256, batch=1, precision=precision, seed=seed, v0=V0_NOM, c0=0.5,
                    c_noise=0.05, dt=ADJOINT_DT)


# Variant workloads of the throughput measurement: the 1024 x 1024 FP32
# production run with the explicit midpoint integrator, and with interface
# composition draws of width INTERFACE_SIGMA on the vapour side.
INTERFACE_SIGMA = 0.1

STEPS = {"dns_small_128_f64": 1000, "dns_1024_f32": 50_000, "batched_32x512_f32": 10_000,
         # the production model at a size far above the 256 MB Infinity Cache
         "dns_8192_f32": 500}
