"""Seeded synthetic inputs shared by the GPU library's callers and the tests.

This module holds parameters and random draws only: no step of the
phase-field method is computed here.  The parameter ranges follow the
paper's dataset description (Materials and Methods, "Dataset"): deposition
rate 0.3-1.0 in simulation units, deposition angle 50-90 degrees, varied
species mobilities, 50 % initial composition, dimensionless uniform 2-D
meshes.  The defaults are this build's frozen parameter set P0.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014),
counter-based: output n of the stream started at `seed` is
mix(seed + (n + 1) * gamma).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
# key of the per-realisation parameter stream (first digits of pi)
_PARAM_KEY = 0x243F6A8885A308D3


@dataclass
class PFParams:
    """Grid, model constants and run controls of one phase-field problem."""

    nx: int = 128
    ny: int = 128
    batch: int = 1
    precision: str = "f64"        # "f32" or "f64" (storage and arithmetic)
    bc_mode: str = "pvd"          # "pvd" (substrate + inlet) or "periodic"
    flux_on: bool = True          # False: incident vapour velocity is zero
    seed: int = 0
    h: float = 1.0
    dt: float = 0.0               # <= 0: dt_factor * stability limit
    dt_factor: float = 0.2
    # free energy: double wells and gradient energies
    W_c: float = 1.0
    W_phi: float = 1.0
    kappa_c: float = 1.0
    kappa_phi: float = 2.0
    # composition mobility (bulk and surface, species A and B), phi mobility
    MA_bulk: float = 1.0
    MB_bulk: float = 0.5
    MA_surf: float = 5.0
    MB_surf: float = 2.5
    sigma_surf: float = 0.4
    M_phi: float = 1.0
    M_scale: float = 1.0
    # vapour transport
    D_rho: float = 1.0
    v0: float = 0.5
    theta_deg: float = 90.0
    rho_in: float = 1.0
    # initial condition
    c0: float = 0.5
    c_noise: float = 0.01
    film_h: float = 0.0           # <= 0: ny * h / 8
    # model variants: "euler" or "midpoint" time integration; standard
    # deviation of the per-step interface composition draw (0: off)
    integrator: str = "euler"
    interface_noise: float = 0.0
    # optional per-realisation incident speed and mean composition
    v0_per: Optional[np.ndarray] = field(default=None, repr=False)
    c0_per: Optional[np.ndarray] = field(default=None, repr=False)

    def replace(self, **kw) -> "PFParams":
        return dataclasses.replace(self, **kw)

    def v0_of(self, b: int) -> float:
        return float(self.v0_per[b]) if self.v0_per is not None else float(self.v0)

    def c0_of(self, b: int) -> float:
        return float(self.c0_per[b]) if self.c0_per is not None else float(self.c0)

    def vmax(self) -> float:
        if self.v0_per is not None:
            return float(np.max(np.abs(self.v0_per)))
        return abs(float(self.v0))


def splitmix64(seed: int, counters) -> np.ndarray:
    """Output `counters` (array of n) of the SplitMix64 stream of `seed`."""
    n = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (n + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counters) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each SplitMix64 output."""
    return (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def realisation_draws(seed: int, batch: int, v0_nom: float = 0.5):
    """Per-realisation (v0, c0): realisation b uses seed + b and draws the
    rate from [0.5, 2] x nominal and the composition from [0.3, 0.7]."""
    v0 = np.empty(batch)
    c0 = np.empty(batch)
    for b in range(batch):
        u = uniform01((seed + b) ^ _PARAM_KEY, [0, 1])
        v0[b] = v0_nom * (0.5 + 1.5 * u[0])
        c0[b] = 0.3 + 0.4 * u[1]
    return v0, c0


def initial_state(p: PFParams):
    """Seeded initial condition as float64 arrays [batch, ny, nx]:
    c = c0 + c_noise (2U - 1) everywhere; a flat film of height film_h as the
    equilibrium tanh profile of the phi double well; rho = rho_in (1-phi)/2.
    Realisation b uses the noise stream of seed + b, counter j*nx + i."""
    nx, ny, B = p.nx, p.ny, p.batch
    H0 = p.film_h if p.film_h > 0 else ny * p.h / 8.0
    width = np.sqrt(2.0 * p.kappa_phi / p.W_phi)
    y = (np.arange(ny) + 0.5) * p.h
    prof = np.tanh((H0 - y) / width)
    ctr = np.arange(ny * nx, dtype=np.uint64)
    c = np.empty((B, ny, nx))
    for b in range(B):
        U = uniform01(p.seed + b, ctr).reshape(ny, nx)
        c[b] = p.c0_of(b) + p.c_noise * (2.0 * U - 1.0)
    phi = np.broadcast_to(prof[None, :, None], (B, ny, nx)).copy()
    rho = p.rho_in * (1.0 - phi) / 2.0
    return c, phi, rho


def random_state(seed: int, batch: int, ny: int, nx: int, film: bool = True):
    """A rough, far-from-equilibrium state for parity tests: every field
    carries O(1) seeded noise so that every term of the step is active."""
    ctr = np.arange(3 * batch * ny * nx, dtype=np.uint64)
    U = uniform01(seed ^ 0x13198A2E03707344, ctr).reshape(3, batch, ny, nx)
    c = 0.2 + 0.6 * U[0]
    if film:
        y = np.arange(ny)[None, :, None]
        base = np.tanh((ny / 3.0 - y) / 2.0)
        phi = np.clip(base + 0.3 * (2 * U[1] - 1), -1.2, 1.2)
    else:
        phi = 2 * U[1] - 1
    rho = np.clip(0.5 * (1 - phi) + 0.2 * U[2], 0.0, None)
    return c, phi, rho
