"""Pins of the oracle's discrete adjoint (reverse mode of the explicit step).

The adjoint is pinned to the forward oracle, which the pins in
test_oracle_pins.py tie to the mathematics: the transpose identity
<J^T w, v> = <w, J v> for the one-step Jacobian J (J v by central
differences of the forward step, in the state and in both parameters), and
the full checkpointed gradient of a final-state loss against central finite
differences of that loss (h = 1e-4).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2312_05410_amd.inputs import PFParams, random_state, uniform01


def one_step(p, v0, dt, u):
    return oracle.run(p, v0, dt, 1, u)


@pytest.mark.parametrize("bc,theta", [("pvd", 60.0), ("pvd", 90.0), ("periodic", 35.0)])
def test_adjoint_transpose_identity(bc, theta):
    nx, ny = 12, 10
    p = PFParams(nx=nx, ny=ny, bc_mode=bc, theta_deg=theta, v0=0.8, M_scale=1.2, h=0.9)
    dt = 0.2 * oracle.dt_limit(p)
    c, phi, rho = random_state(41, 1, ny, nx)
    u = (c[0], phi[0], rho[0])
    R = uniform01(42, np.arange(6 * nx * ny)).reshape(6, ny, nx) - 0.5
    v, w = R[:3], R[3:]
    eps = 1e-6
    up = [a + eps * b for a, b in zip(u, v)]
    um = [a - eps * b for a, b in zip(u, v)]
    Jv = [(a - b) / (2 * eps) for a, b in zip(one_step(p, p.v0, dt, up), one_step(p, p.v0, dt, um))]
    JTw, g = oracle.adjoint_step(p, p.v0, dt, u, w)
    lhs = sum(float(np.sum(a * b)) for a, b in zip(JTw, v))
    rhs = sum(float(np.sum(a * b)) for a, b in zip(w, Jv))
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1.0)
    # parameter directions: one step is linear in M_scale and in v0, so a
    # large central difference is exact up to rounding
    e2 = 0.1
    dMs = [(a - b) / (2 * e2) for a, b in zip(one_step(p.replace(M_scale=p.M_scale + e2), p.v0, dt, u),
                                               one_step(p.replace(M_scale=p.M_scale - e2), p.v0, dt, u))]
    dv0 = [(a - b) / (2 * e2) for a, b in zip(one_step(p, p.v0 + e2, dt, u), one_step(p, p.v0 - e2, dt, u))]
    gM = sum(float(np.sum(a * b)) for a, b in zip(w, dMs))
    gv = sum(float(np.sum(a * b)) for a, b in zip(w, dv0))
    assert abs(g[0] - gM) <= 1e-9 * max(abs(gM), 1e-3)
    assert abs(g[1] - gv) <= 1e-9 * max(abs(gv), 1e-3)


def test_loss_gradient_matches_central_differences():
    """Final-state loss against a target run with (M_scale, v0) = (1.1, 0.9 v0);
    gradients at (1, v0) by the checkpointed adjoint versus central
    differences with h = 1e-4 (fixed dt)."""
    nx, ny = 32, 32
    p = PFParams(nx=nx, ny=ny, theta_deg=70.0, c_noise=0.05)
    dt = 0.2 * oracle.dt_limit(p.replace(M_scale=1.1))
    c, phi, rho = oracle.init(p)
    u0 = (c[0], phi[0], rho[0])
    n, every = 300, 50
    target = oracle.run(p.replace(M_scale=1.1), 0.9 * p.v0, dt, n, u0)
    L, gM, gv = oracle.loss_grad(p, p.v0, dt, n, every, u0, target)
    assert L == pytest.approx(oracle.loss(p, p.v0, dt, n, u0, target), rel=1e-13)
    h = 1e-4
    fdM = (oracle.loss(p.replace(M_scale=1 + h), p.v0, dt, n, u0, target)
           - oracle.loss(p.replace(M_scale=1 - h), p.v0, dt, n, u0, target)) / (2 * h)
    fdv = (oracle.loss(p, p.v0 + h, dt, n, u0, target) - oracle.loss(p, p.v0 - h, dt, n, u0, target)) / (2 * h)
    assert gM == pytest.approx(fdM, rel=1e-6)
    assert gv == pytest.approx(fdv, rel=1e-6)
    assert abs(gM) > 0 and abs(gv) > 0


def test_checkpoint_interval_does_not_change_gradient():
    p = PFParams(nx=16, ny=24, theta_deg=80.0)
    dt = 0.2 * oracle.dt_limit(p)
    c, phi, rho = oracle.init(p)
    u0 = (c[0], phi[0], rho[0])
    target = oracle.run(p, 0.8 * p.v0, dt, 120, u0)
    a = oracle.loss_grad(p, p.v0, dt, 120, 1000, u0, target)
    b = oracle.loss_grad(p, p.v0, dt, 120, 7, u0, target)
    assert np.array_equal(a, b)
