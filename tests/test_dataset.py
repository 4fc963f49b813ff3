"""Paper-size dataset generator: parameter draws and snapshot schedule
(host only), and on the GPU the snapshots of a trajectory."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2312_05410_amd import dataset as D


def test_draws_cover_the_paper_ranges():
    specs = [D.draw(7, i) for i in range(400)]
    v = np.array([s.v0 for s in specs])
    th = np.array([s.theta_deg for s in specs])
    ratio = np.array([s.MB_bulk / s.MA_bulk for s in specs])
    assert v.min() >= 0.3 and v.max() <= 1.0 and v.max() - v.min() > 0.6
    assert th.min() >= 50 and th.max() <= 90 and th.max() - th.min() > 35
    assert ratio.min() >= 0.3 and ratio.max() <= 0.7
    assert D.draw(7, 3) == D.draw(7, 3) and D.draw(7, 3) != D.draw(8, 3)


def test_schedule_lands_snapshots_on_steps():
    from paper_2312_05410_amd._lib import dt_limit

    for i in range(5):
        p = D.params(D.draw(1, i))
        dt, per = D.schedule(p)
        assert dt <= 0.2 * dt_limit(p) * (1 + 1e-12)
        assert abs(dt * per * D.SNAPSHOTS - D.T_END) < 1e-9


@pytest.mark.gpu
def test_trajectory_snapshots_are_the_stepper_states():
    import torch

    from paper_2312_05410_amd._lib import Simulator

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[case] dataset trajectory 64^2, 5 snapshots", flush=True)
    spec = D.draw(3, 2)
    snaps = D.trajectory(spec, n=64, snapshots=5, t_end=1.0, fields="cpr")
    p = D.params(spec, 64)
    dt, per = D.schedule(p, 5, 1.0)
    sim = Simulator(p.replace(dt=dt))
    solid = []
    for k in range(5):
        sim.step(per)
        for f, u in enumerate((sim.c, sim.phi, sim.rho)):
            assert torch.equal(snaps[k, f], u[0])
        solid.append(float(sim.phi.double().mean()))   # grows with the film
    assert solid[-1] > solid[0]
    sim.close()
