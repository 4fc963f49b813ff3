"""The surrogate pipeline on the GPU: training pairs come from the stepper
exactly, the blended schedule hands states between stepper and U-Net
exactly, and training reduces the held-out loss."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def test_training_set_is_the_stepper_trajectory():
    import torch

    from paper_2312_05410_amd import surrogate as S
    from paper_2312_05410_amd._lib import Simulator

    announce("training set 3 x 64^2 staggered")
    snaps = S.make_training_set(seed0=7, n_traj=3, n_jumps=4, jump=20, stagger=40, n=64)
    for j in range(3):
        sim = Simulator(S.blend_params(7 + j, n=64))
        sim.step(40 * j)
        for k in range(5):
            got = snaps[j, k]
            for f, u in enumerate((sim.c, sim.phi, sim.rho)):
                assert torch.equal(got[f], u[0]), (j, k, f)
            sim.step(20)
        sim.close()


def _zero_head_net(n):
    from paper_2312_05410_amd.unet import UNet, UNetConfig

    net = UNet(UNetConfig(height=n, width=n, base=8, levels=3, groups=4, mlp_hidden=16, basis=16, max_batch=1),
               seed=3)
    p = net.param_dict()
    p["head.gamma"][:] = 0
    p["head.beta"][:] = 0
    net.set_params(p)
    return net


@pytest.mark.parametrize("mode", ["leap", "chain"])
def test_blended_schedule_hands_states_exactly(mode):
    """With a zero output head the U-Net returns its input, so the blended
    run equals the plain DNS with the leapt steps left out, bit for bit."""
    import torch

    from paper_2312_05410_amd import surrogate as S
    from paper_2312_05410_amd._lib import Simulator

    announce(f"blended schedule {mode} 64^2")
    net = _zero_head_net(64)
    steps, dns, jumps = 2000, 200, 2
    state, _, _ = S.blended_run(net, seed=5, steps=steps, dns_block=dns, jumps=jumps, mode=mode, n=64)
    cycles = 0
    t = 0
    while t + dns + jumps * S.JUMP <= steps:
        t += dns + jumps * S.JUMP
        cycles += 1
    sim = Simulator(S.blend_params(5, n=64))
    sim.step(steps - cycles * jumps * S.JUMP)
    torch.cuda.synchronize()
    for a, b in zip(state, (sim.c, sim.phi, sim.rho)):
        assert torch.equal(a, b)
    sim.close()
    net.close()


def test_training_reduces_held_out_loss():
    from paper_2312_05410_amd import surrogate as S
    from paper_2312_05410_amd.unet import UNet, UNetConfig

    announce("training 3 epochs on 4 x 64^2 trajectories")
    snaps = S.make_training_set(seed0=11, n_traj=4, n_jumps=10, jump=50, stagger=500, n=64)
    val = S.make_training_set(seed0=21, n_traj=1, n_jumps=10, jump=50, stagger=500, n=64)
    net = UNet(UNetConfig(height=64, width=64, base=8, levels=3, groups=4, mlp_hidden=16, basis=16, max_batch=5),
               seed=4)
    before = S.evaluate(net, val)
    hist = S.train(net, snaps, 3, val=val, lr=1e-3, log=None)
    print("held-out loss", before, [h.val_loss for h in hist], flush=True)
    assert hist[-1].val_loss < 0.5 * before
    net.close()
