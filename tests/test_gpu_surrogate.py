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


# Composition tolerance (increments of the whole run, per field): the leaps
# dominate the error.  The network computes in BF16 operands with FP32
# accumulation against the oracle's FP64 arithmetic on the same BF16-rounded
# operands, and where the FP32 stepper state and the FP64 oracle state lie on
# opposite sides of a BF16 rounding boundary the two networks see inputs one
# BF16 step (2^-8 relative) apart.
BLEND_INC_TOL = 2e-2


def test_blended_run_matches_oracle_composition():
    """The blended schedule on 64^2 FP32 (two cycles of [200 DNS steps, one
    leap of 2 units], then a 200-step DNS tail; a seeded network whose head
    is live, gamma 0.02) against the oracle's composition: its FP64 stepper
    for the DNS blocks and its FP64 U-Net forward with the GPU's BF16
    roundings for the leaps, from the same seeded initial condition (FP32-
    rounded, as the GPU stores it).  Per field, the increment of the whole
    run (final - initial) agrees within BLEND_INC_TOL relative L2, and
    pointwise within BLEND_INC_TOL of the largest increment."""
    import torch

    import oracle
    from oracle import unet_oracle as uo
    from paper_2312_05410_amd import surrogate as S
    from paper_2312_05410_amd.inputs import initial_state
    from paper_2312_05410_amd.unet import UNet, UNetConfig

    announce("blended run vs oracle composition 64^2")
    n, seed, dns, jumps, steps = 64, 5, 200, 2, 1000
    cfg = UNetConfig(height=n, width=n, base=8, levels=3, groups=4, mlp_hidden=16, basis=16, max_batch=1)
    net = UNet(cfg, seed=3)
    prm = net.param_dict()
    prm["head.gamma"][:] = 0.02
    net.set_params(prm)
    state, _, _ = S.blended_run(net, seed=seed, steps=steps, dns_block=dns, jumps=jumps, mode="leap", n=n)
    got = [u[0].double().cpu().numpy() for u in state]

    p = S.blend_params(seed, n=n)
    dt = 0.2 * oracle.dt_limit(p)
    q = p.replace(dt=dt)
    u0 = [np.float32(a).astype(np.float64) for a in initial_state(q)]
    ref_net = uo.Net(cfg, net.param_dict())
    st = oracle.State(q, *u0, dt=dt)
    t = 0
    while t + dns + jumps * S.JUMP <= steps:
        st.step(dns)
        pred = ref_net.forward(st.c, st.phi, st.rho, np.array([float(jumps)]), bf16=True)
        st = oracle.State(q, *(x.detach().numpy() for x in pred), Q=st.Q, dt=dt, nstep=st.nstep)
        t += dns + jumps * S.JUMP
    assert t == 800
    st.step(steps - t)
    for name, g, r, a in zip(("c", "phi", "rho"), got, (st.c[0], st.phi[0], st.rho[0]), u0):
        inc = r - a[0]
        e = np.linalg.norm(g - r) / np.linalg.norm(inc)
        m = np.abs(g - r).max() / np.abs(inc).max()
        print(f"{name}: increment rel L2 {e:.2e}, max abs / max increment {m:.2e}, "
              f"|increment| {np.linalg.norm(inc):.3e}", flush=True)
        assert e <= BLEND_INC_TOL and m <= BLEND_INC_TOL, name
    net.close()
