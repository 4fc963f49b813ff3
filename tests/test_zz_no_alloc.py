"""The allocation-free diagnostics entry point (pf_diagnostics_noalloc,
through the C ABI) against the handle's pf_mass and pf_energy on the same
fields: same kernels and summation order, so the values agree bit for bit.
Two calls in a row, the second with a smaller input (another precision path
of the reduction: a row length that is not a multiple of four)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2312_05410_amd.inputs import PFParams, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_05410_amd import _lib

    _lib.load()


def _check(p, seed):
    import torch

    from paper_2312_05410_amd import _lib

    print(f"\n[case] noalloc diagnostics {p.batch} x {p.ny} x {p.nx} {p.precision} {p.bc_mode}", flush=True)
    state = random_state(seed, p.batch, p.ny, p.nx)
    sim = _lib.Simulator(p, state=state)
    m, e = sim.mass(), sim.energy()
    out = torch.full((p.batch, 4), float("nan"), dtype=torch.float64, device=sim.c.device)
    _lib.diagnostics_noalloc(p, sim.c, sim.phi, sim.rho, out, sim.stream)
    got = out.cpu().numpy()
    assert np.array_equal(got[:, :3], m[:, :3])
    assert np.array_equal(got[:, 3], e)
    sim.close()


def test_noalloc_diagnostics_equal_pf_mass_and_energy():
    _check(PFParams(nx=512, ny=384, batch=3, precision="f32"), 41)
    _check(PFParams(nx=100, ny=77, batch=1, precision="f32", bc_mode="periodic"), 42)


def test_noalloc_diagnostics_fp64():
    _check(PFParams(nx=258, ny=130, batch=2, precision="f64"), 43)
    _check(PFParams(nx=64, ny=33, batch=1, precision="f64"), 44)


def test_noalloc_rejects_inputs_beyond_its_scratch():
    """batch x partial sums beyond the static array: PF_ESCRATCH before
    anything is enqueued (the buffers are real and of the stated size)."""
    import torch

    from paper_2312_05410_amd import _lib

    p = PFParams(nx=8, ny=8, batch=40000, precision="f32")
    u = [torch.zeros((p.batch, p.ny, p.nx), dtype=torch.float32, device="cuda") for _ in range(3)]
    out = torch.zeros((p.batch, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.PFError) as ei:
        _lib.diagnostics_noalloc(p, *u, out)
    assert ei.value.code == _lib.PF_ESCRATCH
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out)) == 0
