"""GPU parity of the HIP stepper (through the C ABI) against the FP64 oracle.

Tolerances: FP64 fields within 1e-12 relative L2 per field; FP32 fields
within 1e-5 relative L2 per field after 1000 steps (FP32 arithmetic, FP64
diagnostics).  GPU self-consistency (temporal blocking, batching, resume,
repeat runs) is bitwise.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2312_05410_amd import workloads
from paper_2312_05410_amd.inputs import PFParams, initial_state, random_state, realisation_draws

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_05410_amd import _lib

    _lib.load()  # fails loudly if the HIP library is missing


def Sim(*a, **kw):
    from paper_2312_05410_amd._lib import Simulator

    return Simulator(*a, **kw)


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def compare(sim_state, ref: oracle.State, tol, label=""):
    for name, got, want in zip(("c", "phi", "rho"), sim_state, (ref.c, ref.phi, ref.rho)):
        e = rel_l2(got, want)
        assert e <= tol, f"{label} {name}: rel L2 {e:.3e} > {tol:.1e}"


def check_increments(got, want, start, steps, prec, label="", rel=None):
    """Cell by cell: the GPU's increment over the run (got - start) against
    the oracle's (want - start).  Bound per cell: rel |oracle increment| +
    2 steps ulp(u) (each step rounds the stored state once; errors carried
    in from neighbours are of the same order), in the run's precision.  A
    wrong seam, rim, boundary row or ghost changes that cell's increment by
    a large fraction of itself, far above this bound, however small the
    cell's share of the whole-field norm."""
    if rel is None:
        rel = 1e-4 if prec == "f32" else 1e-9
    ftype = np.float32 if prec == "f32" else np.float64
    for name, g, w, a in zip(("c", "phi", "rho"), got, want, start):
        g, w, a = (np.asarray(x, dtype=np.float64).reshape(np.shape(w)) for x in (g, w, a))
        inc = w - a
        ulp = np.spacing(np.maximum(np.abs(w), np.abs(a)).astype(ftype)).astype(np.float64)
        bound = rel * np.abs(inc) + 2.0 * steps * ulp
        err = np.abs(g - w)
        bad = err > bound
        if bad.any():
            k = np.unravel_index(np.argmax(err - bound), err.shape)
            raise AssertionError(f"{label} {name}: {int(bad.sum())} cells outside the increment bound; worst at "
                                 f"{tuple(int(i) for i in k)}: |err| {err[k]:.3e}, bound {bound[k]:.3e}, "
                                 f"increment {inc[k]:.3e}")
        e = np.linalg.norm(g - w) / max(np.linalg.norm(inc), 1e-300)
        print(f"{label} {name}: increment rel L2 {e:.2e}, max err/bound {float((err / bound).max()):.2f}",
              flush=True)


def run_pair(p: PFParams, state, n, tol, temporal_block=0, dt=None):
    dt = oracle.resolve_dt(p) if dt is None else dt
    p = p.replace(dt=dt)
    sim = Sim(p, state=state, temporal_block=temporal_block)
    ref = oracle.State(p, *state, dt=dt)
    sim.step(n)
    ref.step(n)
    compare(sim.state(), ref, tol, f"{p.precision} n={n} K={temporal_block}")
    return sim, ref


# ------------------------------------------------------------ initial condition

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_seeded_init_matches_oracle(prec):
    announce(f"seeded init {prec}")
    p = PFParams(nx=96, ny=80, batch=3, seed=11, precision=prec, c0_per=np.array([0.3, 0.5, 0.7]))
    sim = Sim(p)
    c, phi, rho = oracle.init(p)
    gc, gphi, grho = sim.state()
    if prec == "f64":
        assert np.array_equal(gc, c)
        np.testing.assert_allclose(gphi, phi, rtol=0, atol=4e-16)
        np.testing.assert_allclose(grho, rho, rtol=0, atol=4e-16)
    else:
        for g, w in ((gc, c), (gphi, phi), (grho, rho)):
            np.testing.assert_allclose(g, w.astype(np.float32).astype(np.float64), rtol=0, atol=1.2e-7)
    np.testing.assert_array_equal(sim.inflow(), np.zeros(3))
    sim.close()


# ----------------------------------------------------- the small DNS workload

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_parity_f64_dns_small(seed):
    """128^2 FP64, 1000 steps at 0.2 of the stability limit."""
    announce(f"dns_small f64 seed={seed}")
    p = workloads.dns_small(seed, "f64")
    state = initial_state(p)
    sim, ref = run_pair(p, state, 1000, F64_TOL)
    m, mr = sim.mass(), ref.mass()
    np.testing.assert_allclose(m, mr, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sim.energy(), ref.energy(), rtol=1e-12)
    assert sim.step_count == 1000
    sim.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_parity_f32_dns_small(seed):
    """Same inputs run in FP32: within 1e-5 relative L2 after 1000 steps."""
    announce(f"dns_small f32 seed={seed}")
    p = workloads.dns_small(seed, "f32")
    dt = oracle.resolve_dt(p)
    state = initial_state(p)
    sim, ref = run_pair(p, state, 1000, F32_TOL, dt=dt)
    np.testing.assert_allclose(sim.mass(), ref.mass(), rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(sim.energy(), ref.energy(), rtol=1e-5)
    sim.close()


# ------------------------------------------------ rough states, ragged shapes

@pytest.mark.parametrize("prec,K", [("f64", 1), ("f64", 2), ("f32", 1), ("f32", 2), ("f32", 3), ("f32", 4)])
@pytest.mark.parametrize("shape", [(100, 77), (64, 32), (130, 50)])
def test_parity_rough_ragged(prec, K, shape):
    """Far-from-equilibrium fields (every term active), angled flux, grid
    sizes that leave ragged tiles in x and y."""
    nx, ny = shape
    announce(f"rough {prec} K={K} {nx}x{ny}")
    p = PFParams(nx=nx, ny=ny, precision=prec, theta_deg=62.0, v0=0.8, seed=3)
    state = random_state(21, 1, ny, nx)
    n = 23
    sim, ref = run_pair(p, state, n, F64_TOL if prec == "f64" else 1e-5, temporal_block=K)
    np.testing.assert_allclose(sim.inflow(), ref.Q, rtol=1e-12 if prec == "f64" else 1e-5)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_parity_periodic(prec):
    announce(f"periodic {prec}")
    p = PFParams(nx=72, ny=40, precision=prec, bc_mode="periodic", theta_deg=45.0, v0=0.7)
    state = random_state(22, 1, 40, 72, film=False)
    sim, ref = run_pair(p, state, 31, F64_TOL if prec == "f64" else 1e-5, temporal_block=2)
    sim.close()


@pytest.mark.parametrize("shape", [(8, 8), (5, 4), (1, 16), (200, 3)])
def test_parity_tiny_grids(shape):
    nx, ny = shape
    announce(f"tiny {nx}x{ny}")
    p = PFParams(nx=nx, ny=ny, precision="f64", theta_deg=70.0, film_h=ny / 2.0)
    state = random_state(23, 1, ny, nx)
    sim, ref = run_pair(p, state, 17, F64_TOL, temporal_block=2)
    sim.close()


def test_flux_off_conserves_and_decays():
    announce("flux off f64")
    p = workloads.dns_small(0, "f64").replace(flux_on=False)
    sim = Sim(p)
    m0, e0 = sim.mass(), sim.energy()
    for _ in range(10):
        sim.step(100)
        e = sim.energy()
        assert e[0] <= e0[0] + 1e-14 * abs(e0[0])
        e0 = e
    m1 = sim.mass()
    assert abs(m1[0, 0] - m0[0, 0]) <= 1e-12 * abs(m0[0, 0])
    assert abs(m1[0, 1] - m0[0, 1]) <= 1e-12 * abs(m0[0, 1])
    sim.close()


# ------------------------------------------------------- batched realisations

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_parity_batched(prec):
    announce(f"batched {prec}")
    v0, c0 = realisation_draws(5, 4, 0.5)
    p = PFParams(nx=64, ny=48, batch=4, precision=prec, seed=5, v0_per=v0, c0_per=c0, theta_deg=75.0)
    run_pair(p, initial_state(p), 200, F64_TOL if prec == "f64" else 1e-5)


def test_batch_of_identical_realisations_is_bitwise_identical():
    announce("batch identical")
    B = 3
    p = PFParams(nx=96, ny=64, batch=B, precision="f32", theta_deg=70.0)
    c, phi, rho = random_state(24, 1, 64, 96)
    state = tuple(np.repeat(u, B, axis=0) for u in (c, phi, rho))
    sim = Sim(p, state=state)
    sim.step(41)
    out = sim.state()
    for u in out:
        for b in range(1, B):
            assert np.array_equal(u[0], u[b])
    q = sim.inflow()
    assert q[0] == q[1] == q[2]
    sim.close()


# --------------------------------------------------- bitwise self-consistency

@pytest.mark.parametrize("prec,Ks", [("f32", (2, 3, 4)), ("f64", (2,))])
def test_temporal_blocking_is_bitwise(prec, Ks):
    announce(f"temporal blocking bitwise {prec}")
    p = PFParams(nx=150, ny=100, precision=prec, theta_deg=58.0, v0=0.9)
    state = random_state(25, 1, 100, 150)
    ref = Sim(p, state=state, temporal_block=1)
    ref.step(37)
    base = ref.state()
    qb = ref.inflow()
    for K in Ks:
        sim = Sim(p, state=state, temporal_block=K)
        sim.step(37)
        for u, v in zip(sim.state(), base):
            assert np.array_equal(u, v), f"K={K}"
        assert np.array_equal(sim.inflow(), qb), f"K={K}"
        sim.close()
    ref.close()


@pytest.mark.parametrize("prec,K", [("f32", 1), ("f32", 2), ("f64", 1)])
def test_graph_replay_is_bitwise(prec, K):
    """Long runs replay a HIP graph of launches; it must equal plain launches."""
    announce(f"graph replay {prec} K={K}")
    p = PFParams(nx=192, ny=80, precision=prec, theta_deg=66.0, v0=0.7)
    state = random_state(26, 1, 80, 192)
    n = 64 * 3 * K + 5
    out = []
    for mode in (0, 1):
        sim = Sim(p, state=state, temporal_block=K, graph_mode=mode)
        sim.step(n)
        sim.step(n + 1)
        out.append((sim.state(), sim.inflow()))
        sim.close()
    for u, v in zip(out[0][0], out[1][0]):
        assert np.array_equal(u, v)
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_march_chunk_heights_are_bitwise(prec):
    """The single-step kernel at every chunk height equals the LDS-tiled
    two-step kernel bit for bit (same per-cell arithmetic)."""
    announce(f"march chunk heights {prec}")
    p = PFParams(nx=150, ny=100, precision=prec, theta_deg=58.0, v0=0.9)
    state = random_state(27, 1, 100, 150)
    ref = Sim(p, state=state, temporal_block=2)
    ref.step(37)
    base = ref.state()
    qb = ref.inflow()
    ref.close()
    for rows in (4, 8, 16, 32):
        sim = Sim(p, state=state, temporal_block=1, tile_rows=rows)
        sim.step(37)
        for u, v in zip(sim.state(), base):
            assert np.array_equal(u, v), f"rows={rows}"
        assert np.array_equal(sim.inflow(), qb), f"rows={rows}"
        sim.close()


@pytest.mark.parametrize("shape", [(150, 100), (250, 61), (6, 20), (124, 9)])
def test_two_columns_per_lane_is_bitwise(shape):
    """FP32 single-step kernel with two grid columns per lane (even nx:
    ragged last strip, a strip wider than the grid, one exact strip) equals
    the one-column kernel bit for bit (which equals the LDS-tiled kernel, see
    above), at every chunk height, for Euler, the midpoint method and
    interface draws."""
    nx, ny = shape
    announce(f"two columns per lane f32 {nx}x{ny}")
    p = PFParams(nx=nx, ny=ny, precision="f32", theta_deg=58.0, v0=0.9)
    state = random_state(28, 1, ny, nx)
    ref = Sim(p, state=state, temporal_block=1, lane_cols=1)
    ref.step(37)
    base, qb = ref.state(), ref.inflow()
    ref.close()
    for rows in (4, 8, 16, 32):
        sim = Sim(p, state=state, temporal_block=1, tile_rows=rows, lane_cols=2)
        assert sim.lane_cols == 2
        sim.step(37)
        for u, v in zip(sim.state(), base):
            assert np.array_equal(u, v), f"rows={rows}"
        assert np.array_equal(sim.inflow(), qb), f"rows={rows}"
        sim.close()
    for variant in (dict(integrator="midpoint"), dict(interface_noise=0.1)):
        q = p.replace(**variant)
        out = []
        for cols in (1, 2):
            sim = Sim(q, state=state, lane_cols=cols)
            assert sim.lane_cols == cols
            sim.step(23)
            sim.step(14)
            out.append((sim.state(), sim.inflow()))
            sim.close()
        for u, v in zip(out[0][0], out[1][0]):
            assert np.array_equal(u, v), str(variant)
        assert np.array_equal(out[0][1], out[1][1]), str(variant)


@pytest.mark.parametrize("prec,bc,shape", [("f32", "pvd", (150, 96)), ("f64", "pvd", (130, 64)),
                                           ("f32", "periodic", (120, 48)), ("f32", "pvd", (6, 16)),
                                           ("f32", "pvd", (100, 8)), ("f32", "pvd", (250, 32)),
                                           ("f32", "pvd", (121, 16))])
def test_two_step_march_is_bitwise(prec, bc, shape):
    """The register strip march fusing two steps equals single-step
    launches bit for bit (state and inflow) at every chunk height dividing
    ny, for odd step counts (the last step alone), graph replay and plain
    launches."""
    nx, ny = shape
    announce(f"two-step march {prec} {bc} {nx}x{ny}")
    p = PFParams(nx=nx, ny=ny, precision=prec, bc_mode=bc, theta_deg=61.0, v0=0.85)
    state = random_state(29, 1, ny, nx)
    ref = Sim(p, state=state, temporal_block=1, lane_cols=1)
    ref.step(37)
    ref.step(141)
    base, qb = ref.state(), ref.inflow()
    ref.close()
    for rows in (4, 8, 16):
        if ny % rows:
            continue
        # (a request for two columns per lane applies to single-step
        # launches only: the fused march keeps one)
        for gm, cols in ((0, 1), (1, 1), (0, 2)):
            sim = Sim(p, state=state, temporal_block=2, tile_rows=rows, fused_kernel=2, graph_mode=gm,
                      lane_cols=cols)
            assert sim.fused_kernel == 2 and sim.launch == (2, rows)
            assert sim.lane_cols == 1
            sim.step(37)
            sim.step(141)
            for u, v in zip(sim.state(), base):
                assert np.array_equal(u, v), f"rows={rows} graph_mode={gm} cols={cols}"
            assert np.array_equal(sim.inflow(), qb), f"rows={rows} graph_mode={gm} cols={cols}"
            sim.close()


def test_two_step_march_f64_matches_oracle():
    announce("two-step march f64 vs oracle 96x64")
    p = PFParams(nx=96, ny=64, precision="f64", theta_deg=70.0, v0=0.9, seed=4)
    state = random_state(30, 1, 64, 96)
    sim = Sim(p, state=state, temporal_block=2, fused_kernel=2)
    assert sim.fused_kernel == 2
    sim.step(60)
    s = oracle.State(p, *state).step(60)
    for a, b in zip(sim.state(), (s.c, s.phi, s.rho)):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-12
    np.testing.assert_allclose(sim.mass(), s.mass(), rtol=1e-11, atol=1e-12)
    sim.close()


@pytest.mark.parametrize("bc,shape,th,batch", [
    ("pvd", (128, 96), 8, 1), ("pvd", (192, 64), 16, 2), ("periodic", (128, 64), 32, 1),
    ("pvd", (256, 128), 32, 1), ("pvd", (64, 32), 32, 1), ("periodic", (64, 16), 8, 3),
    ("pvd", (320, 48), 16, 1)])
def test_resident_stepper_is_bitwise(bc, shape, th, batch):
    """The resident stepper (one launch per call, tiles held in
    LDS, inner cells computed while the rims are traded through tagged
    words) equals single-step launches bit for bit, state and inflow, over
    calls of 2, 3, 37, 1 (the single-step kernel) and 141 steps in a row;
    one tile column, one tile row and batches included."""
    nx, ny = shape
    announce(f"resident {bc} {batch}x{nx}x{ny} th={th}")
    p = PFParams(nx=nx, ny=ny, batch=batch, precision="f32", bc_mode=bc, theta_deg=61.0, v0=0.85)
    state = random_state(31, batch, ny, nx)
    ref = Sim(p, state=state, temporal_block=1, lane_cols=1)
    sim = Sim(p, state=state, fused_kernel=3, tile_rows=th)
    assert sim.fused_kernel == 3 and sim.launch == (1, th)
    for n in (2, 3, 37, 1, 141):
        ref.step(n)
        sim.step(n)
        for u, v in zip(sim.state(), ref.state()):
            assert np.array_equal(u, v), f"after a call of {n} steps"
        assert np.array_equal(sim.inflow(), ref.inflow()), f"after a call of {n} steps"
    ref.close()
    sim.close()


@pytest.mark.parametrize("nx,ny,batch", [(512, 512, 1), (512, 512, 4), (1024, 768, 1)])
def test_resident_default_shapes_are_bitwise(nx, ny, batch):
    """Where the library picks the resident stepper by itself (the blended
    run's 512^2 DNS, four realisations of it, a 0.79M-cell grid), production
    initial conditions stepped by it equal single-step launches bit for bit,
    state and inflow."""
    announce(f"resident default {batch}x{nx}x{ny}")
    p = workloads.dns_production(0, n=nx).replace(ny=ny, batch=batch)
    state = initial_state(p)
    sim = Sim(p, state=state)
    ref = Sim(p, state=state, temporal_block=1)
    assert sim.fused_kernel == 3 and ref.fused_kernel == 0
    for n in (64, 201):
        sim.step(n)
        ref.step(n)
    for u, v in zip(sim.state(), ref.state()):
        assert np.array_equal(u, v)
    assert np.array_equal(sim.inflow(), ref.inflow())
    sim.close()
    ref.close()


@pytest.mark.parametrize("bc,shape,th,batch", [("pvd", (128, 96), 8, 1), ("pvd", (192, 64), 16, 2),
                                                ("periodic", (128, 64), 32, 1), ("pvd", (256, 128), 32, 1)])
def test_resident_midpoint_is_bitwise(bc, shape, th, batch):
    """The resident stepper running explicit midpoint steps (the half-step
    state traded like a step's result, the step's base state kept in
    registers) equals the two-launch midpoint path bit for bit, state and
    inflow, over calls of 2, 3, 37, 1 and 141 steps."""
    nx, ny = shape
    announce(f"resident midpoint {bc} {batch}x{nx}x{ny} th={th}")
    p = PFParams(nx=nx, ny=ny, batch=batch, precision="f32", bc_mode=bc, theta_deg=61.0, v0=0.85,
                 integrator="midpoint")
    state = random_state(32, batch, ny, nx)
    ref = Sim(p, state=state, temporal_block=1)
    sim = Sim(p, state=state, fused_kernel=3, tile_rows=th)
    assert sim.fused_kernel == 3 and ref.fused_kernel == 0
    for n in (2, 3, 37, 1, 141):
        ref.step(n)
        sim.step(n)
        for u, v in zip(sim.state(), ref.state()):
            assert np.array_equal(u, v), f"after a call of {n} steps"
        assert np.array_equal(sim.inflow(), ref.inflow()), f"after a call of {n} steps"
    ref.close()
    sim.close()


@pytest.mark.parametrize("integrator,bc,shape,th,batch", [
    ("euler", "pvd", (128, 96), 8, 1), ("euler", "pvd", (192, 64), 16, 2), ("euler", "periodic", (128, 64), 32, 1),
    ("midpoint", "pvd", (128, 64), 32, 2), ("midpoint", "pvd", (256, 96), 16, 1)])
def test_resident_interface_draws_are_bitwise(integrator, bc, shape, th, batch):
    """With interface draws on, the resident stepper draws the same FP32
    compositions on the same cells as single-step launches (keyed by the
    global step across calls of 2, 3, 37, 1 and 141 steps): states and
    inflow equal bit for bit, for both integrators."""
    nx, ny = shape
    announce(f"resident draws {integrator} {bc} {batch}x{nx}x{ny} th={th}")
    p = PFParams(nx=nx, ny=ny, batch=batch, precision="f32", bc_mode=bc, theta_deg=61.0, v0=0.85,
                 integrator=integrator, interface_noise=0.1, seed=17)
    state = random_state(33, batch, ny, nx)
    ref = Sim(p, state=state, temporal_block=1)
    sim = Sim(p, state=state, fused_kernel=3, tile_rows=th)
    assert sim.fused_kernel == 3 and ref.fused_kernel == 0
    vapour = 0
    for n in (2, 3, 37, 1, 141):
        ref.step(n)
        sim.step(n)
        for u, v in zip(sim.state(), ref.state()):
            assert np.array_equal(u, v), f"after a call of {n} steps"
        assert np.array_equal(sim.inflow(), ref.inflow()), f"after a call of {n} steps"
        vapour += int((sim.state()[1] < 0).sum())
    assert vapour > 0   # the draws were exercised
    ref.close()
    sim.close()


def test_resident_interface_draws_default_shape():
    """512^2 production initial condition with draws: the library picks the
    resident stepper and its states equal single-step launches bit for bit."""
    announce("resident draws default 512x512")
    p = workloads.dns_production(0, n=512).replace(interface_noise=0.1)
    state = initial_state(p)
    sim = Sim(p, state=state)
    ref = Sim(p, state=state, temporal_block=1)
    assert sim.fused_kernel == 3 and ref.fused_kernel == 0
    for n in (64, 201):
        sim.step(n)
        ref.step(n)
    for u, v in zip(sim.state(), ref.state()):
        assert np.array_equal(u, v)
    assert np.array_equal(sim.inflow(), ref.inflow())
    sim.close()
    ref.close()


def test_resident_call_replays_as_graph():
    """A captured resident call (one launch that advances the epoch) replays
    correctly: the generation tags of every replay are fresh. Three replays,
    each followed by eager single-step launches of the same steps on a
    second handle and a synchronisation, equal them bit for bit."""
    import torch

    announce("resident call captured in a graph")
    p = workloads.dns_production(0, n=512)
    state = initial_state(p)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        sim = Sim(p, state=state)
    ref = Sim(p, state=state, temporal_block=1)
    assert sim.fused_kernel == 3
    sim.step(6)
    ref.step(6)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=sim.stream):
        sim.step(4)
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        ref.step(4)
        torch.cuda.synchronize()
        for u, v in zip(sim.state(), ref.state()):
            assert np.array_equal(u, v), f"replay {k}"
    sim.close()
    ref.close()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_capture_with_interface_draws_is_refused():
    """Draws are keyed by the step a call starts at: a call with draws on a
    capturing stream is refused before anything is enqueued (the capture
    ends cleanly and holds no work), while the same call outside capture
    runs."""
    import torch

    from paper_2312_05410_amd._lib import PFError

    announce("capture with interface draws refused")
    p = workloads.dns_production(0, n=512).replace(interface_noise=0.1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        sim = Sim(p)
    assert sim.fused_kernel == 3
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(PFError):
        with torch.cuda.graph(g, stream=sim.stream):
            sim.step(4)
    torch.cuda.synchronize()
    sim.step(4)
    assert np.isfinite(sim.mass()).all()
    sim.close()


def test_resident_stepper_matches_oracle():
    """FP32 resident stepper against the FP64 oracle: 128^2, 1000 steps, the
    library's tile height."""
    announce("resident vs oracle 128x128 f32")
    p = workloads.dns_small(0, "f32")
    dt = oracle.resolve_dt(p)
    p = p.replace(dt=dt)
    state = initial_state(p)
    sim = Sim(p, state=state, fused_kernel=3)
    assert sim.fused_kernel == 3
    ref = oracle.State(p, *state, dt=dt)
    sim.step(1000)
    ref.step(1000)
    compare(sim.state(), ref, F32_TOL, "resident")
    np.testing.assert_allclose(sim.mass(), ref.mass(), rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(sim.energy(), ref.energy(), rtol=1e-5)
    sim.close()


def test_resident_abort_word_poisons_the_state():
    """A set abort word (forced from the host; the kernel only reads it) makes
    every tile stop at once and write NaN; the next diagnostic call reports
    the abort (PF_EABORTED, not a plain non-finite value); a new handle on
    the same workspace size starts clean."""
    announce("resident abort word")
    import torch
    from paper_2312_05410_amd._lib import PFError, PF_EABORTED

    p = PFParams(nx=128, ny=64, precision="f32")
    sim = Sim(p, fused_kernel=3)
    assert sim.fused_kernel == 3
    ws = sim.workspace
    # the control words (epoch, abort, completion count) are the workspace's last 256-byte block
    ws[-256 + 8:-256 + 16] = torch.tensor([1, 0, 0, 0, 0, 0, 0, 0], dtype=torch.uint8, device=ws.device)
    torch.cuda.synchronize()
    sim.step(5)
    assert np.isnan(sim.state()[0]).all()
    for call in (sim.mass, sim.energy, sim.inflow):
        with pytest.raises(PFError) as ei:
            call()
        assert ei.value.code == PF_EABORTED
    sim.close()
    again = Sim(p, fused_kernel=3)
    again.step(5)
    assert np.isfinite(again.mass()).all()
    again.close()


def test_two_columns_need_even_rows_and_fp32():
    announce("two columns per lane fallback")
    for q in (PFParams(nx=151, ny=40, precision="f32"), PFParams(nx=150, ny=40, precision="f64")):
        sim = Sim(q, temporal_block=1, lane_cols=2)
        assert sim.lane_cols == 1
        sim.close()


def test_runs_are_deterministic():
    announce("determinism")
    p = workloads.dns_small(1, "f32").replace(nx=256, ny=192)
    out = []
    for _ in range(2):
        sim = Sim(p)
        sim.step(300)
        out.append((sim.state(), sim.mass(), sim.energy()))
        sim.close()
    for u, v in zip(out[0][0], out[1][0]):
        assert np.array_equal(u, v)
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_resume_is_bitwise():
    announce("resume")
    p = workloads.dns_small(2, "f32").replace(nx=160, ny=96)
    full = Sim(p, temporal_block=2)
    full.step(120)
    want = full.state()
    half = Sim(p, temporal_block=2)
    half.step(60)
    mid = half.state()
    q = half.inflow()
    resumed = Sim(p.replace(dt=half.dt), state=mid, temporal_block=2)
    resumed.set_inflow(q)
    resumed.step(60)
    for u, v in zip(resumed.state(), want):
        assert np.array_equal(u, v)
    np.testing.assert_allclose(resumed.inflow(), full.inflow(), rtol=1e-14)
    for s in (full, half, resumed):
        s.close()


def test_zero_steps_is_noop_and_nonfinite_is_reported():
    announce("noop + nonfinite")
    from paper_2312_05410_amd._lib import PFError, PF_ENONFINITE

    p = PFParams(nx=32, ny=32, precision="f64")
    sim = Sim(p)
    before = sim.state()
    sim.step(0)
    for u, v in zip(sim.state(), before):
        assert np.array_equal(u, v)
    sim.c[0, 5, 7] = float("nan")
    with pytest.raises(PFError) as ei:
        sim.mass()
    assert ei.value.code == PF_ENONFINITE
    with pytest.raises(PFError):
        sim.energy()
    sim.close()


# ------------------------------------------- full sizes, bench launch shape

def test_full_size_production_parity():
    """1024^2 FP32 (the throughput workload) in the launch configuration the
    benchmark times, from its seeded initial condition, against the oracle on
    the whole grid."""
    announce("dns_1024 f32 full-size")
    p = workloads.dns_production(0)
    K = workloads.BENCH_TEMPORAL_BLOCK["f32"]
    start = [np.float32(u).astype(np.float64) for u in initial_state(p)]
    sim, ref = run_pair(p, start, 20, 1e-6, temporal_block=K)
    assert sim.fused_kernel == 3 and sim.launch == (1, 32)   # the resident stepper
    assert sim.step_count == 20
    check_increments(sim.state(), (ref.c, ref.phi, ref.rho), start, 20, "f32", "dns_1024")
    np.testing.assert_allclose(sim.mass(), ref.mass(), rtol=1e-6)
    sim.close()


@pytest.mark.parametrize("n,prec,steps,tol", [(8192, "f32", 4, 1e-6), (4096, "f64", 6, F64_TOL)])
def test_full_size_large_grids(n, prec, steps, tol):
    """The large-grid throughput shapes (two fused steps in the register
    march by default) against the oracle on the whole grid."""
    announce(f"dns_{n} {prec} full-size")
    p = workloads.dns_production(0, n=n, precision=prec)
    K = workloads.BENCH_TEMPORAL_BLOCK[prec]
    ftype = np.float32 if prec == "f32" else np.float64
    start = [ftype(u).astype(np.float64) for u in initial_state(p)]
    sim, ref = run_pair(p, start, steps, tol, temporal_block=K)
    assert sim.launch[0] == 2 and sim.fused_kernel == 2
    check_increments(sim.state(), (ref.c, ref.phi, ref.rho), start, steps, prec, f"dns_{n}")
    np.testing.assert_allclose(sim.mass(), ref.mass(), rtol=1e-6 if prec == "f32" else 1e-11)
    sim.close()


def test_full_size_batched_sampled():
    """32 x 512^2 FP32 batched workload in the benchmark's launch shape; the
    oracle checks a sample of realisations one by one."""
    announce("batched 32x512 f32 sampled")
    p = workloads.batched(0)
    K = workloads.BENCH_TEMPORAL_BLOCK["f32"]
    dt = oracle.resolve_dt(p)
    p = p.replace(dt=dt)
    state = [np.float32(u).astype(np.float64) for u in initial_state(p)]
    n = 12
    sim = Sim(p, state=state, temporal_block=K)
    sim.step(n)
    assert sim.step_count == n
    out = sim.state()
    for b in (0, 13, 31):
        pb = p.replace(batch=1, seed=p.seed + b, v0=float(p.v0_per[b]), c0=float(p.c0_per[b]),
                       v0_per=None, c0_per=None)
        ref = oracle.State(pb, state[0][b:b + 1], state[1][b:b + 1], state[2][b:b + 1], dt=dt)
        ref.step(n)
        for name, got, want in zip("c phi rho".split(), out, (ref.c, ref.phi, ref.rho)):
            e = rel_l2(got[b], want[0])
            assert e <= 1e-6, f"b={b} {name} {e:.2e}"
        check_increments([u[b] for u in out], (ref.c[0], ref.phi[0], ref.rho[0]), [u[b] for u in state], n,
                         "f32", f"batched b={b}")
    sim.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_step_out_equals_one_step(prec):
    """pf_step_out (one step out of place, used by the adjoint's
    recomputation) equals one pf_step_n step bit for bit, and leaves the
    handle's own state, inflow and step counter untouched; refused for the
    midpoint integrator."""
    import torch

    from paper_2312_05410_amd._lib import PFError

    announce(f"step_out {prec}")
    p = PFParams(nx=100, ny=77, batch=2, precision=prec, theta_deg=70.0)
    state = random_state(61, 2, 77, 100)
    sim = Sim(p, state=state, temporal_block=1)
    ref = Sim(p, state=state, temporal_block=1)
    dst = [torch.empty_like(u) for u in (sim.c, sim.phi, sim.rho)]
    before = sim.state()
    sim.step_out((sim.c, sim.phi, sim.rho), dst)
    ref.step(1)
    torch.cuda.synchronize()
    for u, v in zip(dst, ref.state()):
        assert np.array_equal(u.double().cpu().numpy(), v)
    for u, v in zip(sim.state(), before):
        assert np.array_equal(u, v)
    assert sim.step_count == 0 and np.all(sim.inflow() == 0)
    mid = Sim(p.replace(integrator="midpoint"), state=state, temporal_block=1)
    with pytest.raises(PFError):
        mid.step_out((mid.c, mid.phi, mid.rho), dst)
    for s in (sim, ref, mid):
        s.close()
