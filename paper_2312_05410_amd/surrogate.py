"""The surrogate side of the method (Introduction and Results: the DNS and a
time-conditioned U-Net take turns, the U-Net leaping ahead in time and the
DNS resuming from its prediction; Materials and Methods, "Training of the
network"; appendix on trajectory splitting).

* make_training_set: snapshot pairs produced by the GPU stepper only.
* train: Adam on the relative squared error, batch 5, through the U-Net's C
  ABI (forward, backward and the optimiser step run in the library).
* blended_run / dns_run: the alternating schedule and the plain DNS that
  it is measured against, timed with HIP events on the stream both use.

Readings (where the paper leaves the choice open):
  * one U-Net time unit is JUMP = 100 DNS steps; a call may leap
    dt = 1..MAX_DT units from the same input (the paper evaluates its
    operator for dt = 1..lf from one input window);
  * training trajectory j starts at step j * STAGGER of its own seeded run,
    so the 2000 pairs (20 trajectories x 100 jumps) cover the states of a
    whole 50,000-step run while each trajectory spans 10,000 steps;
  * the blended schedule repeats [BLEND_DNS DNS steps, one leap of
    BLEND_JUMPS units] ("leap"), or the same jumps one unit at a time
    ("chain").
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from .inputs import PFParams
from .workloads import V0_NOM

JUMP = 100
MAX_DT = 4
N_TRAJ = 20
N_JUMPS = 100
STAGGER = 2100
BLEND_N = 512
BLEND_STEPS = 50_000
BLEND_DNS = 200
BLEND_JUMPS = 4
TRAIN_SEED = 1000      # training trajectories: seeds TRAIN_SEED + j
VAL_SEED = 2000        # held-out trajectories
TEST_SEED = 3000       # the blended run


def blend_params(seed: int, batch: int = 1, n: int = BLEND_N, dt_factor: float = 0.2) -> PFParams:
    """The P0 model on n x n in FP32, nominal rate, c = 0.5 +- 0.01."""
    return PFParams(nx=n, ny=n, batch=batch, precision="f32", seed=seed, v0=V0_NOM, c0=0.5, dt_factor=dt_factor)


def make_training_set(seed0: int = TRAIN_SEED, n_traj: int = N_TRAJ, n_jumps: int = N_JUMPS, jump: int = JUMP,
                      stagger: int = STAGGER, n: int = BLEND_N):
    """snaps [n_traj][n_jumps + 1][3][n][n] (float32, device): realisation j
    (seed seed0 + j) recorded every `jump` steps from step j * stagger, all
    realisations stepped together by the batched stepper."""
    import torch

    from ._lib import Simulator

    if stagger % jump:
        raise ValueError("stagger must be a multiple of jump")
    sim = Simulator(blend_params(seed0, batch=n_traj, n=n))
    snaps = torch.empty(n_traj, n_jumps + 1, 3, n, n, dtype=torch.float32, device=sim.c.device)
    end = (n_traj - 1) * stagger + n_jumps * jump
    for t in range(0, end + 1, jump):
        for j in range(n_traj):
            k, r = divmod(t - j * stagger, jump)
            if t >= j * stagger and r == 0 and k <= n_jumps:
                for f, u in enumerate((sim.c, sim.phi, sim.rho)):
                    snaps[j, k, f].copy_(u[j])
        if t < end:
            sim.step(jump)
    torch.cuda.synchronize()
    sim.close()
    return snaps


def _fields(x):
    return tuple(x[:, f].contiguous() for f in range(3))


def rel_mse(pred, true) -> float:
    """sum over fields of sum (pred - true)^2 / sum true^2 (evaluation)."""
    return float(sum(((p.double() - t.double()) ** 2).sum() / (t.double() ** 2).sum() for p, t in zip(pred, true)))


@dataclass
class TrainLog:
    epoch: int
    step: int
    train_loss: float
    val_loss: float
    seconds: float


def evaluate(net, snaps, max_dt: int = MAX_DT, batch: int = 5):
    """Mean loss over every (trajectory, start, dt) of a snapshot set."""
    import torch

    T, K1 = snaps.shape[:2]
    losses = []
    for dt in range(1, max_dt + 1):
        idx = [(t, k) for t in range(T) for k in range(K1 - dt)]
        for b0 in range(0, len(idx), batch):
            sel = idx[b0:b0 + batch]
            ti = torch.tensor([s[0] for s in sel], device=snaps.device)
            ki = torch.tensor([s[1] for s in sel], device=snaps.device)
            x, y = snaps[ti, ki], snaps[ti, ki + dt]
            pred = net.forward(*_fields(x), torch.full((len(sel),), float(dt), device=snaps.device), train=False)
            losses.append(rel_mse(pred, _fields(y)))
    return float(np.mean(losses))


def train(net, snaps, epochs: int, val=None, batch: int = 5, lr: float = 1e-4, max_dt: int = MAX_DT, seed: int = 0,
          log=print, time_limit: float = None, loss_every: int = 50):
    """Adam (lr, batch as in the paper) over the pairs (s_k, s_{k+dt}) of
    every trajectory, dt uniform in 1..max_dt (at most the remaining
    jumps), one epoch = one pass over the starting snapshots."""
    import torch

    T, K1 = snaps.shape[:2]
    npairs = T * (K1 - 1)
    g = torch.Generator().manual_seed(seed)
    history, step, t0 = [], 0, time.time()
    for ep in range(epochs):
        perm = torch.randperm(npairs, generator=g)
        dts = torch.randint(1, max_dt + 1, (npairs,), generator=g)
        tl = []
        for b0 in range(0, npairs - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            ti, ki = sel // (K1 - 1), sel % (K1 - 1)
            dt = torch.minimum(dts[b0:b0 + batch], (K1 - 1) - ki)
            ti, ki, dt = ti.to(snaps.device), ki.to(snaps.device), dt.to(snaps.device)
            x, y = snaps[ti, ki], snaps[ti, ki + dt]
            pred = net.forward(*_fields(x), dt.float())
            L = net.backward(pred, _fields(y), want_loss=(step % loss_every == 0))
            if L is not None:
                tl.append(L)
            net.adam_step(lr)
            step += 1
        vl = evaluate(net, val, max_dt) if val is not None else float("nan")
        rec = TrainLog(ep, step, float(np.mean(tl)) if tl else float("nan"), vl, time.time() - t0)
        history.append(rec)
        if log:
            log(f"epoch {ep:3d} step {step:6d} train {rec.train_loss:.4e} val {rec.val_loss:.4e} "
                f"{rec.seconds:7.1f} s")
        if time_limit and time.time() - t0 > time_limit:
            break
    return history


def _events():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def dns_run(seed: int = TEST_SEED, steps: int = BLEND_STEPS, dt_factor: float = 0.2, n: int = BLEND_N,
            record_every: int = 0):
    """Plain DNS to the physical time of `steps` steps at 0.2 of the stability
    limit, with time step dt_factor of the limit (so steps * 0.2 / dt_factor
    steps, rounded).  Returns (state (c, phi, rho) device tensors [1][n][n],
    milliseconds, records {step_at_0.2: state copies})."""
    import torch

    from ._lib import Simulator

    from ._lib import dt_limit

    # the same physical time as `steps` steps at 0.2 of the limit, exactly
    p = blend_params(seed, n=n)
    nsteps = int(round(steps * 0.2 / dt_factor))
    sim = Simulator(p.replace(dt=steps * 0.2 * dt_limit(p) / nsteps))
    rec = {}
    e0, e1 = _events()
    e0.record()
    if record_every:
        ratio = 0.2 / dt_factor
        done = 0
        for t in range(record_every, steps + 1, record_every):
            k = int(round(t * ratio))
            sim.step(k - done)
            done = k
            rec[t] = tuple(u.clone() for u in (sim.c, sim.phi, sim.rho))
        sim.step(nsteps - done)
    else:
        sim.step(nsteps)
    e1.record()
    torch.cuda.synchronize()
    state = (sim.c.clone(), sim.phi.clone(), sim.rho.clone())
    ms = e0.elapsed_time(e1)
    sim.close()
    return state, ms, rec


def blended_run(net, seed: int = TEST_SEED, steps: int = BLEND_STEPS, dns_block: int = BLEND_DNS,
                jumps: int = BLEND_JUMPS, mode: str = "leap", n: int = BLEND_N, record: bool = False,
                dns_factor: float = 0.2):
    """Alternate dns_block DNS steps with `jumps` U-Net units (one leap of
    `jumps`, or `jumps` chained single units), the U-Net writing its
    prediction straight into the stepper's state tensors, then DNS to
    `steps`; `steps`, dns_block and the jumps count steps at 0.2 of the
    stability limit.  dns_factor > 0.2: each DNS segment covers the same
    physical time in round(dns_block 0.2 / dns_factor) larger steps.
    Returns (state, milliseconds, records {step: state copy})."""
    import torch

    from ._lib import Simulator, dt_limit

    if mode not in ("leap", "chain"):
        raise ValueError(mode)
    p = blend_params(seed, n=n)
    seg = max(1, int(round(dns_block * 0.2 / dns_factor)))
    sim = Simulator(p.replace(dt=dns_block * 0.2 * dt_limit(p) / seg))
    u = (sim.c, sim.phi, sim.rho)
    leap = torch.full((1,), float(jumps if mode == "leap" else 1), device=sim.c.device)
    rec = {}
    t = 0
    e0, e1 = _events()
    e0.record()
    while t + dns_block + jumps * JUMP <= steps:
        sim.step(seg)
        t += dns_block
        for _ in range(1 if mode == "leap" else jumps):
            net.forward(*u, leap, out=u, train=False)
        t += jumps * JUMP
        if record:
            rec[t] = tuple(x.clone() for x in u)
    # the tail in segment-sized steps (whole segments when dns_block divides it)
    sim.step(int(round((steps - t) * seg / dns_block)))
    e1.record()
    torch.cuda.synchronize()
    state = tuple(x.clone() for x in u)
    ms = e0.elapsed_time(e1)
    sim.close()
    return state, ms, rec


def compare(net, seed: int = TEST_SEED, steps: int = BLEND_STEPS, dt_factors=(0.4, 0.6, 0.8, 0.95),
            reps: int = 3, n: int = BLEND_N, log=print):
    """The blended runs ("leap", "chain") and plain DNS at larger time steps,
    all compared with plain DNS at 0.2 of the stability limit from the same
    seeded initial condition: final-state relative L2 of each field, relative
    L2 of the phase-A autocorrelation S2 and of its radial average, and the
    best of `reps` timed runs.  "At fixed error": the fastest plain DNS whose
    S2 error does not exceed the blended run's."""
    from . import metrics as M

    ref, ms_ref, _ = dns_run(seed, steps, 0.2, n)
    ms_ref = min([ms_ref] + [dns_run(seed, steps, 0.2, n)[1] for _ in range(reps - 1)])
    s2_ref = M.s2(M.phase_indicator(ref[0][0], ref[1][0]))
    ra_ref = M.radial_average(s2_ref, n // 4)

    def errors(st):
        s2 = M.s2(M.phase_indicator(st[0][0], st[1][0]))
        return {"c": M.rel_l2(st[0], ref[0]), "phi": M.rel_l2(st[1], ref[1]), "rho": M.rel_l2(st[2], ref[2]),
                "S2": M.rel_l2(s2, s2_ref), "S2_radial": M.rel_l2(M.radial_average(s2, n // 4), ra_ref)}

    out = {"steps": steps, "n": n, "seed": seed, "dns_ms": round(ms_ref, 3), "runs": {}}
    fast = max(dt_factors)
    for mode, f in (("leap", 0.2), ("chain", 0.2), ("leap", fast)):
        key = f"blend_{mode}" if f == 0.2 else f"blend_{mode}_dns{f}"
        st, ms, _ = blended_run(net, seed, steps, mode=mode, n=n, dns_factor=f)
        ms = min([ms] + [blended_run(net, seed, steps, mode=mode, n=n, dns_factor=f)[1] for _ in range(reps - 1)])
        out["runs"][key] = {"ms": round(ms, 3), "errors": errors(st)}
        if log:
            log(f"blended {key}: {ms:.2f} ms {out['runs'][key]['errors']}")
    for f in dt_factors:
        st, ms, _ = dns_run(seed, steps, f, n)
        ms = min([ms] + [dns_run(seed, steps, f, n)[1] for _ in range(reps - 1)])
        out["runs"][f"dns_{f}"] = {"ms": round(ms, 3), "errors": errors(st)}
        if log:
            log(f"dns dt {f}: {ms:.2f} ms {out['runs'][f'dns_{f}']['errors']}")
    b = out["runs"]["blend_leap"]
    out["speedup_same_dt"] = round(ms_ref / b["ms"], 3)
    # at fixed error: for each blended run, the fastest plain DNS whose S2
    # error does not exceed the blended run's, over the blended run's time;
    # the headline is the best blended configuration
    best_key, best_ratio = None, 0.0
    for key, r in out["runs"].items():
        if not key.startswith("blend_"):
            continue
        ok = [d["ms"] for k, d in out["runs"].items()
              if k.startswith("dns_") and d["errors"]["S2"] <= r["errors"]["S2"]]
        r["dns_at_same_error_ms"] = min([ms_ref] + ok)
        r["speedup_fixed_error"] = round(r["dns_at_same_error_ms"] / r["ms"], 3)
        if r["speedup_fixed_error"] > best_ratio:
            best_key, best_ratio = key, r["speedup_fixed_error"]
    out["speedup_fixed_error"] = best_ratio
    out["best_blend"] = best_key
    return out


def error_curve(net, seed: int = TEST_SEED, steps: int = BLEND_STEPS, n: int = BLEND_N, mode: str = "leap",
                dt_factor_dns: float = 0.8):
    """S2 relative L2 error at every blended cycle boundary for the blended
    run and for plain DNS at dt_factor_dns, against DNS at 0.2."""
    from . import metrics as M

    _, _, rec_b = blended_run(net, seed, steps, mode=mode, n=n, record=True)
    ts = sorted(rec_b)
    cyc = BLEND_DNS + BLEND_JUMPS * JUMP
    _, _, rec_ref = dns_run(seed, steps, 0.2, n, record_every=cyc)
    _, _, rec_d = dns_run(seed, steps, dt_factor_dns, n, record_every=cyc)
    rows = []
    for t in ts:
        if t not in rec_ref:
            continue
        r = rec_ref[t]
        s2r = M.s2(M.phase_indicator(r[0][0], r[1][0]))
        e = lambda st: M.rel_l2(M.s2(M.phase_indicator(st[0][0], st[1][0])), s2r)
        rows.append((t, e(rec_b[t]), e(rec_d[t]) if t in rec_d else float("nan"),
                     M.rel_l2(rec_b[t][0], r[0])))
    return rows
