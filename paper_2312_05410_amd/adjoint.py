"""Gradients of a final-state loss with respect to the mobility scale and
the deposition rate, through the library's discrete adjoint.

`final_state(M_scale, v0, p, u0, n, every)` runs n explicit steps of the
stepper from u0 = (c, phi, rho) and returns the final fields; as a
torch.autograd.Function its backward sweeps the steps in reverse with the
hand-written adjoint kernels (pf_adjoint_step), recomputing each segment of
`every` steps from a stored checkpoint into a ring of `every` states
allocated once (each state stepped out of place from the previous one), so memory holds n/every checkpoints plus two
segments instead of all n states.  With `overlap` (the default) the
recomputation of the next segment runs on a second stream into a second
ring while the adjoint steps of the current one run on the caller's stream
(events order the two; the results are bitwise those of the serial sweep).
Gradients are taken at fixed dt
(p.dt must be set) and are summed over the realisations of the batch.
Every step, forward and reverse, runs in the HIP library; torch only holds
the buffers and copies checkpoints.
"""
from __future__ import annotations

import torch

from .inputs import PFParams


class _FinalState(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Ms, v0, p: PFParams, c0, phi0, rho0, n: int, every: int, temporal_block: int,
                overlap: bool):
        from ._lib import Simulator

        if not (p.dt > 0):
            raise ValueError("final_state needs a fixed dt (p.dt > 0)")
        if p.integrator != "euler" or p.interface_noise > 0:
            raise ValueError("the adjoint is the transpose of the explicit Euler step without interface "
                             "draws (integrator 'euler', interface_noise 0)")
        q = p.replace(M_scale=float(Ms), v0=float(v0), v0_per=None)
        u = [t.detach().clone().contiguous() for t in (c0, phi0, rho0)]
        sim = Simulator(q, tensors=u, temporal_block=temporal_block)
        ckpts = []
        for s in range(0, n, every):
            ckpts.append([t.clone() for t in u])
            sim.step(min(every, n - s))
        ctx.q, ctx.n, ctx.every, ctx.ckpts = q, n, every, ckpts
        ctx.temporal_block = temporal_block
        ctx.overlap = overlap
        out = tuple(t.clone() for t in u)
        sim.close()
        return out

    @staticmethod
    def backward(ctx, gc, gphi, grho):
        from ._lib import Simulator

        q, n, every = ctx.q, ctx.n, ctx.every
        dtype = ctx.ckpts[0][0].dtype
        lam = [g.detach().to(dtype).contiguous() if g is not None else torch.zeros_like(ctx.ckpts[0][i])
               for i, g in enumerate((gc, gphi, grho))]
        nxt = [torch.empty_like(t) for t in lam]
        # the recomputed states of one segment live in a ring allocated once:
        # slot t holds (c, phi, rho) after t steps of the segment, each slot
        # stepped from the previous one by pf_step_out (one launch, no copy)
        shape = ctx.ckpts[0][0].shape
        dev = lam[0].device
        rings = [torch.empty((every, 3) + tuple(shape), dtype=dtype, device=dev)]
        rec = Simulator(q, tensors=[rings[0][0, 0], rings[0][0, 1], rings[0][0, 2]],
                        temporal_block=ctx.temporal_block)
        ws = rec.adjoint_workspace()
        nseg = len(ctx.ckpts)
        lengths = [min(every, n - sg * every) for sg in range(nseg)]
        if not ctx.overlap:
            for sg in range(nseg - 1, -1, -1):
                for f, ck in enumerate(ctx.ckpts[sg]):
                    rings[0][0, f].copy_(ck)
                # recompute the segment and run its adjoint steps in one call
                if rec.adjoint_segment(rings[0], lengths[sg], lam, nxt, ws):
                    lam, nxt = nxt, lam
        else:
            main = torch.cuda.current_stream(dev)
            side = torch.cuda.Stream(dev)
            rings.append(torch.empty_like(rings[0]))
            with torch.cuda.stream(side):
                side_rec = Simulator(q, tensors=[rings[1][0, 0], rings[1][0, 1], rings[1][0, 2]],
                                     temporal_block=ctx.temporal_block)
            start = torch.cuda.Event()
            start.record(main)
            side.wait_event(start)
            ready, freed = [None, None], [None, None]

            def recompute(sg):
                # segment sg into ring sg % 2 on the side stream, once the
                # sweep that last read that ring has finished
                k = sg % 2
                with torch.cuda.stream(side):
                    if freed[k] is not None:
                        side.wait_event(freed[k])
                    for f, ck in enumerate(ctx.ckpts[sg]):
                        rings[k][0, f].copy_(ck)
                    side_rec.adjoint_recompute(rings[k], lengths[sg])
                    ready[k] = torch.cuda.Event()
                    ready[k].record(side)

            try:
                recompute(nseg - 1)
                for sg in range(nseg - 1, -1, -1):
                    k = sg % 2
                    if sg > 0:
                        recompute(sg - 1)
                    main.wait_event(ready[k])
                    if rec.adjoint_sweep(rings[k], lengths[sg], lam, nxt, ws):
                        lam, nxt = nxt, lam
                    freed[k] = torch.cuda.Event()
                    freed[k].record(main)
            finally:
                # the side stream's last recomputation precedes the last
                # sweep; on an error it may still be writing a ring
                side.synchronize()
                side_rec.close()
        g = rec.adjoint_grad(ws).sum(axis=0)
        rec.close()
        ctx.ckpts = None
        dMs = torch.tensor(g[0], dtype=torch.float64)
        dv0 = torch.tensor(g[1], dtype=torch.float64)
        return dMs, dv0, None, lam[0], lam[1], lam[2], None, None, None, None


def final_state(Ms, v0, p: PFParams, u0, n: int, every: int = 50, temporal_block: int = 0, overlap: bool = True):
    """Final (c, phi, rho) after n steps; differentiable in Ms, v0 and u0.
    `overlap` recomputes the next segment on a second stream during the
    adjoint steps of the current one."""
    Ms = torch.as_tensor(Ms, dtype=torch.float64)
    v0 = torch.as_tensor(v0, dtype=torch.float64)
    return _FinalState.apply(Ms, v0, p, u0[0], u0[1], u0[2], n, every, temporal_block, overlap)


def l2_mismatch(u, target, h: float = 1.0):
    """h^2/2 sum over the three fields of (u - u*)^2, in FP64."""
    return 0.5 * h * h * sum(((a.double() - b.double()) ** 2).sum() for a, b in zip(u, target))
