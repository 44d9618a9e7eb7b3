"""Reverse-mode differentiation of GP-MOOD rollouts through the stage adjoint.

`rollout(g, U0, nsteps, cfl, checkpoint_every)` is a torch.autograd.Function over a
single-problem context `g` (GPMood): the forward advances U0 by nsteps SSP-RK3
steps on the GPU and keeps the state every `checkpoint_every` steps; the backward
recomputes each segment from its checkpoint with the dts recorded in the forward
(keeping that segment's stage inputs and final cell orders) and runs the stage
adjoint stage by stage in reverse, on a twin context's stream, so that the
adjoint of one segment overlaps the recomputation of the one before it.  The recomputation must reproduce the forward
bit for bit: the state it reaches at the end of each segment is compared on the
device with the forward's (the next checkpoint, or the rollout's output), and
the backward raises if any differs.  With checkpoint_every = 0 the forward keeps every stage's
inputs and orders instead (three states and three order masks per step: 50 MB a
step at 1024^2 in FP32) and the backward recomputes nothing.  The backward
accumulates dL/d(ell) on the device (gpm_stage_vjp_acc) and reads it once.  The cell orders and every dt are those of the forward, held fixed (the
detection and the CFL reduction are not differentiated).  The stage adjoint is
deterministic, so a backward gives the same bits every time.  Besides dL/dU0 the backward returns
dL/d(ell) through the GP weights (as the gradient of the `ell` input).

Only control flow and buffer handling live here: every arithmetic step of the
forward and of the adjoint runs in the library's kernels.
"""
from __future__ import annotations

import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, ell, g, nsteps, cfl, every):
        ctx.g, ctx.nsteps, ctx.cfl, ctx.every = g, int(nsteps), float(cfl), int(every)
        U = U0.detach().to(device=g.device, dtype=g.dtype).contiguous().clone()
        checkpoints = []
        dts = []
        tape = []
        with torch.cuda.stream(g.stream):
            for n in range(ctx.nsteps):
                if ctx.every == 0:
                    U, dt, stages, orders = _step(g, U, ctx.cfl, keep=True)
                    tape.append((dt, stages, orders))
                else:
                    if n % ctx.every == 0:
                        checkpoints.append(U.clone())
                    U, dt, _, _ = _step(g, U, ctx.cfl, keep=False)
                dts.append(dt)
        ctx.checkpoints = checkpoints
        ctx.tape = tape
        ctx.dts = dts
        # the end of the last segment, for the check of its recomputation
        ctx.U_T = U.clone() if ctx.every != 0 else None
        return U

    @staticmethod
    def backward(ctx, lam_T):
        g = ctx.g
        lam = lam_T.detach().to(device=g.device, dtype=g.dtype).contiguous().clone()
        with torch.cuda.stream(g.stream):
            dl = torch.zeros(1, dtype=torch.float64, device=g.device)
            if ctx.every == 0:
                lam = _reverse(g, ctx.tape, lam, dl)
            else:
                # the stage adjoints of a segment run on the twin context's stream
                # while this context recomputes the segment before it (the
                # recomputation waits on the host once per stage, and the adjoint
                # kernels fill those gaps); same kernels, same order, same bits
                tw = g.vjp_twin()
                sA, sB = g.stream, tw.stream
                differs = torch.zeros((), dtype=torch.bool, device=g.device)
                sB.wait_stream(sA)  # lam and dl are written
                for t in (lam, dl):
                    t.record_stream(sB)
                for seg in reversed(range(len(ctx.checkpoints))):
                    n0 = seg * ctx.every
                    n1 = min(ctx.nsteps, n0 + ctx.every)
                    # recompute the segment with the recorded dts, keeping every
                    # stage's inputs and orders
                    U = ctx.checkpoints[seg].clone()
                    tape = []
                    for n in range(n0, n1):
                        U, dt, stages, orders = _step(g, U, ctx.cfl, keep=True, dt_forward=ctx.dts[n])
                        tape.append((dt, stages, orders))
                    end = ctx.checkpoints[seg + 1] if seg + 1 < len(ctx.checkpoints) else ctx.U_T
                    differs |= (U != end).any()
                    sB.wait_stream(sA)  # the segment's tape is written
                    for _, stages, orders in tape:
                        for t in (*stages, *orders):
                            t.record_stream(sB)  # kept from reuse until sB has read it
                    with torch.cuda.stream(sB):
                        lam = _reverse(tw, tape, lam, dl)
                sA.wait_stream(sB)
                lam = lam.clone()  # on this context's stream, like the other results
                if bool(differs):
                    raise RuntimeError("the backward's recomputation did not reproduce the forward's states")
            grad_ell = dl.to("cpu").reshape(())
        ctx.tape = None
        ctx.U_T = None
        return lam, grad_ell, None, None, None, None


def _reverse(g, tape, lam, dl):
    """Stage adjoints of the taped steps in reverse order, from lam = dL/dU after the
    last of them; dL/d(ell) is added to the device scalar dl.  Returns dL/dU before
    the first."""
    import torch
    for dt, (Un, U1, U2), (o0, o1, o2) in reversed(tape):
        lam_n = torch.zeros_like(lam)
        l2 = torch.empty_like(lam)
        g.gpm_stage_vjp_acc(2, Un, U2, o2, dt, lam, l2, lam_n, dl)
        l1 = torch.empty_like(lam)
        g.gpm_stage_vjp_acc(1, Un, U1, o1, dt, l2, l1, lam_n, dl)
        l0 = torch.empty_like(lam)
        g.gpm_stage_vjp_acc(0, Un, Un, o0, dt, l1, l0, lam_n, dl)
        lam = l0
    return lam


def _step(g, Un, cfl, keep, dt_forward=None):
    """One SSP-RK3 step of context g from the device tensor Un (4, ny, nx).  With
    dt_forward (the recomputation of a recorded step) the step takes that dt,
    without a reduction or a host round trip."""
    if dt_forward is None:
        dt = g.gpm_compute_dt_dev(Un, cfl)
    else:
        g.gpm_set_dt(dt_forward)
        dt = dt_forward
    U1 = torch.empty_like(Un)
    U2 = torch.empty_like(Un)
    U3 = torch.empty_like(Un)
    orders = []
    g.gpm_stage_dev(0, Un, Un, U1)
    if keep:
        orders.append(g.gpm_order_ptr().clone())
    g.gpm_stage_dev(1, Un, U1, U2)
    if keep:
        orders.append(g.gpm_order_ptr().clone())
    g.gpm_stage_dev(2, Un, U2, U3)
    if keep:
        orders.append(g.gpm_order_ptr().clone())
    return U3, dt, (Un, U1, U2), orders


def rollout(g, U0, nsteps, cfl=0.8, checkpoint_every=20, ell=None):
    """Differentiable nsteps-step rollout of context g from U0 (torch (4, ny, nx)).
    checkpoint_every = 0 keeps the whole tape (no recomputation in the backward).

    `ell` (a 0-dim tensor, default the context's length scale) receives dL/d(ell);
    its value must equal the context's ell (the weights are built by set_scheme).
    """
    if ell is None:
        ell = torch.tensor(g.ell, dtype=torch.float64, requires_grad=True)
    return _Rollout.apply(U0, ell, g, nsteps, cfl, checkpoint_every)
