"""Backpropagation through a short velocity-Verlet trajectory with checkpoints.

Forward: `steps` velocity-Verlet steps on one neighbor list built at step 0
(the window is shorter than the rebuild cadence), storing (x, v, F) every
`checkpoint_every` steps.  Loss on the final positions:
    loss = 1/2 sum_i |x_T,i - x_ref,i|^2     (unwrapped difference)
Reverse: the discrete adjoint of velocity Verlet, newest step first.  Each
segment is recomputed forward from its checkpoint (the FULL-list path is
bitwise deterministic, so the recomputation reproduces the stored
trajectory exactly), then walked backwards; per step n (x_n -> x_{n+1})
    vbar += dt * xbar
    (xbar, pbar) += J^T(x_n) (w_n dt vbar)     w_n = 1 (n > 0), 1/2 (n = 0)
where J^T is ljmd_force_backward: the two half-kick VJPs that meet at every
interior x_n are merged into one call.  Gradients w.r.t. x_0, v_0 and the
packed (eps, sigma) come back in the caller's atom order.
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import FP64, FULL
from .md import LJSim


class TrajectoryResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _forward_sim(L, x0, v0, types, eps, sigma, rc, skin, dt, mass, precision, steps, device):
    sim = LJSim(L, rc=rc, skin=skin, eps=eps, sigma=sigma, precision=precision, kind=FULL, dt=dt,
                mass=mass, rebuild_every=steps + 1, device=device)
    sim.load(x0, v0, types)
    return sim


def run_trajectory(L, x0, v0, types, eps, sigma, steps=20, rc=2.5, skin=0.3, dt=0.005,
                   mass=1.0, precision=FP64, device=None):
    """Forward only; returns final positions in caller order."""
    sim = _forward_sim(L, x0, v0, types, eps, sigma, rc, skin, dt, mass, precision, steps, device)
    sim.step(steps, energy=False)
    return sim.in_caller_order(sim.x)


def backprop_trajectory(L, x0, v0, types, eps, sigma, xref, steps=20, checkpoint_every=5,
                        rc=2.5, skin=0.3, dt=0.005, mass=1.0, precision=FP64, device=None,
                        verify_recompute=True):
    sim = _forward_sim(L, x0, v0, types, eps, sigma, rc, skin, dt, mass, precision, steps, device)
    nl = sim.nl
    ids = sim.ids
    xref_s = ops.gather_rows(ids, torch.as_tensor(xref, dtype=torch.float64,
                                                  device=sim.device).contiguous())
    ckpt = {}
    for k in range(steps):
        if k % checkpoint_every == 0:
            ckpt[k] = (sim.x.clone(), sim.v.clone(), sim.F.clone())
        sim.step(1, energy=False)
    xT = sim.x.clone()
    loss, xbar = ops.traj_loss(sim.L, sim.x, xref_s)
    vbar = torch.zeros_like(xbar)
    g = torch.empty_like(xbar)
    geps = torch.zeros_like(sim.eps)
    gsig = torch.zeros_like(sim.eps)
    ws = torch.empty(ops.workspace_bytes(ops.OP_BACKWARD, sim.n, 0, ops._ntypes(sim.eps)),
                     dtype=torch.uint8, device=sim.device)
    recompute_ok = True
    starts = sorted(ckpt)
    for s in reversed(starts):
        e = min(s + checkpoint_every, steps)
        x, v, F = ckpt[s]
        sim.x.copy_(x)
        sim.v.copy_(v)
        sim.F.copy_(F)
        sim.step_count = s  # keeps the recomputation clear of the rebuild cadence
        xs = [sim.x.clone()]
        for _ in range(s, e - 1):
            sim.step(1, energy=False)
            xs.append(sim.x.clone())
        if verify_recompute:
            sim.step(1, energy=False)
            ref = ckpt[e][0] if e in ckpt else xT
            recompute_ok &= bool(torch.equal(sim.x, ref))
        for n in range(e - 1, s - 1, -1):
            ops.adjoint_kick(dt, 1.0 if n > 0 else 0.5, xbar, vbar, g)
            ops.force_backward(sim.L, precision, rc, sim.eps, sim.sigma, xs[n - s], sim.types,
                               nl.nbr, nl.nnbr, nl.maxn, g, gx=xbar, geps=geps, gsigma=gsig,
                               accumulate=True, ws=ws)
    return TrajectoryResult(
        loss=loss, gx0=sim.in_caller_order(xbar), gv0=sim.in_caller_order(vbar), geps=geps,
        gsigma=gsig, xT=ops.scatter_rows(ids, xT), recompute_bitwise=recompute_ok, sim=sim)
