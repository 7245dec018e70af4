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
interior x_n are merged into one call.  With mass m the kicks add dt/(2m) F,
so the cotangent handed to the VJP carries 1/m: w_n = 1/m (n > 0), 1/(2m) (n = 0).  Gradients w.r.t. x_0, v_0 and the
packed (eps, sigma) come back in the caller's atom order.
"""
from __future__ import annotations

import ctypes
import time

import torch

from . import _lib, ops
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
                        verify_recompute=True, timings=None):
    """timings: optional dict, filled with host wall times (s) of the forward pass and
    of the reverse pass (recomputation included), each bracketed by a device sync."""

    def mark():
        if timings is None:
            return 0.0
        torch.cuda.synchronize(sim.device)
        return time.perf_counter()

    sim = _forward_sim(L, x0, v0, types, eps, sigma, rc, skin, dt, mass, precision, steps, device)
    nl = sim.nl
    ids = sim.ids
    xref_s = ops.gather_rows(ids, torch.as_tensor(xref, dtype=torch.float64,
                                                  device=sim.device).contiguous())
    ckpt = {}
    t0 = mark()
    for k in range(0, steps, checkpoint_every):
        ckpt[k] = (sim.x.clone(), sim.v.clone(), sim.F.clone())
        sim.step(min(checkpoint_every, steps - k), energy=False)
    xT = sim.x.clone()
    t1 = mark()
    loss, xbar = ops.traj_loss(sim.L, sim.x, xref_s)
    vbar = torch.zeros_like(xbar)
    g = torch.empty_like(xbar)
    geps = torch.zeros_like(sim.eps)
    gsig = torch.zeros_like(sim.eps)
    ws = torch.empty(ops.workspace_bytes(ops.OP_BACKWARD, sim.n, 0, ops._ntypes(sim.eps)),
                     dtype=torch.uint8, device=sim.device)
    lib = _lib.load()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    box = _lib.make_box(sim.L)
    stream = ctypes.c_void_p(torch.cuda.current_stream(sim.device).cuda_stream)
    recompute_ok = True
    for s in reversed(sorted(ckpt)):
        e = min(s + checkpoint_every, steps)
        x, v, F = ckpt[s]
        sim.x.copy_(x)
        sim.v.copy_(v)
        sim.F.copy_(F)
        sim.step_count = s  # keeps the recomputation clear of the rebuild cadence
        xs = [x]
        # the force calls of steps s+1 .. e read x_{s+1} .. x_e
        nrec = e - s if verify_recompute else e - s - 1
        sim.step(nrec, energy=False, on_positions=lambda t: xs.append(t.clone()))
        if verify_recompute:
            ref = ckpt[e][0] if e in ckpt else xT
            recompute_ok &= bool(torch.equal(xs.pop(), ref))
        for n in range(e - 1, s - 1, -1):
            wn = (1.0 if n > 0 else 0.5) / mass
            _lib.check(lib.ljmd_adjoint_kick(sim.n, dt, wn, p(xbar), p(vbar), p(g), stream),
                       "ljmd_adjoint_kick")
            _lib.check(lib.ljmd_force_backward(
                ctypes.byref(box), precision, rc, sim.ntypes, p(sim.eps), p(sim.sigma), sim.n,
                p(xs[n - s]), p(sim.types), p(nl.nbr), p(nl.nnbr), nl.maxn, p(g), p(xbar),
                p(geps), p(gsig), 1, p(ws), ws.numel(), stream), "ljmd_force_backward")
    t2 = mark()
    if timings is not None:
        timings.update(forward_s=t1 - t0, reverse_s=t2 - t1)
    return TrajectoryResult(
        loss=loss, gx0=sim.in_caller_order(xbar), gv0=sim.in_caller_order(vbar), geps=geps,
        gsigma=gsig, xT=ops.scatter_rows(ids, xT), recompute_bitwise=recompute_ok, sim=sim)
