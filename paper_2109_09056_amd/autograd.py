"""Differentiable LJ forces: torch.autograd.Function over the HIP adjoint.

Forward calls ljmd_compute_forces, backward calls ljmd_force_backward with
the incoming force cotangent; both walk the same FULL neighbor list, which
(like the set of pairs inside rc) is treated as a constant of the graph.
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import FP64, FULL
from .md import NeighborList, _dev, _to


class ForceContext:
    """Atoms sorted by cell and their FULL Verlet list, for differentiable force calls.

    x (sorted, [n, 3]), types (sorted) and ids (sorted position -> caller id)
    are device tensors; results of LJForce are in this sorted order.
    """

    def __init__(self, L, x, types=None, rc=2.5, skin=0.3, precision=FP64, device=None):
        dev = _dev(device)
        self.L = [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]
        self.rc = float(rc)
        self.rlist = float(rc) + float(skin)
        self.precision = precision
        x = _to(x, torch.float64, dev)
        n = x.shape[0]
        types = (_to(types, torch.int32, dev) if types is not None
                 else torch.zeros(n, dtype=torch.int32, device=dev))
        xs, _, ts, ids, cs = ops.bin(self.L, self.rlist, x, None, types, None)
        self.x, self.types, self.ids = xs, ts, ids
        self.nl = NeighborList(self.L, self.rlist, FULL, device=dev).build(xs, cs)

    def sorted_rows(self, t):
        """Caller-order rows -> sorted order."""
        return ops.gather_rows(self.ids, _to(t, torch.float64, self.x.device))

    def caller_rows(self, t):
        """Sorted-order rows -> caller order."""
        return ops.scatter_rows(self.ids, t.contiguous())


class LJForce(torch.autograd.Function):
    """F = LJForce.apply(x, eps, sigma, ctx): forces on the sorted atoms of ctx."""

    @staticmethod
    def forward(ctx, x, eps, sigma, fc: ForceContext):
        x = x.detach().contiguous()
        eps = eps.detach().contiguous()
        sigma = sigma.detach().contiguous()
        F, _, _ = ops.compute_forces(fc.L, fc.precision, FULL, fc.rc, eps, sigma, x, fc.types,
                                     fc.nl.nbr, fc.nl.nnbr, fc.nl.maxn, want_energy=False)
        ctx.save_for_backward(x, eps, sigma)
        ctx.fc = fc
        return F

    @staticmethod
    def backward(ctx, gF):
        x, eps, sigma = ctx.saved_tensors
        fc = ctx.fc
        gx, geps, gsig = ops.force_backward(fc.L, fc.precision, fc.rc, eps, sigma, x, fc.types,
                                            fc.nl.nbr, fc.nl.nnbr, fc.nl.maxn,
                                            gF.contiguous().to(torch.float64))
        return gx, geps, gsig, None


def lj_forces(x, eps, sigma, fc: ForceContext):
    return LJForce.apply(x, eps, sigma, fc)
