"""Weakly compressible SPH on one MI355X over the MD path's bins and Verlet lists.

SPH is, beside MD, the short-range particle-particle application the paper
names for the same binning and neighbor-list machinery (Introduction; Cabana
"Neighbor List Creation").  Per step, with the list rebuilt on a fixed
cadence (cutoff 2h + skin):
    v += dt/2 a; x += dt v; wrap                 (ljmd_integrate, a in place of F/m)
    every `rebuild_every` steps: re-sort by cell and rebuild the list
    rho = density(x)                             (ljmd_sph_density)
    a = pressure acceleration(x, rho)            (ljmd_sph_accel)
    v += dt/2 a                                  (ljmd_integrate)
The closing half kick of a step and the opening kick + drift of the next run
as one launch (KICK_KICK_DRIFT).  Every arithmetic step runs in libljmd's HIP
kernels; this module owns buffers and the rebuild cadence only.
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import FULL, KICK, KICK_DRIFT, KICK_KICK_DRIFT, KINETIC
from .md import NeighborList, _dev, _to


class SPHSim:
    """State in cell-sorted order; `ids` maps sorted position k to the caller's id."""

    def __init__(self, L, h, mass=1.0, c0=10.0, rho0=1.0, skin=0.4, dt=0.01, rebuild_every=10,
                 device=None):
        self.device = _dev(device)
        self.L = [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]
        self.h, self.mass, self.c0, self.rho0 = float(h), float(mass), float(c0), float(rho0)
        self.rlist = 2.0 * self.h + float(skin)
        self.dt = float(dt)
        self.rebuild_every = int(rebuild_every)
        self.nl = NeighborList(self.L, self.rlist, FULL, device=self.device)
        self.step_count = 0

    def load(self, x, v=None, ids=None):
        dev = self.device
        self.x = _to(x, torch.float64, dev)
        n = self.n = self.x.shape[0]
        self.v = _to(v, torch.float64, dev) if v is not None else torch.zeros_like(self.x)
        self.ids = _to(ids, torch.int64, dev) if ids is not None else None
        self._alt = (torch.empty_like(self.x), torch.empty_like(self.v), None,
                     torch.empty(n, dtype=torch.int64, device=dev))
        self.cell_start = None
        self.rho = torch.empty(n, dtype=torch.float64, device=dev)
        self.acc = torch.empty_like(self.x)
        self.u = torch.zeros(1, dtype=torch.float64, device=dev)   # internal energy U
        self.ke = torch.zeros(1, dtype=torch.float64, device=dev)  # 1/2 sum v^2 (unit mass)
        self.ws = torch.empty(max(ops.workspace_bytes(ops.OP_SPH, n), 8), dtype=torch.uint8,
                              device=dev)
        self.ws_int = torch.empty(max(ops.workspace_bytes(ops.OP_INTEGRATE, n), 8),
                                  dtype=torch.uint8, device=dev)
        self.rebuild()
        self.forces(energy=True)
        ops.integrate(KINETIC, self.dt, 1.0, self.L, None, self.v, None, ke=self.ke,
                      ws=self.ws_int)
        return self

    def rebuild(self):
        self.nl.check()  # the previous build's deferred row check, before anything moves
        xo, vo, _, io, self.cell_start = ops.bin(self.L, self.rlist, self.x, self.v, None,
                                                 self.ids, out=self._alt,
                                                 cell_start=self.cell_start)
        self._alt = (self.x, self.v, None,
                     self.ids if self.ids is not None else torch.empty_like(io))
        self.x, self.v, self.ids = xo, vo, io
        # after the first build, the row-capacity check of each rebuild is left to the next
        # one (or energy()), so the host does not wait for the GPU at every rebuild
        self.nl.build(self.x, self.cell_start, defer=True)

    def forces(self, energy=False):
        """Density (and U when energy) then the pressure acceleration at the current x."""
        nl = self.nl
        ops.sph_density(self.L, self.h, self.mass, self.c0, self.rho0, self.x, nl.nbr, nl.nnbr,
                        nl.maxn, rho=self.rho, u_total=self.u if energy else None, ws=self.ws)
        ops.sph_accel(self.L, self.h, self.mass, self.c0, self.rho0, self.x, self.rho, nl.nbr,
                      nl.nnbr, nl.maxn, acc=self.acc, ws=self.ws)

    def step(self, nsteps=1, energy=False, fused=True):
        """nsteps velocity-Verlet steps; with energy, U and the kinetic energy of the last.
        fused: every step but the last runs its acceleration and integration as one
        pass (ljmd_sph_accel_step; bitwise the separate calls).  acc holds the last
        step's accelerations."""
        if nsteps <= 0:
            return self
        ops.integrate(KICK_DRIFT, self.dt, 1.0, self.L, self.x, self.v, self.acc)
        for s in range(nsteps):
            last = s == nsteps - 1
            self.step_count += 1
            if self.step_count % self.rebuild_every == 0:
                self.rebuild()
            if last:
                self.forces(energy=energy)
                ops.integrate(KICK, self.dt, 1.0, self.L, self.x, self.v, self.acc,
                              ke=self.ke if energy else None, ws=self.ws_int)
            elif fused:
                # acceleration, closing kick and the next opening kick + drift in one pass
                nl = self.nl
                ops.sph_density(self.L, self.h, self.mass, self.c0, self.rho0, self.x, nl.nbr,
                                nl.nnbr, nl.maxn, rho=self.rho, ws=self.ws)
                ops.sph_accel_step(self.L, self.h, self.mass, self.c0, self.rho0, self.x, self.v,
                                   self.rho, nl.nbr, nl.nnbr, nl.maxn, self.dt, ws=self.ws)
            else:
                self.forces()
                ops.integrate(KICK_KICK_DRIFT, self.dt, 1.0, self.L, self.x, self.v, self.acc)
        self.nl.check(block=False)
        return self

    def energy(self):
        """(kinetic m/2 sum v^2, internal U) as of the last step taken with energy (syncs)."""
        self.nl.check()
        return self.mass * float(self.ke.item()), float(self.u.item())

    def in_caller_order(self, t):
        """Rows of a sorted-order tensor rearranged into the caller's order (ids)."""
        return ops.scatter_rows(self.ids, t.contiguous())
