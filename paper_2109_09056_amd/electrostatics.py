"""LJ molecular dynamics with point-charge electrostatics by smooth particle-mesh
Ewald, on one MI355X.

CabanaMD composes the short-range path with SPME: real-space energies and forces
through the same neighbor loops, reciprocal space by spline spreading, 3-D FFTs
and a gradient gather (CabanaMD subsection).  Per step, velocity Verlet with the
list rebuilt on the fixed cadence:
    v += dt/2 F/m; x += dt v; wrap                      (ljmd_integrate)
    every `rebuild_every` steps: re-sort and rebuild; charges follow the ids
    F = F_LJ + F_dir + F_rec                             (ljmd_compute_forces,
                                                          ljmd_ewald_real, ljmd_spme_recip)
    v += dt/2 F/m                                        (ljmd_integrate)
The closing kick of a step and the opening kick + drift of the next run as one
launch.  Every arithmetic step runs in libljmd's HIP kernels; this module only
owns buffers and the order of the calls.
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import FULL, KICK, KICK_DRIFT, KICK_KICK_DRIFT
from .md import LJSim, _to


class ChargedLJSim(LJSim):
    """12-6 LJ plus Coulomb (Gaussian units) between point charges; full lists only.
    The real-space Ewald cutoff is the LJ cutoff rc."""

    def __init__(self, L, alpha=1.2, order=4, grid=(32, 32, 32), **kw):
        kw["kind"] = FULL
        super().__init__(L, **kw)
        self.alpha = float(alpha)
        self.order = int(order)
        self.grid = tuple(int(k) for k in grid)
        self.q_caller = None

    def load(self, x, v, charges, types=None, ids=None):
        dev = self.device
        self.q_caller = _to(charges, torch.float64, dev).reshape(-1)
        n = self.q_caller.shape[0]
        # E_LJ .. W (7), kinetic (1) in ev; E_dir, E_rec + E_self here
        self.ec = torch.zeros(2, dtype=torch.float64, device=dev)
        self._ws_real = torch.empty(ops.workspace_bytes(ops.OP_EWALD_REAL, n), dtype=torch.uint8,
                                    device=dev)
        g = self.grid
        self._ws_rec = torch.empty(ops.workspace_bytes(ops.OP_SPME, n, ncells=g[0] * g[1] * g[2]),
                                   dtype=torch.uint8, device=dev)
        return super().load(x, v, types, ids)

    def rebuild(self):
        super().rebuild()
        self.q = ops.gather_rows(self.ids, self.q_caller)

    def compute_forces(self, energy=True):
        super().compute_forces(energy=energy)
        nl = self.nl
        ops.ewald_real(self.L, self.alpha, self.rc, self.x, self.q, nl.nbr, nl.nnbr, nl.maxn,
                       F=self.F, e_total=self.ec[:1] if energy else None, accumulate=True,
                       ws=self._ws_real)
        ops.spme_recip(self.L, self.alpha, self.order, self.grid, self.x, self.q, F=self.F,
                       e_total=self.ec[1:] if energy else None, accumulate=True,
                       ws=self._ws_rec)

    def step(self, nsteps=1, energy=True, **_):
        """nsteps velocity-Verlet steps; energies (LJ, Coulomb, kinetic) of the last one
        when energy is true."""
        if nsteps <= 0:
            return self
        ws = self._ws[ops.OP_INTEGRATE]
        ops.integrate(KICK_DRIFT, self.dt, self.mass, self.L, self.x, self.v, self.F)
        for s in range(nsteps):
            last = s == nsteps - 1
            self.step_count += 1
            if self.step_count % self.rebuild_every == 0:
                self.rebuild()
            self.compute_forces(energy=energy and last)
            if last:
                ops.integrate(KICK, self.dt, self.mass, self.L, self.x, self.v, self.F,
                              ke=self.ke if energy else None, ws=ws)
            else:
                ops.integrate(KICK_KICK_DRIFT, self.dt, self.mass, self.L, self.x, self.v,
                              self.F)
        return self

    def thermo(self):
        """LJ thermo plus the Coulomb energy (E_dir + E_rec + E_self); the pressure
        is the LJ part only (no Coulomb virial is formed)."""
        t = super().thermo()
        ec = self.ec.cpu()
        t["e_lj"] = t["pe"]
        t["e_coul"] = float(ec[0] + ec[1])
        t["pe"] = t["e_lj"] + t["e_coul"]
        t["etot"] = t["pe"] + t["ke"]
        return t


__all__ = ["ChargedLJSim"]
