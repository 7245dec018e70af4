"""LJ + SPME electrostatics in the MD loop: the forces of the composed step against
the sum of the oracles (LJ, Ewald direct sum, SPME reference steps) on the same
input, and total-energy conservation of a charged liquid under velocity Verlet."""
import numpy as np
import pytest

import lj_inputs as li
from helpers import gpu_device, pairs_within

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _sim(dev, w, grid, order, v=None):
    from paper_2109_09056_amd import electrostatics as es, ops
    sim = es.ChargedLJSim(w.box, alpha=li.EWALD_ALPHA, order=order, grid=grid, rc=w.rc,
                          skin=w.skin, precision=ops.FP64, dt=w.dt,
                          rebuild_every=w.rebuild_every, device=dev)
    return sim.load(li.positions(w), v, li.charges(w))


@pytest.mark.parametrize("name,grid,order", [("lj256", (16, 16, 16), 6),
                                             ("lj32k", (64, 64, 64), 4)])
def test_composed_forces_vs_oracles(dev, orc, name, grid, order):
    w = li.WORKLOADS[name]
    x, q = li.positions(w), li.charges(w)
    sim = _sim(dev, w, grid, order)
    F_lj, e_lj, _, _ = orc.forces(x, w.box, w.rc)
    e_d, F_d = orc.ewald_direct(x, q, w.box, li.EWALD_ALPHA, w.rc)
    E_r, F_r = orc.spme_recip(x, q, w.box, li.EWALD_ALPHA, grid, order)
    F_o = F_lj + F_d + F_r
    Fg = sim.in_caller_order(sim.F).cpu().numpy()
    assert np.abs(Fg - F_o).max() <= 1e-11 * np.abs(F_o).max()
    t = sim.thermo()
    assert t["e_lj"] == pytest.approx(e_lj.sum(), rel=1e-12)
    assert t["e_coul"] == pytest.approx(e_d.sum() + E_r + orc.ewald_self(q, li.EWALD_ALPHA),
                                        rel=1e-11)


def test_charged_liquid_conserves_energy(dev, orc):
    """256 unit charges in the LJ liquid, 200 steps (10 list rebuilds): the total energy,
    with the LJ truncation jumps removed (E - n_pairs(r < rc) u(rc), as for the LJ
    runs), stays within 1e-3 per atom of its start (velocity Verlet's O(dt^2) error;
    the real-space truncation jumps are ~1e-5 per crossing pair), and the total
    momentum stays small."""
    w = li.WORKLOADS["lj256"]
    sim = _sim(dev, w, (16, 16, 16), 6, v=li.velocities(w))
    u_rc = orc.pair_energy(w.rc * (1 - 1e-15))[0]
    esh = []
    for _ in range(10):
        sim.step(20)
        th = sim.thermo()
        esh.append(th["etot"] - pairs_within(sim.x.cpu().numpy(), w.box, w.rc) * u_rc)
    esh = np.array(esh)
    assert np.abs(esh - esh[0]).max() / w.natoms < 1e-3, esh
    # momentum: the pair forces conserve it exactly, SPME's gathered forces only to
    # its interpolation error (their sum is not zero), so a small bounded drift
    v = sim.v
    assert v.sum(dim=0).abs().max().item() < 1e-3 * v.abs().sum().item()
    assert sim.nl.overflows == 0
