"""Compressed (CSR) neighbor lists and team-per-atom force traversal: rows equal to the
tiled list they come from, forces and energies against the oracle for every team size,
the tiled kernel's team bitwise equal to its forces, every team deterministic."""
import numpy as np
import pytest

import lj_inputs as li
from helpers import decode_rows, gpu_device, max_rel_vec

pytestmark = pytest.mark.gpu

TEAMS = (1, 2, 4, 8, 16)


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _case(name):
    """(box, caller-order positions, types, eps, sigma) of a named input."""
    if name == "gas1000":  # ragged n, uniform random, one type
        rng = np.random.default_rng(11)
        L = np.array([12.0, 13.0, 14.0])
        return L, rng.uniform(0, 1, (1000, 3)) * L, np.zeros(1000, np.int32), [1.0], [1.0]
    # 70,304 atoms, two types: beyond the four-lane small-grid size of the tiled kernel
    w = li.Workload("lj70k_2t", 7, cells=26, ntypes=2) if name == "lj70k_2t" else li.WORKLOADS[name]
    if w.ntypes == 1:
        return w.box, li.positions(w), np.zeros(w.natoms, np.int32), [1.0], [1.0]
    eps, sig = li.params(w)
    return w.box, li.positions(w), li.types(w), eps, sig


_ORACLE = {}


def _oracle(orc, name):
    if name not in _ORACLE:
        L, x, ty, eps, sig = _case(name)
        _ORACLE[name] = orc.forces(x, L, 2.5, eps, sig, ty if len(eps) > 1 else None)
    return _ORACLE[name]


def _sim(dev, name):
    from paper_2109_09056_amd import md, ops
    L, x, ty, eps, sig = _case(name)
    sim = md.LJSim(L, eps=eps, sigma=sig, precision=ops.FP64, kind=ops.FULL, device=dev)
    sim.load(x, None, ty)
    return sim


@pytest.mark.parametrize("name", ["lj256", "gas1000", "lj32k", "lj32k_fm"])
def test_csr_rows_equal_tiled(dev, name):
    import torch
    from paper_2109_09056_amd import ops
    sim = _sim(dev, name)
    nl = sim.nl
    off, csr = ops.list_to_csr(nl.nbr, nl.nnbr, nl.maxn)
    rows = decode_rows(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn)
    off_h, csr_h = off.cpu().numpy(), csr.cpu().numpy()
    cnt = np.array([r.size for r in rows])
    assert off_h[0] == 0 and np.array_equal(np.diff(off_h), cnt)
    for i, r in enumerate(rows):
        assert np.array_equal(csr_h[off_h[i]:off_h[i + 1]], r), i  # same order
    # a capacity below the total: offsets unchanged, nothing written at or past cap
    total = int(off_h[-1])
    cap = total - 37
    sentinel = torch.full((total + 16,), -7, dtype=torch.int32, device=dev)
    off2, _ = ops.list_to_csr(nl.nbr, nl.nnbr, nl.maxn, cap=cap, csr=sentinel)
    s = sentinel.cpu().numpy()
    assert np.array_equal(off2.cpu().numpy(), off_h)
    assert np.array_equal(s[:cap], csr_h[:cap]) and np.all(s[cap:] == -7)


def test_csr_empty(dev):
    import torch
    from paper_2109_09056_amd import ops
    nbr = torch.zeros(64 * 8, dtype=torch.int32, device=dev)
    nnbr = torch.zeros(0, dtype=torch.int32, device=dev)
    off, _ = ops.list_to_csr(nbr, nnbr, 8, cap=0)
    assert off.cpu().tolist() == [0]
    x = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    one = torch.ones(1, dtype=torch.float64, device=dev)
    _, _, ev = ops.compute_forces_csr([10.0, 10.0, 10.0], ops.FP64, 2.5, one, one, x,
                                      torch.zeros(0, dtype=torch.int32, device=dev), off,
                                      torch.zeros(1, dtype=torch.int32, device=dev), team=4)
    assert torch.count_nonzero(ev).item() == 0


@pytest.mark.parametrize("name", ["lj256", "gas1000", "lj32k", "lj32k_fm"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_csr_forces_vs_oracle(dev, orc, name, prec):
    """Every team size against the oracle (FP64 1e-12; mixed 1e-5 F_rms, 1e-6 per-atom e)."""
    from paper_2109_09056_amd import ops
    Fo, eo, Wo, _ = _oracle(orc, name)
    sim = _sim(dev, name)
    nl = sim.nl
    off, csr = ops.list_to_csr(nl.nbr, nl.nnbr, nl.maxn)
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    for team in TEAMS:
        F, e, ev = ops.compute_forces_csr(sim.L, P, 2.5, sim.eps, sim.sigma, sim.x, sim.types,
                                          off, csr, team=team)
        Fg = sim.in_caller_order(F).cpu().numpy()
        eg = sim.in_caller_order(e).cpu().numpy()
        ev = ev.cpu().numpy()
        if P == ops.FP64:
            assert max_rel_vec(Fg, Fo) <= 1e-12, team
            assert np.abs(eg - eo).max() <= 1e-12 * np.abs(eo).max(), team
            assert ev[0] == pytest.approx(eo.sum(), rel=1e-12)
            assert np.abs(ev[1:] - Wo).max() <= 1e-12 * np.abs(Wo[:3]).max()
        else:
            frms = np.sqrt((Fo * Fo).sum() / Fo.shape[0])
            assert np.linalg.norm(Fg - Fo, axis=1).max() <= 1e-5 * frms, team
            assert (np.abs(eg - eo) / np.maximum(np.abs(eo), 1e-3)).max() <= 1e-6, team
            assert ev[0] == pytest.approx(eo.sum(), rel=1e-6)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["lj32k_fm", "lj70k_2t"])
def test_csr_team_bitwise_tiled_and_teams_deterministic(dev, prec, name):
    """The tiled kernel walks rows with four lanes per atom up to SMALL_GRID_ATOMS atoms
    (32,000 here) and two beyond (70,304): CSR with that team gives bitwise the same
    forces and per-atom energies; every team size is deterministic."""
    import torch
    from paper_2109_09056_amd import _lib, ops
    sim = _sim(dev, name)
    nl = sim.nl
    tiled_team = 4 if sim.n <= _lib.SMALL_GRID_ATOMS else 2
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    off, csr = ops.list_to_csr(nl.nbr, nl.nnbr, nl.maxn)
    Ft, et, evt = ops.compute_forces(sim.L, P, ops.FULL, 2.5, sim.eps, sim.sigma, sim.x,
                                     sim.types, nl.nbr, nl.nnbr, nl.maxn)
    F2, e2, ev2 = ops.compute_forces_csr(sim.L, P, 2.5, sim.eps, sim.sigma, sim.x, sim.types,
                                         off, csr, team=tiled_team)
    assert torch.equal(F2, Ft) and torch.equal(e2, et)
    np.testing.assert_allclose(ev2.cpu().numpy(), evt.cpu().numpy(), rtol=1e-12, atol=0)
    if name != "lj32k_fm":
        return
    for team in TEAMS:
        a = ops.compute_forces_csr(sim.L, P, 2.5, sim.eps, sim.sigma, sim.x, sim.types, off, csr,
                                   team=team)
        b = ops.compute_forces_csr(sim.L, P, 2.5, sim.eps, sim.sigma, sim.x, sim.types, off, csr,
                                   team=team)
        assert all(torch.equal(u, v) for u, v in zip(a, b)), team
        # forces only (no energy): the same forces
        Fn, _, _ = ops.compute_forces_csr(sim.L, P, 2.5, sim.eps, sim.sigma, sim.x, sim.types,
                                          off, csr, team=team, want_energy=False)
        assert torch.equal(Fn, a[0]), team


# ------------------------------------------------------------- AoSoA layouts --

@pytest.mark.parametrize("vlen", [0, 1, 8, 64])
@pytest.mark.parametrize("name", ["gas1000", "lj256", "lj32k", "lj32k_fm"])
def test_aosoa_forces_bitwise_equal_and_vs_oracle(dev, orc, name, vlen):
    """Positions and forces in AoSoA(vlen) (0: SoA): forces, per-atom energies, energy and
    virial bitwise those of the [n][3] kernel (same traversal and order) for FP64 and
    mixed, and the FP64 forces against the oracle; the conversion round-trips exactly."""
    import torch
    from paper_2109_09056_amd import ops
    sim = _sim(dev, name)
    nl = sim.nl
    xa = ops.aosoa_convert(sim.x, vlen, True)
    assert torch.equal(ops.aosoa_convert(xa, vlen, False, n=sim.n), sim.x)
    if vlen not in (0, 1):  # chunk-major; the last chunk holds the remaining atoms
        for i in (0, vlen + 3, sim.n - 1):
            c = i // vlen
            wid = min(vlen, sim.n - c * vlen)
            base = c * 3 * vlen + i - c * vlen
            assert float(xa[base + wid].item()) == float(sim.x[i, 1].item())
            assert float(xa[base + 2 * wid].item()) == float(sim.x[i, 2].item())
    for prec in (ops.FP64, ops.MIXED):
        F, e, ev = ops.compute_forces(sim.L, prec, ops.FULL, 2.5, sim.eps, sim.sigma, sim.x,
                                      sim.types, nl.nbr, nl.nnbr, nl.maxn)
        Fa, ea, eva = ops.compute_forces_aosoa(sim.L, prec, 2.5, sim.eps, sim.sigma, xa,
                                               sim.types, nl.nbr, nl.nnbr, nl.maxn, vlen)
        assert torch.equal(ops.aosoa_convert(Fa, vlen, False, n=sim.n), F)
        assert torch.equal(ea, e) and torch.equal(eva, ev)
        if prec == ops.FP64:
            Fo = _oracle(orc, name)[0]
            Fg = ops.scatter_rows(sim.ids, ops.aosoa_convert(Fa, vlen, False, n=sim.n))
            assert max_rel_vec(Fg.cpu().numpy(), Fo) <= 1e-12


def test_aosoa_rejects_other_vector_lengths(dev):
    import torch
    from paper_2109_09056_amd import _lib, ops
    x = torch.zeros(10, 3, dtype=torch.float64, device=dev)
    with pytest.raises(_lib.LjmdError):
        ops.aosoa_convert(x, 16, True)


# ------------------------------------------------- compressed rows from the cells --

@pytest.mark.parametrize("kind", ["full", "half"])
@pytest.mark.parametrize("name", ["lj256", "gas1000", "lj32k", "lj32k_fm"])
def test_direct_csr_build_equals_tiled_rows(dev, name, kind):
    """Rows built straight into CSR equal the tiled build's rows entry by entry (same order),
    full and half; a capacity below the total keeps the offsets and drops only the tail."""
    import torch
    from paper_2109_09056_amd import md, ops
    sim = _sim(dev, name)
    K = ops.FULL if kind == "full" else ops.HALF
    nl = md.NeighborList(sim.L, sim.rlist, K, device=dev).build(sim.x, sim.cell_start)
    off, csr = ops.build_neighbors_csr(sim.L, sim.rlist, K, sim.x, sim.cell_start)
    rows = decode_rows(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn)
    assert int(nl.max_count.item()) <= nl.maxn
    off_h, csr_h = off.cpu().numpy(), csr.cpu().numpy()
    cnt = np.array([r.size for r in rows])
    assert np.array_equal(np.diff(off_h), cnt) and off_h[0] == 0
    assert np.array_equal(csr_h[:off_h[-1]], np.concatenate(rows))
    cap = int(off_h[-1]) // 2
    small = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    off2, _ = ops.build_neighbors_csr(sim.L, sim.rlist, K, sim.x, sim.cell_start, cap=cap,
                                      csr=small)
    assert torch.equal(off2, off) and np.array_equal(small.cpu().numpy(), csr_h[:cap])


def test_direct_csr_forces_vs_oracle(dev, orc):
    """Team traversal over the direct CSR list: the oracle's forces and energies."""
    from paper_2109_09056_amd import ops
    name = "lj32k_fm"
    sim = _sim(dev, name)
    off, csr = ops.build_neighbors_csr(sim.L, sim.rlist, ops.FULL, sim.x, sim.cell_start)
    Fo, eo, _, _ = _oracle(orc, name)
    for team in (1, 4):
        F, e, _ = ops.compute_forces_csr(sim.L, ops.FP64, 2.5, sim.eps, sim.sigma, sim.x,
                                         sim.types, off, csr, team=team)
        assert max_rel_vec(ops.scatter_rows(sim.ids, F).cpu().numpy(), Fo) <= 1e-12
        eg = ops.scatter_rows(sim.ids, e.reshape(-1, 1)).cpu().numpy().reshape(-1)
        assert np.abs(eg - eo).max() <= 1e-12 * np.abs(eo).max()
