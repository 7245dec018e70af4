"""Integrator and MD-loop parity of the HIP path against the oracle."""
import numpy as np
import pytest

import lj_inputs as li
from helpers import gpu_device, pairs_within

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def T(a, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def test_integrate_stages_bitwise(dev, orc):
    import torch
    from paper_2109_09056_amd import ops
    rng = np.random.default_rng(0)
    L = np.array([10.0, 11.0, 12.0])
    n = 1000
    x = rng.uniform(0, 1, (n, 3)) * L
    x[:3] = [[np.nextafter(10.0, 0), 0.0, 5.0], [0.0, 1e-18, 5.0], [5.0, 5.0, 11.9999999]]
    v = rng.normal(size=(n, 3)) * 50.0
    F = rng.normal(size=(n, 3)) * 30.0
    for mass in (1.0, 2.5):
        xg, vg = T(x, dev), T(v, dev)
        ke = torch.zeros(1, dtype=torch.float64, device=dev)
        ops.integrate(ops.KICK_DRIFT, 0.005, mass, L, xg, vg, T(F, dev))
        xo, vo = x.copy(), v.copy()
        orc.kick_drift(xo, vo, F, 0.005, L, mass=mass)
        assert np.array_equal(xg.cpu().numpy(), xo)
        assert np.array_equal(vg.cpu().numpy(), vo)
        assert np.all(xo >= 0) and np.all(xo < L)
        ops.integrate(ops.KICK, 0.005, mass, L, xg, vg, T(F, dev), ke=ke)
        orc.kick(vo, F, 0.005, mass=mass)
        assert np.array_equal(vg.cpu().numpy(), vo)
        assert float(ke.item()) == pytest.approx(0.5 * mass * (vo * vo).sum(), rel=1e-13)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("ntypes", [1, 2])
def test_md_step_matches_separate_calls(dev, prec, ntypes):
    """ljmd_md_step == compute_forces + integrate(KICK) + integrate(KICK_DRIFT), bitwise."""
    import torch
    from paper_2109_09056_amd import md, ops
    w = li.Workload("t", 3, cells=8, ntypes=ntypes)
    s = li.make_system(w)
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    sim = md.LJSim(w.box, eps=s["eps"], sigma=s["sigma"], precision=P, device=dev)
    sim.load(s["x"], s["v"], s["types"])
    sim.step(3)
    x0, v0 = sim.x.clone(), sim.v.clone()
    for mass in (1.0, 1.7):
        # fused
        v1 = v0.clone()
        xn, F1, ev1 = ops.md_step(w.box, P, w.rc, sim.eps, sim.sigma, x0, sim.types, sim.nl.nbr,
                                  sim.nl.nnbr, sim.nl.maxn, w.dt, mass, v1, F=torch.empty_like(x0))
        # separate calls
        x2, v2 = x0.clone(), v0.clone()
        F2, _, ev2 = ops.compute_forces(w.box, P, ops.FULL, w.rc, sim.eps, sim.sigma, x2,
                                        sim.types, sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn)
        ke = torch.zeros(1, dtype=torch.float64, device=dev)
        ops.integrate(ops.KICK, w.dt, mass, w.box, x2, v2, F2, ke=ke)
        ops.integrate(ops.KICK_DRIFT, w.dt, mass, w.box, x2, v2, F2)
        assert torch.equal(F1, F2)
        assert torch.equal(v1, v2)
        assert torch.equal(xn, x2)
        assert torch.equal(ev1[:7], ev2)
        assert float(ev1[7]) == pytest.approx(float(ke), rel=1e-13)
        # closing a call: velocities kicked once, no drift
        v3 = v0.clone()
        ops.md_step(w.box, P, w.rc, sim.eps, sim.sigma, x0, sim.types, sim.nl.nbr, sim.nl.nnbr,
                    sim.nl.maxn, w.dt, mass, v3, open_next=False)
        v4 = v0.clone()
        ops.integrate(ops.KICK, w.dt, mass, w.box, x0.clone(), v4, F2)
        assert torch.equal(v3, v4)


@pytest.mark.parametrize("cells", [0, 1, 5, 10])
def test_chained_steps_match_md_step(dev, cells):
    """A run of ljmd_md_step_chained calls (halves 0, 1, 0, ...) gives bitwise the
    positions, velocities and forces of ljmd_md_step; ljmd_md_step_sums of each half
    is bitwise the inline ev, and the sums a chained launch forms for the previous
    step agree with it to rounding.  cells 0 and 1 are the empty and one-atom boxes;
    5 and 10 the fcc lattices of 500 and 4000 atoms (ragged last blocks)."""
    import torch
    from paper_2109_09056_amd import md, ops
    if cells >= 2:
        w = li.Workload("t", 4, cells=cells)
        sys_ = li.make_system(w)
        L, x, v = w.box, sys_["x"], sys_["v"]
    else:
        L = np.array([9.0, 10.0, 11.0])
        x = np.array([[1.0, 2.0, 3.0]])[:cells]
        v = np.array([[0.3, -0.2, 0.1]])[:cells]
    n = x.shape[0]
    xt = torch.as_tensor(x, dtype=torch.float64, device=dev).reshape(n, 3).contiguous()
    types = torch.zeros(n, dtype=torch.int32, device=dev)
    if n:
        xs, _, _, _, cs = ops.bin(L, 2.8, xt)
        nl = md.NeighborList(L, 2.8, ops.FULL, device=dev).build(xs, cs)
        nbr, nnbr, maxn = nl.nbr, nl.nnbr, nl.maxn
        vt = torch.as_tensor(v, dtype=torch.float64, device=dev).contiguous()
    else:
        xs, vt = xt, torch.zeros((0, 3), dtype=torch.float64, device=dev)
        nbr = torch.zeros(64 * 8, dtype=torch.int32, device=dev)
        nnbr, maxn = torch.zeros(0, dtype=torch.int32, device=dev), 8
    one = torch.ones(1, dtype=torch.float64, device=dev)
    args = lambda xx: (L, ops.MIXED, 2.5, one, one, xx, types, nbr, nnbr, maxn, 0.005, 1.0)
    ws = torch.empty(max(ops.workspace_bytes(ops.OP_MD_CHAIN, n), 8), dtype=torch.uint8,
                     device=dev)
    xa, va, xb, vb = xs.clone(), vt.clone(), xs.clone(), vt.clone()
    prev = None
    for k in range(5):
        Fa, Fb = torch.empty_like(xa), torch.empty_like(xb)
        xa2, _, ev = ops.md_step(*args(xa), va, F=Fa)
        ev_prev = torch.full((8,), float("nan"), dtype=torch.float64, device=dev)
        xb2 = ops.md_step_chained(*args(xb), vb, k % 2, ws, F=Fb,
                                  ev_prev=ev_prev if k else None)
        assert torch.equal(xa2, xb2) and torch.equal(va, vb) and torch.equal(Fa, Fb)
        if k:
            scale = prev.abs().max().item()
            assert (ev_prev - prev).abs().max().item() <= 1e-12 * scale
        prev = ev.clone()
        assert torch.equal(ops.md_step_sums(n, k % 2, ws), prev)  # this step's half
        if n == 0:
            assert float(prev.abs().max()) == 0.0
        xa, xb = xa2, xb2


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lj_sim_chained_matches_inline(dev, prec):
    """LJSim stepping with chained launches (the default) gives bitwise the
    trajectory and E, W, KE of one ljmd_md_step per step, across rebuilds, energy on
    and off, and calls of one step."""
    import torch
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj32k"]
    s = li.make_system(w)
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    runs = []
    for chain in (False, True):
        sim = md.LJSim(w.box, precision=P, device=dev)
        sim.load(s["x"], s["v"])
        out = []
        for chunk, energy in ((1, True), (1, False), (2, True), (19, True), (41, False),
                              (37, True)):
            sim.step(chunk, energy=energy, chain=chain)
            out.append((sim.x.clone(), sim.v.clone(), sim.F.clone(), sim.ev.clone(),
                        sim.e_atom.clone() if energy else None))
        runs.append(out)
    for a, b in zip(*runs):
        for ta, tb in zip(a, b):
            assert (ta is None and tb is None) or torch.equal(ta, tb)


def test_nve_lj256_matches_oracle_trajectory(dev, orc):
    """100 FP64 steps with rebuilds every 20: GPU and oracle Verlet-mirror trajectories agree."""
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj256"]
    s = li.make_system(w)
    sim = md.LJSim(w.box, precision=ops.FP64, kind=ops.FULL, dt=w.dt, device=dev)
    sim.load(s["x"], s["v"])
    th0 = sim.thermo()
    rec = {20, 50, 100}
    got = {}
    for k in range(1, 101):
        sim.step(1)
        if k in rec:
            got[k] = (sim.in_caller_order(sim.x).cpu().numpy(), sim.thermo())
    _, _, _, thermo, snaps, _ = orc.run_nve(s["x"], s["v"], w.box, w.rc, w.rlist, w.dt, 100,
                                            mode="verlet", record=rec)
    for k in sorted(rec):
        xg, th = got[k]
        d = xg - snaps[k][0]
        d -= w.box * np.round(d / w.box)
        assert np.abs(d).max() < 1e-9, (k, np.abs(d).max())
        pe_o, ke_o = thermo[k][1], thermo[k][2]
        assert th["pe"] == pytest.approx(pe_o, rel=1e-10)
        assert th["ke"] == pytest.approx(ke_o, rel=1e-10)
    assert th0["temp"] == pytest.approx(1.44, rel=1e-12)


def test_nve_energy_and_momentum_lj256(dev, orc):
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj256"]
    s = li.make_system(w)
    u_rc = orc.pair_energy(w.rc * (1 - 1e-15))[0]
    for prec in (ops.FP64, ops.MIXED):
        sim = md.LJSim(w.box, precision=prec, kind=ops.FULL, dt=w.dt, device=dev)
        sim.load(s["x"], s["v"])
        esh = []
        for _ in range(10):
            sim.step(10)
            th = sim.thermo()
            esh.append(th["etot"] - pairs_within(sim.x.cpu().numpy(), w.box, w.rc) * u_rc)
        esh = np.array(esh)
        assert np.abs(esh - esh[0]).max() / w.natoms < 1e-3
        assert sim.v.sum(dim=0).abs().max().item() < 1e-10


def test_md_bitwise_repeatable(dev):
    import torch
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj32k"]
    s = li.make_system(w)
    outs = []
    for _ in range(2):
        sim = md.LJSim(w.box, precision=ops.MIXED, kind=ops.FULL, dt=w.dt, device=dev)
        sim.load(s["x"], s["v"])
        sim.step(45)
        outs.append((sim.x.clone(), sim.v.clone(), sim.ev.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


@pytest.fixture(scope="module")
def oracle_32k_run(orc):
    """The oracle's own Verlet-list trajectory of the 32,000-atom liquid, 1,000 steps (the
    lattice start melts; by step 1,000 it is an equilibrated liquid at T ~ 0.7)."""
    w = li.WORKLOADS["lj32k"]
    s = li.make_system(w)
    _, _, _, thermo, snaps, _ = orc.run_nve(s["x"], s["v"], w.box, w.rc, w.rlist, w.dt, 1000,
                                            mode="verlet", record={20, 100, 1000})
    return w, s, thermo, snaps


@pytest.mark.parametrize("prec,kind", [("fp64", "full"), ("mixed", "full"), ("fp64", "half"),
                                       ("mixed", "half")])
def test_lj32k_trajectory_vs_oracle(dev, oracle_32k_run, prec, kind):
    """32,000 atoms, rebuild every 20 steps: positions and energies track the oracle's own
    trajectory at steps 20 and 100, then 900 more steps keep momentum and energy."""
    from paper_2109_09056_amd import md, ops
    w, s, thermo, snaps = oracle_32k_run
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    K = ops.FULL if kind == "full" else ops.HALF
    sim = md.LJSim(w.box, precision=P, kind=K, dt=w.dt, device=dev)
    sim.load(s["x"], s["v"])
    tol = {20: 1e-11, 100: 1e-9} if P == ops.FP64 else {20: 1e-6, 100: 1e-4}
    done = 0
    for snap in (20, 100):
        sim.step(snap - done)
        done = snap
        d = sim.in_caller_order(sim.x).cpu().numpy() - snaps[snap][0]
        d -= w.box * np.round(d / w.box)
        assert np.abs(d).max() < tol[snap], (snap, np.abs(d).max())
        th = sim.thermo()
        etol = 1e-10 if P == ops.FP64 else 1e-6
        assert th["pe"] == pytest.approx(thermo[snap][1], rel=etol)
    e100 = sim.thermo()["etot"]
    sim.step(900)
    th = sim.thermo()
    assert th["builds"] == 51 and np.isfinite(th["etot"])
    assert abs(th["etot"] - e100) / w.natoms < 5e-3
    assert sim.v.sum(dim=0).abs().max().item() < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replay_matches_eager(dev, prec):
    """Steps replayed from captured HIP graphs give bitwise the eager trajectory,
    across rebuilds (eager work between replays) and repeated replays."""
    import torch
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj32k"]
    s = li.make_system(w)
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    runs = []
    for graphs in (False, True):
        sim = md.LJSim(w.box, precision=P, device=dev)
        sim.load(s["x"], s["v"])
        out = []
        for chunk in (7, 45, 1, 60):
            sim.step(chunk, graphs=graphs)
            out.append((sim.x.clone(), sim.v.clone(), sim.F.clone(), sim.ev.clone()))
        runs.append(out)
        if graphs:
            assert len(sim._graphs) >= 1
    for (xa, va, fa, ea), (xb, vb, fb, eb) in zip(*runs):
        assert torch.equal(xa, xb) and torch.equal(va, vb) and torch.equal(fa, fb)
        assert torch.equal(ea, eb)


@pytest.mark.parametrize("snap", [100, 1000])
@pytest.mark.parametrize("kind", ["full", "half"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_forces_at_oracle_snapshot(dev, orc, oracle_32k_run, snap, kind, prec):
    """Every atom's force and energy, and E and W, at the oracle's own positions of the
    32,000-atom run, against the oracle there: step 100 (the lattice melting) and step
    1,000 (the equilibrated liquid, where per-atom energies are smallest), on full and
    half lists; the lists themselves against the oracle's brute-force sets."""
    import torch
    from helpers import list_pairs
    from paper_2109_09056_amd import md, ops
    w, s, thermo, snaps = oracle_32k_run
    x = snaps[snap][0]
    n = w.natoms
    Fo, eo, Wo, _ = orc.forces(x, w.box, w.rc)
    Eo = eo.sum()
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    K = ops.FULL if kind == "full" else ops.HALF
    sim = md.LJSim(w.box, precision=P, kind=K, device=dev)
    sim.load(x, None)
    up = orc.upper_pairs(x, w.box, w.rlist)
    i, j = list_pairs(sim.nl.nbr.cpu().numpy(), sim.nl.nnbr.cpu().numpy(), sim.nl.maxn)
    ids = sim.ids.cpu().numpy()
    a, b = ids[i], ids[j]
    want = up[:, 0] * n + up[:, 1]
    if K == ops.FULL:  # both directions of every pair, nothing else
        lo = a < b
        assert a.size == 2 * want.size
        assert np.array_equal(np.sort(a[lo] * n + b[lo]), want)
        assert np.array_equal(np.sort(b[~lo] * n + a[~lo]), want)
    else:
        assert np.array_equal(np.sort(np.minimum(a, b) * n + np.maximum(a, b)), want)
    F, e, ev = ops.compute_forces(w.box, P, K, w.rc, sim.eps, sim.sigma, sim.x,
                                  sim.types, sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn)
    Fg = sim.in_caller_order(F).cpu().numpy()
    eg = sim.in_caller_order(e.reshape(-1, 1)).cpu().numpy().reshape(-1)
    ev = ev.cpu().numpy()
    if P == ops.FP64:
        assert np.linalg.norm(Fg - Fo, axis=1).max() <= 1e-12 * np.linalg.norm(Fo, axis=1).max()
        assert np.abs(eg - eo).max() <= 1e-12 * np.abs(eo).max()
        assert ev[0] == pytest.approx(Eo, rel=1e-12)
        assert np.abs(ev[1:] - Wo).max() <= 1e-12 * np.abs(Wo).max()
    else:
        frms = np.sqrt((Fo * Fo).sum() / Fo.shape[0])
        assert np.linalg.norm(Fg - Fo, axis=1).max() <= 1e-5 * frms
        assert (np.abs(eg - eo) / np.abs(eo)).max() <= 1e-6
        assert ev[0] == pytest.approx(Eo, rel=1e-6)
        assert np.abs(ev[1:] - Wo).max() <= 1e-6 * np.abs(Wo).max()


@pytest.mark.parametrize("every,steps", [(50, 100), (10, 40), (5, 40)])
def test_dangerous_build_check_vs_oracle(dev, orc, every, steps):
    """256-atom liquid with the list rebuilt every `every` steps: the largest displacement
    of each window (checked on the GPU at every rebuild) equals the oracle's, from its
    own trajectory, and every window in which the oracle's stale list misses pairs inside
    rc is flagged (some atom moved more than skin/2); with a 50-step window the oracle
    misses pairs, with 5 steps nothing is missed or flagged."""
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj256"]
    s = li.make_system(w)
    missed = []
    rec = set(range(0, steps + 1, every))
    _, _, _, _, snaps, _ = orc.run_nve(s["x"], s["v"], w.box, w.rc, w.rlist, w.dt, steps,
                                       rebuild_every=every, record=rec, missed=missed)
    sim = md.LJSim(w.box, precision=ops.FP64, rebuild_every=every, dt=w.dt, device=dev)
    sim.load(s["x"], s["v"])
    sim.step(steps)
    got = sim.displacement_history()
    assert len(got) == steps // every
    flagged = 0
    for k, dk in enumerate(got):
        d = snaps[(k + 1) * every][0] - snaps[k * every][0]
        d -= w.box * np.round(d / w.box)
        want = np.sqrt((d * d).sum(axis=1)).max()
        assert dk == pytest.approx(want, abs=1e-9)
        miss = max(missed[k * every + 1:(k + 1) * every + 1])
        if miss > 0:
            assert dk > 0.5 * w.skin
        flagged += dk > 0.5 * w.skin
    checked, dangerous, dmax = sim.displacement_report()
    assert (checked, dangerous) == (len(got), flagged) and dmax == max(got)
    if every == 50:
        assert max(missed) > 0 and dangerous == 2
    if every == 5:
        assert max(missed) == 0 and dangerous == 0


def test_deferred_row_capacity_check(dev):
    """LJSim rebuilds leave the longest-row check of a build to the next one (no host wait
    per rebuild): the trajectory is bitwise the one checked (and waited for) at every
    build, and a deferred build that cut rows raises RuntimeError at its check."""
    import torch
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj32k"]
    s = li.make_system(w)
    runs = []
    for headroom in (md.NeighborList.HEADROOM, 10 ** 6):  # deferred / checked at once
        sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=ops.MIXED, device=dev)
        sim.nl.HEADROOM = headroom
        sim.load(s["x"], s["v"])
        sim.step(45)
        sim.thermo()
        runs.append((sim.x.clone(), sim.v.clone(), sim.nl.builds, sim.nl.deferred,
                     sim.nl.last_need, sim.nl.maxn, sim.nl.overflows))
    (xa, va, ba, da, *ra), (xb, vb, bb, db, *rb) = runs
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    assert ba == bb == 3 and da == 2 and db == 0 and ra == rb and ra[2] == 0
    # a build cut at a capacity below its longest row, with the check deferred
    xs, _, _, _, cs = ops.bin(w.box, w.rlist, torch.as_tensor(li.positions(w), device=dev))
    nl = md.NeighborList(w.box, w.rlist, ops.FULL, device=dev).build(xs, cs)
    need = nl.last_need
    nl.maxn, nl.last_need = need - 4, 0
    nl.build(xs, cs, defer=True)
    assert nl.deferred == 1 and nl._pending
    with pytest.raises(RuntimeError, match="cut rows"):
        nl.check()
    assert nl.overflows == 1 and nl.last_need == need
    # in a simulation the failed check surfaces at the next rebuild, before it moves anything
    sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=ops.MIXED, device=dev)
    sim.load(s["x"], s["v"])
    sim.step(19)  # the rebuild at step 20 is the next one
    # a deferred build that cuts rows (no force call reads the list after it: the
    # row capacity changes only here, and the rebuild below raises)
    sim.nl.maxn, sim.nl.last_need = sim.nl.last_need - 4, 0
    sim.nl.build(sim.x, sim.cell_start, defer=True)
    x_before, cs_before = sim.x.clone(), sim.cell_start.clone()
    with pytest.raises(RuntimeError, match="cut rows"):
        sim.rebuild()
    assert torch.equal(sim.x, x_before) and torch.equal(sim.cell_start, cs_before)
