#!/usr/bin/env python3
"""Benchmark of the short-range LJ MD hot path on one MI355X.

A step is one velocity-Verlet MD step of the whole path: the binned re-sort
and Verlet-list rebuild every 20 steps, LJ forces with per-atom energy,
energy and virial, the closing half kick with the kinetic energy and the
next step's opening half kick, drift and wrap: one fused launch per step on
the full list, which also sums the previous step's energy/virial/KE partial
rows, and one reduction launch closing the run.  Workload: the 500,000-atom dense LJ liquid (fcc 50^3 cells
at rho* = 0.8442, T* = 1.44, rc 2.5, skin 0.3, dt 0.005), synthetic and
seeded, inputs resident in HBM before the timed region.

Prints ONE JSON line: the mixed-precision path's atom-steps/s (headline), the
FP64 path beside it, backward/forward time ratios (32k force matching and the
256k checkpointed trajectory), the dominant kernel's roofline figures and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import statistics
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Counter figures of the fused step kernel k_force_full<mixed, one type, EV, 6, interior,
# step, narrow, team 2, [n][3]> on the 500,000-atom workload, from the rocprofv3 summaries
# committed in profiles/ (k_force_full_step_lj500k_hbm_counters.txt, ..._pipeline_counters.txt):
# HBM bytes per dispatch = FETCH_SIZE x 2 + WRITE_SIZE x 1 (the scales a 512 MiB copy
# gives the two counters); set to None whenever the kernel changes until re-measured.
FORCE_COUNTERS_FROM = ("profiles/k_force_full_step_lj500k_hbm_counters.txt and "
                       "..._pipeline_counters.txt (rocprofv3 --pmc on this kernel build)")
FORCE_TRAFFIC = 234.56e6
FORCE_VALU_BUSY = 0.540
FORCE_TA_BUSY = 0.766


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="lj500k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the headline path only (no FP64 run, no bwd/fwd ratios)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target length of the oracle's CPU sample")
    ap.add_argument("--sph-only", action="store_true",
                    help="run only the SPH leg (512,000 particles) and print its JSON object")
    ap.add_argument("--spme-only", action="store_true",
                    help="run only the SPME leg (500,000 charges) and print its JSON object")
    ap.add_argument("--charged-only", action="store_true",
                    help="run only the charged LJ + SPME MD leg and print its JSON object")
    ap.add_argument("--half-only", action="store_true",
                    help="run only the half-list force calls (32,000 and 500,000 atoms) beside the "
                         "full-list ones and print their JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 512 MiB (x5), to calibrate HBM "
                         "byte counters")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch
    nbytes = 512 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 5}), flush=True)


EVENT_SPAN = 10
WINDOWS = 3


def span_events(first_step, steps, rebuild_every):
    """Per-step items for LJSim.step's force_events: one event pair spanning the launches
    of EVENT_SPAN consecutive steps with no rebuild between them (a rebuild runs before its
    step's start event), so the average launch is the pair's time / EVENT_SPAN and the
    timed window carries two event records; with no such run, every launch alone.
    Returns (items, [(start, end, launches)])."""
    import torch
    new = lambda: torch.cuda.Event(enable_timing=True)
    rebuild = [(first_step + k) % rebuild_every == 0 for k in range(steps)]
    span = min(EVENT_SPAN, steps)
    for k0 in range(steps - span + 1):
        if span > 1 and not any(rebuild[k0 + 1:k0 + span]):
            a, b = new(), new()
            items = [None] * steps
            items[k0], items[k0 + span - 1] = (a, None), (None, b)
            return items, [(a, b, span)]
    items = [(new(), new()) for _ in range(steps)]
    return items, [(a, b, 1) for a, b in items]


def md_run(w, s, precision, steps, warmup, dev, windows=WINDOWS, kind=None):
    """Time `windows` consecutive windows of `steps` MD steps each after `warmup` steps;
    returns (median window seconds, all window seconds, per-launch force-call ms list, sim).

    Python's garbage collector is run before and held off during the windows: a full
    collection of this process's objects costs tens of milliseconds, which would land
    inside a short window as a host-side stall between launches."""
    import gc
    import torch
    from paper_2109_09056_amd import md, ops
    sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=precision,
                   kind=ops.FULL if kind is None else kind, dt=w.dt,
                   rebuild_every=w.rebuild_every, device=dev)
    sim.load(s["x"], s["v"])
    # every window's timing events, created (at their first record) before anything is timed
    plan = []
    for k in range(windows):
        events, pairs = span_events(sim.step_count + warmup + k * steps + 1, steps,
                                    w.rebuild_every)
        for a, b, _ in pairs:
            a.record()
            b.record()
        plan.append((events, pairs))
    times = []
    gc.collect()
    gc.disable()
    try:
        sim.step(warmup)
        # windows back to back: only the synchronizations that bracket each one in between,
        # so the GPU does not idle (and clock down) between them
        torch.cuda.synchronize()
        for events, _ in plan:
            t0 = time.perf_counter()
            sim.step(steps, force_events=iter(events))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            times.append(t1 - t0)
    finally:
        gc.enable()
    force_ms = [a.elapsed_time(b) / m for _, pairs in plan for a, b, m in pairs]
    return statistics.median(times), times, force_ms, sim


def event_time(fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def bwd_fwd_forcematching(dev, reps=100):
    """Force-matching workload (32,000 atoms, two types): t(force_backward)/t(compute_forces)."""
    import numpy as np
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import autograd, ops
    w = li.WORKLOADS["lj32k_fm"]
    x, ty = li.positions(w), li.types(w)
    eps, sig = (torch.as_tensor(a, device=dev) for a in li.params(w))
    out = {}
    for name, prec in (("mixed", ops.MIXED), ("fp64", ops.FP64)):
        fc = autograd.ForceContext(w.box, x, ty, rc=w.rc, skin=w.skin, precision=prec, device=dev)
        g = torch.as_tensor(np.random.default_rng(0).normal(size=x.shape), device=dev)
        F = torch.empty_like(fc.x)
        gx = torch.empty_like(fc.x)
        ge, gs = torch.empty_like(eps), torch.empty_like(eps)
        wsf = torch.empty(ops.workspace_bytes(ops.OP_FORCES, x.shape[0]), dtype=torch.uint8,
                          device=dev)
        wsb = torch.empty(ops.workspace_bytes(ops.OP_BACKWARD, x.shape[0], 0, 2),
                          dtype=torch.uint8, device=dev)
        nl = fc.nl
        tf = event_time(lambda: ops.compute_forces(w.box, prec, ops.FULL, w.rc, eps, sig, fc.x,
                                                   fc.types, nl.nbr, nl.nnbr, nl.maxn, F=F,
                                                   want_energy=False, ws=wsf), reps)
        tb = event_time(lambda: ops.force_backward(w.box, prec, w.rc, eps, sig, fc.x, fc.types,
                                                   nl.nbr, nl.nnbr, nl.maxn, g, gx=gx, geps=ge,
                                                   gsigma=gs, ws=wsb), reps)
        out[name] = {"fwd_ms": round(tf, 5), "bwd_ms": round(tb, 5), "ratio": round(tb / tf, 3)}
    return out


def bwd_fwd_trajectory(dev):
    """Backprop through 20 steps of the 256,000-atom two-type system (mixed), checkpoints
    every 5: trajectory-level t(reverse pass, recomputation included) / t(forward pass
    with checkpoint stores), best of 3, and the kernel-level ratio on the same list."""
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import ops, trajectory
    w = li.WORKLOADS["lj256k_traj"]
    x0, v0, ty = li.positions(w), li.velocities(w), li.types(w)
    eps, sig = li.params(w)
    et, st = li.perturbed_params(w)
    xref = trajectory.run_trajectory(w.box, x0, v0, ty, et, st, steps=w.steps, precision=ops.MIXED,
                                     device=dev)
    sim = trajectory._forward_sim(w.box, x0, v0, ty, eps, sig, w.rc, w.skin, w.dt, 1.0,
                                  ops.MIXED, w.steps, dev)
    sim.step(w.steps, energy=False)  # warm-up of the forward kernels
    best = None
    for _ in range(3):
        tm = {}
        r = trajectory.backprop_trajectory(w.box, x0, v0, ty, eps, sig, xref.cpu().numpy(),
                                           steps=w.steps, checkpoint_every=w.checkpoint_every,
                                           precision=ops.MIXED, device=dev,
                                           verify_recompute=False, timings=tm)
        if best is None or tm["forward_s"] + tm["reverse_s"] < best["forward_s"] + best["reverse_s"]:
            best = tm
    s2 = r.sim
    nl = s2.nl
    g = torch.randn_like(s2.x)
    tf = event_time(lambda: ops.compute_forces(w.box, ops.MIXED, ops.FULL, w.rc, s2.eps, s2.sigma,
                                               s2.x, s2.types, nl.nbr, nl.nnbr, nl.maxn,
                                               want_energy=False), 20)
    tb = event_time(lambda: ops.force_backward(w.box, ops.MIXED, w.rc, s2.eps, s2.sigma, s2.x,
                                               s2.types, nl.nbr, nl.nnbr, nl.maxn, g), 20)
    return {"steps": w.steps, "checkpoint_every": w.checkpoint_every,
            "forward_s": round(best["forward_s"], 5), "reverse_s": round(best["reverse_s"], 5),
            "trajectory_ratio": round(best["reverse_s"] / best["forward_s"], 3),
            "kernel_fwd_ms": round(tf, 5), "kernel_bwd_ms": round(tb, 5),
            "kernel_ratio": round(tb / tf, 3)}


def config1_matrix(dev, steps=1000, warmup=50):
    """The 32,000-atom liquid (fcc 20^3 cells), 1,000 steps rebuilding every 20, in each of
    FP64 / mixed x full / half lists: atom-steps/s (median of three windows) and the
    average force launch (full lists: the fused step launch; half lists: the force
    call, whose integration runs as separate launches)."""
    import lj_inputs as li
    from paper_2109_09056_amd import ops
    w = li.WORKLOADS["lj32k"]
    s = li.make_system(w)
    out = {}
    for pname, prec in (("fp64", ops.FP64), ("mixed", ops.MIXED)):
        for kname, kind in (("full", ops.FULL), ("half", ops.HALF)):
            t, tw, fms, sim = md_run(w, s, prec, steps, warmup, dev, kind=kind)
            out[f"{pname}_{kname}"] = {
                "value": round(w.natoms * steps / t, 1), "ms_per_step": round(t * 1e3 / steps, 5),
                "force_launch_us": round(statistics.mean(fms) * 1e3, 3),
                "mean_list_length": round(float(sim.nl.nnbr.double().mean().item()), 3)}
            del sim
    out["natoms"], out["steps"], out["unit"] = w.natoms, steps, "atom-steps/s"
    return out


def half_bench(dev, reps=20):
    """Force calls on the 32,000- and 500,000-atom starts (mixed): the half list (each pair
    once, partner sums through LDS tiles and FP64 atomics) against the full list, with
    per-atom energies and virial and forces only, HIP events around `reps` calls each."""
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import md, ops
    out = {}
    for name in ("lj32k", "lj500k"):
        w = li.WORKLOADS[name]
        s = li.make_system(w)
        sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=ops.MIXED, device=dev)
        sim.load(s["x"], s["v"])
        hl = md.NeighborList(sim.L, sim.rlist, ops.HALF, device=dev).build(sim.x, sim.cell_start)
        F, e = torch.empty_like(sim.F), torch.empty_like(sim.e_atom)
        ev = torch.empty(7, dtype=torch.float64, device=dev)
        row = {}
        for lname, nl, kind in (("full", sim.nl, ops.FULL), ("half", hl, ops.HALF)):
            for ename, want in (("energies", True), ("forces_only", False)):
                row[f"{lname}_{ename}_us"] = round(event_time(lambda: ops.compute_forces(
                    w.box, ops.MIXED, kind, w.rc, sim.eps, sim.sigma, sim.x, sim.types, nl.nbr,
                    nl.nnbr, nl.maxn, F=F, e_atom=e if want else None, ev=ev if want else None,
                    want_energy=want, ws=sim._ws[ops.OP_FORCES]), reps) * 1e3, 2)
        row["half_over_full_energies"] = round(row["half_energies_us"] / row["full_energies_us"], 3)
        row["half_over_full_forces_only"] = round(row["half_forces_only_us"] /
                                                  row["full_forces_only_us"], 3)
        out[name] = row
        del sim, hl
    return out


def mixed_error(w, sim):
    """Mixed against FP64 forces and energies at the final positions of the mixed run."""
    import torch
    from paper_2109_09056_amd import ops
    out = {}
    for name, prec in (("mixed", ops.MIXED), ("fp64", ops.FP64)):
        out[name] = ops.compute_forces(w.box, prec, ops.FULL, w.rc, sim.eps, sim.sigma, sim.x,
                                       sim.types, sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn)
    (Fm, em, evm), (Fd, ed, evd) = out["mixed"], out["fp64"]
    frms = torch.sqrt((Fd * Fd).sum(dim=1).mean())
    return {"max_dF_over_Frms": float((Fm - Fd).norm(dim=1).max() / frms),
            "max_rel_de_atom": float(((em - ed).abs() / ed.abs()).max()),
            "max_de_atom_over_mean_abs_e": float((em - ed).abs().max() / ed.abs().mean()),
            "atoms_rel_de_above_1e-6": int(((em - ed).abs() > 1e-6 * ed.abs()).sum()),
            "rel_dE": float(abs((evm[0] - evd[0]) / evd[0])),
            "max_rel_dW": float(((evm[1:] - evd[1:]).abs().max() / evd[1:].abs().max()))}


def rebuild_time(sim, reps=20):
    """Average wall time of one re-sort + list build (bin, build, overflow check)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.rebuild()
    torch.cuda.synchronize()
    return round((time.perf_counter() - t0) / reps * 1e6, 2)


def traversal_study(w, sim, reps=50):
    """Forces + energy/virial of the 500k workload (mixed) over the same pairs: the dense
    tiled list walked by two lanes per atom (the production kernel) against its CSR copy
    walked by 1, 2, 4, 8 and 16 lanes per atom, positions in AoSoA layouts (SoA, 8, 64),
    and the half list; plus the tiled -> CSR conversion."""
    import torch
    from paper_2109_09056_amd import ops
    nl = sim.nl
    off, csr = ops.list_to_csr(nl.nbr, nl.nnbr, nl.maxn)
    cap = csr.numel()
    wsc = torch.empty(ops.workspace_bytes(ops.OP_CSR, sim.n), dtype=torch.uint8, device=sim.device)
    wsf = torch.empty(ops.workspace_bytes(ops.OP_FORCES_CSR, sim.n), dtype=torch.uint8,
                      device=sim.device)
    F, e = torch.empty_like(sim.F), torch.empty_like(sim.e_atom)
    ev = torch.empty(7, dtype=torch.float64, device=sim.device)
    out = {"list_to_csr_us": round(event_time(lambda: ops.list_to_csr(
        nl.nbr, nl.nnbr, nl.maxn, cap=cap, offsets=off, csr=csr, ws=wsc), reps) * 1e3, 2)}
    # building the lists: tiled (the production build) and CSR straight from the cells
    wsb = torch.empty(ops.workspace_bytes(ops.OP_BUILD_CSR, sim.n), dtype=torch.uint8,
                      device=sim.device)
    off2 = torch.empty_like(off)
    csr2 = torch.empty(cap + 64, dtype=torch.int32, device=sim.device)
    out["build_tiled_us"] = round(event_time(lambda: ops.build_neighbors(
        w.box, sim.rlist, ops.FULL, sim.x, sim.cell_start, nl.maxn, nl.nbr, nl.nnbr,
        nl.max_count), reps) * 1e3, 2)
    out["build_csr_direct_us"] = round(event_time(lambda: ops.build_neighbors_csr(
        w.box, sim.rlist, ops.FULL, sim.x, sim.cell_start, cap=csr2.numel(), offsets=off2,
        csr=csr2, ws=wsb), reps) * 1e3, 2)
    out["tiled_team2_us"] = round(event_time(lambda: ops.compute_forces(
        w.box, ops.MIXED, ops.FULL, w.rc, sim.eps, sim.sigma, sim.x, sim.types, nl.nbr,
        nl.nnbr, nl.maxn, F=F, e_atom=e, ev=ev, ws=sim._ws[ops.OP_FORCES]), reps) * 1e3, 2)
    for team in (1, 2, 4, 8, 16):
        out[f"csr_team{team}_us"] = round(event_time(lambda: ops.compute_forces_csr(
            w.box, ops.MIXED, w.rc, sim.eps, sim.sigma, sim.x, sim.types, off, csr, team=team,
            F=F, e_atom=e, ev=ev, ws=wsf), reps) * 1e3, 2)
    # positions and forces in AoSoA(V) layouts (0: SoA) over the same tiled list, team 2
    for vlen in (0, 8, 64):
        xa = ops.aosoa_convert(sim.x, vlen, True)
        Fa = torch.empty_like(xa)
        out[f"aosoa_v{vlen}_us"] = round(event_time(lambda: ops.compute_forces_aosoa(
            w.box, ops.MIXED, w.rc, sim.eps, sim.sigma, xa, sim.types, nl.nbr, nl.nnbr,
            nl.maxn, vlen, F=Fa, e_atom=e, ev=ev, ws=sim._ws[ops.OP_FORCES]), reps) * 1e3, 2)
    # half list (each pair once, j-side sums through LDS tiles and atomics), same positions
    from paper_2109_09056_amd import md
    hl = md.NeighborList(sim.L, sim.rlist, ops.HALF, device=sim.device).build(sim.x,
                                                                            sim.cell_start)
    # with per-atom energies, and with E and W only
    for name, ea in (("half_list_us", e), ("half_list_no_eatom_us", None)):
        out[name] = round(event_time(lambda: ops.compute_forces(
            w.box, ops.MIXED, ops.HALF, w.rc, sim.eps, sim.sigma, sim.x, sim.types, hl.nbr,
            hl.nnbr, hl.maxn, F=F, e_atom=ea, ev=ev, ws=sim._ws[ops.OP_FORCES],
            atom_energy=ea is not None), reps) * 1e3, 2)
    out["tiled_team2_forces_only_us"] = round(event_time(lambda: ops.compute_forces(
        w.box, ops.MIXED, ops.FULL, w.rc, sim.eps, sim.sigma, sim.x, sim.types, nl.nbr,
        nl.nnbr, nl.maxn, F=F, want_energy=False, ws=sim._ws[ops.OP_FORCES]), reps) * 1e3, 2)
    out["half_list_forces_only_us"] = round(event_time(lambda: ops.compute_forces(
        w.box, ops.MIXED, ops.HALF, w.rc, sim.eps, sim.sigma, sim.x, sim.types, hl.nbr,
        hl.nnbr, hl.maxn, F=F, want_energy=False, ws=sim._ws[ops.OP_FORCES]), reps) * 1e3, 2)
    return out


def shard_share(dev, steps=200, warmup=40):
    """One GPU's share of the 500,000-atom box split 2x2x2 over eight GPUs: the owned
    brick (edge L/2) plus its ghost shell of thickness rlist, cut from the same input
    and placed in a periodic box with an empty gap >= rlist, so that no pair reaches
    across the boundary.  Ghost rows are computed too (no owned-only launch exists),
    and ghosts move without exchange: a timing of the kernels at the shard's shape."""
    import numpy as np
    import lj_inputs as li
    from paper_2109_09056_amd import ops
    w = li.WORKLOADS["lj500k"]
    s = li.make_system(w)
    L, rl = w.box, w.rlist
    xs = np.mod(s["x"] + rl, L)  # owned brick -> [rl, L/2 + rl) per dimension
    keep = np.all(xs < L / 2 + 2 * rl, axis=1)
    owned = np.all((xs >= rl) & (xs < L / 2 + rl), axis=1)
    edge = L / 2 + 3 * rl
    sub = {"x": np.ascontiguousarray(xs[keep]), "v": np.ascontiguousarray(s["v"][keep])}
    shard = types.SimpleNamespace(box=edge, rc=w.rc, skin=w.skin, dt=w.dt,
                                  rebuild_every=w.rebuild_every)
    t, _, fms, sim = md_run(shard, sub, ops.MIXED, steps, warmup, dev)
    n_all, n_own = int(keep.sum()), int(owned.sum())
    return {"owned_atoms": n_own, "ghost_atoms": n_all - n_own, "box_edge": round(float(edge[0]), 4),
            "steps": steps, "ms_per_step": round(t * 1e3 / steps, 5),
            "owned_atom_steps_per_s": round(n_own * steps / t, 1),
            "step_launch_us": round(statistics.mean(fms) * 1e3, 3)}


def sph_bench(dev, steps=300, warmup=50, reps=50):
    """SPH over the same bins and lists: the 512,000-particle lattice fluid (h 1.3,
    support 2.6, skin 0.4, rebuild every 10 steps), velocity-Verlet steps with the
    density and pressure passes, then each pass alone (HIP events).  Algorithmic
    bytes per particle: density 4 nbar + 4 (count) + 24 (x) + 8 (rho written);
    acceleration 32 + 32 (packing x, rho into records) + 4 nbar + 4 + 32 (own
    record) + 24 (a written); neighbour records are gathered through L1/L2."""
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import ops, sph
    w = li.SPH_WORKLOADS["sph512k"]
    sim = sph.SPHSim(w.box, w.h, mass=w.mass, c0=w.c0, rho0=w.rho0, skin=w.skin, dt=w.dt,
                     rebuild_every=w.rebuild_every, device=dev)
    sim.load(li.sph_positions(w), li.sph_velocities(w))
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    nl, n = sim.nl, sim.n
    nb = float(nl.nnbr.double().mean().item())
    td = event_time(lambda: ops.sph_density(sim.L, sim.h, sim.mass, sim.c0, sim.rho0, sim.x,
                                            nl.nbr, nl.nnbr, nl.maxn, rho=sim.rho), reps)
    ta = event_time(lambda: ops.sph_accel(sim.L, sim.h, sim.mass, sim.c0, sim.rho0, sim.x,
                                          sim.rho, nl.nbr, nl.nnbr, nl.maxn, acc=sim.acc,
                                          ws=sim.ws), reps)
    bd = n * (4.0 * nb + 36)
    ba = n * (4.0 * nb + 124)
    return {"natoms": n, "steps": steps, "value": round(n * steps / t, 1),
            "unit": "particle-steps/s", "ms_per_step": round(t * 1e3 / steps, 5),
            "mean_list_length": round(nb, 3), "rebuild_every": w.rebuild_every,
            "density_us": round(td * 1e3, 2), "accel_us": round(ta * 1e3, 2),
            "density_GBps": round(bd / (td * 1e-3) / 1e9, 1),
            "accel_GBps": round(ba / (ta * 1e-3) / 1e9, 1),
            "density_frac": round(bd / (td * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "accel_frac": round(ba / (ta * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def spme_bench(dev, reps=30):
    """Long-range electrostatics on the 500,000-atom liquid with unit charges (half +1,
    half -1): Ewald real space over the MD list (rc 2.5, alpha 1.2) and the SPME
    reciprocal part (order-4 B-splines, 128^3 grid), each timed alone with HIP events.
    Algorithmic bytes: real space per particle 4 nbar + 4 + 32 (own record) + 24 (F)
    + 56 (packing x, q into records); reciprocal: the real grid (8 B per point) is
    zeroed, spread into, read by the x transform, written by the inverse x transform
    and read by the gather (5 passes); the half grid (16 B per point, K0/2 + 1
    columns) is written by the x transform, read and written by the y transform
    each way and by the fused z / influence / inverse z pass, and read by the
    inverse x transform (8 passes); per particle 32 (x, q for spreading) + 32 (for
    the gather) + 48 (F read and written).  Interpolation points are not counted:
    the spread and gather revisit grid points in cache."""
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj500k"]
    x = torch.as_tensor(li.positions(w), dtype=torch.float64, device=dev)
    q = torch.as_tensor(li.charges(w), dtype=torch.float64, device=dev)
    L, K, order, alpha = w.box, li.ewald_grid(w.box), li.EWALD_ORDER, li.EWALD_ALPHA
    xs, _, _, ids, cs = ops.bin(L, w.rlist, x)
    qs = ops.gather_rows(ids, q)
    nl = md.NeighborList(L, w.rlist, ops.FULL, device=dev).build(xs, cs)
    F = torch.zeros_like(xs)
    E = torch.zeros(2, dtype=torch.float64, device=dev)
    wr = torch.empty(ops.workspace_bytes(ops.OP_EWALD_REAL, w.natoms), dtype=torch.uint8,
                     device=dev)
    wk = torch.empty(ops.workspace_bytes(ops.OP_SPME, w.natoms, ncells=K[0] * K[1] * K[2]),
                     dtype=torch.uint8, device=dev)
    real = lambda: ops.ewald_real(L, alpha, w.rc, xs, qs, nl.nbr, nl.nnbr, nl.maxn, F=F,
                                  e_total=E[:1], ws=wr)
    recip = lambda: ops.spme_recip(L, alpha, order, K, xs, qs, F=F, e_total=E[1:],
                                   accumulate=True, ws=wk)
    tr = event_time(real, reps)
    tk = event_time(recip, reps)
    tb = event_time(lambda: (real(), recip()), reps)
    n = w.natoms
    nb = float(nl.nnbr.double().mean().item())
    npts = K[0] * K[1] * K[2]
    br = n * (4.0 * nb + 116)
    hpts = (K[0] // 2 + 1) * K[1] * K[2]
    bk = 5 * 8 * npts + 8 * 16 * hpts + n * (32 + 32 + 48)
    return {"natoms": n, "grid": list(K), "order": order, "alpha": alpha, "rc": w.rc,
            "real_us": round(tr * 1e3, 2), "recip_us": round(tk * 1e3, 2),
            "both_us": round(tb * 1e3, 2),
            "value": round(n / (tb * 1e-3), 1), "unit": "atom-evaluations/s",
            "real_GBps": round(br / (tr * 1e-3) / 1e9, 1),
            "recip_GBps": round(bk / (tk * 1e-3) / 1e9, 1),
            "real_frac": round(br / (tr * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "recip_frac": round(bk / (tk * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "energy": [float(v) for v in E.cpu()]}


def charged_md_bench(dev, steps=100, warmup=20):
    """The 500,000-atom LJ liquid with unit charges (half +1, half -1) as CabanaMD
    composes it: per step LJ forces (mixed) + Ewald real space over the same list +
    SPME reciprocal part (128^3, order 4), then velocity Verlet; rebuild every 20."""
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import electrostatics as es, ops
    w = li.WORKLOADS["lj500k"]
    sim = es.ChargedLJSim(w.box, alpha=li.EWALD_ALPHA, order=li.EWALD_ORDER,
                          grid=li.ewald_grid(w.box), rc=w.rc, skin=w.skin, precision=ops.MIXED,
                          dt=w.dt, rebuild_every=w.rebuild_every, device=dev)
    sim.load(li.positions(w), li.velocities(w), li.charges(w))
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    th = sim.thermo()
    return {"natoms": w.natoms, "steps": steps, "value": round(w.natoms * steps / t, 1),
            "unit": "atom-steps/s", "ms_per_step": round(t * 1e3 / steps, 5),
            "grid": list(sim.grid), "order": sim.order, "temp": round(th["temp"], 4)}


def sph_cpu_oracle(rows=4096):
    """The SPH oracle (all pairs, FP64, OpenMP) on a sample of the 512,000-particle
    fluid: density and pressure acceleration of `rows` sampled particles (the
    acceleration with uniform densities as input: the same pair work)."""
    import numpy as np
    import lj_inputs as li
    import oracle
    w = li.SPH_WORKLOADS["sph512k"]
    x = li.sph_positions(w)
    sel = np.sort(np.random.default_rng(1).choice(w.natoms, rows, replace=False))
    t0 = time.perf_counter()
    oracle.sph_density(x, w.box, w.h, w.mass, sel=sel)
    oracle.sph_accel(x, w.box, w.h, w.mass, w.c0, w.rho0, np.full(w.natoms, w.rho0), sel=sel)
    dt = time.perf_counter() - t0
    return {"value": round(rows / dt, 3), "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"density + acceleration of {rows} sampled particles of "
                                        f"{w.natoms}, all pairs ({dt:.1f} s)"}


def spme_cpu_oracle(rows=256):
    """The SPME reference steps (NumPy spreading, FFTs, sampled gathers) and the Ewald
    direct-sum oracle on the same 500,000-charge input: the grid part once, the
    per-particle parts on `rows` sampled atoms, scaled to one whole evaluation."""
    import numpy as np
    import lj_inputs as li
    import oracle
    w = li.WORKLOADS["lj500k"]
    x, q = li.positions(w), li.charges(w)
    K = li.ewald_grid(w.box)
    sel = np.sort(np.random.default_rng(2).choice(w.natoms, rows, replace=False))
    t0 = time.perf_counter()
    oracle.spme_recip(x, q, w.box, li.EWALD_ALPHA, K, li.EWALD_ORDER, sel=sel[:1])
    t_grid = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.spme_recip(x, q, w.box, li.EWALD_ALPHA, K, li.EWALD_ORDER, sel=sel)
    t_gather = max(time.perf_counter() - t0 - t_grid, 0.0) / rows
    t0 = time.perf_counter()
    oracle.ewald_direct(x, q, w.box, li.EWALD_ALPHA, w.rc, sel=sel)
    t_direct = (time.perf_counter() - t0) / rows
    total = t_grid + w.natoms * (t_gather + t_direct)
    return {"value": round(w.natoms / total, 3), "unit": "atom-evaluations/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"grid part once ({t_grid:.1f} s), gathers and all-pairs direct sums of "
                      f"{rows} sampled atoms, scaled to {w.natoms} atoms ({total:.0f} s)"}


def cpu_model():
    """The host CPU's model name and logical CPU count, from /proc/cpuinfo."""
    names = []
    try:
        with open("/proc/cpuinfo") as f:
            names = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")]
    except OSError:
        pass
    return (names[0] if names else "unknown"), len(names)


def _oracle_rate(w, s, target_s, rng):
    """Oracle atom-evaluations/s on a sample sized to about target_s of CPU time."""
    import numpy as np
    import oracle
    n = w.natoms
    probe = np.sort(rng.choice(n, 128, replace=False))
    t0 = time.perf_counter()
    oracle.forces(s["x"], w.box, w.rc, sel=probe)
    per_atom = (time.perf_counter() - t0) / probe.size
    m = int(min(n, max(128, target_s / max(per_atom, 1e-9))))
    rows = np.sort(rng.choice(n, m, replace=False))
    t0 = time.perf_counter()
    oracle.forces(s["x"], w.box, w.rc, sel=rows)
    dt = time.perf_counter() - t0
    return m / dt, m, dt


def cpu_baseline(w, s, target_s):
    """The oracle (plain all-pairs FP64, OpenMP) on sampled atoms of the same input, with
    all the threads OpenMP gives it and with one thread."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    cores = oracle.num_threads()
    model, logical = cpu_model()
    v_all, m_all, dt_all = _oracle_rate(w, s, target_s, rng)
    oracle.set_threads(1)
    try:
        v_one, m_one, dt_one = _oracle_rate(w, s, target_s / 2, rng)
    finally:
        oracle.set_threads(cores)
    return {"value": round(v_all, 3), "unit": "atom-steps/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "logical_cpus": logical,
            "one_thread": {"value": round(v_one, 3), "cores": 1,
                           "sample": f"{m_one} sampled atoms ({dt_one:.1f} s)"},
            "sample": f"all-pairs FP64 forces+energy for {m_all} sampled atoms of the "
                      f"{w.natoms}-atom input (one force evaluation each, {dt_all:.1f} s, "
                      f"{cores} threads); the same on one thread beside it"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(the spatial decomposition across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch
    import lj_inputs as li
    from paper_2109_09056_amd import _lib, ops

    dev = torch.device("cuda:0")
    _lib.load()
    if args.sph_only:
        print(json.dumps({"sph_512k": sph_bench(dev)}), flush=True)
        return
    if args.spme_only:
        print(json.dumps({"spme_500k": spme_bench(dev)}), flush=True)
        return
    if args.half_only:
        print(json.dumps({"half_list": half_bench(dev)}), flush=True)
        return
    if args.charged_only:
        print(json.dumps({"charged_md_500k": charged_md_bench(dev)}), flush=True)
        return
    w = li.WORKLOADS[args.workload]
    s = li.make_system(w)
    n = w.natoms
    log(f"[bench] workload {w.name}: {n} atoms, box {w.box[0]:.4f}, mixed path, "
        f"{args.warmup} warmup + {args.steps} timed steps")
    t_mixed, tw_mixed, fms, sim = md_run(w, s, ops.MIXED, args.steps, args.warmup, dev)
    value = n * args.steps / t_mixed
    nbar = float(sim.nl.nnbr.double().mean().item())
    force_ms = statistics.mean(fms)
    # fused step kernel, per atom: list row 4*nbar + count 4 + x 24 + F 24 + e 8
    # + v read/write 48 + next positions 24 (neighbor positions are cache hits)
    force_bytes = n * (4.0 * nbar + 4 + 24 + 24 + 8 + 48 + 24)
    achieved = force_bytes / (force_ms * 1e-3) / 1e9
    th = sim.thermo()
    log(f"[bench] mixed: {t_mixed * 1e3 / args.steps:.4f} ms/step, {value:.4e} atom-steps/s, "
        f"fused step launch {force_ms * 1e3:.1f} us, mean list {nbar:.2f}, T {th['temp']:.4f}")
    line = {
        "metric": "atom-steps/s LJ force+neighbor, mixed vs FP64, 500k atoms; bwd/fwd time ratio",
        "value": round(value, 1), "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_mixed * 1e3 / args.steps, 5),
        "timing": {"windows": len(tw_mixed), "statistic": "median window",
                   "window_ms_per_step": [round(t * 1e3 / args.steps, 5) for t in tw_mixed]},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed: f64 displacement/cutoff/accumulation, f32 pair math",
        "data": "synthetic (seeded jittered fcc LJ liquid, Maxwell velocities)",
        "config": {"workload": f"{w.name}: fcc {w.cells}^3 cells, {n} atoms, rho 0.8442, "
                               f"T 1.44, rc 2.5, skin 0.3, dt 0.005, rebuild every 20, full list",
                   "natoms": n, "precision": "mixed", "list": "full",
                   "mean_list_length": round(nbar, 3), "maxn": sim.nl.maxn},
        "roofline": {"bound": "hbm",
                     "kernel": "k_force_full<mixed, step, team 2> fused force+integration "
                               "(block 0 also sums the previous step's energy/virial/KE rows)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(FORCE_TRAFFIC) if FORCE_TRAFFIC else None,
                     "valu_busy": FORCE_VALU_BUSY, "texture_addr_busy": FORCE_TA_BUSY,
                     "counters_from": FORCE_COUNTERS_FROM,
                     "bytes_per_launch": round(force_bytes), "avg_launch_us": round(force_ms * 1e3, 3),
                     "launch_timing": f"HIP events around {EVENT_SPAN} consecutive chained launches "
                                      f"per timed window, on the launch stream"},
    }
    checked, dangerous, dmax = sim.displacement_report()
    line["stale_list_check"] = {
        "rebuilds_checked": checked, "dangerous_rebuilds": dangerous,
        "max_displacement": round(dmax, 4), "skin_half": 0.5 * w.skin,
        "note": "a window is dangerous when some atom moved more than skin/2 since the list "
                "was built (pairs inside rc may then be missing from it)"}
    if not args.no_extras:
        t64, tw64, f64ms, sim64 = md_run(w, s, ops.FP64, args.steps, args.warmup, dev)
        line["fp64"] = {"value": round(n * args.steps / t64, 1), "unit": "atom-steps/s",
                        "ms_per_step": round(t64 * 1e3 / args.steps, 5),
                        "window_ms_per_step": [round(t * 1e3 / args.steps, 5) for t in tw64],
                        "step_launch_us": round(statistics.mean(f64ms) * 1e3, 3),
                        "mixed_over_fp64": round(t64 / t_mixed, 4),
                        "mixed_over_fp64_step_kernel": round(statistics.mean(f64ms) / force_ms, 4)}
        log(f"[bench] fp64: {t64 * 1e3 / args.steps:.4f} ms/step")
        line["fp64"]["mixed_error_vs_fp64"] = mixed_error(w, sim)
        line["traversal_study"] = traversal_study(w, sim)
        log(f"[bench] traversal study: {line['traversal_study']}")
        line["rebuild_us"] = rebuild_time(sim)
        line["lj32k_matrix"] = config1_matrix(dev)
        log(f"[bench] 32k matrix: {line['lj32k_matrix']}")
        line["bwd_fwd"] = {"force_matching_32k": bwd_fwd_forcematching(dev),
                           "trajectory_256k": bwd_fwd_trajectory(dev)}
        w2 = li.WORKLOADS["lj2m"]
        s2 = li.make_system(w2)
        t2, _, f2ms, sim2 = md_run(w2, s2, ops.MIXED, w2.steps, 40, dev)
        nb2 = float(sim2.nl.nnbr.double().mean().item())
        line["scale_2m"] = {"natoms": w2.natoms, "steps": w2.steps,
                            "value": round(w2.natoms * w2.steps / t2, 1), "unit": "atom-steps/s",
                            "ms_per_step": round(t2 * 1e3 / w2.steps, 5),
                            "step_launch_us": round(statistics.mean(f2ms) * 1e3, 3),
                            "achieved_GBps": round(w2.natoms * (4.0 * nb2 + 132) /
                                                   (statistics.mean(f2ms) * 1e-3) / 1e9, 2)}
        log(f"[bench] 2M atoms: {t2 * 1e3 / w2.steps:.4f} ms/step")
        del sim2, s2
        line["sph_512k"] = sph_bench(dev)
        if not args.no_cpu_baseline:
            line["sph_512k"]["cpu_oracle"] = sph_cpu_oracle()
        log(f"[bench] SPH 512k: {line['sph_512k']}")
        line["spme_500k"] = spme_bench(dev)
        if not args.no_cpu_baseline:
            line["spme_500k"]["cpu_oracle"] = spme_cpu_oracle()
        log(f"[bench] SPME 500k: {line['spme_500k']}")
        line["charged_md_500k"] = charged_md_bench(dev)
        log(f"[bench] charged LJ + SPME MD 500k: {line['charged_md_500k']}")
        line["shard_share_2x2x2"] = shard_share(dev)
        log(f"[bench] one 2x2x2 shard: {line['shard_share_2x2x2']}")
        log(f"[bench] bwd/fwd: {json.dumps(line['bwd_fwd'])}")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample")
        line["cpu_baseline"] = cpu_baseline(w, s, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    _ = np


if __name__ == "__main__":
    main()
