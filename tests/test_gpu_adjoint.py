"""Adjoint parity: force VJP vs the oracle, autograd, finite differences, and
checkpointed backprop through a short trajectory.  The oracle only ever sees
generator inputs in the caller's atom order; GPU results are mapped back to
that order through the ids the sort returns."""
import numpy as np
import pytest

import lj_inputs as li
from helpers import gpu_device, max_rel_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def T(a, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


@pytest.fixture(scope="module")
def fm(dev, orc):
    """32,000 atoms, two types: force-matching loss against perturbed-parameter targets."""
    from paper_2109_09056_amd import autograd, ops
    w = li.WORKLOADS["lj32k_fm"]
    x, ty = li.positions(w), li.types(w)
    eps, sig = li.params(w)
    et, st = li.perturbed_params(w)
    lst = orc.neighbor_lists(x, w.box, w.rlist)
    Ft, _, _ = orc.forces_list(x, w.box, w.rc, *lst, et, st, ty)
    fc = autograd.ForceContext(w.box, x, ty, rc=w.rc, skin=w.skin, precision=ops.FP64, device=dev)
    return dict(w=w, fc=fc, x=x, ty=ty, eps=eps, sig=sig, Ft=Ft, lst=lst)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_vjp_vs_oracle(dev, orc, fm, prec):
    from paper_2109_09056_amd import ops
    w, fc = fm["w"], fm["fc"]
    g = np.random.default_rng(7).normal(size=fm["x"].shape)
    gxo, geo, gso = orc.force_vjp(fm["x"], w.box, w.rc, g, fm["eps"], fm["sig"], fm["ty"],
                                  *fm["lst"])
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    gx, ge, gs = ops.force_backward(w.box, P, w.rc, T(fm["eps"], dev), T(fm["sig"], dev), fc.x,
                                    fc.types, fc.nl.nbr, fc.nl.nnbr, fc.nl.maxn,
                                    fc.sorted_rows(g))
    gx = fc.caller_rows(gx).cpu().numpy()
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    ex = max_rel_vec(gx, gxo)
    ee = np.abs(ge - geo).max() / np.abs(geo).max()
    es = np.abs(gs - gso).max() / np.abs(gso).max()
    print(f"[{prec}] vjp rel err x {ex:.2e} eps {ee:.2e} sigma {es:.2e}")
    tol = 1e-12 if prec == "fp64" else 1e-4
    assert ex <= tol and ee <= tol and es <= tol


@pytest.fixture(scope="module")
def vjp70k(orc):
    """70,304 atoms (fcc 26^3 cells): above the 65,536-atom bound where the VJP kernel
    leaves four lanes per atom for two, two types 50/50, and the oracle's full list."""
    w = li.Workload("lj70k_fm", 7, cells=26, ntypes=2)
    x, ty = li.positions(w), li.types(w)
    eps, sig = li.params(w)
    lst = orc.neighbor_lists(x, w.box, w.rlist)
    g = np.random.default_rng(13).normal(size=x.shape)
    return dict(w=w, x=x, ty=ty, eps=eps, sig=sig, lst=lst, g=g)


@pytest.mark.parametrize("ntypes", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_vjp_two_lane_path_vs_oracle(dev, orc, vjp70k, ntypes, prec):
    """The VJP kernel's two-lanes-per-atom path (n > 65,536, as at 256,000 atoms), with one
    type and with two, against the oracle element by element: gx per atom, geps, gsigma."""
    from paper_2109_09056_amd import autograd, ops
    d = vjp70k
    w, x = d["w"], d["x"]
    assert x.shape[0] > 65536
    if ntypes == 1:
        ty, eps, sig = np.zeros(x.shape[0], dtype=np.int32), d["eps"][:1], d["sig"][:1]
    else:
        ty, eps, sig = d["ty"], d["eps"], d["sig"]
    gxo, geo, gso = orc.force_vjp(x, w.box, w.rc, d["g"], eps, sig, ty, *d["lst"])
    fc = autograd.ForceContext(w.box, x, ty, rc=w.rc, skin=w.skin, device=dev)
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    gx, ge, gs = ops.force_backward(w.box, P, w.rc, T(eps, dev), T(sig, dev), fc.x, fc.types,
                                    fc.nl.nbr, fc.nl.nnbr, fc.nl.maxn, fc.sorted_rows(d["g"]))
    gx = fc.caller_rows(gx).cpu().numpy()
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    ex = max_rel_vec(gx, gxo)
    ee = np.abs(ge - geo).max() / np.abs(geo).max()
    es = np.abs(gs - gso).max() / np.abs(gso).max()
    print(f"[{prec}, {ntypes} type(s), n {x.shape[0]}] vjp rel err x {ex:.2e} eps {ee:.2e} "
          f"sigma {es:.2e}")
    tol = 1e-12 if prec == "fp64" else 1e-4
    assert ex <= tol and ee <= tol and es <= tol


def test_force_vjp_three_types(dev, orc):
    """General type count (per-lane LDS accumulators): 256 atoms, three types."""
    from paper_2109_09056_amd import autograd, ops
    w = li.WORKLOADS["lj256"]
    x = li.positions(w)
    ty = (np.arange(w.natoms) % 3).astype(np.int32)
    eps = np.array([1.0, 0.9, 1.1, 1.2, 0.8, 1.05])
    sig = np.array([1.0, 0.95, 1.02, 1.05, 0.92, 0.97])
    g = np.random.default_rng(9).normal(size=x.shape)
    lst = orc.neighbor_lists(x, w.box, w.rlist)
    gxo, geo, gso = orc.force_vjp(x, w.box, w.rc, g, eps, sig, ty, *lst)
    fc = autograd.ForceContext(w.box, x, ty, rc=w.rc, skin=w.skin, device=dev)
    for prec, tol in ((ops.FP64, 1e-12), (ops.MIXED, 1e-4)):
        gx, ge, gs = ops.force_backward(w.box, prec, w.rc, T(eps, dev), T(sig, dev), fc.x,
                                        fc.types, fc.nl.nbr, fc.nl.nnbr, fc.nl.maxn,
                                        fc.sorted_rows(g))
        assert max_rel_vec(fc.caller_rows(gx).cpu().numpy(), gxo) <= tol
        assert np.abs(ge.cpu().numpy() - geo).max() <= tol * np.abs(geo).max()
        assert np.abs(gs.cpu().numpy() - gso).max() <= tol * np.abs(gso).max()


def test_force_vjp_accumulate_and_deterministic(dev, fm):
    import torch
    from paper_2109_09056_amd import ops
    w, fc = fm["w"], fm["fc"]
    g = fc.sorted_rows(np.random.default_rng(3).normal(size=fm["x"].shape))
    args = (w.box, ops.FP64, w.rc, T(fm["eps"], dev), T(fm["sig"], dev), fc.x, fc.types,
            fc.nl.nbr, fc.nl.nnbr, fc.nl.maxn, g)
    a = [t.clone() for t in ops.force_backward(*args)]
    b = ops.force_backward(*args)
    for p, q in zip(a, b):
        assert torch.equal(p, q)
    c = ops.force_backward(*args, gx=b[0].clone(), geps=b[1].clone(), gsigma=b[2].clone(),
                           accumulate=True)
    for p, q in zip(a, c):
        assert torch.allclose(2 * p, q, rtol=1e-14, atol=0)


def test_autograd_force_matching_loss(dev, orc, fm):
    """loss = sum |F - F_target|^2 through LJForce; gradients vs the oracle and FD."""
    import torch
    from paper_2109_09056_amd import autograd
    w, fc = fm["w"], fm["fc"]
    x = fc.x.clone().requires_grad_(True)
    eps = T(fm["eps"], dev).requires_grad_(True)
    sig = T(fm["sig"], dev).requires_grad_(True)
    Ft = fc.sorted_rows(fm["Ft"])
    F = autograd.lj_forces(x, eps, sig, fc)
    loss = ((F - Ft) ** 2).sum()
    loss.backward()
    Fo, _, _ = orc.forces_list(fm["x"], w.box, w.rc, *fm["lst"], fm["eps"], fm["sig"], fm["ty"])
    gxo, geo, gso = orc.force_vjp(fm["x"], w.box, w.rc, 2.0 * (Fo - fm["Ft"]), fm["eps"],
                                  fm["sig"], fm["ty"], *fm["lst"])
    assert float(loss.item()) == pytest.approx(((Fo - fm["Ft"]) ** 2).sum(), rel=1e-11)
    assert max_rel_vec(fc.caller_rows(x.grad).cpu().numpy(), gxo) <= 1e-11
    np.testing.assert_allclose(eps.grad.cpu().numpy(), geo, rtol=1e-11)
    np.testing.assert_allclose(sig.grad.cpu().numpy(), gso, rtol=1e-11)

    def L_of(xx, ee, ss):  # central finite differences of the GPU loss itself (FP64 path)
        with torch.no_grad():
            return float(((autograd.lj_forces(xx, ee, ss, fc) - Ft) ** 2).sum().item())
    h = 1e-6
    rng = np.random.default_rng(5)
    for _ in range(6):
        i, k = int(rng.integers(0, x.shape[0])), int(rng.integers(0, 3))
        xp, xm = x.detach().clone(), x.detach().clone()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (L_of(xp, eps.detach(), sig.detach()) - L_of(xm, eps.detach(), sig.detach())) / (2 * h)
        assert x.grad[i, k].item() == pytest.approx(fd, rel=1e-5, abs=1e-4)
    hp = 1e-7
    for p in range(3):
        for which in (0, 1):
            up = [eps.detach().clone(), sig.detach().clone()]
            dn = [eps.detach().clone(), sig.detach().clone()]
            up[which][p] += hp
            dn[which][p] -= hp
            fd = (L_of(x.detach(), *up) - L_of(x.detach(), *dn)) / (2 * hp)
            grad = (eps.grad if which == 0 else sig.grad)[p].item()
            assert grad == pytest.approx(fd, rel=1e-5)


@pytest.mark.parametrize("mass", [1.0, 2.0])
def test_trajectory_backprop_vs_oracle_small(dev, orc, mass):
    """256 atoms, two types, 20 steps, checkpoints every 5, FP64: GPU gradient vs the
    oracle's (uncheckpointed, unmerged) discrete adjoint; mass 2 checks the 1/m of the
    kicks in the reverse pass."""
    from paper_2109_09056_amd import ops, trajectory
    w = li.Workload("traj_small", 4, cells=4, ntypes=2, steps=20, checkpoint_every=5)
    x0, v0, ty = li.positions(w), li.velocities(w), li.types(w)
    eps, sig = li.params(w)
    et, st = li.perturbed_params(w)
    _, _, xref, _ = orc.trajectory(x0, v0, w.box, w.rc, w.rlist, w.dt, 20, et, st, ty, mass=mass)
    r = trajectory.backprop_trajectory(w.box, x0, v0, ty, eps, sig, xref, steps=20,
                                       checkpoint_every=5, mass=mass, precision=ops.FP64,
                                       device=dev)
    assert r.recompute_bitwise
    xs, vT, xT_unw, lst = orc.trajectory(x0, v0, w.box, w.rc, w.rlist, w.dt, 20, eps, sig, ty,
                                         mass=mass)
    d = xT_unw - xref
    gx0, gv0, ge, gs = orc.trajectory_adjoint(xs, w.box, w.rc, w.dt, eps, sig, d,
                                              np.zeros_like(d), ty, lst, mass=mass)
    assert float(r.loss.item()) == pytest.approx(0.5 * (d * d).sum(), rel=1e-9)
    assert max_rel_vec(r.gx0.cpu().numpy(), gx0) <= 1e-9
    assert max_rel_vec(r.gv0.cpu().numpy(), gv0) <= 1e-9
    np.testing.assert_allclose(r.geps.cpu().numpy(), ge, rtol=1e-9)
    np.testing.assert_allclose(r.gsigma.cpu().numpy(), gs, rtol=1e-9)


@pytest.fixture(scope="module")
def traj256k(orc):
    """The 256,000-atom two-type trajectory workload and the oracle's side of it: the
    reference end positions from 20 steps at the perturbed parameters, the 20 steps at
    the model parameters (positions of every step, pairs inside rc per step) on the
    oracle's own list built at step 0, and the oracle's discrete adjoint."""
    w = li.WORKLOADS["lj256k_traj"]
    x0, v0, ty = li.positions(w), li.velocities(w), li.types(w)
    eps, sig = li.params(w)
    et, st = li.perturbed_params(w)
    _, _, xref, lst = orc.trajectory(x0, v0, w.box, w.rc, w.rlist, w.dt, w.steps, et, st, ty)
    pairs = []
    xs, _, xT, _ = orc.trajectory(x0, v0, w.box, w.rc, w.rlist, w.dt, w.steps, eps, sig, ty,
                                  lst=lst, pairs=pairs)
    d = xT - xref
    adj = orc.trajectory_adjoint(xs, w.box, w.rc, w.dt, eps, sig, d, np.zeros_like(d), ty, lst)
    del xs
    return dict(w=w, x0=x0, v0=v0, ty=ty, eps=eps, sig=sig, xref=xref, lst=lst, pairs=pairs,
                loss=0.5 * (d * d).sum(), adj=adj)


@pytest.mark.timeout(900)
def test_trajectory_backprop_256k_vs_oracle(dev, orc, traj256k):
    """256,000 atoms, two types, 20 steps, checkpoints every 5.  FP64: the checkpointed GPU
    gradient against the oracle's discrete adjoint (x0, v0 per atom; every eps and sigma
    entry), and central differences of the GPU loss on coordinates of x0 and on all six
    parameters, each with the set of pairs inside rc checked unchanged at +-h along the
    whole trajectory (the oracle's per-step pair counts).  Mixed: its gradient's error
    against the oracle's."""
    from paper_2109_09056_amd import ops, trajectory
    t = traj256k
    w, x0, v0, ty, eps, sig, xref = (t[k] for k in ("w", "x0", "v0", "ty", "eps", "sig", "xref"))
    gx0, gv0, ge, gs = t["adj"]
    r64 = trajectory.backprop_trajectory(w.box, x0, v0, ty, eps, sig, xref, steps=w.steps,
                                         checkpoint_every=w.checkpoint_every,
                                         precision=ops.FP64, device=dev)
    assert r64.recompute_bitwise
    assert float(r64.loss.item()) == pytest.approx(t["loss"], rel=1e-9)
    ex, ev_ = max_rel_vec(r64.gx0.cpu().numpy(), gx0), max_rel_vec(r64.gv0.cpu().numpy(), gv0)
    ee = np.abs(r64.geps.cpu().numpy() - ge) / np.abs(ge)
    es = np.abs(r64.gsigma.cpu().numpy() - gs) / np.abs(gs)
    print(f"256k FP64 gradient vs oracle: x0 {ex:.2e} v0 {ev_:.2e} eps {ee.max():.2e} "
          f"sigma {es.max():.2e}")
    assert ex <= 1e-9 and ev_ <= 1e-9 and ee.max() <= 1e-9 and es.max() <= 1e-9

    def end_diff(x, e, s):
        xt = trajectory.run_trajectory(w.box, x, v0, ty, e, s, steps=w.steps, device=dev)
        d = xt.cpu().numpy() - xref
        return d - w.box * np.round(d / w.box)

    def central(a, b, h):
        """(loss(b) - loss(a)) / 2h from the two end-point differences, formed as
        1/2 sum (d_b - d_a)(d_b + d_a): the terms of atoms the perturbation never
        reached vanish exactly instead of cancelling in a sum of 768,000 squares."""
        return 0.5 * ((b - a) * (b + a)).sum() / (2 * h)

    def same_pairs(x, e, s):
        got = []
        orc.trajectory(x, v0, w.box, w.rc, w.rlist, w.dt, w.steps, e, s, ty, lst=t["lst"],
                       pairs=got)
        return got == t["pairs"]

    gx = r64.gx0.cpu().numpy()
    rng = np.random.default_rng(11)
    h = 1e-6
    # a perturbation that moves a pair across rc somewhere along the trajectory makes the
    # loss jump: such a coordinate is replaced by another one, such a parameter step by
    # a smaller one (the adjoint holds the pair set fixed)
    done = tried = 0
    while done < 3:
        tried += 1
        assert tried <= 8, "every sampled coordinate moved a pair across rc"
        i, k = int(rng.integers(0, w.natoms)), int(rng.integers(0, 3))
        xp, xm = x0.copy(), x0.copy()
        xp[i, k] += h
        xm[i, k] -= h
        if not (same_pairs(xp, eps, sig) and same_pairs(xm, eps, sig)):
            print(f"x0[{i},{k}]: a pair crosses rc at +-h, resampled")
            continue
        fd = central(end_diff(xm, eps, sig), end_diff(xp, eps, sig), h)
        print(f"x0[{i},{k}]: grad {gx[i, k]:.10e} fd {fd:.10e}")
        assert abs(gx[i, k] - fd) <= 1e-5 * abs(fd) + 1e-9
        done += 1
    for which, base, grad in ((0, eps, r64.geps), (1, sig, r64.gsigma)):
        for p in range(base.size):
            for hp in (1e-7, 2e-8, 5e-9):
                up, dn = [eps.copy(), sig.copy()], [eps.copy(), sig.copy()]
                up[which][p] += hp
                dn[which][p] -= hp
                if same_pairs(x0, *up) and same_pairs(x0, *dn):
                    break
                print(f"{'eps' if which == 0 else 'sigma'}[{p}]: a pair crosses rc at "
                      f"+-{hp:g}, smaller step")
            else:
                pytest.fail(f"parameter {which},{p}: pairs cross rc at every step tried")
            fd = central(end_diff(x0, *dn), end_diff(x0, *up), hp)
            print(f"{'eps' if which == 0 else 'sigma'}[{p}]: grad {grad[p].item():.10e} "
                  f"fd {fd:.10e}")
            assert grad[p].item() == pytest.approx(fd, rel=1e-5)
    rm = trajectory.backprop_trajectory(w.box, x0, v0, ty, eps, sig, xref, steps=w.steps,
                                        checkpoint_every=w.checkpoint_every,
                                        precision=ops.MIXED, device=dev)
    assert rm.recompute_bitwise
    rel = np.linalg.norm(rm.gx0.cpu().numpy() - gx0) / np.linalg.norm(gx0)
    rel_p = max(np.abs(rm.geps.cpu().numpy() - ge).max() / np.abs(ge).max(),
                np.abs(rm.gsigma.cpu().numpy() - gs).max() / np.abs(gs).max())
    print(f"mixed trajectory gradient vs oracle: x0 rel L2 {rel:.3e}, parameters {rel_p:.3e}")
    assert rel < 1e-3 and rel_p < 1e-3
