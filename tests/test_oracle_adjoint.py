"""Pins of the oracle's force adjoint and trajectory adjoint.

Central finite differences of the force-matching loss with the pair set
checked unchanged, the linearity of F in eps (one-type closed form), the
scaling identity that ties the sigma gradient to the position gradient, a
dot-product test, and finite differences through a short trajectory.
"""
import numpy as np
import pytest

import lj_inputs as li


def system(index=3, cells=4, ntypes=2):
    tw = li.Workload("t", index, cells=cells, ntypes=ntypes)
    x = li.positions(tw)
    types = li.types(tw) if ntypes > 1 else None
    eps, sig = li.params(tw)
    return tw, x, types, eps, sig


def loss_and_g(orc, x, L, rc, eps, sig, types, lst, Ft):
    F, _, _ = orc.forces_list(x, L, rc, lst[0], lst[1], eps, sig, types)
    return ((F - Ft) ** 2).sum(), 2.0 * (F - Ft)


def pairs_within(orc, x, L, rc):
    return orc.neighbor_lists(x, L, rc)[1]


def test_force_matching_fd(orc):
    tw, x, types, eps, sig = system()
    L, rc = tw.box, tw.rc
    lst = orc.neighbor_lists(x, L, tw.rlist)
    et, st = li.perturbed_params(tw)
    Ft, _, _ = orc.forces_list(x, L, rc, lst[0], lst[1], et, st, types)
    loss, g = loss_and_g(orc, x, L, rc, eps, sig, types, lst, Ft)
    gx, ge, gs = orc.force_vjp(x, L, rc, g, eps, sig, types, *lst)
    # all-pairs mode gives the same VJP
    gx2, ge2, gs2 = orc.force_vjp(x, L, rc, g, eps, sig, types)
    np.testing.assert_allclose(gx2, gx, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(ge2, ge, rtol=1e-12)
    rng = np.random.default_rng(4)
    base = pairs_within(orc, x, L, rc)
    h = 1e-6
    for _ in range(16):
        i, k = rng.integers(0, x.shape[0]), rng.integers(0, 3)
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        assert np.array_equal(pairs_within(orc, xp, L, rc), base)
        assert np.array_equal(pairs_within(orc, xm, L, rc), base)
        fd = (loss_and_g(orc, xp, L, rc, eps, sig, types, lst, Ft)[0]
              - loss_and_g(orc, xm, L, rc, eps, sig, types, lst, Ft)[0]) / (2 * h)
        assert gx[i, k] == pytest.approx(fd, rel=1e-6, abs=1e-5)
    hp = 1e-7
    for p in range(eps.size):
        for arr, grad in ((eps, ge), (sig, gs)):
            ap, am = arr.copy(), arr.copy()
            ap[p] += hp
            am[p] -= hp
            args = (lambda a: (a, sig)) if arr is eps else (lambda a: (eps, a))
            lp = loss_and_g(orc, x, L, rc, *args(ap), types, lst, Ft)[0]
            lm = loss_and_g(orc, x, L, rc, *args(am), types, lst, Ft)[0]
            assert grad[p] == pytest.approx((lp - lm) / (2 * hp), rel=1e-6)


def test_one_type_eps_closed_form(orc):
    # F is linear in eps, so dL/deps = (1/eps) sum_i g_i . F_i
    tw, x, _, _, _ = system(index=5, ntypes=1)
    eps, sig = np.array([1.3]), np.array([0.97])
    F, _, _, _ = orc.forces(x, tw.box, tw.rc, eps, sig)
    g = np.random.default_rng(2).normal(size=F.shape)
    _, ge, _ = orc.force_vjp(x, tw.box, tw.rc, g, eps, sig)
    assert ge[0] == pytest.approx((g * F).sum() / eps[0], rel=1e-12)


def test_sigma_scaling_identity(orc):
    # For an isolated cluster F(lam x; eps, lam sigma) = F(x; eps, sigma)/lam with the
    # pair set fixed; at lam = 1:  sigma dL/dsigma = -sum g.F - sum_k x_k . gx_k
    rng = np.random.default_rng(8)
    grid = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = 1.12 * grid + rng.uniform(-0.05, 0.05, size=grid.shape) + 30.0
    L = np.full(3, 100.0)
    eps, sig = np.array([0.9]), np.array([1.04])
    F, _, _, _ = orc.forces(x, L, 2.5, eps, sig)
    g = rng.normal(size=F.shape)
    gx, _, gs = orc.force_vjp(x, L, 2.5, g, eps, sig)
    lhs = sig[0] * gs[0]
    rhs = -(g * F).sum() - (x * gx).sum()
    assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-9)


def test_dot_product(orc):
    # <J v, w> = <v, J^T w>, J = dF/dx taken by central differences along v
    tw, x, types, eps, sig = system(index=6)
    L, rc = tw.box, tw.rc
    rng = np.random.default_rng(3)
    v = rng.normal(size=x.shape)
    wv = rng.normal(size=x.shape)
    h = 1e-7
    lst = orc.neighbor_lists(x, L, tw.rlist)
    Fp = orc.forces_list(x + h * v, L, rc, *lst, eps, sig, types)[0]
    Fm = orc.forces_list(x - h * v, L, rc, *lst, eps, sig, types)[0]
    Jv = (Fp - Fm) / (2 * h)
    gx, _, _ = orc.force_vjp(x, L, rc, wv, eps, sig, types, *lst)
    assert (Jv * wv).sum() == pytest.approx((v * gx).sum(), rel=1e-6)


def traj_loss(orc, x0, v0, L, rc, rlist, dt, steps, eps, sig, types, xref, mass=1.0):
    xs, vT, xT, lst = orc.trajectory(x0, v0, L, rc, rlist, dt, steps, eps, sig, types, mass=mass)
    d = xT - xref
    return 0.5 * (d * d).sum(), xs, d, lst


@pytest.mark.parametrize("mass", [1.0, 2.0])
def test_trajectory_adjoint_fd(orc, mass):
    """FD through 20 velocity-Verlet steps; mass 2 fixes where 1/m enters the adjoint."""
    tw, x0, types, eps, sig = system(index=4)
    L, rc, rl, dt, T = tw.box, tw.rc, tw.rlist, tw.dt, 20
    v0 = li.velocities(tw)
    et, st = li.perturbed_params(tw)
    _, _, xref, _ = orc.trajectory(x0, v0, L, rc, rl, dt, T, et, st, types, mass=mass)
    loss, xs, xbarT, lst = traj_loss(orc, x0, v0, L, rc, rl, dt, T, eps, sig, types, xref, mass)
    gx0, gv0, ge, gs = orc.trajectory_adjoint(xs, L, rc, dt, eps, sig, xbarT,
                                              np.zeros_like(xbarT), types, lst, mass=mass)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(6):
        i, k = rng.integers(0, x0.shape[0]), rng.integers(0, 3)
        for arr, grad in ((x0, gx0), (v0, gv0)):
            ap, am = arr.copy(), arr.copy()
            ap[i, k] += h
            am[i, k] -= h
            if arr is x0:
                lp = traj_loss(orc, ap, v0, L, rc, rl, dt, T, eps, sig, types, xref, mass)[0]
                lm = traj_loss(orc, am, v0, L, rc, rl, dt, T, eps, sig, types, xref, mass)[0]
            else:
                lp = traj_loss(orc, x0, ap, L, rc, rl, dt, T, eps, sig, types, xref, mass)[0]
                lm = traj_loss(orc, x0, am, L, rc, rl, dt, T, eps, sig, types, xref, mass)[0]
            assert grad[i, k] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9)
    hp = 1e-7
    for p in range(eps.size):
        for which, grad in ((0, ge), (1, gs)):
            pp = [eps.copy(), sig.copy()]
            pm = [eps.copy(), sig.copy()]
            pp[which][p] += hp
            pm[which][p] -= hp
            lp = traj_loss(orc, x0, v0, L, rc, rl, dt, T, *pp, types, xref, mass)[0]
            lm = traj_loss(orc, x0, v0, L, rc, rl, dt, T, *pm, types, xref, mass)[0]
            assert grad[p] == pytest.approx((lp - lm) / (2 * hp), rel=1e-5)
