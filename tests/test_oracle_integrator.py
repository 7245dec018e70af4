"""Pins of the oracle's velocity-Verlet integrator.

Free flight is exact up to rounding, the scheme is time reversible and
conserves momentum, its energy error shrinks as dt^2, and a short NVE run of
the 256-atom liquid keeps the (cutoff-shifted) total energy bounded.
"""
import numpy as np
import pytest

import lj_inputs as li


def test_free_flight(orc):
    L = np.array([10.0, 12.0, 14.0])
    rng = np.random.default_rng(0)
    x0 = rng.uniform(0, 1, size=(5, 3)) * L
    v = rng.normal(size=(5, 3)) * 3.0
    x = x0.copy()
    vv = v.copy()
    F = np.zeros_like(x)
    dt = 0.005
    img = np.zeros((5, 3), dtype=np.int32)
    for _ in range(400):
        orc.kick_drift(x, vv, F, dt, L, img=img)
        orc.kick(vv, F, dt)
        assert np.all(x >= 0) and np.all(x < L)
    np.testing.assert_array_equal(vv, v)
    np.testing.assert_allclose(x + img * L, x0 + 400 * dt * v, rtol=0, atol=1e-11)


def dimer(r=1.3):
    L = np.full(3, 30.0)
    x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    v = np.array([[0.3, 0.1, 0.0], [-0.3, -0.1, 0.0]])
    return x, v, L


def test_dimer_energy_and_momentum(orc):
    x, v, L = dimer()
    x, v, F, thermo, _, _ = orc.run_nve(x, v, L, 2.5, 2.8, 0.002, 2000, mode="allpairs")
    E = np.array([pe + ke for _, pe, ke in thermo])
    # bounded fluctuation (O(dt^2)) and no secular drift
    assert np.abs(E - E[0]).max() < 1e-4
    half = E.size // 2
    assert abs(E[half:].mean() - E[:half].mean()) < 1e-5
    assert np.abs(v.sum(axis=0)).max() < 1e-13


def test_time_reversibility(orc):
    w = li.WORKLOADS["lj256"]
    s = li.make_system(w)
    x1, v1, _, _, _, _ = orc.run_nve(s["x"], s["v"], w.box, w.rc, w.rlist, w.dt, 60,
                                    mode="allpairs")
    x2, v2, _, _, _, _ = orc.run_nve(x1, -v1, w.box, w.rc, w.rlist, w.dt, 60, mode="allpairs")
    d = x2 - s["x"]
    d -= w.box * np.round(d / w.box)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-v2, s["v"], atol=1e-9)


def test_energy_error_scales_as_dt2(orc):
    x, v, L = dimer(1.15)
    amp = []
    for dt in (0.004, 0.002):
        steps = int(round(4.0 / dt))
        _, _, _, thermo, _, _ = orc.run_nve(x, v, L, 2.5, 2.8, dt, steps, mode="allpairs")
        E = np.array([pe + ke for _, pe, ke in thermo])
        amp.append(E.max() - E.min())
    assert amp[0] / amp[1] == pytest.approx(4.0, rel=0.2)


def test_nve_lj256(orc):
    """100 steps of the 256-atom liquid with the oracle's own Verlet lists.

    The truncated potential jumps by u(rc) when a pair crosses rc, so energy
    conservation is judged on E - npairs(r < rc) * u(rc).
    """
    w = li.WORKLOADS["lj256"]
    s = li.make_system(w)
    x, v, F, thermo, snaps, _ = orc.run_nve(s["x"], s["v"], w.box, w.rc, w.rlist, w.dt,
                                            w.steps, mode="verlet",
                                            record=set(range(0, 101, 10)))
    u_rc = orc.pair_energy(w.rc * (1 - 1e-15))[0]
    Esh = []
    for step in sorted(snaps):
        xs, vs, _ = snaps[step]
        _, e, _, npairs = orc.forces(xs, w.box, w.rc)
        Esh.append(e.sum() - npairs[0] * u_rc + 0.5 * (vs * vs).sum())
    Esh = np.array(Esh)
    n = w.natoms
    assert np.abs(Esh - Esh[0]).max() / n < 1e-3
    assert np.abs(v.sum(axis=0)).max() < 1e-11
