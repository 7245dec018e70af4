"""Pins of the oracle's 12-6 pair interaction against closed forms.

Three facts fix a 12-6 potential A r^-12 - B r^-6 completely: its zero at
r = sigma, its minimum at r = 2^(1/6) sigma with depth -eps, and the tail
-4 eps (sigma/r)^6.  The force is then pinned against -du/dr by central
differences.  None of these re-types the oracle's formula.
"""
import numpy as np
import pytest

PARAMS = [(1.0, 1.0), (0.8, 0.9), (1.2, 1.1), (2.5, 0.7)]


@pytest.mark.parametrize("eps,sigma", PARAMS)
def test_zero_at_sigma(orc, eps, sigma):
    u, F = orc.pair_energy(sigma, eps, sigma)
    assert abs(u) < 1e-13 * eps
    # |F| = 24 eps / sigma at r = sigma (derivative of the closed form there)
    assert F[0, 0] == pytest.approx(-24.0 * eps / sigma, rel=1e-13)
    assert F[1, 0] == pytest.approx(24.0 * eps / sigma, rel=1e-13)
    assert np.all(F[:, 1:] == 0.0)


@pytest.mark.parametrize("eps,sigma", PARAMS)
def test_minimum(orc, eps, sigma):
    rmin = 2.0 ** (1.0 / 6.0) * sigma
    u, F = orc.pair_energy(rmin, eps, sigma)
    assert u == pytest.approx(-eps, rel=1e-13)
    assert abs(F[0, 0]) < 1e-12 * eps / sigma
    # strictly a minimum: higher on both sides
    assert orc.pair_energy(rmin * 0.99, eps, sigma)[0] > u
    assert orc.pair_energy(rmin * 1.01, eps, sigma)[0] > u


@pytest.mark.parametrize("eps,sigma", PARAMS)
def test_tail(orc, eps, sigma):
    for r in (8.0 * sigma, 20.0 * sigma):
        u, _ = orc.pair_energy(r, eps, sigma)
        tail = -4.0 * eps * (sigma / r) ** 6
        assert u == pytest.approx(tail, rel=2.0 * (sigma / r) ** 6)


@pytest.mark.parametrize("eps,sigma", PARAMS)
def test_force_is_minus_gradient(orc, eps, sigma):
    h = 1e-6
    for r in np.array([0.95, 1.05, 1.3, 1.7, 2.3]) * sigma:
        up = orc.pair_energy(r + h, eps, sigma)[0]
        um = orc.pair_energy(r - h, eps, sigma)[0]
        dudr = (up - um) / (2 * h)
        _, F = orc.pair_energy(r, eps, sigma)
        # atom 0 at origin, atom 1 at +r x: force on atom 1 is -du/dr along +x
        assert F[1, 0] == pytest.approx(-dudr, rel=1e-7, abs=1e-9)
        assert F[0, 0] == -F[1, 0]


def test_scaling_law(orc):
    # u(r; eps, sigma) = eps * u(r/sigma; 1, 1)
    for eps, sigma in PARAMS:
        for rr in (0.97, 1.2, 1.9):
            u1 = orc.pair_energy(rr * sigma, eps, sigma)[0]
            u0 = orc.pair_energy(rr, 1.0, 1.0)[0]
            assert u1 == pytest.approx(eps * u0, rel=1e-13)


def test_strict_cutoff(orc):
    # pairs at r >= rc contribute nothing; just inside they do
    L = np.full(3, 50.0)
    rc = 2.5
    for r, inside in ((rc * (1 - 1e-12), True), (rc, False), (rc * (1 + 1e-12), False)):
        x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
        F, e, W, npairs = orc.forces(x, L, rc)
        assert (npairs[0] == 1) == inside
        assert (e[0] != 0.0) == inside


def test_minimum_image(orc):
    # two atoms across the periodic boundary interact through the short image
    L = np.array([10.0, 11.0, 12.0])
    x = np.array([[0.2, 5.0, 6.0], [9.5, 5.0, 6.0]])
    F, e, _, _ = orc.forces(x, L, rc=2.5)
    u_direct, Fd = orc.pair_energy(0.7)
    assert 2 * e[0] == pytest.approx(u_direct, rel=1e-14)
    # image at -0.5: atom 0 is to the right of atom 1's image, so it is pushed +x
    assert F[0, 0] == pytest.approx(Fd[1, 0], rel=1e-14)
