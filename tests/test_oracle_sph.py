"""Pins of the SPH oracle against what the mathematics fixes, independent of its own
formulas: the kernel's unit integral and its derivative, compact support and
continuity, the lattice sum against the continuum density, the acceleration
as minus the gradient of the internal energy (finite differences), momentum
conservation, symmetry zeros, the sign of pressure, and energy conservation
under velocity Verlet."""
import numpy as np
import pytest
from scipy import integrate

import lj_inputs as li


def _lattice(m, spacing=1.0):
    idx = np.arange(m, dtype=np.float64)
    X = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3) + 0.5
    return X * spacing


@pytest.mark.parametrize("h", [0.7, 1.3])
def test_kernel_unit_integral(orc, h):
    """4 pi int_0^2h r^2 W(r) dr = 1: fixes the normalisation and every coefficient
    of the polynomial pieces (each one moves the integral)."""
    f = lambda r: 4.0 * np.pi * r * r * orc.sph_kernel([r], h)[0][0]
    val, err = integrate.quad(f, 0.0, 2.0 * h, points=[h], epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-10
    # the second moment of the cubic spline: int r^2 W dV = 9/10 h^2 (no free constant)
    g = lambda r: 4.0 * np.pi * r ** 4 * orc.sph_kernel([r], h)[0][0]
    m2, _ = integrate.quad(g, 0.0, 2.0 * h, points=[h], epsabs=1e-13, epsrel=1e-13)
    assert m2 == pytest.approx(0.9 * h * h, rel=1e-10)


@pytest.mark.parametrize("h", [0.7, 1.3])
def test_kernel_gradient_is_derivative(orc, h):
    """G(r) r equals the central difference of W at points away from the joins."""
    r = np.concatenate([np.linspace(0.01, 0.99, 37), np.linspace(1.01, 1.99, 37)]) * h
    W, G = orc.sph_kernel(r, h)
    e = 1e-6 * h
    Wp, _ = orc.sph_kernel(r + e, h)
    Wm, _ = orc.sph_kernel(r - e, h)
    fd = (Wp - Wm) / (2 * e)
    assert np.abs(G * r - fd).max() <= 1e-7 * np.abs(fd).max()
    assert np.all(G < 0)  # monotone decreasing inside the support


def test_kernel_support_and_continuity(orc):
    h = 1.1
    W, G = orc.sph_kernel([2 * h, 2 * h + 1e-9, 5.0], h)
    assert np.all(W == 0) and np.all(G == 0)
    # W, dW/dr and G continuous at r = h (q = 1) and vanishing at r = 2h
    r = np.array([h * (1 - 1e-12), h * (1 + 1e-12), 2 * h * (1 - 1e-9)])
    W, G = orc.sph_kernel(r, h)
    assert W[0] == pytest.approx(W[1], rel=1e-10) and G[0] == pytest.approx(G[1], rel=1e-10)
    assert W[2] < 1e-20 and abs(G[2]) < 1e-12


def test_single_particle_density_is_self_term(orc):
    """Alone in the box: rho = m W(0, h) = m / (pi h^3) (the kernel's peak)."""
    rho = orc.sph_density(np.array([[1.0, 2.0, 3.0]]), [20.0, 20.0, 20.0], 1.5, mass=2.0)
    assert rho[0] == pytest.approx(2.0 / (np.pi * 1.5 ** 3), rel=1e-14)


@pytest.mark.parametrize("h", [1.0, 1.3, 1.5])
def test_lattice_density_matches_continuum(orc, h):
    """On a simple-cubic lattice of spacing a the summed density approaches m/a^3; at
    h >= a the discrete sum is within 0.5 % (a dropped self term is off by 15-30 %)."""
    X = _lattice(10, 1.0)
    rho = orc.sph_density(X, [10.0] * 3, h, mass=1.0)
    assert np.ptp(rho) <= 1e-12  # every site equivalent
    assert abs(rho[0] - 1.0) < 5e-3


def test_lattice_has_zero_acceleration(orc):
    """Uniform pressure (rho0 != lattice density) on a perfect lattice: no net force."""
    X = _lattice(8)
    L = [8.0] * 3
    rho = orc.sph_density(X, L, 1.3)
    a = orc.sph_accel(X, L, 1.3, 1.0, 10.0, 0.5, rho)
    assert np.abs(a).max() < 1e-10


def test_pressure_sign_of_a_pair(orc):
    """Two particles: compressed (p > 0) they repel, in tension (p < 0) they attract."""
    x = np.array([[5.0, 5.0, 5.0], [5.9, 5.3, 5.1]])
    L = [20.0] * 3
    rho = orc.sph_density(x, L, 1.0)
    d = x[0] - x[1]
    push = orc.sph_accel(x, L, 1.0, 1.0, 3.0, 0.0, rho)  # rho0 = 0: p > 0
    pull = orc.sph_accel(x, L, 1.0, 1.0, 3.0, 10.0, rho)  # rho0 above rho: p < 0
    assert push[0] @ d > 0 and pull[0] @ d < 0
    for a in (push, pull):  # along the line of centres, equal and opposite
        assert np.abs(np.cross(a[0], d)).max() < 1e-12 * np.abs(a).max()
        assert np.abs(a[0] + a[1]).max() < 1e-13 * np.abs(a).max()


def _random_fluid(n, L, seed, jitter=0.3):
    m = round(n ** (1 / 3))
    g = np.random.default_rng(seed)
    X = _lattice(m, L / m) + g.uniform(-jitter, jitter, (m ** 3, 3))
    return np.mod(X, L)


def test_acceleration_is_minus_energy_gradient(orc):
    """m a_k = -dU/dx_k with U = sum_i m u(rho_i), du/drho = p/rho^2: central
    differences of the oracle's own density-based energy fix the pair form, the
    factor m, the equation of state and every sign."""
    L, h, m, c0, rho0 = 5.0, 1.2, 1.3, 4.0, 1.1
    x = _random_fluid(125, L, 3)
    rho = orc.sph_density(x, [L] * 3, h, m)
    a = orc.sph_accel(x, [L] * 3, h, m, c0, rho0, rho)
    U = lambda y: orc.sph_internal_energy(orc.sph_density(y, [L] * 3, h, m), m, c0, rho0)
    e = 1e-6
    for k in (0, 17, 64, 124):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, c] += e
            xm[k, c] -= e
            grad = (U(xp) - U(xm)) / (2 * e)
            assert -grad / m == pytest.approx(a[k, c], abs=2e-6 * np.abs(a).max())


def test_momentum_conserved_and_rows_selectable(orc):
    L = 6.0
    x = _random_fluid(216, L, 5)
    rho = orc.sph_density(x, [L] * 3, 1.3)
    a = orc.sph_accel(x, [L] * 3, 1.3, 1.0, 10.0, 1.0, rho)
    assert np.abs(a.sum(axis=0)).max() < 1e-12 * np.abs(a).sum()
    sel = np.array([3, 0, 200, 17])
    assert np.array_equal(orc.sph_density(x, [L] * 3, 1.3, sel=sel), rho[sel])
    assert np.array_equal(orc.sph_accel(x, [L] * 3, 1.3, 1.0, 10.0, 1.0, rho, sel=sel), a[sel])


def test_velocity_verlet_conserves_energy(orc):
    """E = m/2 sum v^2 + U drifts at O(dt^2): halving dt cuts the spread ~4x."""
    w = li.SPH_WORKLOADS["sph4k"]
    x0 = _random_fluid(216, 6.0, 9, jitter=0.1)
    v0 = np.random.default_rng(2).normal(0.0, 0.2, x0.shape)
    spreads = []
    for dt, steps in ((0.02, 20), (0.01, 40)):
        _, _, E = orc.sph_run(x0, v0, [6.0] * 3, w.h, w.mass, w.c0, w.rho0, dt, steps)
        spreads.append(np.ptp(E))
    assert spreads[0] < 5e-3 * abs(E[0])
    assert 3.5 < spreads[0] / spreads[1] < 4.5
