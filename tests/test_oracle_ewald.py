"""Pins of the Ewald and SPME oracles against what the mathematics fixes: the
Madelung constants of rock salt and caesium chloride, independence of the Ewald
energy from the splitting parameter, forces as minus the energy gradient,
cardinal B-spline identities, SPME converging to the Ewald sum, and exact
invariances of the SPME grid."""
import numpy as np
import pytest

NACL = 1.747564594633182   # Madelung constant of rock salt (nearest-neighbour distance)
CSCL = 1.762674773070988   # Madelung constant of caesium chloride (nearest-neighbour distance)


def _ewald_total(orc, x, q, L, alpha, rc, nmax):
    e, F = orc.ewald_direct(x, q, L, alpha, rc)
    Er, Fr = orc.ewald_recip(x, q, L, alpha, nmax)
    return e.sum() + Er + orc.ewald_self(q, alpha), F + Fr


def test_rock_salt_madelung(orc):
    """Simple-cubic lattice with alternating charges (two interpenetrating fcc):
    E per ion pair = -M / a for nearest-neighbour distance a."""
    m, a = 4, 1.0
    idx = np.arange(m)
    I = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    x = (I + 0.25) * a
    q = np.where(I.sum(1) % 2 == 0, 1.0, -1.0)
    E, F = _ewald_total(orc, x, q, [m * a] * 3, 3.0, 1.99, 16)
    assert E / (len(q) / 2) * a == pytest.approx(-NACL, rel=1e-9)
    assert np.abs(F).max() < 1e-12  # every ion at a centre of symmetry


def test_caesium_chloride_madelung(orc):
    """Cube corners +1, body centres -1: E per ion pair = -M / r_nn, r_nn = a sqrt(3)/2."""
    m, a = 3, 1.0
    idx = np.arange(m)
    I = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3).astype(float)
    x = np.concatenate([I + 0.1, I + 0.6]) * a
    q = np.concatenate([np.ones(len(I)), -np.ones(len(I))])
    E, _ = _ewald_total(orc, x, q, [m * a] * 3, 3.5, 1.49, 18)
    assert E / len(I) * (a * np.sqrt(3) / 2) == pytest.approx(-CSCL, rel=1e-8)


def _random_neutral(n, L, seed):
    g = np.random.default_rng(seed)
    x = g.uniform(0.0, 1.0, (n, 3)) * np.asarray(L)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * g.uniform(0.5, 1.5, n)
    q -= q.mean()
    return x, q


def test_energy_independent_of_alpha(orc):
    L = np.array([6.0, 6.5, 7.0])
    x, q = _random_neutral(60, L, 3)
    E1, F1 = _ewald_total(orc, x, q, L, 1.4, 2.99, 14)
    E2, F2 = _ewald_total(orc, x, q, L, 1.8, 2.99, 18)
    assert E1 == pytest.approx(E2, rel=1e-8)
    assert np.abs(F1 - F2).max() < 1e-6 * np.abs(F1).max()


def test_ewald_forces_are_minus_gradient(orc):
    L = np.array([6.0, 6.5, 7.0])
    x, q = _random_neutral(40, L, 5)
    E, F = _ewald_total(orc, x, q, L, 1.5, 2.99, 14)
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).sum()
    e = 1e-6
    for i in (0, 7, 33):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += e
            xm[i, c] -= e
            g = (_ewald_total(orc, xp, q, L, 1.5, 2.99, 14)[0] -
                 _ewald_total(orc, xm, q, L, 1.5, 2.99, 14)[0]) / (2 * e)
            assert -g == pytest.approx(F[i, c], abs=1e-6 * np.abs(F).max())


@pytest.mark.parametrize("n", [4, 6, 8])
def test_bspline_identities(orc, n):
    w = np.linspace(0.0, 1.0, 11)[:-1]
    vals = np.stack([orc.bspline(w + j, n) for j in range(n)])
    assert np.abs(vals.sum(0) - 1.0).max() < 1e-14      # partition of unity
    u = np.linspace(0.0, n, 4001)
    M = orc.bspline(u, n)
    assert np.abs(M - orc.bspline(n - u, n)).max() < 1e-14  # symmetric about n/2
    assert np.trapezoid(M, u) == pytest.approx(1.0, abs=1e-6)
    assert M.min() >= 0.0 and orc.bspline(np.array([-0.1, n + 0.1]), n).max() == 0.0
    if n == 4:  # closed form at the knots
        assert orc.bspline(np.array([1.0, 2.0, 3.0]), 4) == pytest.approx([1 / 6, 2 / 3, 1 / 6])


def test_spme_converges_to_ewald(orc):
    L = np.array([7.0, 8.0, 9.0])
    x, q = _random_neutral(120, L, 1)
    Er, Fr = orc.ewald_recip(x, q, L, 1.2, 14)
    errs = []
    for K, n in (((16, 16, 16), 4), ((32, 32, 32), 4), ((32, 32, 32), 6), ((64, 64, 64), 8)):
        Es, Fs = orc.spme_recip(x, q, L, 1.2, K, n)
        errs.append((abs(Es - Er) / abs(Er), np.abs(Fs - Fr).max() / np.abs(Fr).max()))
    assert all(a[0] > b[0] and a[1] > b[1] for a, b in zip(errs, errs[1:]))
    assert errs[-1][0] < 1e-8 and errs[-1][1] < 1e-7


def test_spme_forces_are_minus_gradient(orc):
    L = np.array([5.0, 5.5, 6.0])
    x, q = _random_neutral(30, L, 7)
    K = (16, 16, 20)
    _, F = orc.spme_recip(x, q, L, 1.1, K, 4)
    e = 1e-6
    for i in (0, 11, 29):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += e
            xm[i, c] -= e
            g = (orc.spme_recip(xp, q, L, 1.1, K, 4)[0] - orc.spme_recip(xm, q, L, 1.1, K, 4)[0])
            assert -g / (2 * e) == pytest.approx(F[i, c], abs=1e-7 * np.abs(F).max())


def test_spme_grid_invariances(orc):
    """The spread charge sums to the total charge; a shift of every particle by one grid
    spacing permutes the grid, so E_rec is unchanged and the forces too."""
    L = np.array([6.0, 6.0, 8.0])
    x, q = _random_neutral(50, L, 9)
    q = q + 0.3  # a non-zero total for the sum check
    K = (12, 16, 20)
    Q = orc.spme_grid_charge(x, q, L, K, 6)
    assert Q.sum() == pytest.approx(q.sum(), rel=1e-13)
    q -= q.mean()
    E0, F0 = orc.spme_recip(x, q, L, 1.3, K, 6)
    shift = np.array([L[0] / K[0], 2 * L[1] / K[1], -L[2] / K[2]])
    E1, F1 = orc.spme_recip(np.mod(x + shift, L), q, L, 1.3, K, 6)
    assert E1 == pytest.approx(E0, rel=1e-12)
    assert np.abs(F1 - F0).max() < 1e-11 * np.abs(F0).max()
