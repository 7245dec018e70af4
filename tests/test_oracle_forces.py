"""Pins of the oracle's forces, energies and virial on disordered systems.

Newton's third law, F = -grad E by central differences, the virial as minus
the strain derivative of E, and the packed type-pair table checked through
sub-system energies.
"""
import numpy as np
import pytest

import lj_inputs as li


def jittered(cells=4, jitter=0.05, index=0):
    w = li.Workload("t", index, cells=cells, jitter=jitter)
    return w, li.positions(w)


def test_newton3_and_energy_sum(orc):
    w, x = jittered()
    F, e, W, npairs = orc.forces(x, w.box, w.rc)
    assert np.abs(F.sum(axis=0)).max() < 1e-11
    assert np.abs(F).max() > 1.0  # the jitter produces real forces


def pair_set(orc, x, L, rc):
    off, nb = orc.neighbor_lists(x, L, rc)
    return nb.copy(), off.copy()


@pytest.mark.parametrize("two_types", [False, True])
def test_force_is_minus_gradient(orc, two_types):
    w, x = jittered(index=11)
    if two_types:
        tw = li.Workload("t", 3, cells=4, ntypes=2)
        types, (eps, sig) = li.types(tw), li.params(tw)
    else:
        types, eps, sig = None, [1.0], [1.0]
    F, _, _, _ = orc.forces(x, w.box, w.rc, eps, sig, types)
    rng = np.random.default_rng(5)
    h = 1e-5
    base = pair_set(orc, x, w.box, w.rc)
    for _ in range(24):
        i, k = rng.integers(0, x.shape[0]), rng.integers(0, 3)
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        for xx in (xp, xm):
            s = pair_set(orc, xx, w.box, w.rc)
            assert np.array_equal(s[0], base[0])
        Ep = orc.forces(xp, w.box, w.rc, eps, sig, types)[1].sum()
        Em = orc.forces(xm, w.box, w.rc, eps, sig, types)[1].sum()
        assert F[i, k] == pytest.approx(-(Ep - Em) / (2 * h), rel=1e-6, abs=1e-6)


def test_virial_is_minus_diagonal_strain_derivative(orc):
    w, x = jittered(index=12)
    _, _, W, _ = orc.forces(x, w.box, w.rc)
    h = 1e-6
    for a in range(3):
        s = np.ones(3)
        s[a] = 1 + h
        Ep = orc.forces(x * s, w.box * s, w.rc)[1].sum()
        s[a] = 1 - h
        Em = orc.forces(x * s, w.box * s, w.rc)[1].sum()
        assert W[a] == pytest.approx(-(Ep - Em) / (2 * h), rel=1e-6)


def test_virial_shear_on_cluster(orc):
    # isolated cluster in a large box: shear x_a += lam * x_b changes every
    # displacement the same way, so dE/dlam = -W_ab
    rng = np.random.default_rng(9)
    g = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = 40.0 + 1.12 * g + rng.uniform(-0.05, 0.05, size=g.shape)
    L = np.full(3, 100.0)
    _, _, W, _ = orc.forces(x, L, 2.5)
    h = 1e-6
    for q, (a, b) in zip(range(3, 6), [(0, 1), (0, 2), (1, 2)]):
        xp, xm = x.copy(), x.copy()
        xp[:, a] += h * x[:, b]
        xm[:, a] -= h * x[:, b]
        dE = (orc.forces(xp, L, 2.5)[1].sum() - orc.forces(xm, L, 2.5)[1].sum()) / (2 * h)
        assert W[q] == pytest.approx(-dE, rel=1e-6, abs=1e-6)


def test_packed_type_table_by_subsystems(orc):
    # E with only eps_00 on equals the energy of the type-0 atoms alone; with
    # only eps_11 on, of the type-1 atoms alone; eps_01 carries the rest.
    tw = li.Workload("t", 3, cells=4, ntypes=2)
    w, x = jittered(index=3)
    types = li.types(tw)
    sig = np.array([0.95, 1.05, 1.0])
    E_all = orc.forces(x, w.box, w.rc, [1, 1, 1], sig, types)[1].sum()
    E00 = orc.forces(x, w.box, w.rc, [1, 0, 0], sig, types)[1].sum()
    E11 = orc.forces(x, w.box, w.rc, [0, 0, 1], sig, types)[1].sum()
    E01 = orc.forces(x, w.box, w.rc, [0, 1, 0], sig, types)[1].sum()
    sub0 = orc.forces(x[types == 0], w.box, w.rc, [1], [sig[0]])[1].sum()
    sub1 = orc.forces(x[types == 1], w.box, w.rc, [1], [sig[2]])[1].sum()
    assert E00 == pytest.approx(sub0, rel=1e-12)
    assert E11 == pytest.approx(sub1, rel=1e-12)
    assert E01 == pytest.approx(E_all - E00 - E11, rel=1e-10)
    # relabelling the types and swapping the diagonal entries changes nothing
    F1 = orc.forces(x, w.box, w.rc, [0.9, 1.1, 1.2], sig, types)[0]
    F2 = orc.forces(x, w.box, w.rc, [1.2, 1.1, 0.9], sig[::-1].copy(), 1 - types)[0]
    np.testing.assert_allclose(F1, F2, rtol=1e-12, atol=1e-12)


def test_selected_rows_and_list_mode_agree(orc):
    w, x = jittered(index=13)
    F, e, W, _ = orc.forces(x, w.box, w.rc)
    sel = np.array([3, 99, 200, 7])
    Fs, es, _, _ = orc.forces(x, w.box, w.rc, sel=sel)
    np.testing.assert_array_equal(Fs, F[sel])
    np.testing.assert_array_equal(es, e[sel])
    off, nb = orc.neighbor_lists(x, w.box, w.rlist)
    Fl, el, Wl = orc.forces_list(x, w.box, w.rc, off, nb)
    np.testing.assert_allclose(Fl, F, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Wl, W, rtol=1e-13)


def test_pair_counts_within_cutoff(orc):
    """Unordered pairs within rc per packed type pair, over all pairs and over a list,
    against a NumPy count by type that shares no code with the oracle."""
    from helpers import pairs_within
    w, x = jittered(index=17, jitter=0.2)
    types = (np.arange(x.shape[0]) % 2).astype(np.int32)
    eps, sig = [1.0, 0.9, 1.1], [1.0, 1.05, 0.95]
    _, _, _, npairs = orc.forces(x, w.box, w.rc, eps, sig, types)
    off, nb = orc.neighbor_lists(x, w.box, w.rlist)
    _, _, _, np_list = orc.forces_list(x, w.box, w.rc, off, nb, eps, sig, types,
                                       with_pairs=True)
    a, b = x[types == 0], x[types == 1]
    n00, n11 = pairs_within(a, w.box, w.rc), pairs_within(b, w.box, w.rc)
    n01 = pairs_within(x, w.box, w.rc) - n00 - n11
    assert list(npairs) == [n00, n01, n11] and list(np_list) == [n00, n01, n11]
    assert n01 > 0 and n00 > 0
