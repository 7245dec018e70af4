"""Pins of the oracle's many-body sums on the perfect fcc lattice.

Crystallographic facts (tests/golden/fcc_shells.txt) fix the neighbor counts,
inversion symmetry fixes the forces to zero, and the per-atom energy and the
virial trace are shell sums of the (separately pinned) pair interaction.
"""
import os

import numpy as np
import pytest

import lj_inputs as li

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fcc_shells.txt")


def shells(a):
    tab = np.loadtxt(GOLDEN, comments="#")
    return np.sqrt(tab[:, 0] * a * a / 2.0), tab[:, 1].astype(int)


@pytest.mark.parametrize("cells", [4, 6])
def test_fcc_neighbor_counts(orc, cells):
    w = li.Workload("t", 0, cells=cells)
    x = li.fcc_lattice(cells, w.lattice_constant)
    r, cnt = shells(w.lattice_constant)
    for cut in (w.rc, w.rlist):
        expect = int(cnt[r < cut].sum())
        off, nb = orc.neighbor_lists(x, w.box, cut)
        assert np.all(np.diff(off) == expect)
    # 78 within rlist = 2.8 and 54 within rc = 2.5 at rho* = 0.8442
    assert int(cnt[r < w.rlist].sum()) == 78
    assert int(cnt[r < w.rc].sum()) == 54


@pytest.mark.parametrize("cells", [4, 6])
def test_fcc_energy_forces_virial(orc, cells):
    w = li.Workload("t", 0, cells=cells)
    x = li.fcc_lattice(cells, w.lattice_constant)
    n = x.shape[0]
    F, e, W, npairs = orc.forces(x, w.box, w.rc)
    assert np.abs(F).max() < 1e-12
    r, cnt = shells(w.lattice_constant)
    inside = r < w.rc
    u_sh = np.array([orc.pair_energy(rk)[0] for rk in r[inside]])
    f_sh = np.array([orc.pair_energy(rk)[1][1, 0] for rk in r[inside]])  # force along r
    e_expect = 0.5 * np.sum(cnt[inside] * u_sh)
    np.testing.assert_allclose(e, e_expect, rtol=1e-13)
    assert e_expect == pytest.approx(-6.773368053252957, rel=1e-13)
    # virial trace: 1/2 sum_i sum_j r f(r);  cubic symmetry: equal diagonal, zero shear
    tr_expect = 0.5 * n * np.sum(cnt[inside] * r[inside] * f_sh)
    assert W[:3].sum() == pytest.approx(tr_expect, rel=1e-12)
    np.testing.assert_allclose(W[:3], tr_expect / 3, rtol=1e-12)
    assert np.abs(W[3:]).max() < 1e-9 * abs(tr_expect)
    assert npairs[0] == n * 54 // 2


def test_fcc_translation_invariance(orc):
    w = li.WORKLOADS["lj256"]
    x = li.fcc_lattice(w.cells, w.lattice_constant)
    shift = np.array([0.31, 0.77, 1.13])
    x2 = np.mod(x + shift, w.box)
    _, e1, _, _ = orc.forces(x, w.box, w.rc)
    _, e2, _, _ = orc.forces(x2, w.box, w.rc)
    np.testing.assert_allclose(e1, e2, rtol=1e-12)
