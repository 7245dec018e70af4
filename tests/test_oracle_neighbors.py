"""Pins of the oracle's Verlet lists and binning against independent NumPy code.

The brute force here forms the minimum image as d - L*round(d/L), a different
formula from the oracle's single shift; both give the same representative for
any pair within rlist < L/2, so the sets must agree exactly.
"""
import numpy as np
import pytest

import lj_inputs as li


def numpy_full_sets(x, L, rlist):
    L = np.asarray(L, dtype=np.float64)
    d = x[:, None, :] - x[None, :, :]
    d = d - L * np.round(d / L)
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    m = r2 < rlist * rlist
    np.fill_diagonal(m, False)
    return m


CASES = [
    ("lj256", None, None),
    ("gas_ragged", 331, (6.0, 7.5, 9.0)),
    ("gas_2cells", 500, (6.0, 6.0, 6.0)),
    ("gas_1cell", 97, (5.7, 5.9, 5.61)),
    ("gas_long", 450, (5.8, 5.8, 17.0)),
]


@pytest.mark.parametrize("name,n,L", CASES)
def test_full_list_matches_bruteforce(orc, name, n, L):
    rlist = 2.8
    if name == "lj256":
        w = li.WORKLOADS["lj256"]
        x, L = li.positions(w), w.box
    else:
        x = li.random_gas(n, L, seed=7 + n)
    off, nb = orc.neighbor_lists(x, L, rlist)
    m = numpy_full_sets(x, L, rlist)
    for i in range(x.shape[0]):
        assert np.array_equal(nb[off[i]:off[i + 1]], np.flatnonzero(m[i]))
    assert np.array_equal(m, m.T)  # symmetric relation


def test_selected_rows_match_full(orc):
    w = li.WORKLOADS["lj256"]
    x = li.positions(w)
    off, nb = orc.neighbor_lists(x, w.box, w.rlist)
    sel = np.array([0, 5, 17, 255, 128])
    so, sn = orc.neighbor_lists(x, w.box, w.rlist, sel=sel)
    for k, i in enumerate(sel):
        assert np.array_equal(sn[so[k]:so[k + 1]], nb[off[i]:off[i + 1]])


@pytest.mark.parametrize("case", ["liquid4000", "clump"])
def test_pair_pass_matches_row_passes(orc, case):
    """Whole lists (one pass over the unordered pairs, rows cut at a capacity and
    re-run when cut) equal the row-by-row count and fill passes over all j."""
    if case == "liquid4000":
        w = li.Workload("liquid4000", 9, cells=10)
        x, L = li.positions(w), w.box
    else:  # 300 atoms inside one rlist-sized ball: rows far beyond the first capacity
        L = np.array([20.0, 21.0, 22.0])
        x = li.random_gas(300, np.array([1.6, 1.6, 1.6]), seed=4) + 18.9
        x = np.where(x >= L, x - L, x)
    n = x.shape[0]
    off, nb = orc.neighbor_lists(x, L, 2.8)
    so, sn = orc.neighbor_lists(x, L, 2.8, sel=np.arange(n))
    assert np.array_equal(off, so) and np.array_equal(nb, sn)
    up = orc.upper_pairs(x, L, 2.8)
    assert np.array_equal(up, orc.half_pairs(so, sn))
    if case == "clump":
        assert np.diff(off).max() > 96


def test_half_pairs(orc):
    w = li.WORKLOADS["lj256"]
    x = li.positions(w)
    off, nb = orc.neighbor_lists(x, w.box, w.rlist)
    hp = orc.half_pairs(off, nb)
    assert hp.shape[0] * 2 == nb.size
    assert np.all(hp[:, 0] < hp[:, 1])


@pytest.mark.parametrize("L,rlist", [((6.718, 6.718, 6.718), 2.8), ((33.59,) * 3, 2.8),
                                     ((5.6, 8.4, 30.0), 2.8), ((2.0, 3.0, 4.0), 2.8)])
def test_grid(orc, L, rlist):
    nc = orc.grid(L, rlist)
    for k in range(3):
        assert nc[k] >= 1
        if nc[k] > 1:
            assert L[k] / nc[k] >= rlist  # an edge never shorter than rlist
        assert L[k] / (nc[k] + 1) < rlist * (1 + 1e-10)  # and no finer grid would do


def test_bin_order(orc):
    L = np.array([9.0, 10.0, 11.5])
    x = li.random_gas(700, L, seed=3)
    ids = np.random.default_rng(1).permutation(700).astype(np.int64) * 3 + 11
    perm, cell_start, nc = orc.bin_order(x, ids, L, 2.8)
    h = L / nc
    c3 = np.minimum(np.floor(x / h).astype(np.int64), nc - 1)
    cell = (c3[:, 2] * nc[1] + c3[:, 1]) * nc[0] + c3[:, 0]
    assert np.array_equal(np.sort(perm), np.arange(700))
    cs = cell[perm]
    assert np.all(np.diff(cs) >= 0)
    same = np.diff(cs) == 0
    assert np.all(np.diff(ids[perm])[same] > 0)
    for c in range(int(np.prod(nc))):
        assert np.all(cs[cell_start[c]:cell_start[c + 1]] == c)
    assert cell_start[-1] == 700


def test_bin_upper_edge(orc):
    # box edges where x just below L gives x/h == nc after rounding: such atoms
    # belong to the last cell, never to cell 0
    L = np.array([15.980117845432297, 26.507607108814266, 27.54778587512588])
    x = li.random_gas(50, L, seed=2)
    edge = np.nextafter(L, 0.0)
    x[:3] = [[edge[0], 1.0, 1.0], [1.0, edge[1], 1.0], [1.0, 1.0, edge[2]]]
    x[3] = [0.0, 0.0, 0.0]
    nc = orc.grid(L, 2.8)
    assert np.any(np.floor(edge / (L / nc)) >= nc)  # the rounding case is exercised
    cell = orc.cell_index(x, L, nc)
    cx = cell % nc[0]
    cy = (cell // nc[0]) % nc[1]
    cz = cell // (nc[0] * nc[1])
    assert cx[0] == nc[0] - 1 and cy[1] == nc[1] - 1 and cz[2] == nc[2] - 1
    assert cell[3] == 0
