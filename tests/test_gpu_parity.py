"""Parity of the HIP path (through the C ABI) against the CPU FP64 oracle.

Bars: bin permutation and cell starts bit-exact; neighbor sets identical as
sorted sets of original-id pairs; FP64 forces max_i |dF_i| <= 1e-12 max_i |F_i|
and per-atom energy, E and each virial component to relative 1e-12; mixed
forces max_i |dF_i| <= 1e-5 F_rms and per-atom energy relative 1e-6.
"""
import numpy as np
import pytest

import lj_inputs as li
from helpers import gpu_device, gpu_pairs_by_id, max_rel_vec, oracle_pairs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_F_TOL = 1e-5
MIXED_E_TOL = 1e-6


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def T(a, dev, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev, dtype=dtype)


def gas(n, L, seed):
    return li.random_gas(n, L, seed)


def clumped(n_bulk, n_clump, L, seed):
    """Bulk gas plus a dense clump that overfills a few cells (ragged, big candidate sets)."""
    rng = np.random.default_rng(seed)
    x = li.random_gas(n_bulk, L, seed)
    c = rng.uniform(0.3, 0.7, size=3) * np.asarray(L)
    clump = c + rng.uniform(-1.2, 1.2, size=(n_clump, 3))
    return np.concatenate([x, clump])


def gpu_sort(dev, x, L, rlist, v=None, types=None):
    import torch
    from paper_2109_09056_amd import ops
    xs, vs, ts, ids, cs = ops.bin(L, rlist, T(x, dev, torch.float64),
                                  None if v is None else T(v, dev, torch.float64),
                                  None if types is None else T(types, dev, torch.int32))
    return xs, vs, ts, ids, cs


# ---------------------------------------------------------------------- bin --

BIN_CASES = [
    ("lj256", None), ("lj32k", None), ("gas_ragged", (331, (6.0, 7.5, 9.0))),
    ("gas_one", (1, (6.0, 6.0, 6.0))), ("gas_five", (5, (9.0, 9.1, 9.2))),
    ("clump", None),
    # 15,625 and 24,389 cells: the cell scan runs over several 4,096-cell chunks
    ("gas_many_cells", (40000, (70.0, 71.0, 72.5))), ("lj500k", None),
]


@pytest.mark.parametrize("name,spec", BIN_CASES)
def test_bin_matches_oracle(dev, orc, name, spec):
    if name in li.WORKLOADS:
        w = li.WORKLOADS[name]
        x, L = li.positions(w), w.box
    elif name == "clump":
        L = np.array([14.0, 15.0, 16.0])
        x = clumped(900, 700, L, 5)
    else:
        n, L = spec
        x = gas(n, L, 11)
    L = np.asarray(L, dtype=np.float64)
    perm, cell_start, nc = orc.bin_order(x, np.arange(x.shape[0]), L, 2.8)
    xs, _, _, ids, cs = gpu_sort(dev, x, L, 2.8)
    assert np.array_equal(ids.cpu().numpy(), perm)
    assert np.array_equal(cs.cpu().numpy().astype(np.int64), cell_start)
    assert np.array_equal(xs.cpu().numpy(), x[perm])


def test_bin_permutes_every_field_and_keeps_given_ids(dev, orc):
    import torch
    from paper_2109_09056_amd import ops
    L = np.array([9.0, 10.0, 11.5])
    x = gas(700, L, 3)
    rng = np.random.default_rng(1)
    ids = rng.permutation(700).astype(np.int64) * 3 + 11
    v = rng.normal(size=(700, 3))
    ty = rng.integers(0, 3, 700).astype(np.int32)
    perm, cell_start, _ = orc.bin_order(x, ids, L, 2.8)
    xs, vs, ts, io, cs = ops.bin(L, 2.8, T(x, dev), T(v, dev), T(ty, dev), T(ids, dev))
    assert np.array_equal(io.cpu().numpy(), ids[perm])
    assert np.array_equal(vs.cpu().numpy(), v[perm])
    assert np.array_equal(ts.cpu().numpy(), ty[perm])
    assert np.array_equal(cs.cpu().numpy(), cell_start)
    # deterministic: a second sort of the sorted output is the identity
    xs2, _, _, io2, _ = ops.bin(L, 2.8, xs, None, None, io)
    assert torch.equal(xs2, xs) and torch.equal(io2, io)


def test_bin_empty(dev):
    import torch
    from paper_2109_09056_amd import ops
    x = torch.zeros(0, 3, dtype=torch.float64, device=dev)
    xs, _, _, ids, cs = ops.bin((9.0, 9.0, 9.0), 2.8, x)
    assert xs.shape == (0, 3) and int(cs.cpu().max()) == 0


# ---------------------------------------------------------------- neighbors --

def gpu_lists(dev, x, L, rlist, kind, maxn=None):
    from paper_2109_09056_amd import md
    xs, _, _, ids, cs = gpu_sort(dev, x, L, rlist)
    nl = md.NeighborList(L, rlist, kind, maxn=maxn, device=dev).build(xs, cs)
    return nl, ids, xs


NBR_CASES = ["lj256", "lj32k", "gas_ragged", "gas_long", "clump", "tiny", "slab",
             "cutoff_lattice", "gas_three_cells", "gas_tight_cells"]


def cutoff_lattice():
    """Simple-cubic lattice of spacing rlist / 2 = 1.4 on 16^3 sites (7 binning cells per
    axis), every coordinate moved by at most 1e-9: each atom's six second-axis neighbours
    sit at rlist to within ~3e-9, so about half of those pairs are in the list and which
    ones is decided by FP64 rounding -- the build's integer pre-test must hand every such
    pair to the FP64 test."""
    a = 1.4
    g = np.stack(np.meshgrid(*[np.arange(16)] * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    L = np.full(3, 16 * a)
    x = (g + 0.5) * a + np.random.default_rng(31).uniform(-1e-9, 1e-9, g.shape)
    return np.mod(x, L), L


def slab_positions():
    """A jittered simple-cubic lattice at the liquid's number density (0.8442) in a
    22 x 28 x 150 lattice-cell slab: 92,400 atoms, 8 x 10 x 56 binning cells at rlist 2.8
    (unequal counts per axis), every row of the list and every force at that size."""
    a = (1.0 / 0.8442) ** (1.0 / 3.0)
    nx, ny, nz = 22, 28, 150
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                 axis=-1).reshape(-1, 3).astype(np.float64)
    L = a * np.array([nx, ny, nz], dtype=np.float64)
    x = (g + 0.5 + np.random.default_rng(29).uniform(-0.1, 0.1, g.shape)) * a
    return np.mod(x, L), L


def case_positions(name):
    if name in li.WORKLOADS:
        w = li.WORKLOADS[name]
        return li.positions(w), w.box
    if name == "gas_ragged":
        L = np.array([6.0, 7.5, 9.0])
        return gas(331, L, 17), L
    if name == "gas_long":
        L = np.array([5.8, 5.8, 17.0])
        return gas(450, L, 19), L
    if name == "clump":
        L = np.array([14.0, 15.0, 16.0])
        return clumped(900, 700, L, 5), L
    if name == "tiny":
        L = np.array([6.0, 6.0, 6.0])
        return gas(3, L, 23), L
    if name == "slab":
        return slab_positions()
    if name == "cutoff_lattice":
        return cutoff_lattice()
    if name == "gas_three_cells":
        # 3 x 3 x 4 binning cells: the fewest per axis that take the build's integer
        # pre-test, where the stencil wraps on every side
        L = np.array([8.5, 8.9, 11.5])
        return gas(800, L, 41), L
    if name == "gas_tight_cells":
        # 3 x 3 x 4 cells whose edge exceeds rlist = 2.8 by 1e-7
        L = np.array([8.4000003, 8.4000003, 11.2000004])
        return gas(700, L, 43), L
    raise KeyError(name)


@pytest.mark.parametrize("kind", ["full", "half"])
@pytest.mark.parametrize("name", NBR_CASES)
def test_neighbor_sets_match_oracle(dev, orc, name, kind):
    from paper_2109_09056_amd import ops
    x, L = case_positions(name)
    k = ops.FULL if kind == "full" else ops.HALF
    nl, ids, _ = gpu_lists(dev, x, L, 2.8, k)
    got = gpu_pairs_by_id(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn,
                          ids.cpu().numpy(), half=(kind == "half"))
    off, nb = orc.neighbor_lists(x, L, 2.8)
    want = oracle_pairs(off, nb, half=(kind == "half"))
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    if kind == "half":
        # each unordered pair stored once, owned by the lower sorted index
        rows_total = int(nl.nnbr.sum().item())
        assert rows_total == want.shape[0]


@pytest.mark.parametrize("kind", ["full", "half"])
@pytest.mark.parametrize("case", ["sph4k", "lj32k"])
def test_neighbor_sets_dense_build_shape(dev, orc, case, kind):
    """Row capacity above 128 selects the build's dense shape (16 register slots, rows of
    up to 256 entries compacted in LDS): the SPH fluid at rlist 3.0 (~790 candidates per
    stencil) and the LJ liquid, both against the oracle."""
    from paper_2109_09056_amd import ops
    if case == "sph4k":
        w = li.SPH_WORKLOADS[case]
        x, L, rl = li.sph_positions(w), w.box, w.rlist
    else:
        w = li.WORKLOADS[case]
        x, L, rl = li.positions(w), w.box, w.rlist
    k = ops.FULL if kind == "full" else ops.HALF
    nl, ids, _ = gpu_lists(dev, x, L, rl, k, maxn=200)
    assert nl.maxn == 200 and nl.overflows == 0
    got = gpu_pairs_by_id(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn,
                          ids.cpu().numpy(), half=(kind == "half"))
    off, nb = orc.neighbor_lists(x, L, rl)
    assert np.array_equal(got, oracle_pairs(off, nb, half=(kind == "half")))


def stencil_pairs(x, L, rlist):
    """(i, j) pairs, i != j, that the cell build tests when positions may lie outside
    [0, L): atom j's cell (floor(x / h), clamped to the grid as binning clamps it) is one
    of the 27 around atom i's cell, and the minimum-image r^2 = (dx^2 + dy^2) + dz^2 is
    below rlist^2.  For positions inside the box this is every pair within rlist."""
    L = np.asarray(L, dtype=np.float64)
    nc = np.floor(L / rlist).astype(np.int64)
    for k in range(3):
        while nc[k] > 1 and L[k] / nc[k] < rlist * (1.0 + 1e-10):
            nc[k] -= 1
    h = L / nc
    cell = np.clip(np.floor(x / h).astype(np.int64), 0, nc - 1)
    n = x.shape[0]
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i, j = i.ravel(), j.ravel()
    dc = (cell[i] - cell[j]) % nc
    adj = np.all((dc == 0) | (dc == 1) | (dc == nc - 1), axis=1) & (i != j)
    d = x[i] - x[j]
    d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    keep = adj & (r2 < rlist * rlist)
    return i[keep], j[keep]


@pytest.mark.parametrize("kind", ["full", "half"])
def test_neighbor_sets_positions_outside_the_box(dev, kind):
    """Outside the documented range (positions in [0, L) at build time): atoms up to 1.4
    cell edges beyond a face are binned into the face cells.  The build then matches the
    stencil-restricted FP64 test exactly -- the wavefronts that see such atoms leave the
    integer pre-test for the FP64 path."""
    from paper_2109_09056_amd import ops
    L = np.array([15.0, 16.0, 17.0])
    x = li.random_gas(2000, L, 37)
    h = L / np.array([5, 5, 6])
    x[:40, 0] = L[0] + np.linspace(0.05, 1.4, 40) * h[0]
    x[40:60, 2] = -np.linspace(0.05, 1.4, 20) * h[2]
    k = ops.FULL if kind == "full" else ops.HALF
    nl, ids, _ = gpu_lists(dev, x, L, 2.8, k)
    got = gpu_pairs_by_id(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn,
                          ids.cpu().numpy(), half=(kind == "half"))
    i, j = stencil_pairs(x, L, 2.8)
    if kind == "half":
        i, j = np.minimum(i, j), np.maximum(i, j)
        a = np.unique(np.stack([i, j], 1), axis=0)
        i, j = a[:, 0], a[:, 1]
    from helpers import pair_array
    assert np.array_equal(got, pair_array(i, j))


@pytest.mark.parametrize("case", ["lj256", "lj32k"])
def test_neighbor_capacity_overflow_reported(dev, orc, case):
    """Rows cut at maxn = 10 keep true neighbours and report the longest row: on a
    2-cell grid (FP64-staged build) and an 11-cell grid (integer pre-test)."""
    from paper_2109_09056_amd import ops
    w = li.WORKLOADS[case]
    x = li.positions(w)
    xs, _, _, ids, cs = gpu_sort(dev, x, w.box, w.rlist)
    nbr, nnbr, mc = ops.build_neighbors(w.box, w.rlist, ops.FULL, xs, cs, 10)
    off, nb = orc.neighbor_lists(x, w.box, w.rlist)
    assert int(mc.item()) == int(np.diff(off).max())
    assert int(nnbr.max().item()) == 10
    # the first 10 entries kept in each cut row are true neighbours
    got = gpu_pairs_by_id(nbr.cpu().numpy(), nnbr.cpu().numpy(), 10, ids.cpu().numpy())
    want = oracle_pairs(off, nb)
    assert got.shape[0] == 10 * x.shape[0]
    assert np.all(np.isin(got[:, 0] * x.shape[0] + got[:, 1], want[:, 0] * x.shape[0] + want[:, 1]))
    # the driver grows maxn until nothing is cut
    from paper_2109_09056_amd import md
    nl = md.NeighborList(w.box, w.rlist, ops.FULL, maxn=10, device=dev).build(xs, cs)
    assert nl.overflows == 1 and nl.maxn >= int(np.diff(off).max())
    got = gpu_pairs_by_id(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn, ids.cpu().numpy())
    assert np.array_equal(got, oracle_pairs(off, nb))


# ------------------------------------------------------------------- forces --

def gpu_forces(dev, x, L, precision, kind, eps=(1.0,), sigma=(1.0,), types=None, rc=2.5,
               skin=0.3):
    import torch
    from paper_2109_09056_amd import ops
    nl, ids, xs = gpu_lists(dev, x, L, rc + skin, kind)
    n = x.shape[0]
    ty = T(types if types is not None else np.zeros(n, np.int32), dev, torch.int32)
    ts = ops.gather_rows(ids, ty.to(torch.float64)).to(torch.int32)
    F, e, ev = ops.compute_forces(L, precision, kind, rc, T(eps, dev, torch.float64),
                                  T(sigma, dev, torch.float64), xs, ts, nl.nbr, nl.nnbr, nl.maxn)
    F = ops.scatter_rows(ids, F).cpu().numpy()
    e = ops.scatter_rows(ids, e).cpu().numpy()
    return F, e, ev.cpu().numpy()


def check_fp64(F, e, ev, Fo, eo, Wo):
    assert max_rel_vec(F, Fo) <= FP64_TOL
    assert np.abs(e - eo).max() <= FP64_TOL * np.abs(eo).max()
    assert abs(ev[0] - eo.sum()) <= FP64_TOL * abs(eo.sum())
    wscale = np.abs(Wo[:3]).max()
    assert np.abs(ev[1:] - Wo).max() <= FP64_TOL * wscale


def check_mixed(F, e, Fo, eo):
    frms = np.sqrt((Fo * Fo).sum() / Fo.shape[0])
    err_f = np.linalg.norm(F - Fo, axis=1).max() / frms
    err_e = (np.abs(e - eo) / np.maximum(np.abs(eo), 1e-3)).max()
    assert err_f <= MIXED_F_TOL, err_f
    assert err_e <= MIXED_E_TOL, err_e
    return err_f, err_e


SYSTEMS = {
    "lj256": lambda: (li.positions(li.WORKLOADS["lj256"]), li.WORKLOADS["lj256"].box, None, [1.0],
                      [1.0]),
    "lj32k": lambda: (li.positions(li.WORKLOADS["lj32k"]), li.WORKLOADS["lj32k"].box, None, [1.0],
                      [1.0]),
    "lj32k_fm": lambda: (li.positions(li.WORKLOADS["lj32k_fm"]), li.WORKLOADS["lj32k_fm"].box,
                         li.types(li.WORKLOADS["lj32k_fm"]), *li.params(li.WORKLOADS["lj32k_fm"])),
    "three_types": lambda: (li.positions(li.WORKLOADS["lj256"]), li.WORKLOADS["lj256"].box,
                            (np.arange(256) % 3).astype(np.int32),
                            np.array([1.0, 0.9, 1.1, 1.2, 0.8, 1.05]),
                            np.array([1.0, 0.95, 1.02, 1.05, 0.92, 0.97])),
    # 70,304 atoms, two types: the kernels' mid-size shapes (two lanes per atom on the
    # full list, 128-atom blocks with four lanes on the half list)
    "lj70k_2t": lambda: (lambda w: (li.positions(w), w.box, li.types(w), *li.params(w)))(
        li.Workload("lj70k_2t", 7, cells=26, ntypes=2)),
    "slab": lambda: (*slab_positions(), None, [1.0], [1.0]),
}


@pytest.fixture(scope="module")
def oracle_forces_cache(orc):
    cache = {}

    def get(name):
        if name not in cache:
            x, L, ty, eps, sig = SYSTEMS[name]()
            cache[name] = (x, L, ty, eps, sig, orc.forces(x, L, 2.5, eps, sig, ty))
        return cache[name]
    return get


@pytest.mark.parametrize("kind", ["full", "half"])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_forces_fp64(dev, oracle_forces_cache, name, kind):
    from paper_2109_09056_amd import ops
    x, L, ty, eps, sig, (Fo, eo, Wo, _) = oracle_forces_cache(name)
    k = ops.FULL if kind == "full" else ops.HALF
    F, e, ev = gpu_forces(dev, x, L, ops.FP64, k, eps, sig, ty)
    check_fp64(F, e, ev, Fo, eo, Wo)


@pytest.mark.parametrize("kind", ["full", "half"])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_forces_mixed(dev, oracle_forces_cache, name, kind):
    from paper_2109_09056_amd import ops
    x, L, ty, eps, sig, (Fo, eo, Wo, _) = oracle_forces_cache(name)
    k = ops.FULL if kind == "full" else ops.HALF
    F, e, ev = gpu_forces(dev, x, L, ops.MIXED, k, eps, sig, ty)
    err_f, err_e = check_mixed(F, e, Fo, eo)
    print(f"[{name}/{kind}] mixed max|dF|/Frms = {err_f:.3e}  max rel de = {err_e:.3e}")
    assert abs(ev[0] - eo.sum()) <= 1e-6 * abs(eo.sum())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_half_forces_in_scrambled_order(dev, orc, oracle_forces_cache, prec):
    """The half-list kernel on the 32k liquid with its atoms (and list indices) put in a
    random order: every block then touches far more 64-atom tiles than it keeps j-side
    sums for, so most pairs take the direct-atomic path.  Forces, energies and virial
    against the oracle."""
    import torch
    from helpers import list_pairs
    from paper_2109_09056_amd import ops
    x, L, _, eps, sig, (Fo, eo, Wo, _) = oracle_forces_cache("lj32k")
    n = x.shape[0]
    nl, ids, xs = gpu_lists(dev, x, L, 2.8, ops.HALF)
    i, j = list_pairs(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn)
    perm = np.random.default_rng(3).permutation(n)  # sorted position k -> new position perm[k]
    ni, nj = perm[i], perm[j]
    order = np.argsort(ni, kind="stable")
    ni, nj = ni[order], nj[order]
    cnt = np.bincount(ni, minlength=n)
    maxn = int(cnt.max())
    tiles = (n + 63) // 64
    nbr = np.zeros((tiles, maxn, 64), dtype=np.int32)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    k = np.arange(ni.size) - start[ni]
    nbr[ni // 64, k, ni % 64] = nj
    x_new = np.empty((n, 3))
    x_new[perm] = xs.cpu().numpy()
    ids_new = np.empty(n, dtype=np.int64)
    ids_new[perm] = ids.cpu().numpy()
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    one = T([1.0], dev, torch.float64)
    F, e, ev = ops.compute_forces(L, P, ops.HALF, 2.5, one, one, T(x_new, dev),
                                  torch.zeros(n, dtype=torch.int32, device=dev),
                                  T(nbr.reshape(-1), dev), T(cnt.astype(np.int32), dev), maxn)
    Fg, eg = np.empty((n, 3)), np.empty(n)
    Fg[ids_new] = F.cpu().numpy()
    eg[ids_new] = e.cpu().numpy()
    if P == ops.FP64:
        check_fp64(Fg, eg, ev.cpu().numpy(), Fo, eo, Wo)
    else:
        check_mixed(Fg, eg, Fo, eo)


def test_forces_full_list_bitwise_deterministic(dev):
    import torch
    from paper_2109_09056_amd import ops
    w = li.WORKLOADS["lj32k"]
    x = li.positions(w)
    nl, ids, xs = gpu_lists(dev, x, w.box, w.rlist, ops.FULL)
    one = T([1.0], dev, torch.float64)
    ty = torch.zeros(x.shape[0], dtype=torch.int32, device=dev)
    for prec in (ops.FP64, ops.MIXED):
        a = ops.compute_forces(w.box, prec, ops.FULL, 2.5, one, one, xs, ty, nl.nbr, nl.nnbr,
                               nl.maxn)
        a = [t.clone() for t in a]
        b = ops.compute_forces(w.box, prec, ops.FULL, 2.5, one, one, xs, ty, nl.nbr, nl.nnbr,
                               nl.maxn)
        for p, q in zip(a, b):
            assert torch.equal(p, q)


def test_forces_without_energy_outputs(dev, oracle_forces_cache):
    import torch
    from paper_2109_09056_amd import ops
    x, L, ty, eps, sig, (Fo, eo, Wo, _) = oracle_forces_cache("lj256")
    nl, ids, xs = gpu_lists(dev, x, L, 2.8, ops.FULL)
    one = T([1.0], dev, torch.float64)
    tz = torch.zeros(x.shape[0], dtype=torch.int32, device=dev)
    F, e, ev = ops.compute_forces(L, ops.FP64, ops.FULL, 2.5, one, one, xs, tz, nl.nbr, nl.nnbr,
                                  nl.maxn, want_energy=False)
    assert e is None and ev is None
    assert max_rel_vec(ops.scatter_rows(ids, F).cpu().numpy(), Fo) <= FP64_TOL


@pytest.mark.parametrize("kind", ["full", "half"])
def test_energy_and_virial_without_atom_energies(dev, orc, oracle_forces_cache, kind):
    """E and W with no per-atom energy array (e_atom NULL): the half list then takes its
    three-accumulator kernel.  Forces, E and W against the oracle at the FP64 bar, on a
    32,000-atom liquid (the half list's 128-atom, eight-lane shape)."""
    import torch
    from paper_2109_09056_amd import ops
    x, L, ty, eps, sig, (Fo, eo, Wo, _) = oracle_forces_cache("lj32k")
    k = ops.FULL if kind == "full" else ops.HALF
    nl, ids, xs = gpu_lists(dev, x, L, 2.8, k)
    one = T([1.0], dev, torch.float64)
    tz = torch.zeros(x.shape[0], dtype=torch.int32, device=dev)
    F, e, ev = ops.compute_forces(L, ops.FP64, k, 2.5, one, one, xs, tz, nl.nbr, nl.nnbr,
                                  nl.maxn, atom_energy=False)
    assert e is None
    assert max_rel_vec(ops.scatter_rows(ids, F).cpu().numpy(), Fo) <= FP64_TOL
    ev = ev.cpu().numpy()
    assert abs(ev[0] - eo.sum()) <= FP64_TOL * abs(eo.sum())
    assert np.abs(ev[1:] - Wo).max() <= FP64_TOL * np.abs(Wo[:3]).max()


def test_forces_empty(dev):
    import torch
    from paper_2109_09056_amd import ops
    x = torch.zeros(0, 3, dtype=torch.float64, device=dev)
    one = T([1.0], dev, torch.float64)
    nbr = torch.zeros(64 * 8, dtype=torch.int32, device=dev)
    nnbr = torch.zeros(0, dtype=torch.int32, device=dev)
    t = torch.zeros(0, dtype=torch.int32, device=dev)
    for kind in (ops.FULL, ops.HALF):
        F, e, ev = ops.compute_forces((9.0, 9.0, 9.0), ops.FP64, kind, 2.5, one, one, x, t, nbr,
                                      nnbr, 8)
        assert F.shape == (0, 3) and float(ev.abs().sum().item()) == 0.0


# ------------------------------------------------------- 500k, sampled rows --

@pytest.fixture(scope="module")
def big(dev):
    """500,000-atom jittered fcc liquid start, sorted and listed exactly as the benchmark does."""
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj500k"]
    s = li.make_system(w)
    sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=ops.MIXED, kind=ops.FULL, dt=w.dt,
                   rebuild_every=w.rebuild_every, device=dev)
    sim.load(s["x"], s["v"])
    return w, s, sim


def test_500k_sampled_neighbors_and_forces(dev, orc, big):
    """Sampled atoms of the 500k start: oracle rows over all 500k atoms, by original id."""
    import torch
    from helpers import decode_rows
    from paper_2109_09056_amd import ops
    w, s, sim = big
    n = w.natoms
    x = s["x"]
    ids = sim.ids.cpu().numpy()
    assert np.array_equal(np.sort(ids), np.arange(n))
    pos_of = np.empty(n, dtype=np.int64)
    pos_of[ids] = np.arange(n)
    atoms = np.sort(np.random.default_rng(0).choice(n, 1500, replace=False))  # original ids
    rows = decode_rows(sim.nl.nbr.cpu().numpy(), sim.nl.nnbr.cpu().numpy(), sim.nl.maxn)
    off, nb = orc.neighbor_lists(x, w.box, w.rlist, sel=atoms)
    for k, a in enumerate(atoms):
        got = np.sort(ids[rows[pos_of[a]]])
        assert np.array_equal(got, nb[off[k]:off[k + 1]])
    Fo, eo, _, _ = orc.forces(x, w.box, w.rc, sel=atoms)
    one = T([1.0], dev, torch.float64)
    for prec in (ops.MIXED, ops.FP64):
        F, e, _ = ops.compute_forces(w.box, prec, ops.FULL, w.rc, one, one, sim.x, sim.types,
                                     sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn)
        Fs = F.cpu().numpy()[pos_of[atoms]]
        es = e.cpu().numpy()[pos_of[atoms]]
        if prec == ops.FP64:
            assert (np.linalg.norm(Fs - Fo, axis=1).max()
                    <= FP64_TOL * np.linalg.norm(Fo, axis=1).max())
            assert np.abs(es - eo).max() <= FP64_TOL * np.abs(eo).max()
        else:
            frms = np.sqrt((Fo * Fo).sum() / Fo.shape[0])
            assert np.linalg.norm(Fs - Fo, axis=1).max() <= MIXED_F_TOL * frms
            assert (np.abs(es - eo) / np.abs(eo)).max() <= MIXED_E_TOL


@pytest.mark.timeout(900)
def test_500k_every_row_full_and_half(dev, orc):
    """Every row of the 500k start's full and half lists, by original id, against the
    oracle's brute-force relation over all pairs (1.25e11 pair tests): the full list holds
    each unordered pair in both directions and nothing else, the half list each once."""
    from helpers import list_pairs
    from paper_2109_09056_amd import md, ops
    w = li.WORKLOADS["lj500k"]
    x = li.positions(w)
    n = w.natoms
    up = orc.upper_pairs(x, w.box, w.rlist)
    key = up[:, 0] * n + up[:, 1]  # ascending: rows by i, then j
    del up
    xs, _, _, ids, cs = ops.bin(w.box, w.rlist, T(x, dev, None))
    ids = ids.cpu().numpy()
    for kind in (ops.FULL, ops.HALF):
        nl = md.NeighborList(w.box, w.rlist, kind, device=dev).build(xs, cs)
        i, j = list_pairs(nl.nbr.cpu().numpy(), nl.nnbr.cpu().numpy(), nl.maxn)
        a, b = ids[i], ids[j]
        del i, j, nl
        if kind == ops.FULL:
            assert a.size == 2 * key.size
            lo = a < b
            assert np.array_equal(np.sort(a[lo] * n + b[lo]), key)
            assert np.array_equal(np.sort(b[~lo] * n + a[~lo]), key)
        else:
            assert a.size == key.size
            assert np.array_equal(np.sort(np.minimum(a, b) * n + np.maximum(a, b)), key)


def test_500k_steps_properties(dev, big):
    """40 steps (two rebuilds) at 500k: momentum stays zero, mixed and FP64 runs from the
    same start stay together, and the full list stays symmetric."""
    import torch
    from paper_2109_09056_amd import md, ops
    w, s, sim = big
    ref = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=ops.FP64, kind=ops.FULL, dt=w.dt,
                   device=dev)
    ref.load(s["x"], s["v"])
    e0 = sim.thermo()["etot"]
    sim.step(40)
    ref.step(40)
    th = sim.thermo()
    assert th["builds"] >= 3 and np.isfinite(th["etot"])
    assert abs(th["etot"] - e0) / w.natoms < 1e-2
    assert sim.v.sum(dim=0).abs().max().item() < 1e-8
    xm = sim.in_caller_order(sim.x).cpu().numpy()
    xf = ref.in_caller_order(ref.x).cpu().numpy()
    d = xm - xf
    d -= w.box * np.round(d / w.box)
    # FP32 pair-math noise (~1e-7 relative in F) grows chaotically in a few colliding atoms
    assert np.sqrt((d * d).mean()) < 1e-7 and np.abs(d).max() < 1e-3
    nn = sim.nl.nnbr.to(torch.int64)
    assert int(nn.sum().item()) % 2 == 0


def test_wide_indices_17m(dev, orc):
    """17,006,112 atoms (fcc 162^3 cells): sorted indices above 2^24 take the wide
    (64-bit) gather addressing.  Sampled rows and forces, several of them above 2^24,
    against the oracle over all atoms; the fused step against the separate calls."""
    import torch
    from paper_2109_09056_amd import md, ops
    w = li.Workload("fcc162", 5, cells=162)
    x = li.positions(w)
    n = x.shape[0]
    assert n > (1 << 24)
    sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, precision=ops.MIXED, kind=ops.FULL, dt=w.dt,
                   device=dev)
    sim.load(x, None)
    # samples chosen from the generator's positions: atoms of the top cell layer in z
    # sort last (cell-major order), so their sorted indices lie above 2^24
    nc = orc.grid(w.box, w.rlist)
    hz = w.box[2] / nc[2]
    rng = np.random.default_rng(1)
    top = np.nonzero(x[:, 2] >= (nc[2] - 1) * hz * (1 + 1e-12))[0]
    ids = np.sort(np.concatenate([rng.choice(n, 16, replace=False),
                                  rng.choice(top, 32, replace=False)]))
    ids = np.unique(ids)
    inv = torch.empty(n, dtype=torch.int64, device=dev)
    inv[sim.ids] = torch.arange(n, device=dev)
    p = inv[torch.as_tensor(ids, device=dev)]
    pos = p.cpu().numpy()
    assert (pos >= (1 << 24)).sum() >= 32
    cnt = sim.nl.nnbr[p].to(torch.int64)
    k = torch.arange(sim.nl.maxn, device=dev)
    flat = ((p[:, None] >> 6) * sim.nl.maxn + k[None, :]) * 64 + (p[:, None] & 63)
    ent = sim.nl.nbr.reshape(-1)[flat.clamp(max=sim.nl.nbr.numel() - 1)].to(torch.int64)
    # slots past a row's count are unused memory: clamp before indexing, keep only :cnt
    rows = sim.ids[ent.clamp(min=0, max=n - 1)].cpu().numpy()
    cnt = cnt.cpu().numpy()
    off, nb = orc.neighbor_lists(x, w.box, w.rlist, sel=ids)
    for q in range(len(ids)):
        assert np.array_equal(np.sort(rows[q, :cnt[q]]), nb[off[q]:off[q + 1]]), q
    Fo, eo, _, _ = orc.forces(x, w.box, w.rc, sel=ids)
    one = T([1.0], dev, torch.float64)
    for prec in (ops.MIXED, ops.FP64):
        F, e, _ = ops.compute_forces(w.box, prec, ops.FULL, w.rc, one, one, sim.x, sim.types,
                                     sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn)
        Fs, es = F[p].cpu().numpy(), e[p].cpu().numpy()
        if prec == ops.FP64:
            assert (np.linalg.norm(Fs - Fo, axis=1).max()
                    <= FP64_TOL * np.linalg.norm(Fo, axis=1).max())
            assert np.abs(es - eo).max() <= FP64_TOL * np.abs(eo).max()
        else:
            frms = np.sqrt((Fo * Fo).sum() / Fo.shape[0])
            assert np.linalg.norm(Fs - Fo, axis=1).max() <= MIXED_F_TOL * frms
            assert (np.abs(es - eo) / np.abs(eo)).max() <= MIXED_E_TOL
        del F, e
    # Ewald real space on the wide path: unit charges, the same sampled rows against the
    # oracle's direct sum over all atoms
    q = li.charges(w)
    qs = ops.gather_rows(sim.ids, torch.as_tensor(q, dtype=torch.float64, device=dev))
    Fq, _ = ops.ewald_real(w.box, li.EWALD_ALPHA, w.rc, sim.x, qs, sim.nl.nbr, sim.nl.nnbr,
                           sim.nl.maxn)
    _, Fq_o = orc.ewald_direct(x, q, w.box, li.EWALD_ALPHA, w.rc, sel=ids)
    assert np.abs(Fq[p].cpu().numpy() - Fq_o).max() <= 1e-12 * np.abs(Fq_o).max()
    del Fq, qs
    # fused step == forces + closing kick + opening kick/drift, bitwise, on the wide path
    v1 = torch.zeros_like(sim.x)
    xn, F1, ev1 = ops.md_step(w.box, ops.MIXED, w.rc, one, one, sim.x, sim.types, sim.nl.nbr,
                              sim.nl.nnbr, sim.nl.maxn, w.dt, 1.0, v1, F=torch.empty_like(sim.x))
    F2, _, ev2 = ops.compute_forces(w.box, ops.MIXED, ops.FULL, w.rc, one, one, sim.x, sim.types,
                                    sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn)
    assert torch.equal(F1, F2) and torch.equal(ev1[:7], ev2)
    x2, v2 = sim.x.clone(), torch.zeros_like(sim.x)
    ops.integrate(ops.KICK, w.dt, 1.0, w.box, x2, v2, F2)
    ops.integrate(ops.KICK_DRIFT, w.dt, 1.0, w.box, x2, v2, F2)
    assert torch.equal(v1, v2) and torch.equal(xn, x2)
    del xn, F1, F2, v1, v2, x2
    # adjoint on the wide path (FP64): directional derivatives of g.F by central
    # differences, along a displacement of 64 atoms (half of them above 2^24) and
    # along eps and sigma; the pair set is fixed (no moved pair within 1e-4 of rc)
    h = 1e-6
    g = torch.as_tensor(np.random.default_rng(2).normal(size=(n, 3)), device=dev)
    gx, geps, gsig = ops.force_backward(w.box, ops.FP64, w.rc, one, one, sim.x, sim.types,
                                        sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn, g)
    mids = np.unique(np.concatenate([rng.choice(n, 32, replace=False),
                                     rng.choice(top, 32, replace=False)]))
    off2, nb2 = orc.neighbor_lists(x, w.box, w.rlist, sel=mids)
    for q, a_ in enumerate(mids):
        d = x[nb2[off2[q]:off2[q + 1]]] - x[a_]
        d -= w.box * np.round(d / w.box)
        assert np.abs(np.sqrt((d * d).sum(1)) - w.rc).min() > 1e-4
    moved = inv[torch.as_tensor(mids, device=dev)]
    assert int((moved >= (1 << 24)).sum()) >= 32
    wdir = torch.zeros_like(sim.x)
    wdir[moved] = torch.as_tensor(np.random.default_rng(3).normal(size=(len(mids), 3)),
                                  device=dev)

    def gF(xx, e=one, sg=one):
        F, _, _ = ops.compute_forces(w.box, ops.FP64, ops.FULL, w.rc, e, sg, xx, sim.types,
                                     sim.nl.nbr, sim.nl.nnbr, sim.nl.maxn, want_energy=False)
        return float((g * F).sum().item())

    fd = (gF(sim.x + h * wdir) - gF(sim.x - h * wdir)) / (2 * h)
    assert fd == pytest.approx(float((wdir * gx).sum().item()), rel=1e-5)
    fe = (gF(sim.x, e=one * (1 + h)) - gF(sim.x, e=one * (1 - h))) / (2 * h)
    assert fe == pytest.approx(float(geps.item()), rel=1e-6)
    fs = (gF(sim.x, sg=one * (1 + h)) - gF(sim.x, sg=one * (1 - h))) / (2 * h)
    assert fs == pytest.approx(float(gsig.item()), rel=1e-5)
