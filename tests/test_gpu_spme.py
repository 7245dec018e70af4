"""Smooth particle-mesh Ewald on the GPU against the CPU oracles: the direct-space
pair kernel against the Ewald direct sum, the reciprocal part against the SPME
reference steps (same grid and order), the whole sum against the exact Ewald sum
and the rock-salt Madelung constant, a 500,000-particle sampled check, edge cases."""
import numpy as np
import pytest

import lj_inputs as li
from helpers import gpu_device

pytestmark = pytest.mark.gpu

ALPHA = li.EWALD_ALPHA
RC = 2.5


@pytest.fixture(scope="module")
def dev():
    return gpu_device()


def _sorted(dev, x, q, L, rlist):
    """Cell-sorted positions, charges in that order, ids and a FULL list."""
    import torch
    from paper_2109_09056_amd import md, ops
    xt = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    xs, _, _, ids, cs = ops.bin(L, rlist, xt)
    qs = ops.gather_rows(ids, torch.as_tensor(q, dtype=torch.float64, device=dev).contiguous())
    nl = md.NeighborList(L, rlist, ops.FULL, device=dev).build(xs, cs)
    return xs, qs, ids, nl


def _case(name):
    if name in li.WORKLOADS:
        w = li.WORKLOADS[name]
        return li.positions(w), li.charges(w), w.box
    if name == "gas1000":  # ragged n, random charges of both signs, neutral
        L = np.array([11.0, 12.0, 13.0])
        g = np.random.default_rng(8)
        q = g.uniform(-1.5, 1.5, 1000)
        return li.random_gas(1000, L, 31), q - q.mean(), L
    if name == "gas400":  # small box: the k-space reference sum converges at nmax 18
        L = np.array([8.0, 9.0, 10.0])
        g = np.random.default_rng(9)
        q = g.uniform(-1.5, 1.5, 400)
        return li.random_gas(400, L, 33), q - q.mean(), L
    raise KeyError(name)


@pytest.mark.parametrize("name", ["lj256", "gas1000", "lj32k"])
def test_real_space_vs_oracle(dev, orc, name):
    from paper_2109_09056_amd import ops
    x, q, L = _case(name)
    xs, qs, ids, nl = _sorted(dev, x, q, L, RC + 0.3)
    F, E = ops.ewald_real(L, ALPHA, RC, xs, qs, nl.nbr, nl.nnbr, nl.maxn, want_energy=True)
    e_o, F_o = orc.ewald_direct(x, q, L, ALPHA, RC)
    Fg = ops.scatter_rows(ids, F).cpu().numpy()
    assert np.abs(Fg - F_o).max() <= 1e-12 * np.abs(F_o).max()
    assert E.item() == pytest.approx(e_o.sum(), rel=1e-12)


SPME_CASES = [("lj256", (16, 16, 16), 4), ("gas1000", (16, 32, 8), 6),
              ("gas1000", (32, 32, 32), 8), ("lj32k", (64, 64, 64), 4),
              # the smallest and largest x edges (x pass of 4 and 128 complex points)
              ("lj256", (8, 16, 32), 4), ("gas1000", (256, 8, 16), 6)]


@pytest.mark.parametrize("name,K,order", SPME_CASES)
def test_spme_recip_vs_oracle(dev, orc, name, K, order):
    """Same grid and order as the reference steps: only rounding differs (FFT order,
    atomic spreading), so 1e-11 of the largest force and of the energy."""
    import torch
    from paper_2109_09056_amd import ops
    x, q, L = _case(name)
    xt = torch.as_tensor(x, dtype=torch.float64, device=dev)
    qt = torch.as_tensor(q, dtype=torch.float64, device=dev)
    F, E = ops.spme_recip(L, ALPHA, order, K, xt, qt, want_energy=True)
    E_o, F_o = orc.spme_recip(x, q, L, ALPHA, K, order)
    E_o += orc.ewald_self(q, ALPHA)
    assert np.abs(F.cpu().numpy() - F_o).max() <= 1e-11 * np.abs(F_o).max()
    assert E.item() == pytest.approx(E_o, rel=1e-11)


def test_full_sum_matches_exact_ewald(dev, orc):
    """Direct + reciprocal (K = 64, order 8) + self against the k-space Ewald sum."""
    import torch
    from paper_2109_09056_amd import ops
    x, q, L = _case("gas400")
    xs, qs, ids, nl = _sorted(dev, x, q, L, RC + 0.3)
    F, Ed = ops.ewald_real(L, ALPHA, RC, xs, qs, nl.nbr, nl.nnbr, nl.maxn, want_energy=True)
    F, Er = ops.spme_recip(L, ALPHA, 8, (64, 64, 64), xs, qs, F=F, want_energy=True,
                           accumulate=True)
    e_o, Fd_o = orc.ewald_direct(x, q, L, ALPHA, RC)
    Er_o, Fr_o = orc.ewald_recip(x, q, L, ALPHA, 18)
    E_o = e_o.sum() + Er_o + orc.ewald_self(q, ALPHA)
    F_o = Fd_o + Fr_o
    Fg = ops.scatter_rows(ids, F).cpu().numpy()
    assert Ed.item() + Er.item() == pytest.approx(E_o, rel=1e-7)
    assert np.abs(Fg - F_o).max() <= 1e-6 * np.abs(F_o).max()
    assert torch.isfinite(F).all()


def test_rock_salt_madelung_on_gpu(dev):
    """512 ions of rock salt, spacing 1: E per ion pair = -1.747565 (nearest distance 1)."""
    import torch
    from paper_2109_09056_amd import ops
    m = 8
    idx = np.arange(m)
    I = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    x = I + 0.25
    q = np.where(I.sum(1) % 2 == 0, 1.0, -1.0)
    L = np.full(3, float(m))
    alpha, rc = 1.0, 3.9
    xs, qs, ids, nl = _sorted(dev, x, q, L, rc)
    _, Ed = ops.ewald_real(L, alpha, rc, xs, qs, nl.nbr, nl.nnbr, nl.maxn, want_energy=True)
    _, Er = ops.spme_recip(L, alpha, 8, (64, 64, 64), xs, qs, want_energy=True)
    assert (Ed.item() + Er.item()) / (len(q) / 2) == pytest.approx(-1.747564594633182, rel=1e-6)


def test_accumulate_and_empty(dev):
    import torch
    from paper_2109_09056_amd import ops
    x, q, L = _case("lj256")
    xs, qs, ids, nl = _sorted(dev, x, q, L, RC + 0.3)
    F0, _ = ops.ewald_real(L, ALPHA, RC, xs, qs, nl.nbr, nl.nnbr, nl.maxn)
    F1 = torch.ones_like(xs)
    ops.ewald_real(L, ALPHA, RC, xs, qs, nl.nbr, nl.nnbr, nl.maxn, F=F1, accumulate=True)
    assert torch.equal(F1, F0 + 1.0)
    R0, _ = ops.spme_recip(L, ALPHA, 4, (16, 16, 16), xs, qs)
    R1 = torch.full_like(xs, 2.0)
    ops.spme_recip(L, ALPHA, 4, (16, 16, 16), xs, qs, F=R1, accumulate=True)
    assert torch.allclose(R1, R0 + 2.0, rtol=0, atol=1e-12 * R0.abs().max().item())
    # empty inputs: no launch faults, zero energies
    e = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    eq = torch.zeros(0, dtype=torch.float64, device=dev)
    nbr = torch.zeros(64 * 8, dtype=torch.int32, device=dev)
    nn = torch.zeros(0, dtype=torch.int32, device=dev)
    _, Ed = ops.ewald_real([10.0] * 3, ALPHA, RC, e, eq, nbr, nn, 8, want_energy=True)
    _, Er = ops.spme_recip([10.0] * 3, ALPHA, 4, (8, 8, 8), e, eq, want_energy=True)
    assert Ed.item() == 0.0 and Er.item() == 0.0


def test_sampled_500k_vs_oracle(dev, orc):
    """Full size (K = 128, order 4): E_rec + E_self and 64 sampled forces from the
    reference steps; the direct part of the same samples from the oracle's pair sum."""
    import torch
    from paper_2109_09056_amd import ops
    w = li.WORKLOADS["lj500k"]
    x, q, L = li.positions(w), li.charges(w), w.box
    K = li.ewald_grid(L)
    xs, qs, ids, nl = _sorted(dev, x, q, L, w.rlist)
    Fd, Ed = ops.ewald_real(L, ALPHA, RC, xs, qs, nl.nbr, nl.nnbr, nl.maxn, want_energy=True)
    Fr, Er = ops.spme_recip(L, ALPHA, li.EWALD_ORDER, K, xs, qs, want_energy=True)
    samp = np.random.default_rng(3).choice(x.shape[0], 64, replace=False)
    E_o, Fr_o = orc.spme_recip(x, q, L, ALPHA, K, li.EWALD_ORDER, sel=samp)
    E_o += orc.ewald_self(q, ALPHA)
    idsh = ids.cpu().numpy()
    pos = np.empty_like(idsh)
    pos[idsh] = np.arange(idsh.size)  # sorted position of each caller id
    Frg = Fr.cpu().numpy()[pos[samp]]
    assert np.abs(Frg - Fr_o).max() <= 1e-10 * np.abs(Fr_o).max()
    assert Er.item() == pytest.approx(E_o, rel=1e-11)
    # direct part of the same samples from the oracle's pair sum over all particles
    _, Fd_o = orc.ewald_direct(x, q, L, ALPHA, RC, sel=samp)
    Fdg = Fd.cpu().numpy()[pos[samp]]
    assert np.abs(Fdg - Fd_o).max() <= 1e-12 * np.abs(Fd_o).max()
    assert torch.isfinite(Fd).all() and torch.isfinite(Fr).all()
