"""CPU checks of the seeded input generators and of the host-side logic that does
not need a GPU: the generators are deterministic and have the shapes, ranges and
statistics the workloads state; the row-capacity guess and the bench's
multi-GPU refusal behave as documented."""
import os
import subprocess
import sys

import numpy as np
import pytest

import lj_inputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name", ["lj256", "lj32k"])
def test_lj_generators(name):
    w = li.WORKLOADS[name]
    a, b = li.make_system(w), li.make_system(w)
    for k in ("x", "v", "types", "eps", "sigma"):
        assert np.array_equal(a[k], b[k])  # seeded: identical on every call
    x, v = a["x"], a["v"]
    assert x.shape == (w.natoms, 3) and x.min() >= 0.0 and np.all(x < w.box)
    assert np.abs(v.sum(0)).max() < 1e-9 * w.natoms
    t = (v * v).sum() / (3 * w.natoms - 3)
    assert t == pytest.approx(w.temperature, rel=1e-12)
    # jitter bounded by the workload's amplitude (minimum image against the lattice)
    d = x - li.fcc_lattice(w.cells, w.lattice_constant)
    d -= w.box * np.round(d / w.box)
    assert np.abs(d).max() <= w.jitter + 1e-12


def test_two_type_and_charge_draws():
    w = li.WORKLOADS["lj32k_fm"]
    t = li.types(w)
    assert np.bincount(t).tolist() == [w.natoms // 2, w.natoms // 2]
    eps, sig = li.params(w)
    assert eps.size == sig.size == 3 and eps.min() >= 0.8 and eps.max() <= 1.2
    q = li.charges(li.WORKLOADS["lj256"])
    assert q.sum() == 0.0 and set(np.unique(q).tolist()) == {-1.0, 1.0}


def test_ewald_grid_rule():
    for L in (6.7, 33.6, 84.0, 150.0):
        K = li.ewald_grid(L)
        assert all(k >= 8 and k & (k - 1) == 0 for k in K)
        assert all(L / k <= 0.7 and (k == 8 or L / (k // 2) > 0.7) for k in K)


@pytest.mark.parametrize("name", ["sph4k", "sph32k"])
def test_sph_generators(name):
    w = li.SPH_WORKLOADS[name]
    x, v = li.sph_positions(w), li.sph_velocities(w)
    assert np.array_equal(x, li.sph_positions(w)) and np.array_equal(v, li.sph_velocities(w))
    assert x.shape == (w.natoms, 3) and x.min() >= 0.0 and np.all(x < w.box)
    assert np.abs(v.mean(0)).max() < 1e-12
    assert np.std(v) == pytest.approx(w.vel, rel=0.05)
    assert w.rlist == pytest.approx(2 * w.h + w.skin) and w.rlist < 0.5 * w.box.min()


def test_initial_row_capacity():
    """The row-capacity guess covers the ideal-gas mean with margin, in multiples of 4;
    half lists get about half."""
    from paper_2109_09056_amd import md, _lib
    w = li.WORKLOADS["lj500k"]
    full = md.initial_maxn(w.natoms, w.box, w.rlist, _lib.FULL)
    half = md.initial_maxn(w.natoms, w.box, w.rlist, _lib.HALF)
    mean = 4.0 / 3.0 * np.pi * w.rlist ** 3 * w.density
    assert full % 4 == 0 and half % 4 == 0
    assert full >= 1.3 * mean and half >= 0.65 * mean and half < full


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
