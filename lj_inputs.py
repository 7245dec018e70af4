"""Seeded synthetic inputs for the short-range Lennard-Jones MD hot path and the
SPH pass built on the same lists.

This module only draws inputs: an fcc lattice at a given reduced density,
uniform positional jitter, Maxwell velocities, a 50/50 two-type assignment and
per-type-pair (epsilon, sigma) draws; for SPH a jittered simple-cubic lattice
with small Gaussian velocities.  It holds none of the method's
arithmetic (no distances, forces, neighbor tests or integration) and imports
neither the oracle nor the HIP package; both of those consume what it returns.

The state point is the classic dense LJ liquid used for the LJ benchmark kernel
the paper names (CabanaMD proxy-app section): fcc at rho* = 0.8442,
T* = 1.44, cutoff 2.5 sigma, skin 0.3 sigma.  All quantities are in LJ reduced
units (mass 1, k_B 1).
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 20210919

# fcc conventional-cell basis, in units of the lattice constant
_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


@dataclasses.dataclass(frozen=True)
class Workload:
    """One benchmark/parity configuration (sizes follow the paper's dense-LJ state point)."""
    name: str
    index: int              # seeds derive from SEED_BASE + index
    cells: int              # fcc unit cells per box edge
    density: float = 0.8442
    temperature: float = 1.44
    rc: float = 2.5
    skin: float = 0.3
    dt: float = 0.005
    steps: int = 0
    rebuild_every: int = 20
    ntypes: int = 1
    jitter: float = 0.05
    checkpoint_every: int = 0

    @property
    def natoms(self) -> int:
        return 4 * self.cells ** 3

    @property
    def rlist(self) -> float:
        return self.rc + self.skin

    @property
    def lattice_constant(self) -> float:
        return (4.0 / self.density) ** (1.0 / 3.0)

    @property
    def box(self) -> np.ndarray:
        return np.full(3, self.cells * self.lattice_constant)


WORKLOADS = {
    "lj256": Workload("lj256", 0, cells=4, steps=100),
    "lj32k": Workload("lj32k", 1, cells=20, steps=1000),
    "lj500k": Workload("lj500k", 2, cells=50, steps=1000),
    "lj32k_fm": Workload("lj32k_fm", 3, cells=20, ntypes=2),
    "lj256k_traj": Workload("lj256k_traj", 4, cells=40, steps=20, ntypes=2,
                            checkpoint_every=5),
    # the same liquid at 2,048,000 atoms: a working set well beyond the 256 MiB
    # Infinity Cache (the uncached-HBM regime of the 500k benchmark)
    "lj2m": Workload("lj2m", 6, cells=80, steps=200),
}


def rng(workload: Workload, stream: int) -> np.random.Generator:
    """PCG64 stream: 0 jitter, 1 velocities, 2 types, 3 parameters, 4 perturbation,
    5 charges."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + workload.index + stream))


def fcc_lattice(cells: int, a: float) -> np.ndarray:
    """Perfect fcc positions, loop order ix, iy, iz, basis atom; shape [4*cells^3, 3]."""
    idx = np.arange(cells)
    ix, iy, iz = np.meshgrid(idx, idx, idx, indexing="ij")
    origins = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = (origins[:, None, :] + _FCC_BASIS[None, :, :]).reshape(-1, 3)
    return pos * a


def _into_box(x: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Fold freshly drawn positions into [0, L) (input preparation only)."""
    x = np.where(x < 0.0, x + L, x)
    x = np.where(x >= L, x - L, x)
    return np.where(x >= L, x - L, x)


def positions(workload: Workload, jitter: float | None = None) -> np.ndarray:
    """Jittered fcc positions in [0, L)^3, FP64 [N, 3]."""
    j = workload.jitter if jitter is None else jitter
    x = fcc_lattice(workload.cells, workload.lattice_constant)
    if j > 0.0:
        x = x + rng(workload, 0).uniform(-j, j, size=x.shape)
    return _into_box(x, workload.box)


def velocities(workload: Workload, n: int | None = None) -> np.ndarray:
    """Maxwell velocities at T (m = 1), zero total momentum, kinetic T exact with 3N-3 dof."""
    n = workload.natoms if n is None else n
    v = rng(workload, 1).normal(0.0, np.sqrt(workload.temperature), size=(n, 3))
    v -= v.mean(axis=0)
    t_now = (v * v).sum() / (3 * n - 3)
    return v * np.sqrt(workload.temperature / t_now)


def types(workload: Workload, n: int | None = None) -> np.ndarray:
    """int32 types: exactly floor(N/T) of each type via a seeded permutation (0 for one type)."""
    n = workload.natoms if n is None else n
    t = np.zeros(n, dtype=np.int32)
    if workload.ntypes > 1:
        perm = rng(workload, 2).permutation(n)
        per = n // workload.ntypes
        for k in range(1, workload.ntypes):
            t[perm[k * per:(k + 1) * per]] = k
    return t


def charges(workload: Workload, n: int | None = None) -> np.ndarray:
    """Unit point charges for the long-range (SPME) path: +1 on exactly floor(N/2)
    atoms chosen by a seeded permutation, -1 on the rest (neutral for even N)."""
    n = workload.natoms if n is None else n
    q = -np.ones(n)
    q[rng(workload, 5).permutation(n)[:n // 2]] = 1.0
    return q


# SPME settings for the charged liquid: erfc(alpha rc) = 2.2e-5 at rc = 2.5, cubic
# (order 4) B-splines, grid of a power of two points per edge with spacing <= 0.7 sigma
EWALD_ALPHA = 1.2
EWALD_ORDER = 4


def ewald_grid(L) -> tuple[int, int, int]:
    """Smallest power of two K >= L / 0.7 per edge (at least 8)."""
    out = []
    for v in np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)):
        k = 8
        while v / k > 0.7:
            k *= 2
        out.append(k)
    return tuple(out)


def npacked(ntypes: int) -> int:
    return ntypes * (ntypes + 1) // 2


def params(workload: Workload) -> tuple[np.ndarray, np.ndarray]:
    """Packed upper-triangle (eps, sigma), entry order (0,0),(0,1),...,(0,T-1),(1,1),...

    One type: eps = sigma = 1.  Several types: eps ~ U[0.8, 1.2], sigma ~ U[0.9, 1.1].
    """
    p = npacked(workload.ntypes)
    if workload.ntypes == 1:
        return np.ones(1), np.ones(1)
    g = rng(workload, 3)
    eps = g.uniform(0.8, 1.2, size=p)
    sigma = g.uniform(0.9, 1.1, size=p)
    return eps, sigma


def perturbed_params(workload: Workload, rel: float = 0.05) -> tuple[np.ndarray, np.ndarray]:
    """Target parameters: each packed entry scaled by (1 + delta), delta ~ U[-rel, rel]."""
    eps, sigma = params(workload)
    g = rng(workload, 4)
    return (eps * (1.0 + g.uniform(-rel, rel, size=eps.shape)),
            sigma * (1.0 + g.uniform(-rel, rel, size=sigma.shape)))


def make_system(workload: Workload):
    """Everything one run needs: x, v, types, ids, packed eps/sigma, box."""
    x = positions(workload)
    n = x.shape[0]
    eps, sigma = params(workload)
    return dict(x=x, v=velocities(workload, n), types=types(workload, n),
                ids=np.arange(n, dtype=np.int64), eps=eps, sigma=sigma,
                box=workload.box.copy())


def random_gas(n: int, L, seed: int) -> np.ndarray:
    """Uniform random positions in [0, L)^3 (ragged/edge-case tests)."""
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    g = np.random.Generator(np.random.PCG64(seed))
    return _into_box(g.uniform(0.0, 1.0, size=(n, 3)) * L, L)


@dataclasses.dataclass(frozen=True)
class SphWorkload:
    """Weakly compressible SPH fluid at rest density 1: a simple-cubic lattice of
    spacing 1 (particle mass 1), jittered, smoothing length h = 1.3 spacings
    (support 2.6, about 74 neighbours inside it), sound speed 10."""
    name: str
    index: int              # seeds derive from SEED_BASE + 100 + index
    cells: int              # particles per box edge
    h: float = 1.3
    mass: float = 1.0
    c0: float = 10.0
    rho0: float = 1.0
    skin: float = 0.4
    dt: float = 0.01
    rebuild_every: int = 10
    jitter: float = 0.1     # uniform positional jitter, spacings
    vel: float = 0.2        # Gaussian velocity scale per component
    steps: int = 0

    @property
    def natoms(self) -> int:
        return self.cells ** 3

    @property
    def support(self) -> float:
        return 2.0 * self.h

    @property
    def rlist(self) -> float:
        return self.support + self.skin

    @property
    def box(self) -> np.ndarray:
        return np.full(3, float(self.cells))


SPH_WORKLOADS = {
    "sph4k": SphWorkload("sph4k", 0, cells=16, steps=50),
    "sph32k": SphWorkload("sph32k", 1, cells=32, steps=100),
    "sph512k": SphWorkload("sph512k", 2, cells=80, steps=500),
}


def sph_rng(workload: SphWorkload, stream: int) -> np.random.Generator:
    """PCG64 stream: 0 jitter, 1 velocities."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 + 10 * workload.index + stream))


def sph_positions(workload: SphWorkload) -> np.ndarray:
    """Jittered simple-cubic positions in [0, L)^3, FP64 [N, 3], loop order ix, iy, iz."""
    idx = np.arange(workload.cells, dtype=np.float64)
    ix, iy, iz = np.meshgrid(idx, idx, idx, indexing="ij")
    x = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) + 0.5
    if workload.jitter > 0.0:
        x = x + sph_rng(workload, 0).uniform(-workload.jitter, workload.jitter, size=x.shape)
    return _into_box(x, workload.box)


def sph_velocities(workload: SphWorkload) -> np.ndarray:
    """Gaussian velocities of scale `vel` per component, zero mean."""
    v = sph_rng(workload, 1).normal(0.0, workload.vel, size=(workload.natoms, 3))
    return v - v.mean(axis=0)
