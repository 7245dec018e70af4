"""Python face of the SPH part of the CPU FP64 oracle (test infrastructure only).

The pair sums live in sph.c (all pairs, minimum image, FP64; definitions and
citations there).  Written out here in NumPy: the equation of state
p = c0^2 (rho - rho0), the internal energy U = sum_i m u(rho_i) with
u(rho) = c0^2 (ln(rho/rho0) + rho0/rho - 1), and a velocity-Verlet loop over
the pass for conservation checks.
"""
from __future__ import annotations

import numpy as np

from .oracle import _box, _f64, _ptr, lib

__all__ = ["sph_kernel", "sph_density", "sph_accel", "sph_pressure", "sph_internal_energy",
           "sph_run"]


def _sel(sel, n):
    if sel is None:
        return None, n
    s = np.ascontiguousarray(sel, dtype=np.int64)
    assert s.ndim == 1 and (s.size == 0 or (s.min() >= 0 and s.max() < n))
    return s, s.size


def sph_kernel(r, h):
    """(W(r, h), G(r, h) = W'(r)/r) of the cubic spline for an array of distances r >= 0."""
    r = _f64(np.atleast_1d(r))
    W = np.empty_like(r)
    G = np.empty_like(r)
    lib().orc_sph_kernel(r.size, r, float(h), _ptr(W), _ptr(G))
    return W, G


def sph_density(x, L, h, mass=1.0, sel=None):
    """rho of every particle (or of the rows in sel), all-pairs summation."""
    x = _f64(x)
    n = x.shape[0]
    s, ns = _sel(sel, n)
    out = np.empty(ns)
    lib().orc_sph_density(n, x, _box(L), float(h), float(mass), ns, _ptr(s), out)
    return out


def sph_accel(x, L, h, mass, c0, rho0, rho, sel=None):
    """Symmetric pressure acceleration [n or len(sel), 3] from the densities of all particles."""
    x = _f64(x)
    n = x.shape[0]
    rho = _f64(rho)
    assert rho.shape == (n,)
    s, ns = _sel(sel, n)
    out = np.empty((ns, 3))
    lib().orc_sph_accel(n, x, _box(L), float(h), float(mass), float(c0), float(rho0), rho, ns,
                        _ptr(s), out)
    return out


def sph_pressure(rho, c0, rho0):
    """Linear weakly compressible equation of state p = c0^2 (rho - rho0)."""
    return c0 * c0 * (np.asarray(rho, dtype=np.float64) - rho0)


def sph_internal_energy(rho, mass, c0, rho0):
    """U = sum_i m c0^2 (ln(rho_i/rho0) + rho0/rho_i - 1); du/drho = p/rho^2."""
    rho = np.asarray(rho, dtype=np.float64)
    return float(np.sum(mass * c0 * c0 * (np.log(rho / rho0) + rho0 / rho - 1.0)))


def _wrap(x, L):
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    x = np.where(x >= L, x - L, x)
    return np.where(x < 0.0, x + L, x)


def sph_run(x, v, L, h, mass, c0, rho0, dt, steps):
    """Velocity Verlet over the pressure pass (small n): returns final (x, v) and the
    total energy m/2 sum v^2 + U after every step (index 0: the start)."""
    x, v = _f64(x).copy(), _f64(v).copy()
    rho = sph_density(x, L, h, mass)
    a = sph_accel(x, L, h, mass, c0, rho0, rho)
    energy = [0.5 * mass * float(np.sum(v * v)) + sph_internal_energy(rho, mass, c0, rho0)]
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = _wrap(x + dt * v, L)
        rho = sph_density(x, L, h, mass)
        a = sph_accel(x, L, h, mass, c0, rho0, rho)
        v = v + 0.5 * dt * a
        energy.append(0.5 * mass * float(np.sum(v * v)) + sph_internal_energy(rho, mass, c0, rho0))
    return x, v, np.array(energy)
