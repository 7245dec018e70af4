"""Ewald sum and smooth particle-mesh Ewald (SPME) references, FP64 (test
infrastructure only).

Ewald (ewald.c): direct-space sum over minimum-image pairs inside rc,
reciprocal sum over the k-vectors |n_a| <= nmax, self term; definitions and
citations in ewald.c.

SPME (Essmann, Perera, Berkowitz, Darden, Lee, Pedersen 1995, J. Chem. Phys.
103, 8577), written out here in NumPy in that paper's order and notation:
  u_ai = K_a x_ai / L_a                       scaled fractional coordinates
  M_2(u) = 1 - |u - 1| on [0, 2], 0 elsewhere
  M_n(u) = u/(n-1) M_{n-1}(u) + (n-u)/(n-1) M_{n-1}(u-1)     cardinal B-splines
  Q(k) = sum_i q_i prod_a M_n(u_ai - k_a - s_a K_a), summed over the periodic
         images s_a (only points k_a = floor(u_ai) - j, j = 0..n-1, mod K_a)
  b_a(m) = exp(2 pi i (n-1) m/K_a) / sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k/K_a)
  B(m) = prod_a |b_a(m_a)|^2
  C(m) = exp(-pi^2 |m'|^2 / alpha^2) / (pi V |m'|^2), C(0) = 0, with
         m'_a = m_a / L_a for m_a <= K_a/2, (m_a - K_a) / L_a otherwise
  E_rec = 1/2 sum_m B(m) C(m) |F(Q)(m)|^2     (F: the 3-D discrete Fourier transform)
  F_i = -dE_rec/dx_i = -sum_k dQ(k)/dx_i phi(k),  phi = F^-1 applied to B C F(Q),
        unnormalised, i.e. phi(k) = sum_m B C F(Q)(m) exp(2 pi i m.k/K)
  dM_n(u)/du = M_{n-1}(u) - M_{n-1}(u-1)
Even orders n only (the b_a denominators of odd n vanish at m = K/2).
"""
from __future__ import annotations

import numpy as np

from .oracle import _box, _f64, _ptr, lib

__all__ = ["ewald_direct", "ewald_recip", "ewald_self", "bspline", "spme_recip",
           "spme_grid_charge"]


def ewald_direct(x, q, L, alpha, rc, sel=None):
    """(per-particle direct energies, direct forces [., 3]) of every particle or of the
    rows in sel."""
    x = _f64(x)
    q = _f64(q)
    n = x.shape[0]
    s = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    ns = n if s is None else s.size
    e = np.empty(ns)
    F = np.empty((ns, 3))
    lib().orc_ewald_direct(n, x, q, _box(L), float(alpha), float(rc), ns, _ptr(s), e, F)
    return e, F


def ewald_recip(x, q, L, alpha, nmax):
    """(E_rec, F_rec [n, 3]) from the k-space sum over |n_a| <= nmax."""
    x = _f64(x)
    q = _f64(q)
    F = np.empty((x.shape[0], 3))
    E = lib().orc_ewald_recip(x.shape[0], x, q, _box(L), float(alpha), int(nmax), F)
    return float(E), F


def ewald_self(q, alpha):
    return float(-alpha / np.sqrt(np.pi) * np.sum(np.asarray(q, dtype=np.float64) ** 2))


def bspline(u, n):
    """M_n(u) by the recursion, for an array u (the definition, evaluated directly)."""
    u = np.asarray(u, dtype=np.float64)
    if n == 2:
        return np.where((u >= 0.0) & (u <= 2.0), 1.0 - np.abs(u - 1.0), 0.0)
    return (u * bspline(u, n - 1) + (n - u) * bspline(u - 1.0, n - 1)) / (n - 1)


def _dbspline(u, n):
    return bspline(u, n - 1) - bspline(u - 1.0, n - 1)


def _weights(x, L, K, n):
    """Per particle and dimension: grid indices [n_p, 3, n], M_n and dM_n/du values."""
    L = np.asarray(L, dtype=np.float64)
    K = np.asarray(K)
    u = K * x / L                                    # [n_p, 3]
    base = np.floor(u)
    j = np.arange(n)
    idx = (base[:, :, None].astype(np.int64) - j) % K[None, :, None]
    arg = u[:, :, None] - (base[:, :, None] - j)     # u - k for k = floor(u) - j
    return idx, bspline(arg, n), _dbspline(arg, n)


def spme_grid_charge(x, q, L, K, n):
    """Q(k) on the K_0 x K_1 x K_2 grid (index order [k0, k1, k2])."""
    x = _f64(x)
    q = _f64(q)
    idx, w, _ = _weights(x, L, K, n)
    Q = np.zeros(tuple(K))
    # every particle's n^3 products q_i M(u_0 - k_0) M(u_1 - k_1) M(u_2 - k_2), added at their points
    wt = q[:, None, None, None] * w[:, 0, :, None, None] * w[:, 1, None, :, None] * \
        w[:, 2, None, None, :]
    i0 = np.broadcast_to(idx[:, 0, :, None, None], wt.shape)
    i1 = np.broadcast_to(idx[:, 1, None, :, None], wt.shape)
    i2 = np.broadcast_to(idx[:, 2, None, None, :], wt.shape)
    np.add.at(Q, (i0.ravel(), i1.ravel(), i2.ravel()), wt.ravel())
    return Q


def _bmod2(K, n):
    m = np.arange(K)
    k = np.arange(n - 1)
    den = (bspline(k + 1.0, n)[None, :] * np.exp(2j * np.pi * m[:, None] * k[None, :] / K)).sum(1)
    return 1.0 / np.abs(den) ** 2


def spme_recip(x, q, L, alpha, K, n=4, sel=None):
    """(E_rec, F_rec) by SPME with grid K = (K0, K1, K2) and spline order n; the forces
    of every particle [n_p, 3], or of the rows in sel [len(sel), 3]."""
    x = _f64(x)
    q = _f64(q)
    L = np.asarray(L, dtype=np.float64)
    K = tuple(int(k) for k in K)
    assert n % 2 == 0 and n >= 4
    V = float(np.prod(L))
    Q = spme_grid_charge(x, q, L, K, n)
    mp = [np.where(np.arange(k) <= k // 2, np.arange(k), np.arange(k) - k) / l
          for k, l in zip(K, L)]
    m2 = mp[0][:, None, None] ** 2 + mp[1][None, :, None] ** 2 + mp[2][None, None, :] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        C = np.exp(-np.pi ** 2 * m2 / alpha ** 2) / (np.pi * V * m2)
    C[0, 0, 0] = 0.0
    B = _bmod2(K[0], n)[:, None, None] * _bmod2(K[1], n)[None, :, None] * \
        _bmod2(K[2], n)[None, None, :]
    FQ = np.fft.fftn(Q)
    E = 0.5 * float(np.sum(B * C * np.abs(FQ) ** 2))
    phi = np.real(np.fft.ifftn(B * C * FQ)) * (K[0] * K[1] * K[2])
    rows = np.arange(x.shape[0]) if sel is None else np.asarray(sel, dtype=np.int64)
    idx, w, dw = _weights(x[rows], L, K, n)
    F = np.empty((rows.size, 3))
    Ka = np.asarray(K, dtype=np.float64)
    for i in range(rows.size):
        P = phi[np.ix_(idx[i, 0], idx[i, 1], idx[i, 2])]
        g0 = np.einsum("a,b,c,abc->", dw[i, 0], w[i, 1], w[i, 2], P) * Ka[0] / L[0]
        g1 = np.einsum("a,b,c,abc->", w[i, 0], dw[i, 1], w[i, 2], P) * Ka[1] / L[1]
        g2 = np.einsum("a,b,c,abc->", w[i, 0], w[i, 1], dw[i, 2], P) * Ka[2] / L[2]
        F[i] = -q[rows[i]] * np.array([g0, g1, g2])
    return E, F
