"""Python face of the CPU FP64 oracle (test infrastructure only).

The arithmetic lives in oracle.c (O(N^2) all pairs, minimum image, FP64);
this module marshals NumPy arrays and writes out, in plain Python, the few
steps that are pure bookkeeping: the counting-sort order as a lexicographic
sort, the half list as the unordered pairs of the full relation, the
velocity-Verlet loop with its fixed rebuild cadence, and the discrete adjoint
of that loop.  See oracle.c for the definitions and their citations.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None
_lock = threading.Lock()

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_VP = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


def lib():
    """Load liborc.so, building it from oracle.c if it is missing or stale."""
    global _lib
    with _lock:
        if _lib is None:
            srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "sph.c", "ewald.c")]
            if (not os.path.exists(_LIB_PATH)
                    or os.path.getmtime(_LIB_PATH) < max(map(os.path.getmtime, srcs))):
                from . import build as _b
                _b.build()
            L = ctypes.CDLL(_LIB_PATH)
            L.orc_grid.argtypes = [_D, _dbl, _I32]
            L.orc_cell_index.argtypes = [_i64, _D, _D, _I32, _I64]
            L.orc_neighbor_count.argtypes = [_i64, _D, _D, _dbl, _i64, _VP, _I32]
            L.orc_neighbor_count.restype = _i64
            L.orc_neighbor_fill.argtypes = [_i64, _D, _D, _dbl, _i64, _VP, _I64, _I32]
            L.orc_neighbor_upper.argtypes = [_i64, _D, _D, _dbl, ctypes.c_int32, _I32, _I32]
            L.orc_forces.argtypes = [_i64, _D, _VP, ctypes.c_int, _D, _D, _D, _dbl, _i64,
                                     _VP, _D, _D, _D, _VP]
            L.orc_forces_list.argtypes = [_i64, _D, _VP, ctypes.c_int, _D, _D, _D, _dbl,
                                          _I64, _I32, _D, _D, _D, _VP]
            L.orc_force_vjp.argtypes = [_i64, _D, _VP, ctypes.c_int, _D, _D, _D, _dbl, _VP,
                                        _VP, _D, _D, _D, _D]
            L.orc_kick_drift.argtypes = [_i64, _D, _D, _D, _dbl, _dbl, _D, _VP]
            L.orc_kick.argtypes = [_i64, _D, _D, _dbl, _dbl]
            L.orc_num_threads.restype = ctypes.c_int
            L.orc_set_threads.argtypes = [ctypes.c_int]
            L.orc_sph_kernel.argtypes = [_i64, _D, _dbl, _VP, _VP]
            L.orc_sph_density.argtypes = [_i64, _D, _D, _dbl, _dbl, _i64, _VP, _D]
            L.orc_sph_accel.argtypes = [_i64, _D, _D, _dbl, _dbl, _dbl, _dbl, _D, _i64, _VP, _D]
            L.orc_ewald_direct.argtypes = [_i64, _D, _D, _D, _dbl, _dbl, _i64, _VP, _D, _D]
            L.orc_ewald_recip.argtypes = [_i64, _D, _D, _D, _dbl, ctypes.c_int, _D]
            L.orc_ewald_recip.restype = _dbl
            _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _box(L):
    return _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def ntypes_of(eps) -> int:
    p = int(np.asarray(eps).size)
    t = int(round((np.sqrt(8 * p + 1) - 1) / 2))
    assert t * (t + 1) // 2 == p, "packed parameter length must be T(T+1)/2"
    return t


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


# ------------------------------------------------------------------ binning --

def grid(L, rlist) -> np.ndarray:
    nc = np.zeros(3, dtype=np.int32)
    lib().orc_grid(_box(L), float(rlist), nc)
    return nc


def cell_index(x, L, nc) -> np.ndarray:
    x = _f64(x)
    out = np.zeros(x.shape[0], dtype=np.int64)
    lib().orc_cell_index(x.shape[0], x, _box(L), np.ascontiguousarray(nc, dtype=np.int32), out)
    return out


def bin_order(x, ids, L, rlist):
    """Counting sort by cell, ascending id inside a cell: a stable order on (cell, id).

    Returns (perm, cell_start, nc): sorted position k holds input atom perm[k];
    cell_start[c] is the first sorted position of cell c (length ncells + 1).
    """
    nc = grid(L, rlist)
    cell = cell_index(x, L, nc)
    perm = np.lexsort((np.asarray(ids), cell))
    ncell = int(np.prod(nc.astype(np.int64)))
    counts = np.bincount(cell, minlength=ncell)
    cell_start = np.zeros(ncell + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_start[1:])
    return perm, cell_start, nc


# ---------------------------------------------------------------- neighbors --

def neighbor_lists(x, L, rlist, sel=None):
    """Full Verlet list by brute force: CSR (offsets, nbr), each row j-ascending.

    Rows are all atoms, or the atoms in sel (then offsets has len(sel)+1 entries).
    All rows are formed from the unordered pairs (one brute-force pass over j > i);
    selected rows by a count pass and a fill pass over all j.
    """
    x = _f64(x)
    n = x.shape[0]
    if sel is None and n > 0:
        return full_from_upper(upper_pairs(x, L, rlist), n)
    sel_a = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    rows = n if sel_a is None else sel_a.size
    counts = np.zeros(rows, dtype=np.int32)
    lib().orc_neighbor_count(n, x, _box(L), float(rlist), rows, _ptr(sel_a), counts)
    offsets = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    nbr = np.zeros(max(int(offsets[-1]), 1), dtype=np.int32)
    lib().orc_neighbor_fill(n, x, _box(L), float(rlist), rows, _ptr(sel_a), offsets, nbr)
    return offsets, nbr[:offsets[-1]]


def upper_pairs(x, L, rlist, cap=96):
    """Every unordered pair within rlist once, by brute force over j > i: a [P, 2]
    int64 array of (i, j), i < j, sorted by i then j."""
    x = _f64(x)
    n = x.shape[0]
    while True:
        upper = np.zeros(max(n * cap, 1), dtype=np.int32)
        ln = np.zeros(max(n, 1), dtype=np.int32)
        lib().orc_neighbor_upper(n, x, _box(L), float(rlist), cap, upper, ln)
        top = int(ln[:n].max()) if n else 0
        if top <= cap:
            break
        cap = top
    ln = ln[:n]
    keep = np.arange(cap)[None, :] < ln[:, None]
    j = upper[:n * cap].reshape(n, cap)[keep].astype(np.int64)
    i = np.repeat(np.arange(n, dtype=np.int64), ln)
    return np.stack([i, j], axis=1)


def full_from_upper(pairs, n):
    """CSR full list (offsets, nbr), rows j-ascending, from the unordered pairs."""
    i = np.concatenate([pairs[:, 0], pairs[:, 1]])
    j = np.concatenate([pairs[:, 1], pairs[:, 0]])
    order = np.argsort(i * n + j, kind="stable")
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(i, minlength=n), out=offsets[1:])
    return offsets, j[order].astype(np.int32)


def half_pairs(offsets, nbr, rows=None) -> np.ndarray:
    """Unordered pairs {min, max} of a full relation, as a sorted [P, 2] int64 array."""
    n = offsets.size - 1
    rows = np.arange(n) if rows is None else np.asarray(rows)
    i = np.repeat(rows, np.diff(offsets))
    j = nbr.astype(np.int64)
    a = np.minimum(i, j)
    b = np.maximum(i, j)
    pairs = np.unique(np.stack([a, b], axis=1), axis=0)
    return pairs


# ------------------------------------------------------------------- forces --

def forces(x, L, rc, eps=(1.0,), sigma=(1.0,), types=None, sel=None):
    """All-pairs F, e (per row), W[6] and unordered pair counts within rc per type pair."""
    x = _f64(x)
    n = x.shape[0]
    eps = _f64(np.atleast_1d(eps))
    sigma = _f64(np.atleast_1d(sigma))
    T = ntypes_of(eps)
    t = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
    sel_a = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    rows = n if sel_a is None else sel_a.size
    F = np.zeros((rows, 3))
    e = np.zeros(rows)
    W = np.zeros(6)
    npairs = np.zeros(eps.size, dtype=np.int64)
    lib().orc_forces(n, x, _ptr(t), T, eps, sigma, _box(L), float(rc), rows, _ptr(sel_a),
                     F, e, W, _ptr(npairs))
    return F, e, W, npairs


def forces_list(x, L, rc, offsets, nbr, eps=(1.0,), sigma=(1.0,), types=None,
                with_pairs=False):
    """F, e, W over a given CSR full list; with_pairs adds the list's unordered pairs
    within rc per packed type pair."""
    x = _f64(x)
    n = x.shape[0]
    eps = _f64(np.atleast_1d(eps))
    sigma = _f64(np.atleast_1d(sigma))
    t = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
    F = np.zeros((n, 3))
    e = np.zeros(n)
    W = np.zeros(6)
    npairs = np.zeros(eps.size, dtype=np.int64) if with_pairs else None
    lib().orc_forces_list(n, x, _ptr(t), ntypes_of(eps), eps, sigma, _box(L), float(rc),
                          np.ascontiguousarray(offsets, dtype=np.int64),
                          np.ascontiguousarray(nbr, dtype=np.int32), F, e, W, _ptr(npairs))
    return (F, e, W, npairs) if with_pairs else (F, e, W)


def force_vjp(x, L, rc, g, eps=(1.0,), sigma=(1.0,), types=None, offsets=None, nbr=None):
    """(gx, geps, gsigma) = g^T dF/d(x, eps, sigma) with the pair set held fixed."""
    x = _f64(x)
    n = x.shape[0]
    eps = _f64(np.atleast_1d(eps))
    sigma = _f64(np.atleast_1d(sigma))
    t = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
    off = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int64)
    nb = None if nbr is None else np.ascontiguousarray(nbr, dtype=np.int32)
    gx = np.zeros((n, 3))
    ge = np.zeros(eps.size)
    gs = np.zeros(eps.size)
    lib().orc_force_vjp(n, x, _ptr(t), ntypes_of(eps), eps, sigma, _box(L), float(rc),
                        _ptr(off), _ptr(nb), _f64(g), gx, ge, gs)
    return gx, ge, gs


def pair_energy(r, eps=1.0, sigma=1.0):
    """12-6 pair energy for scalar r (no cutoff), via the oracle's two-atom force call."""
    L = np.full(3, 1e3)
    x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]]) + 10.0
    F, e, _, _ = forces(x, L, rc=1e2, eps=[eps], sigma=[sigma])
    return 2.0 * e[0], F


# --------------------------------------------------------------- integrator --

def kick_drift(x, v, F, dt, L, mass=1.0, img=None):
    """In place: v += dt/2 F/m; x += dt v; wrap into [0, L)."""
    lib().orc_kick_drift(x.shape[0], x, v, _f64(F), float(dt), float(mass), _box(L),
                         _ptr(img))


def kick(v, F, dt, mass=1.0):
    lib().orc_kick(v.shape[0], v, _f64(F), float(dt), float(mass))


def run_nve(x, v, L, rc, rlist, dt, steps, rebuild_every=20, eps=(1.0,), sigma=(1.0,),
            types=None, mode="verlet", record=None, missed=None):
    """Velocity-Verlet NVE run.

    mode "verlet": the oracle's own brute-force list, rebuilt every
    rebuild_every steps from step 0 with no displacement check; "allpairs":
    every force call over all pairs.  Returns (x, v, F, thermo) where thermo is
    a list of (step, PE, KE) and `record` (a set of steps) selects snapshots
    returned in thermo-side dict `snaps`.  missed (verlet mode): optional list
    that receives, for every force call, the number of pairs inside rc that the
    current list does not hold (all pairs inside rc minus the list's).
    """
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[0]
    img = np.zeros((n, 3), dtype=np.int32)
    lst = None

    def force(step):
        nonlocal lst
        if mode == "allpairs":
            F, e, W, _ = forces(x, L, rc, eps, sigma, types)
            return F, e
        if step % rebuild_every == 0 or lst is None:
            lst = neighbor_lists(x, L, rlist)
        if missed is None:
            F, e, W = forces_list(x, L, rc, lst[0], lst[1], eps, sigma, types)
        else:
            F, e, W, held = forces_list(x, L, rc, lst[0], lst[1], eps, sigma, types,
                                        with_pairs=True)
            missed.append(int(forces(x, L, rc, eps, sigma, types)[3].sum() - held.sum()))
        return F, e

    F, e = force(0)
    thermo = [(0, e.sum(), 0.5 * (v * v).sum())]
    snaps = {}
    if record and 0 in record:
        snaps[0] = (x.copy(), v.copy(), F.copy())
    for step in range(1, steps + 1):
        kick_drift(x, v, F, dt, L, img=img)
        F, e = force(step)
        kick(v, F, dt)
        thermo.append((step, e.sum(), 0.5 * (v * v).sum()))
        if record and step in record:
            snaps[step] = (x.copy(), v.copy(), F.copy())
    return x, v, F, thermo, snaps, img


# ------------------------------------------------------- trajectory adjoint --

def trajectory(x0, v0, L, rc, rlist, dt, steps, eps, sigma, types=None, mass=1.0, lst=None,
               pairs=None):
    """Forward velocity Verlet with one list built at step 0 (steps <= rebuild cadence),
    or the given list lst.

    Returns (xs, v_T, unwrapped x_T, lst): xs[k] is the wrapped position at step k.
    pairs: optional list that receives, for steps 0..steps, the number of unordered
    pairs of the list within rc (all type pairs).
    """
    x = _f64(x0).copy()
    v = _f64(v0).copy()
    img = np.zeros(x.shape, dtype=np.int32)
    if lst is None:
        lst = neighbor_lists(x, L, rlist)

    def force():
        out = forces_list(x, L, rc, lst[0], lst[1], eps, sigma, types,
                          with_pairs=pairs is not None)
        if pairs is not None:
            pairs.append(int(out[3].sum()))
        return out[0]

    F = force()
    xs = [x.copy()]
    for _ in range(steps):
        kick_drift(x, v, F, dt, L, mass=mass, img=img)
        F = force()
        kick(v, F, dt, mass=mass)
        xs.append(x.copy())
    return xs, v, x + img * _box(L), lst


def trajectory_adjoint(xs, L, rc, dt, eps, sigma, xbar_T, vbar_T, types=None, lst=None,
                       mass=1.0):
    """Discrete adjoint of the velocity-Verlet trajectory, newest step first.

    Step n maps (x_n, v_n) to (x_{n+1}, v_{n+1}) through h = v_n + dt/(2m) F(x_n),
    x_{n+1} = x_n + dt h, v_{n+1} = h + dt/(2m) F(x_{n+1}).  Its reverse, with
    J^T a the force VJP at the stated positions:
        xbar_{n+1} += J^T(x_{n+1}) (dt/(2m) vbar_{n+1});  hbar = vbar_{n+1} + dt xbar_{n+1}
        xbar_n = xbar_{n+1} + J^T(x_n) (dt/(2m) hbar);    vbar_n = hbar
    Parameter cotangents collect the same VJP calls.  Returns
    (xbar_0, vbar_0, geps, gsigma).
    """
    T = len(xs) - 1
    xbar = _f64(xbar_T).copy()
    vbar = _f64(vbar_T).copy()
    ge = np.zeros(np.asarray(eps).size)
    gs = np.zeros(np.asarray(eps).size)
    off, nb = (None, None) if lst is None else lst

    def vjp(x, a):
        return force_vjp(x, L, rc, a, eps, sigma, types, off, nb)

    c = 0.5 * dt / mass
    for n in range(T - 1, -1, -1):
        gx, e1, s1 = vjp(xs[n + 1], c * vbar)
        xbar += gx
        ge += e1
        gs += s1
        hbar = vbar + dt * xbar
        gx, e2, s2 = vjp(xs[n], c * hbar)
        xbar = xbar + gx
        ge += e2
        gs += s2
        vbar = hbar
    return xbar, vbar, ge, gs
