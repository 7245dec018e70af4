"""Python face of the libljmd C ABI: one function per entry point, same names.

Argument marshalling only: tensors must already live on the GPU with the
dtype and layout the ABI states; each call passes their device pointers and
the current torch stream to the library, which does every step in its own
HIP kernels.  PyTorch supplies device memory (including workspaces) and the
stream, nothing else.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (EBOX, EHIP, EINVAL, EWORKSPACE, FP64, FULL, HALF, KICK, KICK_DRIFT,  # noqa: F401
                   KICK_KICK_DRIFT, KINETIC,
                   MAX_TEAM, MAX_TYPES, MIXED, OP_BACKWARD, OP_BIN, OP_CSR, OP_FORCES,
                   OP_BUILD_CSR, OP_DISPLACEMENT, OP_EWALD_REAL, OP_FORCES_CSR, OP_INTEGRATE,
                   OP_LOSS, OP_MD_CHAIN,
                   OP_SPH, OP_SPME,
                   SPME_MAX_GRID, TILE, LjmdError, make_box)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t, name, dtype, shape=None, device=None):
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _ws(op, n, device, ncells=0, ntypes=1, ws=None):
    need = int(_lib.load().ljmd_workspace_bytes(op, n, ncells, ntypes))
    if ws is not None and ws.numel() >= need:
        return ws, need
    return torch.empty(max(need, 8), dtype=torch.uint8, device=device), need


def grid(L, rlist):
    """Cell counts per dimension for binning at rlist (host computation)."""
    nc = (ctypes.c_int32 * 3)()
    b = make_box(L)
    _lib.check(_lib.load().ljmd_grid(ctypes.byref(b), float(rlist), nc), "ljmd_grid")
    return (int(nc[0]), int(nc[1]), int(nc[2]))


def workspace_bytes(op, n, ncells=0, ntypes=1) -> int:
    return int(_lib.load().ljmd_workspace_bytes(op, n, ncells, ntypes))


def bin(L, rlist, x, v=None, types=None, ids=None, out=None, cell_start=None, ws=None):
    """Counting sort into cells.  Returns (x, v, types, ids, cell_start) in sorted order."""
    n = x.shape[0]
    dev = x.device
    _need(x, "x", torch.float64, (n, 3))
    _need(v, "v", torch.float64, (n, 3), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(ids, "ids", torch.int64, (n,), dev)
    nc = grid(L, rlist)
    ncells = nc[0] * nc[1] * nc[2]
    if out is None:
        out = (torch.empty_like(x), None if v is None else torch.empty_like(v),
               None if types is None else torch.empty_like(types),
               torch.empty(n, dtype=torch.int64, device=dev))
    xo, vo, to, io = out
    if cell_start is None or cell_start.numel() < ncells + 1:
        cell_start = torch.empty(ncells + 1, dtype=torch.int32, device=dev)
    _need(cell_start, "cell_start", torch.int32, None, dev)
    ws, need = _ws(OP_BIN, n, dev, ncells=ncells, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_bin(
        ctypes.byref(b), float(rlist), n, _ptr(x), _ptr(v), _ptr(types), _ptr(ids), _ptr(xo),
        _ptr(vo), _ptr(to), _ptr(io), _ptr(cell_start), cell_start.numel(), _ptr(ws), need,
        _stream(dev)), "ljmd_bin")
    return xo, vo, to, io, cell_start


def list_shape(n, maxn):
    tiles = (n + TILE - 1) // TILE
    return (max(tiles, 1) * maxn * TILE,)


def build_neighbors(L, rlist, kind, x, cell_start, maxn, nbr=None, nnbr=None, max_count=None):
    """Tiled-ELL Verlet list.  Returns (nbr, nnbr, max_count) -- max_count is a device scalar."""
    n = x.shape[0]
    dev = x.device
    _need(x, "x", torch.float64, (n, 3))
    _need(cell_start, "cell_start", torch.int32, None, dev)
    if nbr is None or nbr.numel() < list_shape(n, maxn)[0]:
        nbr = torch.empty(list_shape(n, maxn), dtype=torch.int32, device=dev)
    if nnbr is None:
        nnbr = torch.empty(n, dtype=torch.int32, device=dev)
    if max_count is None:
        max_count = torch.empty(1, dtype=torch.int32, device=dev)
    _need(nbr, "nbr", torch.int32, None, dev)
    _need(nnbr, "nnbr", torch.int32, (n,), dev)
    _need(max_count, "max_count", torch.int32, (1,), dev)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_build_neighbors(
        ctypes.byref(b), float(rlist), int(kind), n, _ptr(x), _ptr(cell_start), int(maxn),
        _ptr(nbr), _ptr(nnbr), _ptr(max_count), _stream(dev)), "ljmd_build_neighbors")
    return nbr, nnbr, max_count


def compute_forces(L, precision, kind, rc, eps, sigma, x, types, nbr, nnbr, maxn, F=None,
                   e_atom=None, ev=None, want_energy=True, ws=None, atom_energy=True):
    """Forces (and per-atom energy / [E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz] when wanted).
    atom_energy=False with want_energy: E and W only (no per-atom energies are made
    unless e_atom is given)."""
    n = x.shape[0]
    dev = x.device
    ntypes = _ntypes(eps)
    _need(x, "x", torch.float64, (n, 3))
    _need(eps, "eps", torch.float64, None, dev)
    _need(sigma, "sigma", torch.float64, tuple(eps.shape), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(nbr, "nbr", torch.int32, None, dev)
    _need(nnbr, "nnbr", torch.int32, (n,), dev)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    if F is None:
        F = torch.empty_like(x)
    if want_energy:
        if e_atom is None and atom_energy:
            e_atom = torch.empty(n, dtype=torch.float64, device=dev)
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=dev)
    _need(F, "F", torch.float64, (n, 3), dev)
    _need(e_atom, "e_atom", torch.float64, (n,), dev)
    _need(ev, "ev", torch.float64, (7,), dev)
    ws, need = _ws(OP_FORCES, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_compute_forces(
        ctypes.byref(b), int(precision), int(kind), float(rc), ntypes, _ptr(eps), _ptr(sigma), n,
        _ptr(x), _ptr(types), _ptr(nbr), _ptr(nnbr), int(maxn), _ptr(F), _ptr(e_atom), _ptr(ev),
        _ptr(ws), need, _stream(dev)), "ljmd_compute_forces")
    return F, e_atom, ev


def build_neighbors_csr(L, rlist, kind, x, cell_start, cap=None, offsets=None, csr=None, ws=None):
    """Compressed (CSR) Verlet list straight from the cells: (offsets int64 [n+1],
    csr int32).  With cap None the capacity starts from the mean density and the
    list is built again, once, if the total read back exceeds it (a sync)."""
    n = x.shape[0]
    dev = x.device
    _need(x, "x", torch.float64, (n, 3))
    _need(cell_start, "cell_start", torch.int32, None, dev)
    if offsets is None:
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    _need(offsets, "offsets", torch.int64, (n + 1,), dev)
    ws, need = _ws(OP_BUILD_CSR, n, dev, ws=ws)
    b = make_box(L)
    guess = cap is None
    if guess:
        vol = float(L[0]) * float(L[1]) * float(L[2])
        mean = 4.0 / 3.0 * 3.141592653589793 * rlist ** 3 * n / vol
        cap = int((mean * (0.5 if kind == HALF else 1.0) * 1.1 + 8) * n) + 64
    while True:
        if csr is None or csr.numel() < cap:
            csr = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        _need(csr, "csr", torch.int32, None, dev)
        _lib.check(_lib.load().ljmd_build_neighbors_csr(
            ctypes.byref(b), float(rlist), int(kind), n, _ptr(x), _ptr(cell_start), _ptr(offsets),
            _ptr(csr), int(csr.numel()), _ptr(ws), need, _stream(dev)), "ljmd_build_neighbors_csr")
        if not guess:
            return offsets, csr
        total = int(offsets[n].item())
        if total <= csr.numel():
            return offsets, csr
        cap, csr = total, None


def list_to_csr(nbr, nnbr, maxn, cap=None, offsets=None, csr=None, ws=None):
    """(offsets int64 [n+1], csr int32 [cap]) = compressed copy of a tiled list.  With
    cap None the capacity is the exact total, read back from the device (a sync)."""
    n = nnbr.shape[0]
    dev = nnbr.device
    _need(nnbr, "nnbr", torch.int32, (n,))
    _need(nbr, "nbr", torch.int32, None, dev)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    if cap is None:
        cap = int(nnbr.clamp(max=maxn).to(torch.int64).sum().item())
    if offsets is None:
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    if csr is None:
        csr = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    _need(offsets, "offsets", torch.int64, (n + 1,), dev)
    _need(csr, "csr", torch.int32, None, dev)
    if csr.numel() < cap:
        raise ValueError("csr is smaller than cap")
    ws, need = _ws(OP_CSR, n, dev, ws=ws)
    _lib.check(_lib.load().ljmd_list_to_csr(n, _ptr(nbr), _ptr(nnbr), int(maxn), _ptr(offsets),
                                            _ptr(csr), int(cap), _ptr(ws), need, _stream(dev)),
               "ljmd_list_to_csr")
    return offsets, csr


def compute_forces_csr(L, precision, rc, eps, sigma, x, types, offsets, csr, team=1, F=None,
                       e_atom=None, ev=None, want_energy=True, ws=None):
    """Forces over a CSR list with `team` lanes per atom (FULL rows)."""
    n = x.shape[0]
    dev = x.device
    ntypes = _ntypes(eps)
    _need(x, "x", torch.float64, (n, 3))
    _need(eps, "eps", torch.float64, None, dev)
    _need(sigma, "sigma", torch.float64, tuple(eps.shape), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(offsets, "offsets", torch.int64, (n + 1,), dev)
    _need(csr, "csr", torch.int32, None, dev)
    if F is None:
        F = torch.empty_like(x)
    if want_energy:
        if e_atom is None:
            e_atom = torch.empty(n, dtype=torch.float64, device=dev)
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=dev)
    _need(F, "F", torch.float64, (n, 3), dev)
    _need(e_atom, "e_atom", torch.float64, (n,), dev)
    _need(ev, "ev", torch.float64, (7,), dev)
    ws, need = _ws(OP_FORCES_CSR, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_compute_forces_csr(
        ctypes.byref(b), int(precision), float(rc), ntypes, _ptr(eps), _ptr(sigma), n, _ptr(x),
        _ptr(types), _ptr(offsets), _ptr(csr), int(team), _ptr(F), _ptr(e_atom), _ptr(ev),
        _ptr(ws), need, _stream(dev)), "ljmd_compute_forces_csr")
    return F, e_atom, ev


AOSOA_VLENS = (0, 1, 8, 64)  # 0: plain SoA; 1: [n][3]


def aosoa_convert(src, vlen, to_aosoa, n=None, dst=None):
    """[n][3] rows -> flat AoSoA(vlen) array of 3n (to_aosoa) or back."""
    dev = src.device
    if n is None:
        n = src.shape[0] if to_aosoa else src.numel() // 3
    _need(src, "src", torch.float64, (n, 3) if to_aosoa else (3 * n,))
    if dst is None:
        dst = torch.empty(3 * n, dtype=torch.float64, device=dev) if to_aosoa else \
            torch.empty(n, 3, dtype=torch.float64, device=dev)
    _need(dst, "dst", torch.float64, (3 * n,) if to_aosoa else (n, 3), dev)
    _lib.check(_lib.load().ljmd_aosoa_convert(n, int(vlen), 1 if to_aosoa else 0, _ptr(src),
                                              _ptr(dst), _stream(dev)), "ljmd_aosoa_convert")
    return dst


def compute_forces_aosoa(L, precision, rc, eps, sigma, x, types, nbr, nnbr, maxn, vlen, F=None,
                         e_atom=None, ev=None, want_energy=True, ws=None):
    """FULL-list forces with positions x and forces F flat [3n] in AoSoA(vlen) layout."""
    n = types.shape[0]
    dev = x.device
    ntypes = _ntypes(eps)
    _need(x, "x", torch.float64, (3 * n,))
    _need(eps, "eps", torch.float64, None, dev)
    _need(sigma, "sigma", torch.float64, tuple(eps.shape), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(nbr, "nbr", torch.int32, None, dev)
    _need(nnbr, "nnbr", torch.int32, (n,), dev)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    if F is None:
        F = torch.empty_like(x)
    if want_energy:
        if e_atom is None:
            e_atom = torch.empty(n, dtype=torch.float64, device=dev)
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=dev)
    _need(F, "F", torch.float64, (3 * n,), dev)
    _need(e_atom, "e_atom", torch.float64, (n,), dev)
    _need(ev, "ev", torch.float64, (7,), dev)
    ws, need = _ws(OP_FORCES, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_compute_forces_aosoa(
        ctypes.byref(b), int(precision), float(rc), ntypes, _ptr(eps), _ptr(sigma), n, int(vlen),
        _ptr(x), _ptr(types), _ptr(nbr), _ptr(nnbr), int(maxn), _ptr(F), _ptr(e_atom), _ptr(ev),
        _ptr(ws), need, _stream(dev)), "ljmd_compute_forces_aosoa")
    return F, e_atom, ev


def md_step(L, precision, rc, eps, sigma, x, types, nbr, nnbr, maxn, dt, mass, v, x_next=None,
            open_next=True, F=None, e_atom=None, ev=None, ws=None):
    """Fused velocity-Verlet step on a FULL list; returns (x_next, F, ev[8])."""
    n = x.shape[0]
    dev = x.device
    ntypes = _ntypes(eps)
    _need(x, "x", torch.float64, (n, 3))
    _need(v, "v", torch.float64, (n, 3), dev)
    _need(eps, "eps", torch.float64, None, dev)
    _need(sigma, "sigma", torch.float64, tuple(eps.shape), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(nbr, "nbr", torch.int32, None, dev)
    _need(nnbr, "nnbr", torch.int32, (n,), dev)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    if open_next and x_next is None:
        x_next = torch.empty_like(x)
    if ev is None:
        ev = torch.empty(8, dtype=torch.float64, device=dev)
    _need(x_next, "x_next", torch.float64, (n, 3), dev)
    _need(F, "F", torch.float64, (n, 3), dev)
    _need(e_atom, "e_atom", torch.float64, (n,), dev)
    _need(ev, "ev", torch.float64, (8,), dev)
    ws, need = _ws(OP_FORCES, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_md_step(
        ctypes.byref(b), int(precision), float(rc), ntypes, _ptr(eps), _ptr(sigma), n, _ptr(x),
        _ptr(types), _ptr(nbr), _ptr(nnbr), int(maxn), float(dt), float(mass), _ptr(v),
        _ptr(x_next), 1 if open_next else 0, _ptr(F), _ptr(e_atom), _ptr(ev), _ptr(ws), need,
        _stream(dev)), "ljmd_md_step")
    return x_next, F, ev


def _chain_ws(n, ws, dev):
    """Byte size of the OP_MD_CHAIN workspace, checked against ws: the rows of a run
    live there between calls, so a fresh one cannot be substituted."""
    need = int(_lib.load().ljmd_workspace_bytes(OP_MD_CHAIN, n, 0, 1))
    if ws is None:
        raise ValueError("the chained steps need the workspace kept between the steps of a run")
    _need(ws, "ws", torch.uint8, None, dev)
    if ws.numel() < need:
        raise ValueError(f"ws holds {ws.numel()} bytes, {need} needed")
    return need


def md_step_chained(L, precision, rc, eps, sigma, x, types, nbr, nnbr, maxn, dt, mass, v, half,
                    ws, x_next=None, open_next=True, F=None, e_atom=None, ev_prev=None):
    """md_step whose energy/virial/KE partial rows stay in half `half` of ws (an
    OP_MD_CHAIN workspace); its first workgroup sums the other half, left by the
    previous chained step, into ev_prev when given.  Returns x_next."""
    n = x.shape[0]
    dev = x.device
    ntypes = _ntypes(eps)
    _need(x, "x", torch.float64, (n, 3))
    _need(v, "v", torch.float64, (n, 3), dev)
    _need(eps, "eps", torch.float64, None, dev)
    _need(sigma, "sigma", torch.float64, tuple(eps.shape), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(nbr, "nbr", torch.int32, None, dev)
    _need(nnbr, "nnbr", torch.int32, (n,), dev)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    if open_next and x_next is None:
        x_next = torch.empty_like(x)
    _need(x_next, "x_next", torch.float64, (n, 3), dev)
    _need(F, "F", torch.float64, (n, 3), dev)
    _need(e_atom, "e_atom", torch.float64, (n,), dev)
    _need(ev_prev, "ev_prev", torch.float64, (8,), dev)
    need = _chain_ws(n, ws, dev)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_md_step_chained(
        ctypes.byref(b), int(precision), float(rc), ntypes, _ptr(eps), _ptr(sigma), n, _ptr(x),
        _ptr(types), _ptr(nbr), _ptr(nnbr), int(maxn), float(dt), float(mass), _ptr(v),
        _ptr(x_next), 1 if open_next else 0, _ptr(F), _ptr(e_atom), int(half), _ptr(ev_prev),
        _ptr(ws), need, _stream(dev)), "ljmd_md_step_chained")
    return x_next


def md_step_sums(n, half, ws, ev=None):
    """ev[8] (E, W, KE) of the md_step_chained call that wrote half `half` of ws."""
    dev = ws.device
    if ev is None:
        ev = torch.empty(8, dtype=torch.float64, device=dev)
    _need(ev, "ev", torch.float64, (8,), dev)
    need = _chain_ws(n, ws, dev)
    _lib.check(_lib.load().ljmd_md_step_sums(int(n), int(half), _ptr(ws), need, _ptr(ev),
                                             _stream(dev)), "ljmd_md_step_sums")
    return ev


def integrate(stage, dt, mass, L, x, v, F, ke=None, ws=None):
    """In-place velocity-Verlet stage; ke (device scalar) receives 1/2 m sum v^2 if given."""
    n = v.shape[0]
    dev = v.device
    _need(v, "v", torch.float64, (n, 3))
    if stage != KINETIC or F is not None:
        _need(F, "F", torch.float64, (n, 3), dev)
    if stage != KINETIC or x is not None:
        _need(x, "x", torch.float64, (n, 3), dev)
    _need(ke, "ke", torch.float64, (1,), dev)
    need = 0
    if ke is not None:
        ws, need = _ws(OP_INTEGRATE, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_integrate(
        int(stage), float(dt), float(mass), ctypes.byref(b), n, _ptr(x), _ptr(v), _ptr(F),
        _ptr(ke), _ptr(ws) if ke is not None else None, need, _stream(dev)), "ljmd_integrate")


def force_backward(L, precision, rc, eps, sigma, x, types, nbr, nnbr, maxn, g, gx=None,
                   geps=None, gsigma=None, accumulate=False, ws=None):
    """(gx, geps, gsigma) = VJP of the forces with cotangent g (FULL list)."""
    n = x.shape[0]
    dev = x.device
    ntypes = _ntypes(eps)
    _need(x, "x", torch.float64, (n, 3))
    _need(eps, "eps", torch.float64, None, dev)
    _need(sigma, "sigma", torch.float64, tuple(eps.shape), dev)
    _need(types, "types", torch.int32, (n,), dev)
    _need(nbr, "nbr", torch.int32, None, dev)
    _need(nnbr, "nnbr", torch.int32, (n,), dev)
    _need(g, "g", torch.float64, (n, 3), dev)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    if gx is None:
        gx = torch.empty_like(x)
    if geps is None:
        geps = torch.empty_like(eps)
    if gsigma is None:
        gsigma = torch.empty_like(eps)
    _need(gx, "gx", torch.float64, (n, 3), dev)
    _need(geps, "geps", torch.float64, tuple(eps.shape), dev)
    _need(gsigma, "gsigma", torch.float64, tuple(eps.shape), dev)
    ws, need = _ws(OP_BACKWARD, n, dev, ntypes=ntypes, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_force_backward(
        ctypes.byref(b), int(precision), float(rc), ntypes, _ptr(eps), _ptr(sigma), n, _ptr(x),
        _ptr(types), _ptr(nbr), _ptr(nnbr), int(maxn), _ptr(g), _ptr(gx), _ptr(geps),
        _ptr(gsigma), 1 if accumulate else 0, _ptr(ws), need, _stream(dev)),
        "ljmd_force_backward")
    return gx, geps, gsigma


def adjoint_kick(dt, w, xbar, vbar, g):
    n = xbar.shape[0]
    dev = xbar.device
    for t, name in ((xbar, "xbar"), (vbar, "vbar"), (g, "g")):
        _need(t, name, torch.float64, (n, 3), dev)
    _lib.check(_lib.load().ljmd_adjoint_kick(n, float(dt), float(w), _ptr(xbar), _ptr(vbar),
                                             _ptr(g), _stream(dev)), "ljmd_adjoint_kick")


def max_displacement(L, x, x_ref, out=None, ws=None):
    """Largest squared minimum-image displacement max_i |x_i - x_ref_i|^2 (device scalar;
    out: a one-element FP64 tensor, possibly a view into a longer buffer)."""
    n = x.shape[0]
    dev = x.device
    _need(x, "x", torch.float64, (n, 3))
    _need(x_ref, "x_ref", torch.float64, (n, 3), dev)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=dev)
    if out.device != dev or out.dtype != torch.float64 or out.numel() != 1:
        raise ValueError("out must be one FP64 element on the device of x")
    ws, need = _ws(OP_DISPLACEMENT, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_max_displacement(ctypes.byref(b), n, _ptr(x), _ptr(x_ref),
                                                 _ptr(out), _ptr(ws), need, _stream(dev)),
               "ljmd_max_displacement")
    return out


def traj_loss(L, x, xref, xbar=None, loss=None, ws=None):
    n = x.shape[0]
    dev = x.device
    _need(x, "x", torch.float64, (n, 3))
    _need(xref, "xref", torch.float64, (n, 3), dev)
    if xbar is None:
        xbar = torch.empty_like(x)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=dev)
    _need(xbar, "xbar", torch.float64, (n, 3), dev)
    _need(loss, "loss", torch.float64, (1,), dev)
    ws, need = _ws(OP_LOSS, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_traj_loss(ctypes.byref(b), n, _ptr(x), _ptr(xref), _ptr(xbar),
                                          _ptr(loss), _ptr(ws), need, _stream(dev)),
               "ljmd_traj_loss")
    return loss, xbar


def scatter_rows(ids, src, dst=None):
    """dst[ids[k]] = src[k] (rows); maps sorted-order results back to the caller's order."""
    n = src.shape[0]
    dev = src.device
    width = 1 if src.dim() == 1 else int(src.shape[1])
    _need(ids, "ids", torch.int64, (n,), dev)
    _need(src, "src", torch.float64, tuple(src.shape), dev)
    if dst is None:
        dst = torch.empty_like(src)
    _need(dst, "dst", torch.float64, tuple(src.shape), dev)
    _lib.check(_lib.load().ljmd_scatter_rows(n, width, _ptr(ids), _ptr(src), _ptr(dst),
                                             _stream(dev)), "ljmd_scatter_rows")
    return dst


def gather_rows(ids, src, dst=None):
    """dst[k] = src[ids[k]] (rows); brings caller-order data into sorted order."""
    n = ids.shape[0]
    dev = src.device
    width = 1 if src.dim() == 1 else int(src.shape[1])
    _need(ids, "ids", torch.int64, (n,), dev)
    _need(src, "src", torch.float64, None, dev)
    if src.shape[0] != n:
        raise ValueError("src must have one row per id")
    if dst is None:
        dst = torch.empty_like(src)
    _need(dst, "dst", torch.float64, tuple(src.shape), dev)
    _lib.check(_lib.load().ljmd_gather_rows(n, width, _ptr(ids), _ptr(src), _ptr(dst),
                                            _stream(dev)), "ljmd_gather_rows")
    return dst


def _ntypes(eps) -> int:
    p = int(eps.numel())
    t = int(round(((8 * p + 1) ** 0.5 - 1) / 2))
    if t * (t + 1) // 2 != p or not 1 <= t <= MAX_TYPES:
        raise ValueError(f"packed parameter length {p} is not T(T+1)/2 with 1 <= T <= {MAX_TYPES}")
    return t


def _sph_list(x, nbr, nnbr, maxn):
    n = x.shape[0]
    _need(x, "x", torch.float64, (n, 3))
    _need(nbr, "nbr", torch.int32, None, x.device)
    _need(nnbr, "nnbr", torch.int32, (n,), x.device)
    if nbr.numel() < list_shape(n, maxn)[0]:
        raise ValueError("nbr is smaller than the tiled list of n rows x maxn")
    return n, x.device


def sph_density(L, h, mass, c0, rho0, x, nbr, nnbr, maxn, rho=None, u_total=None,
                want_energy=False, ws=None):
    """SPH density of every particle over a FULL list with rlist >= 2h; with want_energy
    (or u_total given) also U = sum m u(rho) into the one-element u_total."""
    n, dev = _sph_list(x, nbr, nnbr, maxn)
    if rho is None:
        rho = torch.empty(n, dtype=torch.float64, device=dev)
    if want_energy and u_total is None:
        u_total = torch.empty(1, dtype=torch.float64, device=dev)
    _need(rho, "rho", torch.float64, (n,), dev)
    _need(u_total, "u_total", torch.float64, (1,), dev)
    ws, need = _ws(OP_SPH, n, dev, ws=ws) if u_total is not None else (None, 0)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_sph_density(
        ctypes.byref(b), float(h), float(mass), float(c0), float(rho0), n, _ptr(x), _ptr(nbr),
        _ptr(nnbr), int(maxn), _ptr(rho), _ptr(u_total), _ptr(ws), need, _stream(dev)),
        "ljmd_sph_density")
    return rho, u_total


def sph_accel(L, h, mass, c0, rho0, x, rho, nbr, nnbr, maxn, acc=None, ws=None):
    """Symmetric SPH pressure acceleration [n, 3] from the densities rho."""
    n, dev = _sph_list(x, nbr, nnbr, maxn)
    _need(rho, "rho", torch.float64, (n,), dev)
    if acc is None:
        acc = torch.empty_like(x)
    _need(acc, "acc", torch.float64, (n, 3), dev)
    ws, need = _ws(OP_SPH, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_sph_accel(
        ctypes.byref(b), float(h), float(mass), float(c0), float(rho0), n, _ptr(x), _ptr(rho),
        _ptr(nbr), _ptr(nnbr), int(maxn), _ptr(acc), _ptr(ws), need, _stream(dev)),
        "ljmd_sph_accel")
    return acc


def sph_accel_step(L, h, mass, c0, rho0, x, v, rho, nbr, nnbr, maxn, dt, acc=None, ws=None):
    """sph_accel, then the closing and next opening half kicks and the drift with wrap,
    in place on x and v (acc written only when given)."""
    n, dev = _sph_list(x, nbr, nnbr, maxn)
    _need(rho, "rho", torch.float64, (n,), dev)
    _need(v, "v", torch.float64, (n, 3), dev)
    _need(acc, "acc", torch.float64, (n, 3), dev)
    ws, need = _ws(OP_SPH, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_sph_accel_step(
        ctypes.byref(b), float(h), float(mass), float(c0), float(rho0), n, _ptr(x), _ptr(v),
        _ptr(rho), _ptr(nbr), _ptr(nnbr), int(maxn), float(dt), _ptr(acc), _ptr(ws), need,
        _stream(dev)), "ljmd_sph_accel_step")
    return x, v


def ewald_real(L, alpha, rc, x, q, nbr, nnbr, maxn, F=None, e_total=None, want_energy=False,
               accumulate=False, ws=None):
    """Ewald direct-space forces (and E_dir) over a FULL list with rlist >= rc."""
    n, dev = _sph_list(x, nbr, nnbr, maxn)
    _need(q, "q", torch.float64, (n,), dev)
    if F is None:
        F = torch.zeros_like(x)
    if want_energy and e_total is None:
        e_total = torch.empty(1, dtype=torch.float64, device=dev)
    _need(F, "F", torch.float64, (n, 3), dev)
    _need(e_total, "e_total", torch.float64, (1,), dev)
    ws, need = _ws(OP_EWALD_REAL, n, dev, ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_ewald_real(
        ctypes.byref(b), float(alpha), float(rc), n, _ptr(x), _ptr(q), _ptr(nbr), _ptr(nnbr),
        int(maxn), _ptr(F), _ptr(e_total), int(bool(accumulate)), _ptr(ws), need, _stream(dev)),
        "ljmd_ewald_real")
    return F, e_total


def spme_recip(L, alpha, order, K, x, q, F=None, e_total=None, want_energy=False,
               accumulate=False, ws=None):
    """SPME reciprocal-space forces (and E_rec + E_self) on a K[0] x K[1] x K[2] grid."""
    n = x.shape[0]
    dev = x.device
    _need(x, "x", torch.float64, (n, 3))
    _need(q, "q", torch.float64, (n,), dev)
    if F is None:
        F = torch.zeros_like(x)
    if want_energy and e_total is None:
        e_total = torch.empty(1, dtype=torch.float64, device=dev)
    _need(F, "F", torch.float64, (n, 3), dev)
    _need(e_total, "e_total", torch.float64, (1,), dev)
    Kc = (ctypes.c_int32 * 3)(*[int(k) for k in K])
    ws, need = _ws(OP_SPME, n, dev, ncells=int(K[0]) * int(K[1]) * int(K[2]), ws=ws)
    b = make_box(L)
    _lib.check(_lib.load().ljmd_spme_recip(
        ctypes.byref(b), float(alpha), int(order), Kc, n, _ptr(x), _ptr(q), _ptr(F),
        _ptr(e_total), int(bool(accumulate)), _ptr(ws), need, _stream(dev)), "ljmd_spme_recip")
    return F, e_total
