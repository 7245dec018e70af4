"""Short-range LJ molecular dynamics on one MI355X: the timestep loop.

The step follows the paper's timestep anatomy for short-range MD
(Introduction): from the neighbor list, compute each particle's forces,
propagate, and re-sort; with CabanaMD's split (CabanaMD subsection) the
library side sorts and builds lists while the force kernel and the
integration are the application's.  Every arithmetic step runs in libljmd's
HIP kernels; this module only owns buffers, the rebuild cadence and the
neighbor-capacity check.

Velocity Verlet with a fixed rebuild cadence (no displacement check):
    v += dt/2 F/m; x += dt v; wrap            (ljmd_integrate KICK_DRIFT)
    every `rebuild_every` steps: re-sort by cell and rebuild the list
    F = F(x)                                   (ljmd_compute_forces)
    v += dt/2 F/m                              (ljmd_integrate KICK)
With a FULL list the force call and the kicks of a step run as one launch
(ljmd_md_step, bitwise equal to the separate calls); with a HALF list the
closing kick of a step and the opening kick + drift of the next run as one
launch (ljmd_integrate KICK_KICK_DRIFT).
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib, ops
from ._lib import FP64, FULL, HALF, KICK, KICK_DRIFT, KICK_KICK_DRIFT, KINETIC


def _dev(device):
    return torch.device(device if device is not None else "cuda")


def _to(t, dtype, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


def initial_maxn(n, L, rlist, kind):
    """Row capacity guess from the mean density: 1.3x the ideal-gas count plus 16."""
    vol = float(L[0]) * float(L[1]) * float(L[2])
    mean = 4.0 / 3.0 * math.pi * rlist ** 3 * n / vol
    if kind == HALF:
        mean *= 0.5
    return int(math.ceil((1.3 * mean + 16) / 4.0) * 4)


class NeighborList:
    """Atoms sorted by cell plus their tiled-ELL Verlet list (library-owned indexing)."""

    # A build may leave its longest-row check for later (defer=True) only while the
    # last checked build's longest row left at least this many free slots per row.
    HEADROOM = 8

    def __init__(self, L, rlist, kind=FULL, maxn=None, device=None):
        self.L = [float(v) for v in L]
        self.rlist = float(rlist)
        self.kind = kind
        self.device = _dev(device)
        self.maxn = maxn
        self.nbr = self.nnbr = self.cell_start = None
        self.max_count = None
        self.builds = 0
        self.deferred = 0          # builds whose longest-row check was left for later
        self.overflows = 0
        self.last_need = None      # longest row of the last checked build
        self._host_need = None     # pinned copy of a deferred build's longest row
        self._need_ready = None    # event recorded after that copy
        self._pending = False

    def build(self, x_sorted, cell_start, defer=False):
        """Build from cell-sorted positions; grow the row capacity until nothing is cut.

        Reading the longest row back makes the host wait for the build, and the GPU then
        idles until the host has queued the next launches.  With defer, and while the
        last checked build left HEADROOM free slots per row, the count is instead copied
        to pinned host memory in stream order and checked by check() -- at the next
        build at the latest; a row cut there raises RuntimeError (a liquid's longest row
        moves by a few entries between rebuilds, so the headroom covers it)."""
        self.check()
        n = x_sorted.shape[0]
        if self.maxn is None:
            self.maxn = initial_maxn(n, self.L, self.rlist, self.kind)
        nnbr = self.nnbr if self.nnbr is not None and self.nnbr.numel() == n else None
        if defer and self.last_need is not None and self.last_need + self.HEADROOM <= self.maxn:
            self.nbr, self.nnbr, self.max_count = ops.build_neighbors(
                self.L, self.rlist, self.kind, x_sorted, cell_start, self.maxn, self.nbr, nnbr,
                self.max_count)
            if self._host_need is None:
                self._host_need = torch.empty(1, dtype=torch.int32, pin_memory=True)
                self._need_ready = torch.cuda.Event()
            self._host_need.copy_(self.max_count, non_blocking=True)
            self._need_ready.record()
            self._pending = True
            self.deferred += 1
        else:
            while True:
                self.nbr, self.nnbr, self.max_count = ops.build_neighbors(
                    self.L, self.rlist, self.kind, x_sorted, cell_start, self.maxn, self.nbr,
                    nnbr, self.max_count)
                need = int(self.max_count.item())
                if need <= self.maxn:
                    break
                self.overflows += 1
                self.maxn = int(math.ceil((need + 8) / 4.0) * 4)
                self.nbr = nnbr = None
            self.last_need = need
        self.cell_start = cell_start
        self.builds += 1
        return self

    def check(self, block=True):
        """Check a deferred build's longest row against the row capacity (block=False:
        only if the stream has already passed it).  Raises RuntimeError when the build
        cut rows: forces computed from it missed pairs."""
        if not self._pending or (not block and not self._need_ready.query()):
            return self
        self._need_ready.synchronize()
        self._pending = False
        need = int(self._host_need[0])
        self.last_need = need
        if need > self.maxn:
            self.overflows += 1
            raise RuntimeError(
                f"neighbor list build {self.builds} cut rows: longest row {need} > capacity "
                f"{self.maxn} (checked after the build; later forces missed pairs)")
        return self


class LJSim:
    """Velocity-Verlet NVE simulation of a (multi-type) 12-6 LJ system on one GPU.

    State arrays live on the device in cell-sorted order; `ids` maps sorted
    position k to the caller's atom ids[k].
    """

    def __init__(self, L, rc=2.5, skin=0.3, eps=(1.0,), sigma=(1.0,), precision=FP64, kind=FULL,
                 dt=0.005, mass=1.0, rebuild_every=20, device=None):
        self.device = _dev(device)
        self.L = [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]
        self.rc = float(rc)
        self.rlist = float(rc) + float(skin)
        self.eps = _to(eps, torch.float64, self.device).reshape(-1)
        self.sigma = _to(sigma, torch.float64, self.device).reshape(-1)
        self.precision = precision
        self.kind = kind
        self.dt = float(dt)
        self.mass = float(mass)
        self.rebuild_every = int(rebuild_every)
        self.ntypes = ops._ntypes(self.eps)
        self._box = _lib.make_box(self.L)
        self.nl = NeighborList(self.L, self.rlist, kind, device=self.device)
        self.step_count = 0
        self._ws = {}
        self.skin = float(skin)

    # ------------------------------------------------------------------ setup
    def load(self, x, v, types=None, ids=None):
        dev = self.device
        x = _to(x, torch.float64, dev)
        n = x.shape[0]
        self.n = n
        v = _to(v, torch.float64, dev) if v is not None else torch.zeros_like(x)
        types = (_to(types, torch.int32, dev) if types is not None
                 else torch.zeros(n, dtype=torch.int32, device=dev))
        ids = _to(ids, torch.int64, dev) if ids is not None else None
        self.x, self.v, self.types, self.ids = x, v, types, ids
        # ping-pong buffers for the re-sort
        self._alt = (torch.empty_like(x), torch.empty_like(v), torch.empty_like(types),
                     torch.empty(n, dtype=torch.int64, device=dev))
        self.xn = torch.empty_like(x)  # next-step positions of the fused step
        self.F = torch.empty_like(x)
        self.e_atom = torch.empty(n, dtype=torch.float64, device=dev)
        # E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz, kinetic energy
        self.ev = torch.zeros(8, dtype=torch.float64, device=dev)
        self.ke = self.ev[7:]
        self._fargs = {}
        self._graphs = {}
        self.cell_start = None
        for op in (ops.OP_FORCES, ops.OP_INTEGRATE, ops.OP_MD_CHAIN):
            self._ws[op] = torch.empty(max(ops.workspace_bytes(op, n), 8), dtype=torch.uint8,
                                       device=dev)
        # the re-sort's counters and scan rows, allocated once so a rebuild allocates nothing
        nc = ops.grid(self.L, self.rlist)
        self._ws[ops.OP_BIN] = torch.empty(
            max(ops.workspace_bytes(ops.OP_BIN, n, ncells=nc[0] * nc[1] * nc[2]), 8),
            dtype=torch.uint8, device=dev)
        # dangerous-build check: positions at the last build, and per rebuild the largest
        # squared displacement since then, kept on the device until thermo() reads them
        self._ws[ops.OP_DISPLACEMENT] = torch.empty(
            max(ops.workspace_bytes(ops.OP_DISPLACEMENT, n), 8), dtype=torch.uint8, device=dev)
        self._xref = torch.empty_like(x)
        self._have_ref = False
        self._disp2 = torch.zeros(self.DISP_HISTORY, dtype=torch.float64, device=dev)
        self._ndisp = 0
        self._disp_seen = []
        self.rebuild()
        self.compute_forces(energy=True)
        ops.integrate(KINETIC, self.dt, self.mass, self.L, None, self.v, None, ke=self.ke,
                      ws=self._ws[ops.OP_INTEGRATE])
        return self

    DISP_HISTORY = 4096

    def _check_displacement(self):
        """Largest squared displacement since the last build, into the device history."""
        if self._ndisp == self.DISP_HISTORY:
            self._disp_seen.extend(self._disp2.tolist())
            self._ndisp = 0
        ops.max_displacement(self.L, self.x, self._xref, out=self._disp2[self._ndisp:self._ndisp + 1],
                             ws=self._ws[ops.OP_DISPLACEMENT])
        self._ndisp += 1

    def rebuild(self):
        # the previous build's deferred row check first: if it raises, nothing of this
        # rebuild has happened yet (positions still in the order the list belongs to)
        self.nl.check()
        if self._have_ref:
            self._check_displacement()
        xo, vo, to, io, self.cell_start = ops.bin(
            self.L, self.rlist, self.x, self.v, self.types, self.ids, out=self._alt,
            cell_start=self.cell_start, ws=self._ws.get(ops.OP_BIN))
        self._alt = (self.x, self.v, self.types,
                     self.ids if self.ids is not None else torch.empty_like(io))
        self.x, self.v, self.types, self.ids = xo, vo, to, io
        self._xref.copy_(self.x)
        self.nl.build(self.x, self.cell_start, defer=True)
        self._have_ref = True
        self._fargs = {}

    def displacement_history(self):
        """Per rebuild so far, the largest displacement of any atom since the build before."""
        return [math.sqrt(v) for v in self._disp_seen + self._disp2[:self._ndisp].tolist()]

    def displacement_report(self):
        """Dangerous-build check over every rebuild so far: a list of cutoff rc + skin
        holds every pair inside rc only while no atom has moved more than skin/2 since
        it was built.  Returns (windows checked, windows in which some atom moved more
        than skin/2, the largest displacement seen)."""
        d = self.displacement_history()
        return len(d), sum(1 for v in d if v > 0.5 * self.skin), max(d) if d else 0.0

    # ------------------------------------------------------------------- step
    def compute_forces(self, energy=True):
        ops.compute_forces(self.L, self.precision, self.kind, self.rc, self.eps, self.sigma,
                           self.x, self.types, self.nl.nbr, self.nl.nnbr, self.nl.maxn, F=self.F,
                           e_atom=self.e_atom if energy else None,
                           ev=self.ev[:7] if energy else None, want_energy=energy,
                           ws=self._ws[ops.OP_FORCES])

    def _step_args(self, energy):
        """ctypes argument tuples of the three per-step calls for the current buffers."""
        p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        box = ctypes.byref(self._box)
        n = self.n
        wsf, wsi = self._ws[ops.OP_FORCES], self._ws[ops.OP_INTEGRATE]
        kd = (KICK_DRIFT, self.dt, self.mass, box, n, p(self.x), p(self.v), p(self.F), None, None,
              0, st)
        fc = (box, self.precision, self.kind, self.rc, self.ntypes, p(self.eps), p(self.sigma), n,
              p(self.x), p(self.types), p(self.nl.nbr), p(self.nl.nnbr), self.nl.maxn, p(self.F),
              p(self.e_atom) if energy else None, p(self.ev) if energy else None, p(wsf),
              wsf.numel(), st)
        kk = (KICK, self.dt, self.mass, box, n, p(self.x), p(self.v), p(self.F),
              p(self.ke) if energy else None, p(wsi), wsi.numel(), st)
        kkd = (KICK_KICK_DRIFT,) + kk[1:]
        return kd, fc, kk, kkd

    def _fused_args(self, energy):
        """ljmd_md_step argument tuples (opening the next step, closing the call) for the
        current position buffer; cached per buffer until the next rebuild."""
        stream = torch.cuda.current_stream(self.device).cuda_stream
        key = (self.x.data_ptr(), energy, stream)
        if key not in self._fargs:
            p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
            st = ctypes.c_void_p(stream)
            wsf = self._ws[ops.OP_FORCES]
            head = (ctypes.byref(self._box), self.precision, self.rc, self.ntypes, p(self.eps),
                    p(self.sigma), self.n, p(self.x), p(self.types), p(self.nl.nbr),
                    p(self.nl.nnbr), self.nl.maxn, self.dt, self.mass, p(self.v), p(self.xn))
            tail = (p(self.F), p(self.e_atom) if energy else None, p(self.ev), p(wsf),
                    wsf.numel(), st)
            self._fargs[key] = (head + (1,) + tail, head + (0,) + tail)
        return self._fargs[key]

    def _chained_args(self, energy, half, first):
        """ljmd_md_step_chained argument tuples (opening the next step, closing the call)
        writing partial rows to `half`; unless `first`, the launch also sums the
        other half into ev.  Cached per buffer until the next rebuild."""
        stream = torch.cuda.current_stream(self.device).cuda_stream
        key = ("chain", self.x.data_ptr(), energy, stream, half, first)
        if key not in self._fargs:
            p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
            ws = self._ws[ops.OP_MD_CHAIN]
            head = (ctypes.byref(self._box), self.precision, self.rc, self.ntypes, p(self.eps),
                    p(self.sigma), self.n, p(self.x), p(self.types), p(self.nl.nbr),
                    p(self.nl.nnbr), self.nl.maxn, self.dt, self.mass, p(self.v), p(self.xn))
            tail = (p(self.F), p(self.e_atom) if energy else None, half,
                    None if first else p(self.ev), p(ws), ws.numel(), ctypes.c_void_p(stream))
            self._fargs[key] = (head + (1,) + tail, head + (0,) + tail)
        return self._fargs[key]

    def _window_graph(self, m, energy):
        """HIP graph of m fused steps that each open the next one, from the current
        buffers; captured once per buffer arrangement and replayed afterwards."""
        key = (m, energy, self.x.data_ptr(), self.xn.data_ptr(), self.v.data_ptr(),
               self.types.data_ptr(), self.nl.nbr.data_ptr(), self.nl.nnbr.data_ptr(),
               self.nl.maxn)
        g = self._graphs.get(key)
        if g is None:
            mdstep = _lib.load().ljmd_md_step
            x0, xn0 = self.x, self.xn
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(m):
                    _lib.check(mdstep(*self._fused_args(energy)[0]), "ljmd_md_step")
                    self.x, self.xn = self.xn, self.x
            self.x, self.xn = x0, xn0
            self._graphs[key] = g
        return g

    def step(self, nsteps=1, energy=True, force_events=None, graphs=False, on_positions=None,
             chain=True):
        """Advance nsteps velocity-Verlet steps; E, W and KE are produced every step
        (the per-atom energy only when energy is true).

        FULL lists run one fused launch per step (ljmd_md_step_chained, or
        ljmd_md_step without chain); HALF lists run the separate force and
        integration calls.  force_events: optional iterator with one item per step,
        a pre-created (start, end) pair of timing events recorded on the current stream
        just before and just after that step's force launch (either may be None, so one
        pair can span the launches of several steps), or None.  graphs: replay the steps between
        two rebuilds as one captured HIP graph (FULL lists, no timing events; bitwise
        the same trajectory as launching them one by one).  on_positions: optional callable
        given, for every step in order, the positions tensor the force call of that
        step reads (valid until the next launch on the stream; clone to keep it).
        chain: launched steps run as ljmd_md_step_chained, each summing the previous
        step's energy/virial/KE rows in its own launch (one launch per step); the last
        step's sums come from ljmd_md_step_sums, so E, W and KE are bitwise those of
        ljmd_md_step.
        """
        if nsteps <= 0:
            return self
        lib = _lib.load()
        if self.kind != FULL:
            return self._step_unfused(nsteps, energy, force_events, on_positions)
        integrate, mdstep = lib.ljmd_integrate, lib.ljmd_md_step
        use_graphs = graphs and force_events is None and on_positions is None
        name = "ljmd_md_step"
        if chain and not use_graphs:
            mdstep, name = lib.ljmd_md_step_chained, "ljmd_md_step_chained"
        else:
            chain = False
        half = None  # half of the chained workspace the previous launch wrote
        kd = self._step_args(energy)[0]
        _lib.check(integrate(*kd), "ljmd_integrate")
        s = 0
        while s < nsteps:
            self.step_count += 1
            if self.step_count % self.rebuild_every == 0:
                self.rebuild()
            # steps from this one up to (not including) the next rebuild, all of which
            # open a following step: one graph replay
            m = min(self.rebuild_every - self.step_count % self.rebuild_every, nsteps - s - 1)
            if use_graphs and m >= 2:
                self._window_graph(m, energy).replay()
                if m % 2:
                    self.x, self.xn = self.xn, self.x
                self.step_count += m - 1
                s += m
                continue
            last = s == nsteps - 1
            if chain:
                first = half is None
                half = 0 if first else 1 - half
                args = self._chained_args(energy, half, first)[1 if last else 0]
            else:
                args = self._fused_args(energy)[1 if last else 0]
            ab = next(force_events) if force_events is not None else None
            if ab is not None and ab[0] is not None:
                ab[0].record()
            _lib.check(mdstep(*args), name)
            if ab is not None and ab[1] is not None:
                ab[1].record()
            if chain and last:
                ops.md_step_sums(self.n, half, self._ws[ops.OP_MD_CHAIN], ev=self.ev)
            if on_positions is not None:
                on_positions(self.x)
            if not last:
                self.x, self.xn = self.xn, self.x
            s += 1
        self.nl.check(block=False)
        return self

    def _step_unfused(self, nsteps, energy, force_events, on_positions=None):
        lib = _lib.load()
        integrate, forces = lib.ljmd_integrate, lib.ljmd_compute_forces
        kd, fc, kk, kkd = self._step_args(energy)
        _lib.check(integrate(*kd), "ljmd_integrate")
        for s in range(nsteps):
            self.step_count += 1
            if self.step_count % self.rebuild_every == 0:
                self.rebuild()
                kd, fc, kk, kkd = self._step_args(energy)
            ab = next(force_events) if force_events is not None else None
            if ab is not None and ab[0] is not None:
                ab[0].record()
            _lib.check(forces(*fc), "ljmd_compute_forces")
            if ab is not None and ab[1] is not None:
                ab[1].record()
            if on_positions is not None:
                on_positions(self.x)
            # closing half kick of this step fused with the opening kick + drift of the
            # next one (same operations, one pass); the call ends on a plain half kick
            _lib.check(integrate(*(kk if s == nsteps - 1 else kkd)), "ljmd_integrate")
        self.nl.check(block=False)
        return self

    # ---------------------------------------------------------------- reports
    def thermo(self):
        self.nl.check()
        ev = self.ev.cpu()
        ke = float(ev[7])
        pe = float(ev[0])
        vol = self.L[0] * self.L[1] * self.L[2]
        temp = 2.0 * ke / (3 * self.n - 3)
        press = (self.n * temp + float(ev[1] + ev[2] + ev[3]) / 3.0) / vol
        checked, dangerous, dmax = self.displacement_report()
        return dict(step=self.step_count, pe=pe, ke=ke, etot=pe + ke, temp=temp, press=press,
                    virial=ev[1:7].tolist(), builds=self.nl.builds, maxn=self.nl.maxn,
                    checked_builds=checked, dangerous_builds=dangerous, max_displacement=dmax)

    def in_caller_order(self, t):
        """Rows of a sorted-order tensor rearranged into the caller's atom order (ids)."""
        return ops.scatter_rows(self.ids, t.contiguous())
