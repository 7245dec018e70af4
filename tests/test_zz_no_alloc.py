"""The allocation-free step (ljmd_md_step_noalloc) against ljmd_md_step with a caller
workspace, through the C ABI: two calls in a row on one GPU, the second on a smaller
system, each compared bitwise (same kernels) on every output."""
import ctypes

import numpy as np
import pytest

import lj_inputs as li
from helpers import gpu_device

pytestmark = pytest.mark.gpu


def _step_outputs(lib, L, sim, noalloc, open_next, dev):
    """One fused step from sim's current state through either entry point; returns copies
    of (v, x_next, F, e_atom, ev)."""
    import torch
    from paper_2109_09056_amd import _lib, ops
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    n = sim.n
    v = sim.v.clone()
    xn = torch.full_like(sim.x, float("nan"))
    F = torch.full_like(sim.x, float("nan"))
    e = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    ev = torch.full((8,), float("nan"), dtype=torch.float64, device=dev)
    box = _lib.make_box(L)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    head = (ctypes.byref(box), sim.precision, sim.rc, sim.ntypes, p(sim.eps), p(sim.sigma), n,
            p(sim.x), p(sim.types), p(sim.nl.nbr), p(sim.nl.nnbr), sim.nl.maxn, sim.dt, sim.mass,
            p(v), p(xn), open_next, p(F), p(e), p(ev))
    if noalloc:
        rc = lib.ljmd_md_step_noalloc(*head, st)
        name = "ljmd_md_step_noalloc"
    else:
        ws = torch.empty(ops.workspace_bytes(ops.OP_FORCES, n), dtype=torch.uint8, device=dev)
        rc = lib.ljmd_md_step(*head, p(ws), ws.numel(), st)
        name = "ljmd_md_step"
    _lib.check(rc, name)
    torch.cuda.synchronize(dev)
    return v, xn, F, e, ev


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_step_matches_workspace_step(prec):
    import torch
    from paper_2109_09056_amd import _lib, md, ops
    dev = gpu_device()
    lib = _lib.load()
    P = ops.FP64 if prec == "fp64" else ops.MIXED
    # first call: 32,000 atoms, two types; second: 256 atoms, one type (fewer rows than
    # the first call left in the scratch)
    w2 = li.Workload("t", 3, cells=20, ntypes=2)
    for w, eps, sig, open_next in ((w2, *li.params(w2), 1),
                                  (li.WORKLOADS["lj256"], [1.0], [1.0], 0)):
        sim = md.LJSim(w.box, rc=w.rc, skin=w.skin, eps=eps, sigma=sig, precision=P,
                       dt=w.dt, device=dev)
        sim.load(li.positions(w), li.velocities(w), li.types(w))
        print(f"[noalloc] {prec} n={sim.n} ntypes={sim.ntypes} open_next={open_next}",
              flush=True)
        ref = _step_outputs(lib, w.box, sim, False, open_next, dev)
        got = _step_outputs(lib, w.box, sim, True, open_next, dev)
        names = ("v", "x_next", "F", "e_atom", "ev")
        for name, a, b in zip(names, ref, got):
            if name == "x_next" and not open_next:
                continue
            assert torch.equal(a, b), (name, sim.n)
        assert np.isfinite(got[4].cpu().numpy()).all()
