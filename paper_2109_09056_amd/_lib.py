"""ctypes loader for libljmd.so, the gfx950 library behind include/ljmd.h.

Loading fails loudly when the library has not been built: there is no CPU or
PyTorch fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libljmd.so")

# constants mirrored from include/ljmd.h
OK, EINVAL, EBOX, EWORKSPACE, EHIP = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
FULL, HALF = 0, 1
KICK_DRIFT, KICK, KINETIC, KICK_KICK_DRIFT = 0, 1, 2, 3
(OP_BIN, OP_FORCES, OP_BACKWARD, OP_INTEGRATE, OP_LOSS, OP_CSR, OP_FORCES_CSR, OP_SPH,
 OP_EWALD_REAL, OP_SPME, OP_MD_CHAIN, OP_DISPLACEMENT, OP_BUILD_CSR) = range(13)
SPME_MAX_GRID = 256
MAX_TYPES = 8
TILE = 64
MAX_TEAM = 16
SMALL_GRID_ATOMS = 32768  # tiled FULL-list forces: four lanes per atom up to here, then two
NOALLOC_SCRATCH_BYTES = 2 << 20  # static scratch of ljmd_md_step_noalloc
NOALLOC_MAX_ATOMS = 4194304


class Box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3)]


_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_box = ctypes.POINTER(Box)

# name -> (restype, argtypes); exactly the functions declared in include/ljmd.h
SIGNATURES = {
    "ljmd_grid": (_int, [_box, _dbl, ctypes.POINTER(_i32)]),
    "ljmd_workspace_bytes": (_sz, [_int, _i64, _i64, _i32]),
    "ljmd_error_string": (ctypes.c_char_p, [_int]),
    "ljmd_last_error": (ctypes.c_char_p, []),
    "ljmd_bin": (_int, [_box, _dbl, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _i64, _p, _sz, _p]),
    "ljmd_build_neighbors": (_int, [_box, _dbl, _int, _i64, _p, _p, _i32, _p, _p, _p, _p]),
    "ljmd_build_neighbors_csr": (_int, [_box, _dbl, _int, _i64, _p, _p, _p, _p, _i64, _p, _sz,
                                        _p]),
    "ljmd_compute_forces": (_int, [_box, _int, _int, _dbl, _i32, _p, _p, _i64, _p, _p, _p, _p,
                                   _i32, _p, _p, _p, _p, _sz, _p]),
    "ljmd_integrate": (_int, [_int, _dbl, _dbl, _box, _i64, _p, _p, _p, _p, _p, _sz, _p]),
    "ljmd_force_backward": (_int, [_box, _int, _dbl, _i32, _p, _p, _i64, _p, _p, _p, _p, _i32,
                                   _p, _p, _p, _p, _int, _p, _sz, _p]),
    "ljmd_md_step": (_int, [_box, _int, _dbl, _i32, _p, _p, _i64, _p, _p, _p, _p, _i32, _dbl,
                            _dbl, _p, _p, _int, _p, _p, _p, _p, _sz, _p]),
    "ljmd_md_step_noalloc": (_int, [_box, _int, _dbl, _i32, _p, _p, _i64, _p, _p, _p, _p,
                                    _i32, _dbl, _dbl, _p, _p, _int, _p, _p, _p, _p]),
    "ljmd_md_step_chained": (_int, [_box, _int, _dbl, _i32, _p, _p, _i64, _p, _p, _p, _p, _i32,
                                    _dbl, _dbl, _p, _p, _int, _p, _p, _int, _p, _p, _sz, _p]),
    "ljmd_md_step_sums": (_int, [_i64, _int, _p, _sz, _p, _p]),
    "ljmd_list_to_csr": (_int, [_i64, _p, _p, _i32, _p, _p, _i64, _p, _sz, _p]),
    "ljmd_compute_forces_csr": (_int, [_box, _int, _dbl, _i32, _p, _p, _i64, _p, _p, _p, _p,
                                       _i32, _p, _p, _p, _p, _sz, _p]),
    "ljmd_compute_forces_aosoa": (_int, [_box, _int, _dbl, _i32, _p, _p, _i64, _i32, _p, _p,
                                         _p, _p, _i32, _p, _p, _p, _p, _sz, _p]),
    "ljmd_aosoa_convert": (_int, [_i64, _i32, _int, _p, _p, _p]),
    "ljmd_sph_density": (_int, [_box, _dbl, _dbl, _dbl, _dbl, _i64, _p, _p, _p, _i32, _p, _p,
                                _p, _sz, _p]),
    "ljmd_sph_accel": (_int, [_box, _dbl, _dbl, _dbl, _dbl, _i64, _p, _p, _p, _p, _i32, _p, _p,
                              _sz, _p]),
    "ljmd_sph_accel_step": (_int, [_box, _dbl, _dbl, _dbl, _dbl, _i64, _p, _p, _p, _p, _p, _i32,
                                   _dbl, _p, _p, _sz, _p]),
    "ljmd_ewald_real": (_int, [_box, _dbl, _dbl, _i64, _p, _p, _p, _p, _i32, _p, _p, _int, _p,
                               _sz, _p]),
    "ljmd_spme_recip": (_int, [_box, _dbl, _i32, ctypes.POINTER(_i32), _i64, _p, _p, _p, _p,
                               _int, _p, _sz, _p]),
    "ljmd_adjoint_kick": (_int, [_i64, _dbl, _dbl, _p, _p, _p, _p]),
    "ljmd_max_displacement": (_int, [_box, _i64, _p, _p, _p, _p, _sz, _p]),
    "ljmd_traj_loss": (_int, [_box, _i64, _p, _p, _p, _p, _p, _sz, _p]),
    "ljmd_scatter_rows": (_int, [_i64, _i32, _p, _p, _p, _p]),
    "ljmd_gather_rows": (_int, [_i64, _i32, _p, _p, _p, _p]),
}

_lib = None
_lock = threading.Lock()


class LjmdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: error {code}: {detail}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libljmd.so (built by paper_2109_09056_amd.build); raise if it is absent."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build the HIP library first "
                    "(python -m paper_2109_09056_amd.build or __graft_entry__.build())")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(code: int, where: str) -> None:
    if code != OK:
        detail = load().ljmd_last_error().decode(errors="replace")
        raise LjmdError(code, where, detail)


def make_box(L) -> Box:
    b = Box()
    vals = [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]
    if len(vals) != 3:
        raise ValueError("box needs three edges")
    for k in range(3):
        b.L[k] = vals[k]
    return b
