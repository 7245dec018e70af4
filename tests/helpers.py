"""Shared test helpers: GPU availability, list decoding, parity metrics (no arithmetic of the method)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "ljmd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*\*?(ljmd_\w+)\(", src,
                                 re.M)))


def gpu_device():
    """cuda:0 with the HIP library loaded; skip only where there is no GPU at all."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2109_09056_amd import _lib
    _lib.load()  # raises if libljmd.so is missing: no fallback
    return torch.device("cuda:0")


def decode_rows(nbr, nnbr, maxn):
    """Tiled-ELL list -> list of per-row numpy arrays (sorted indices)."""
    nbr = np.asarray(nbr)
    nnbr = np.asarray(nnbr)
    n = nnbr.size
    tiles = max((n + 63) // 64, 1)
    full = nbr[:tiles * maxn * 64].reshape(tiles, maxn, 64).transpose(0, 2, 1).reshape(-1, maxn)
    return [full[i, :nnbr[i]] for i in range(n)]


def list_pairs(nbr, nnbr, maxn):
    """(i, j) arrays of every entry of a tiled-ELL list, in sorted-order indices, row-major
    (vectorised decode for large lists)."""
    nbr = np.asarray(nbr)
    nnbr = np.asarray(nnbr).astype(np.int64)
    n = nnbr.size
    tiles = max((n + 63) // 64, 1)
    full = nbr[:tiles * maxn * 64].reshape(tiles, maxn, 64).transpose(0, 2, 1).reshape(-1, maxn)
    keep = np.arange(maxn)[None, :] < nnbr[:, None]
    return np.repeat(np.arange(n, dtype=np.int64), nnbr), full[:n][keep].astype(np.int64)


def pair_array(rows_i, rows_j):
    """Sorted unique [P, 2] int64 array of (i, j) pairs."""
    a = np.stack([np.asarray(rows_i, dtype=np.int64), np.asarray(rows_j, dtype=np.int64)], 1)
    a = a[np.lexsort((a[:, 1], a[:, 0]))]
    return a


def gpu_pairs_by_id(nbr, nnbr, maxn, ids_sorted, half=False):
    """Pairs (id_i, id_j) of a GPU list in original ids; half lists as {min, max}."""
    rows = decode_rows(nbr, nnbr, maxn)
    ids_sorted = np.asarray(ids_sorted)
    ii = np.concatenate([np.full(r.size, i) for i, r in enumerate(rows)]) if rows else np.zeros(0)
    jj = np.concatenate(rows) if rows else np.zeros(0)
    a = ids_sorted[ii.astype(np.int64)]
    b = ids_sorted[jj.astype(np.int64)]
    if half:
        a, b = np.minimum(a, b), np.maximum(a, b)
    return pair_array(a, b)


def oracle_pairs(offsets, nbr, rows=None, half=False):
    n = offsets.size - 1
    rows = np.arange(n) if rows is None else np.asarray(rows)
    i = np.repeat(rows, np.diff(offsets))
    j = nbr.astype(np.int64)
    if half:
        i, j = np.minimum(i, j), np.maximum(i, j)
        a = np.unique(np.stack([i, j], 1), axis=0)
        return pair_array(a[:, 0], a[:, 1])
    return pair_array(i, j)


def max_rel_vec(a, b):
    """max_i |a_i - b_i|_2 / max_i |b_i|_2 over rows."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=1).max() / max(np.linalg.norm(b, axis=1).max(), 1e-300)


def pairs_within(x, L, rc):
    """Number of unordered pairs closer than rc (NumPy brute force, small n)."""
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r2 = (d * d).sum(-1)
    return int((np.triu(r2 < rc * rc, 1)).sum())
