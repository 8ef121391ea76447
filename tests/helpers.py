"""Shared helpers of the GPU tests: device state allocation through torch and
field comparison metrics (per-variable max-normalised difference and
relative L1)."""
from __future__ import annotations

import numpy as np


def nvars(ndim: int) -> int:
    return 4 + ndim


def cells(cfg: dict) -> int:
    return cfg["n"] ** cfg["ndim"]


def alloc_state(cfg: dict, precision: str):
    from paper_1705_04374_amd.state import alloc_state as _alloc
    return _alloc(cfg, precision)


def read_state(ctx, spec, st) -> np.ndarray:
    """Conserved vector Q of eq. (system) of the current state, as float64
    numpy [nv, cells] (the library's to-conserved kernel adds Pi(a2) back to
    its energy slot)."""
    import torch
    from paper_1705_04374_amd import capi
    q = torch.empty((4 + spec.ndim, spec.n ** spec.ndim), dtype=torch.float64, device="cuda")
    capi.ofm_state_to_conserved(ctx, spec, st, q)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def oracle_shape(cfg: dict, a: np.ndarray) -> np.ndarray:
    nd, n = cfg["ndim"], cfg["n"]
    return a.reshape(nvars(nd), n if nd > 2 else 1, n if nd > 1 else 1, n)


def max_rel_field(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per variable: max |a - b| / max |b| (b the reference)."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / den


def rel_l1(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.abs(a - b).sum(axis=1) / np.maximum(np.abs(b).sum(axis=1), 1e-300)
