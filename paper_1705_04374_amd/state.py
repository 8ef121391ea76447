"""Device state buffers for the low-level stepping calls (torch tensors)."""
from __future__ import annotations

from . import capi


def alloc_state(cfg: dict, precision: str):
    """Three [nv, n^ndim] device arrays (state, ping-pong partner, RK register)
    and the ofm_state_view pointing at them."""
    import torch
    dt = torch.float64 if precision == "f64" else torch.float32
    shp = (4 + cfg["ndim"], cfg["n"] ** cfg["ndim"])
    bufs = [torch.empty(shp, dtype=dt, device="cuda") for _ in range(3)]
    st = capi.StateView(bufs[0].data_ptr(), bufs[1].data_ptr(), bufs[2].data_ptr())
    return st, bufs


def current(st, bufs):
    """The tensor that holds the current state (st.u)."""
    for b in bufs:
        if b.data_ptr() == st.u:
            return b
    raise ValueError("state pointer not among the buffers")
