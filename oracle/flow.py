"""ctypes wrapper of the serial FP64 oracle solver (``flow_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the library.  It builds the C
file with gcc on first use (``-O2 -ffp-contract=off``, no vector intrinsics).

What the C code computes is described in its header (the five-equation model
of Sec. 2.1, the finite-volume scheme of Sec. 2.2 and the cloud set-up of
Sec. 3.1 of arXiv:1705.04374).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flow_oracle.c")
_LIB = os.path.join(_HERE, "_flow_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (plain -O2, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Spec(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("n", C.c_int32), ("bc", C.c_int32), ("n_sub", C.c_int32),
        ("cfl", C.c_double),
        ("gamma1", C.c_double), ("pc1", C.c_double), ("gamma2", C.c_double), ("pc2", C.c_double),
        ("rho1", C.c_double), ("rho2", C.c_double),
        ("p_bubble", C.c_double), ("p_inf", C.c_double),
        ("center", C.c_double * 3),
        ("cloud_radius", C.c_double), ("ramp_delta", C.c_double), ("ramp_width", C.c_double),
        ("weno_eps", C.c_double), ("weno_order", C.c_int32), ("pad", C.c_int32),
    ]


class Box(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("len", C.c_int32 * 3)]


class Qoi(C.Structure):
    _fields_ = [
        ("p_max", C.c_double), ("x", C.c_double * 3), ("t_at_max", C.c_double), ("t", C.c_double),
        ("argmax", C.c_int64), ("steps", C.c_int64), ("status", C.c_int32), ("pad", C.c_int32),
        ("p_sensor", C.c_double), ("t_p_sensor", C.c_double), ("gas_min", C.c_double),
        ("t_gas_min", C.c_double), ("c_max", C.c_double), ("peak_distance", C.c_double),
    ]


class Reduction(C.Structure):
    _fields_ = [
        ("s_max", C.c_double), ("p_max", C.c_double), ("argmax", C.c_int64),
        ("n_nonfinite", C.c_int64), ("n_negc2", C.c_int64),
        ("c_max", C.c_double), ("p_ball", C.c_double), ("a2_ball", C.c_double),
        ("n_ball_p", C.c_int64), ("n_ball_a", C.c_int64),
    ]


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.orc_k_coefficient.restype = C.c_double
        L.orc_k_coefficient.argtypes = [C.POINTER(Spec), C.c_double, C.c_double]
        L.orc_cons_to_prim.argtypes = [C.POINTER(Spec), _dp, _dp]
        L.orc_prim_to_cons.argtypes = [C.POINTER(Spec), _dp, _dp]
        L.orc_weno5_right_edge.restype = C.c_double
        L.orc_weno5_right_edge.argtypes = [C.c_double] * 6
        L.orc_weno3_right_edge.restype = C.c_double
        L.orc_weno3_right_edge.argtypes = [C.c_double] * 4
        L.orc_hllc.argtypes = [C.POINTER(Spec), C.c_int, _dp, _dp, _dp]
        L.orc_cell_edges.restype = C.c_int
        L.orc_char_ghost.argtypes = [C.POINTER(Spec), C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.orc_cell_edges.argtypes = [C.POINTER(Spec)] + [_dp] * 5 + [C.c_double, _dp, _dp]
        L.orc_rhs.argtypes = [C.POINTER(Spec), C.POINTER(Box), _dp, _dp, C.POINTER(C.c_int64)]
        L.orc_rk_coefficients.argtypes = [_dp, _dp]
        L.orc_step.argtypes = [C.POINTER(Spec), C.POINTER(Box), _dp, C.c_double]
        L.orc_reduce.argtypes = [C.POINTER(Spec), C.POINTER(Box), _dp, C.POINTER(Reduction)]
        L.orc_init.argtypes = [C.POINTER(Spec), C.POINTER(Box), _dp, C.c_int32, _dp]
        L.orc_solve.argtypes = [C.POINTER(Spec), _dp, C.c_double, C.c_int64, C.c_int64, C.POINTER(Qoi)]
        L.orc_run_steps.argtypes = [C.POINTER(Spec), _dp, C.c_int64, _dp]
        L.orc_box_steps.argtypes = [C.POINTER(Spec), C.POINTER(Box), _dp, C.c_int32, C.c_int64, _dp, _dp]
        L.orc_initial_reduction.argtypes = [C.POINTER(Spec), _dp, C.c_int32, C.POINTER(Reduction)]
    return _lib


def nvars(ndim: int) -> int:
    return 4 + ndim


def make_spec(cfg: dict) -> Spec:
    """Oracle spec from a plain workload dictionary (see ``workloads.configs``)."""
    s = Spec()
    s.ndim = cfg["ndim"]
    s.n = cfg["n"]
    s.bc = {"zero_gradient": 0, "periodic": 1, "characteristic": 2}[cfg.get("bc", "zero_gradient")]
    s.n_sub = cfg.get("n_sub", 4)
    s.cfl = cfg.get("cfl", 0.3)
    eos = cfg["eos"]
    s.gamma1, s.pc1, s.gamma2, s.pc2 = eos["gamma1"], eos["pc1"], eos["gamma2"], eos["pc2"]
    s.rho1, s.rho2 = cfg.get("rho1", 1000.0), cfg.get("rho2", 1.0)
    s.p_bubble, s.p_inf = cfg.get("p_bubble", 2340.0), cfg.get("p_inf", 1.0e7)
    c = cfg.get("center", (0.5, 0.5, 0.5))
    for a in range(3):
        s.center[a] = c[a]
    R = cfg.get("cloud_radius", 0.3)
    s.cloud_radius = R
    s.ramp_delta = cfg.get("ramp_delta", R / 20.0)
    s.ramp_width = cfg.get("ramp_width", R / 3.0)
    s.weno_eps = cfg.get("weno_eps", 1e-6)
    s.weno_order = cfg.get("weno_order", 5)
    return s


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def shape_of(cfg: dict, box=None):
    nd, n = cfg["ndim"], cfg["n"]
    if box is None:
        dims = [n if a < nd else 1 for a in range(3)]
    else:
        dims = [box[1][a] if a < nd else 1 for a in range(3)]
    return (nvars(nd), dims[2], dims[1], dims[0])


def _box(cfg, box=None) -> Box:
    b = Box()
    nd, n = cfg["ndim"], cfg["n"]
    for a in range(3):
        if box is None:
            b.lo[a] = 0
            b.len[a] = n if a < nd else 1
        else:
            b.lo[a] = box[0][a] if a < nd else 0
            b.len[a] = box[1][a] if a < nd else 1
    return b


def init_state(cfg: dict, bubbles: np.ndarray, box=None) -> np.ndarray:
    """Initial conserved state [nv, nz, ny, nx] of the domain (or of a box)."""
    s = make_spec(cfg)
    U = np.zeros(shape_of(cfg, box), dtype=np.float64)
    bub = np.ascontiguousarray(bubbles, dtype=np.float64).reshape(-1, 4)
    lib().orc_init(C.byref(s), C.byref(_box(cfg, box)), _ptr(bub), bub.shape[0], _ptr(U))
    return U


def prim_to_cons(cfg: dict, W: np.ndarray) -> np.ndarray:
    s = make_spec(cfg)
    nv = nvars(cfg["ndim"])
    Wf = np.ascontiguousarray(W, dtype=np.float64).reshape(nv, -1)
    Q = np.empty_like(Wf)
    w = np.empty(nv)
    q = np.empty(nv)
    for c in range(Wf.shape[1]):
        w[:] = Wf[:, c]
        lib().orc_prim_to_cons(C.byref(s), _ptr(w), _ptr(q))
        Q[:, c] = q
    return Q.reshape(W.shape)


def cons_to_prim(cfg: dict, U: np.ndarray) -> np.ndarray:
    s = make_spec(cfg)
    nv = nvars(cfg["ndim"])
    Uf = np.ascontiguousarray(U, dtype=np.float64).reshape(nv, -1)
    W = np.empty_like(Uf)
    w = np.empty(nv)
    q = np.empty(nv)
    for c in range(Uf.shape[1]):
        q[:] = Uf[:, c]
        lib().orc_cons_to_prim(C.byref(s), _ptr(q), _ptr(w))
        W[:, c] = w
    return W.reshape(U.shape)


def rhs(cfg: dict, U: np.ndarray, box=None):
    s = make_spec(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    L = np.empty_like(U)
    nfb = C.c_int64(0)
    lib().orc_rhs(C.byref(s), C.byref(_box(cfg, box)), _ptr(U), _ptr(L), C.byref(nfb))
    return L, nfb.value


def step(cfg: dict, U: np.ndarray, dt: float, box=None) -> np.ndarray:
    s = make_spec(cfg)
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    lib().orc_step(C.byref(s), C.byref(_box(cfg, box)), _ptr(U), dt)
    return U


def reduce(cfg: dict, U: np.ndarray, box=None) -> dict:
    s = make_spec(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    r = Reduction()
    lib().orc_reduce(C.byref(s), C.byref(_box(cfg, box)), _ptr(U), C.byref(r))
    return dict(s_max=r.s_max, p_max=r.p_max, argmax=r.argmax,
                n_nonfinite=r.n_nonfinite, n_negc2=r.n_negc2, c_max=r.c_max, p_ball=r.p_ball,
                a2_ball=r.a2_ball, n_ball_p=r.n_ball_p, n_ball_a=r.n_ball_a)


def initial_reduction(cfg: dict, bubbles: np.ndarray) -> dict:
    s = make_spec(cfg)
    bub = np.ascontiguousarray(bubbles, dtype=np.float64).reshape(-1, 4)
    r = Reduction()
    lib().orc_initial_reduction(C.byref(s), _ptr(bub), bub.shape[0], C.byref(r))
    return dict(s_max=r.s_max, p_max=r.p_max, argmax=r.argmax,
                n_nonfinite=r.n_nonfinite, n_negc2=r.n_negc2, c_max=r.c_max, p_ball=r.p_ball,
                a2_ball=r.a2_ball, n_ball_p=r.n_ball_p, n_ball_a=r.n_ball_a)


def run_steps(cfg: dict, U: np.ndarray, n_steps: int):
    """Exactly n_steps CFL steps of the whole domain; returns (U, dts)."""
    s = make_spec(cfg)
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    dts = np.zeros(max(n_steps, 1))
    lib().orc_run_steps(C.byref(s), _ptr(U), n_steps, _ptr(dts))
    return U, dts[:n_steps]


def box_steps(cfg: dict, bubbles: np.ndarray, box, dts) -> np.ndarray:
    """Initial state of a box advanced with the given step sizes (cells within
    9 cells per step of an interior box side are not exact)."""
    s = make_spec(cfg)
    U = np.zeros(shape_of(cfg, box), dtype=np.float64)
    bub = np.ascontiguousarray(bubbles, dtype=np.float64).reshape(-1, 4)
    d = np.ascontiguousarray(np.asarray(dts, dtype=np.float64).reshape(-1))
    if d.size == 0:
        d = np.zeros(1)
        nst = 0
    else:
        nst = d.size
    lib().orc_box_steps(C.byref(s), C.byref(_box(cfg, box)), _ptr(bub), bub.shape[0], nst, _ptr(d), _ptr(U))
    return U


def solve(cfg: dict, bubbles: np.ndarray, t_end: float = 0.0, n_steps: int = 0,
          max_steps: int = 10 ** 9, U0: np.ndarray | None = None) -> dict:
    """Full solve with QoI tracking (Sec. 3.3: global maximum pressure, its
    location and time)."""
    s = make_spec(cfg)
    if U0 is None:
        U = init_state(cfg, bubbles)
    else:
        U = np.array(U0, dtype=np.float64, order="C", copy=True)
    q = Qoi()
    lib().orc_solve(C.byref(s), _ptr(U), t_end, n_steps, max_steps, C.byref(q))
    return dict(p_max=q.p_max, x=tuple(q.x), t_at_max=q.t_at_max, t=q.t, argmax=q.argmax,
                steps=q.steps, status=q.status, p_sensor=q.p_sensor, t_p_sensor=q.t_p_sensor,
                gas_min=q.gas_min, t_gas_min=q.t_gas_min, c_max=q.c_max, peak_distance=q.peak_distance, U=U)


def weno5_right_edge(a, b, c, d, e, eps=1e-6) -> float:
    return lib().orc_weno5_right_edge(a, b, c, d, e, eps)


def weno3_right_edge(b, c, d, eps=1e-6) -> float:
    return lib().orc_weno3_right_edge(b, c, d, eps)


def cell_edges(cfg: dict, stencil):
    """Left and right edge primitives of the centre cell of a five-cell
    primitive stencil [5][nv] along one axis, with the positivity checks;
    returns (left, right, replaced)."""
    s = make_spec(cfg)
    nv = nvars(cfg["ndim"])
    st = [np.ascontiguousarray(stencil[k], dtype=np.float64) for k in range(5)]
    assert all(x.size == nv for x in st)
    lo, hi = np.zeros(nv), np.zeros(nv)
    r = lib().orc_cell_edges(C.byref(s), *[_ptr(x) for x in st], s.weno_eps, _ptr(lo), _ptr(hi))
    return lo, hi, bool(r)


def char_ghost(cfg: dict, axis: int, side: int, beta: float, w) -> np.ndarray:
    """Ghost primitives of the characteristic far-field condition outside
    the domain side (axis, side = -1 low / +1 high) next to a cell with
    primitives w."""
    s = make_spec(cfg)
    x = np.ascontiguousarray(w, dtype=np.float64)
    g = np.zeros_like(x)
    lib().orc_char_ghost(C.byref(s), axis, side, beta, _ptr(x), _ptr(g))
    return g


def hllc(cfg: dict, direction: int, wl, wr) -> np.ndarray:
    s = make_spec(cfg)
    nv = nvars(cfg["ndim"])
    a = np.ascontiguousarray(wl, dtype=np.float64)
    b = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(nv + 1)
    lib().orc_hllc(C.byref(s), direction, _ptr(a), _ptr(b), _ptr(f))
    return f


def k_coefficient(cfg: dict, a2: float, p: float) -> float:
    s = make_spec(cfg)
    return lib().orc_k_coefficient(C.byref(s), a2, p)


def rk_coefficients():
    a = np.zeros(3)
    b = np.zeros(3)
    lib().orc_rk_coefficients(_ptr(a), _ptr(b))
    return a, b
