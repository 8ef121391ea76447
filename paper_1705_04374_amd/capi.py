"""Thin ctypes binding of ``libofm.so`` (declared in ``include/ofm.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (tensors, passed by ``data_ptr()``)
and the current HIP stream.  The library must have been built
(``python -m paper_1705_04374_amd.build``); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libofm.so")

OFM_OK, OFM_EINVAL, OFM_ENOMEM, OFM_EHIP, OFM_EUNSUPPORTED, OFM_ESINGULAR, OFM_EINFEASIBLE = 0, -1, -2, -3, -4, -5, -6
OFM_F32, OFM_F64 = 0, 1
OFM_BC_ZERO_GRADIENT, OFM_BC_PERIODIC, OFM_BC_CHARACTERISTIC = 0, 1, 2
OFM_MODE_TOLERANCE, OFM_MODE_BUDGET = 0, 1
OFM_NOALLOC_SCRATCH_BYTES = 4 << 20     # fixed device scratch of ofm_step_noalloc, per GPU
SAMPLE_OK, SAMPLE_NONFINITE, SAMPLE_NEGATIVE_C2, SAMPLE_MAX_STEPS = 0, 1, 2, 3

# Every symbol include/ofm.h declares.
EXPORTS = [
    "ofm_ctx_create", "ofm_ctx_destroy", "ofm_last_error", "ofm_sample_cloud", "ofm_state_init",
    "ofm_state_from_primitive", "ofm_state_to_conserved", "ofm_step", "ofm_step_noalloc", "ofm_solve", "ofm_solve_batch", "ofm_run_begin", "ofm_run_advance", "ofm_run_status", "ofm_run_destroy",
    "ofm_last_solve_stats",
    "ofm_mlmc_moments", "ofm_ofmlmc_coefficients", "ofm_ofmlmc_errors", "ofm_ofmlmc_estimate",
    "ofm_ofmlmc_optimal_M", "ofm_ofmlmc_fit_indicators", "ofm_mlmc_merge_moments", "ofm_tune_set", "ofm_tune_get", "ofm_autotune", "ofm_kernel_timing", "ofm_kernel_times",
    "ofm_nn_create", "ofm_nn_destroy", "ofm_nn_param_count", "ofm_nn_get_params", "ofm_nn_set_params",
    "ofm_nn_set_normalization", "ofm_nn_reset_optimizer", "ofm_nn_features", "ofm_nn_forward", "ofm_nn_grads",
    "ofm_nn_train_step",
]


class OfmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("ofm error %d: %s" % (code, msg))
        self.code = code


class Eos(C.Structure):
    _fields_ = [("gamma1", C.c_double), ("pc1", C.c_double), ("gamma2", C.c_double), ("pc2", C.c_double)]


class SolveSpec(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("n", C.c_int32), ("precision", C.c_int32), ("bc", C.c_int32),
        ("n_sub", C.c_int32), ("weno_order", C.c_int32),
        ("cfl", C.c_double), ("eos", Eos),
        ("rho1", C.c_double), ("rho2", C.c_double), ("p_bubble", C.c_double), ("p_inf", C.c_double),
        ("center", C.c_double * 3), ("cloud_radius", C.c_double), ("ramp_delta", C.c_double),
        ("ramp_width", C.c_double), ("weno_eps", C.c_double), ("t_end", C.c_double),
        ("n_steps", C.c_int64), ("max_steps", C.c_int64),
    ]


class Qoi(C.Structure):
    _fields_ = [
        ("p_max", C.c_double), ("x", C.c_double * 3), ("t_at_max", C.c_double), ("t", C.c_double),
        ("argmax", C.c_int64), ("steps", C.c_int64), ("status", C.c_int32), ("reserved", C.c_int32),
        ("p_sensor", C.c_double), ("t_p_sensor", C.c_double), ("gas_min", C.c_double), ("t_gas_min", C.c_double),
        ("c_max", C.c_double), ("peak_distance", C.c_double),
    ]

    def as_dict(self) -> dict:
        return dict(p_max=self.p_max, x=tuple(self.x), t_at_max=self.t_at_max, t=self.t, argmax=self.argmax,
                    steps=self.steps, status=self.status, p_sensor=self.p_sensor, t_p_sensor=self.t_p_sensor,
                    gas_min=self.gas_min, t_gas_min=self.t_gas_min, c_max=self.c_max,
                    peak_distance=self.peak_distance)


class CloudSpec(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("n_bubbles", C.c_int32), ("cloud_radius", C.c_double), ("center", C.c_double * 3),
        ("r_median", C.c_double), ("r_sigma", C.c_double), ("r_lo", C.c_double), ("r_hi", C.c_double),
    ]


class StateView(C.Structure):
    _fields_ = [("u", C.c_void_p), ("u_tmp", C.c_void_p), ("du", C.c_void_p)]


class BatchItem(C.Structure):
    _fields_ = [("spec", C.POINTER(SolveSpec)), ("bubbles", C.POINTER(C.c_double)), ("n_bubbles", C.c_int32),
                ("reserved", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("tx", C.c_int32), ("ty", C.c_int32), ("zchunk", C.c_int32), ("graph_steps", C.c_int32),
                ("stage_ms_per_step", C.c_double), ("candidates", C.c_int32), ("reserved", C.c_int32)]


class NNSpec(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("width", C.c_int32), ("d_out", C.c_int32), ("reserved", C.c_int32),
                ("pool_scale", C.c_float), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("adam_eps", C.c_float), ("reserved2", C.c_float),
                ("out_mean", C.c_float * 5), ("out_std", C.c_float * 5)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own libamdhip64.so.7: load it first so that this
        # library binds to the same HIP runtime (one runtime per process)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise OfmError(OFM_EUNSUPPORTED, "libofm.so not built: run python -m paper_1705_04374_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.ofm_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.ofm_ctx_destroy.argtypes = [vp]
        L.ofm_ctx_destroy.restype = None
        L.ofm_last_error.argtypes = [vp]
        L.ofm_last_error.restype = C.c_char_p
        L.ofm_sample_cloud.argtypes = [C.POINTER(CloudSpec), C.c_uint64, C.c_uint64, C.c_uint64, dp]
        L.ofm_state_init.argtypes = [vp, C.POINTER(SolveSpec), dp, i32, C.POINTER(StateView), vp]
        L.ofm_state_from_primitive.argtypes = [vp, C.POINTER(SolveSpec), vp, C.POINTER(StateView), vp]
        L.ofm_state_to_conserved.argtypes = [vp, C.POINTER(SolveSpec), C.POINTER(StateView), vp, vp]
        L.ofm_step.argtypes = [vp, C.POINTER(SolveSpec), C.POINTER(StateView), i64, C.POINTER(Qoi), dp, vp]
        L.ofm_step_noalloc.argtypes = [vp, C.POINTER(SolveSpec), C.POINTER(StateView), i64, C.POINTER(Qoi), dp, vp]
        L.ofm_solve.argtypes = [vp, C.POINTER(SolveSpec), dp, i32, C.POINTER(Qoi), vp]
        L.ofm_solve_batch.argtypes = [vp, C.POINTER(BatchItem), i32, C.POINTER(Qoi), vp]
        L.ofm_last_solve_stats.argtypes = [vp, dp, dp, dp]
        L.ofm_run_begin.argtypes = [vp, C.POINTER(BatchItem), i32, C.POINTER(vp), vp]
        L.ofm_run_advance.argtypes = [vp, i64, C.POINTER(i32)]
        L.ofm_run_status.argtypes = [vp, C.POINTER(Qoi), C.POINTER(i64), dp, dp]
        L.ofm_run_destroy.argtypes = [vp]
        L.ofm_run_destroy.restype = None
        L.ofm_mlmc_moments.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.ofm_ofmlmc_coefficients.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.ofm_ofmlmc_errors.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.ofm_ofmlmc_estimate.argtypes = [vp, i32, vp, vp, vp, vp]
        L.ofm_ofmlmc_optimal_M.argtypes = [vp, i32, vp, vp, vp, i32, C.c_double, vp, vp, vp]
        L.ofm_ofmlmc_fit_indicators.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.ofm_mlmc_merge_moments.argtypes = [vp, i32, vp, vp, vp, vp]
        L.ofm_tune_set.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32]
        L.ofm_tune_get.argtypes = [vp, i32, i32, i32, C.POINTER(TuneResult)]
        L.ofm_autotune.argtypes = [vp, C.POINTER(SolveSpec), C.POINTER(StateView), i32, C.POINTER(TuneResult),
                                   C.POINTER(TuneResult), i32, vp]
        L.ofm_kernel_timing.argtypes = [vp, i32]
        L.ofm_kernel_times.argtypes = [vp, C.POINTER(i64), dp, dp]
        L.ofm_nn_create.argtypes = [vp, C.POINTER(NNSpec), C.c_uint64, C.POINTER(vp)]
        L.ofm_nn_destroy.argtypes = [vp]
        L.ofm_nn_destroy.restype = None
        L.ofm_nn_param_count.argtypes = []
        L.ofm_nn_param_count.restype = i64
        L.ofm_nn_get_params.argtypes = [vp, vp, vp]
        L.ofm_nn_set_params.argtypes = [vp, vp, vp]
        L.ofm_nn_set_normalization.argtypes = [vp, vp, vp, vp]
        L.ofm_nn_reset_optimizer.argtypes = [vp, vp]
        L.ofm_nn_features.argtypes = [C.POINTER(CloudSpec), vp, i64, vp, vp]
        L.ofm_nn_forward.argtypes = [vp, vp, vp, i32, vp, vp]
        L.ofm_nn_grads.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        L.ofm_nn_train_step.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        _lib = L
    return _lib


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        self._check(lib().ofm_ctx_create(device, C.byref(h)), None)
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().ofm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, h):
        if rc != OFM_OK:
            msg = lib().ofm_last_error(h)
            raise OfmError(rc, msg.decode() if msg else "")

    def check(self, rc: int):
        self._check(rc, self.h)


def make_spec(cfg: dict, precision: str = "f64", t_end: float = 0.0, n_steps: int = 0,
              max_steps: int = 10 ** 7) -> SolveSpec:
    """SolveSpec from a plain workload dictionary (see ``workloads.configs``)."""
    s = SolveSpec()
    s.ndim = cfg["ndim"]
    s.n = cfg["n"]
    s.precision = {"f32": OFM_F32, "f64": OFM_F64}[precision]
    s.bc = {"zero_gradient": OFM_BC_ZERO_GRADIENT, "periodic": OFM_BC_PERIODIC,
            "characteristic": OFM_BC_CHARACTERISTIC}[cfg.get("bc", "zero_gradient")]
    s.n_sub = cfg.get("n_sub", 4)
    s.cfl = cfg.get("cfl", 0.3)
    e = cfg["eos"]
    s.eos = Eos(e["gamma1"], e["pc1"], e["gamma2"], e["pc2"])
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
    s.t_end = t_end
    s.n_steps = n_steps
    s.max_steps = max_steps
    return s


def cloud_spec(spec: dict) -> CloudSpec:
    c = CloudSpec()
    c.ndim = spec["ndim"]
    c.n_bubbles = spec["n_bubbles"]
    c.cloud_radius = spec["cloud_radius"]
    cen = spec.get("center", (0.5, 0.5, 0.5))
    for a in range(3):
        c.center[a] = cen[a]
    c.r_median, c.r_sigma = spec["r_median"], spec["r_sigma"]
    c.r_lo, c.r_hi = spec.get("r_lo", 0.0), spec.get("r_hi", 0.0)
    return c


def ofm_sample_cloud(spec: dict, seed: int, term: int, index: int) -> np.ndarray:
    cs = cloud_spec(spec)
    out = np.zeros((spec["n_bubbles"], 4))
    rc = lib().ofm_sample_cloud(C.byref(cs), seed, term, index, out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != OFM_OK:
        raise OfmError(rc, lib().ofm_last_error(None).decode())
    return out


def _bub(bubbles):
    b = np.ascontiguousarray(np.asarray(bubbles, dtype=np.float64).reshape(-1, 4))
    return b, b.ctypes.data_as(C.POINTER(C.c_double)), b.shape[0]


def ofm_state_init(ctx: Context, spec: SolveSpec, bubbles, st: StateView, stream=None):
    b, p, nb = _bub(bubbles)
    ctx.check(lib().ofm_state_init(ctx.h, C.byref(spec), p, nb, C.byref(st), _stream(stream)))


def ofm_state_from_primitive(ctx: Context, spec: SolveSpec, w, st: StateView, stream=None):
    ctx.check(lib().ofm_state_from_primitive(ctx.h, C.byref(spec), _dptr(w), C.byref(st), _stream(stream)))


def ofm_state_to_conserved(ctx: Context, spec: SolveSpec, st: StateView, q, stream=None):
    ctx.check(lib().ofm_state_to_conserved(ctx.h, C.byref(spec), C.byref(st), _dptr(q), _stream(stream)))


def ofm_step(ctx: Context, spec: SolveSpec, st: StateView, n_steps: int, stream=None):
    q = Qoi()
    dts = np.zeros(max(n_steps, 1))
    ctx.check(lib().ofm_step(ctx.h, C.byref(spec), C.byref(st), n_steps, C.byref(q),
                             dts.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return q.as_dict(), dts[:n_steps]


def ofm_step_noalloc(ctx: Context, spec: SolveSpec, st: StateView, n_steps: int, stream=None, log_dts=True):
    q = Qoi()
    dts = np.zeros(max(n_steps, 1))
    ptr = dts.ctypes.data_as(C.POINTER(C.c_double)) if log_dts else None
    ctx.check(lib().ofm_step_noalloc(ctx.h, C.byref(spec), C.byref(st), n_steps, C.byref(q), ptr, _stream(stream)))
    return q.as_dict(), (dts[:n_steps] if log_dts else None)


def ofm_solve(ctx: Context, spec: SolveSpec, bubbles, stream=None) -> dict:
    b, p, nb = _bub(bubbles)
    q = Qoi()
    ctx.check(lib().ofm_solve(ctx.h, C.byref(spec), p, nb, C.byref(q), _stream(stream)))
    return q.as_dict()


def ofm_solve_batch(ctx: Context, specs, bubbles_list, stream=None) -> list:
    n = len(specs)
    items = (BatchItem * n)()
    keep = []
    for i, (s, bl) in enumerate(zip(specs, bubbles_list)):
        b, p, nb = _bub(bl)
        keep.append((s, b))
        items[i].spec = C.pointer(s)
        items[i].bubbles = p
        items[i].n_bubbles = nb
    qs = (Qoi * n)()
    ctx.check(lib().ofm_solve_batch(ctx.h, items, n, qs, _stream(stream)))
    return [q.as_dict() for q in qs]


class Run:
    """A batched solve kept on the device and advanced in portions
    (ofm_run_* calls): the same solve as ofm_solve_batch."""

    def __init__(self, ctx: Context, specs, bubbles_list, stream=None):
        n = len(specs)
        items = (BatchItem * n)()
        keep = []
        for i, (s, bl) in enumerate(zip(specs, bubbles_list)):
            b, p, nb = _bub(bl)
            keep.append((s, b))
            items[i].spec = C.pointer(s)
            items[i].bubbles = p
            items[i].n_bubbles = nb
        self.ctx, self.n = ctx, n
        self.h = C.c_void_p()
        ctx.check(lib().ofm_run_begin(ctx.h, items, n, C.byref(self.h), _stream(stream)))

    def advance(self, max_steps: int) -> bool:
        """Advance by at least max_steps steps (or to the end); True once done."""
        done = C.c_int32()
        self.ctx.check(lib().ofm_run_advance(self.h, max_steps, C.byref(done)))
        return bool(done.value)

    def status(self) -> dict:
        qs = (Qoi * self.n)()
        steps, a, b = C.c_int64(), C.c_double(), C.c_double()
        self.ctx.check(lib().ofm_run_status(self.h, qs, C.byref(steps), C.byref(a), C.byref(b)))
        return dict(qoi=[q.as_dict() for q in qs], steps=steps.value, init_s=a.value, step_s=b.value)

    def close(self):
        if self.h:
            lib().ofm_run_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ofm_last_solve_stats(ctx: Context) -> dict:
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    ctx.check(lib().ofm_last_solve_stats(ctx.h, C.byref(a), C.byref(b), C.byref(c)))
    return dict(init_s=a.value, step_s=b.value, cell_steps=c.value)


def ofm_mlmc_moments(ctx: Context, qf, qc, ok, out, stream=None):
    ctx.check(lib().ofm_mlmc_moments(ctx.h, _dptr(qf), _dptr(qc), _dptr(ok), qf.numel(), _dptr(out),
                                     _stream(stream)))


def ofm_ofmlmc_coefficients(ctx: Context, L: int, mom, W, alpha, flag, stream=None):
    ctx.check(lib().ofm_ofmlmc_coefficients(ctx.h, L, _dptr(mom), _dptr(W), _dptr(alpha), _dptr(flag),
                                            _stream(stream)))


def ofm_ofmlmc_errors(ctx: Context, L: int, mom, alpha, sig, eps2, stream=None):
    ctx.check(lib().ofm_ofmlmc_errors(ctx.h, L, _dptr(mom), _dptr(alpha), _dptr(sig), _dptr(eps2),
                                      _stream(stream)))


def ofm_ofmlmc_estimate(ctx: Context, L: int, mom, alpha, E, stream=None):
    ctx.check(lib().ofm_ofmlmc_estimate(ctx.h, L, _dptr(mom), _dptr(alpha), _dptr(E), _stream(stream)))


def ofm_ofmlmc_optimal_M(ctx: Context, L: int, sig, W, have, mode: int, target: float, out, flag, stream=None):
    ctx.check(lib().ofm_ofmlmc_optimal_M(ctx.h, L, _dptr(sig), _dptr(W), _dptr(have), mode, target, _dptr(out),
                                         _dptr(flag), _stream(stream)))


def ofm_mlmc_merge_moments(ctx: Context, a, b, out, stream=None):
    """a, b, out: [n_terms, 6] float64 device tensors (out may be a or b)."""
    ctx.check(lib().ofm_mlmc_merge_moments(ctx.h, a.shape[0], _dptr(a), _dptr(b), _dptr(out), _stream(stream)))


def ofm_ofmlmc_fit_indicators(ctx: Context, L: int, first: int, m_floor: int, mom, v_hat, flag, stream=None):
    ctx.check(lib().ofm_ofmlmc_fit_indicators(ctx.h, L, first, m_floor, _dptr(mom), _dptr(v_hat), _dptr(flag),
                                              _stream(stream)))


def ofm_tune_set(ctx: Context, precision: int, ndim: int, n: int, tx: int, ty: int, zchunk: int,
                 graph_steps: int):
    ctx.check(lib().ofm_tune_set(ctx.h, precision, ndim, n, tx, ty, zchunk, graph_steps))


def ofm_tune_get(ctx: Context, precision: int, ndim: int, n: int) -> dict:
    r = TuneResult()
    ctx.check(lib().ofm_tune_get(ctx.h, precision, ndim, n, C.byref(r)))
    return dict(tx=r.tx, ty=r.ty, zchunk=r.zchunk, graph_steps=r.graph_steps)


def ofm_autotune(ctx: Context, spec: SolveSpec, st: StateView, steps: int = 2, stream=None) -> dict:
    """Time the compiled tile shapes / z-chunks on the (scratch) state st and
    keep the fastest for spec's precision, dimension and size class."""
    r = TuneResult()
    cap = 64
    every = (TuneResult * cap)()
    ctx.check(lib().ofm_autotune(ctx.h, C.byref(spec), C.byref(st), steps, C.byref(r), every, cap,
                                 _stream(stream)))
    return dict(tx=r.tx, ty=r.ty, zchunk=r.zchunk, graph_steps=r.graph_steps,
                stage_ms_per_step=r.stage_ms_per_step, candidates=r.candidates,
                table=[(e.tx, e.ty, e.zchunk, e.stage_ms_per_step) for e in every[:min(r.candidates, cap)]])


def ofm_kernel_timing(ctx: Context, enable: bool):
    ctx.check(lib().ofm_kernel_timing(ctx.h, 1 if enable else 0))


def ofm_kernel_times(ctx: Context) -> dict:
    n, ms, cells = C.c_int64(), C.c_double(), C.c_double()
    ctx.check(lib().ofm_kernel_times(ctx.h, C.byref(n), C.byref(ms), C.byref(cells)))
    return dict(launches=n.value, total_ms=ms.value, cells=cells.value)


class SetNet:
    """The learned control variate (ofm_nn_* calls)."""

    def __init__(self, ctx: Context, pool_scale: float, seed: int = 0, lr: float = 1e-3, beta1: float = 0.9,
                 beta2: float = 0.999, adam_eps: float = 1e-8, out_mean=(0.0,) * 5, out_std=(1.0,) * 5):
        sp = NNSpec()
        sp.d_in, sp.width, sp.d_out = 4, 128, 5
        sp.pool_scale, sp.lr, sp.beta1, sp.beta2, sp.adam_eps = pool_scale, lr, beta1, beta2, adam_eps
        for i in range(5):
            sp.out_mean[i] = out_mean[i]
            sp.out_std[i] = out_std[i]
        h = C.c_void_p()
        ctx.check(lib().ofm_nn_create(ctx.h, C.byref(sp), seed, C.byref(h)))
        self.h, self.ctx = h, ctx

    def close(self):
        if getattr(self, "h", None):
            lib().ofm_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != OFM_OK:
            raise OfmError(rc, lib().ofm_last_error(None).decode())

    @staticmethod
    def param_count() -> int:
        return int(lib().ofm_nn_param_count())

    def get_params(self, out, stream=None):
        self._chk(lib().ofm_nn_get_params(self.h, _dptr(out), _stream(stream)))

    def set_params(self, p, stream=None):
        self._chk(lib().ofm_nn_set_params(self.h, _dptr(p), _stream(stream)))

    def set_normalization(self, mean, std, stream=None):
        self._chk(lib().ofm_nn_set_normalization(self.h, _dptr(mean), _dptr(std), _stream(stream)))

    def reset_optimizer(self, stream=None):
        self._chk(lib().ofm_nn_reset_optimizer(self.h, _stream(stream)))

    def forward(self, x, offsets, y, stream=None):
        self._chk(lib().ofm_nn_forward(self.h, _dptr(x), _dptr(offsets), offsets.numel() - 1, _dptr(y),
                                       _stream(stream)))

    def grads(self, x, offsets, y_true, grads, loss, stream=None):
        self._chk(lib().ofm_nn_grads(self.h, _dptr(x), _dptr(offsets), offsets.numel() - 1, _dptr(y_true),
                                     _dptr(grads), _dptr(loss), _stream(stream)))

    def train_step(self, x, offsets, y_true, loss, stream=None):
        self._chk(lib().ofm_nn_train_step(self.h, _dptr(x), _dptr(offsets), offsets.numel() - 1, _dptr(y_true),
                                          _dptr(loss), _stream(stream)))


def ofm_nn_features(spec: dict, bubbles_dev, x_out, stream=None):
    cs = cloud_spec(spec)
    rc = lib().ofm_nn_features(C.byref(cs), _dptr(bubbles_dev), bubbles_dev.shape[0], _dptr(x_out), _stream(stream))
    if rc != OFM_OK:
        raise OfmError(rc, lib().ofm_last_error(None).decode())
