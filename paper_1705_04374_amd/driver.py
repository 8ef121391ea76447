"""Adaptive OF-MLMC on top of the C ABI (Sec. 2.4.4 of arXiv:1705.04374).

The driver decides which samples to run next.  It does no arithmetic of the
method itself:
  * clouds come from ofm_sample_cloud;
  * solves from ofm_solve_batch (coupled pairs share their bubbles) and the
    learned level from the ofm_nn_* calls;
  * moments, coefficients, errors, estimate and sample allocation come from
    the ofm_mlmc_* / ofm_ofmlmc_* kernels, all FP64 on the device.

Terms (Sec. 2.4.1): with fidelities f_0 < f_1 < ... < f_L, term 0 holds
single samples of f_0 and term l >= 1 holds pairs (f_l, f_{l-1}) drawn with
the same omega.  With a learned level, f_0 is the network and the solver
levels follow.  Every term draws its omegas from its own stream
(seed, term, index), so terms are independent.  W_l is the measured time
per sample of term l (a pair costs both of its solves, Sec. 2.4.1).

Iteration (Sec. 2.4.4): warm-up counts (eq. (warmup), at least 2 per term)
-> solve -> moments -> coefficients (eq. (alpha-matvec)) -> errors
(eq. (ocv-mlmc-err)) -> stop if eps <= tau -> optimal counts (eq. (M-tol),
keeping computed samples) -> solve the additional samples -> ...
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import capi

SAMPLE_OK = capi.SAMPLE_OK


class Fidelity:
    """A solver level (grid n) or the learned network."""

    def __init__(self, kind: str, n: int = 0):
        self.kind, self.n = kind, n

    def __repr__(self):
        return "nn" if self.kind == "nn" else "%d^d" % self.n


class Ledger:
    """JSON lines of every sample: term, index, QoIs, status, seconds.  An
    existing ledger is read back on start (samples are not run again)."""

    def __init__(self, path: str | None):
        self.path = path
        self.rows = {}
        if path and os.path.exists(path):
            with open(path) as f:
                for line in f:
                    r = json.loads(line)
                    self.rows[(r["term"], r["index"])] = r

    def have(self, term: int, index: int):
        return self.rows.get((term, index))

    def add(self, rows: list):
        for r in rows:
            self.rows[(r["term"], r["index"])] = r
        if self.path:
            with open(self.path, "a") as f:
                for r in rows:
                    f.write(json.dumps(r) + "\n")


class OFMLMC:
    def __init__(self, ctx: capi.Context, solver_cfg: dict, cloud: dict, levels: list, precision: str = "f32",
                 t_end: float = 0.0, n_steps: int = 0, seed: int = 0, net=None, net_scale=None,
                 ledger: str | None = None, max_batch_bytes: float = 60e9, max_steps: int = 10 ** 6):
        self.ctx, self.cfg, self.cloud = ctx, solver_cfg, cloud
        self.precision, self.t_end, self.n_steps, self.seed = precision, t_end, n_steps, seed
        self.net = net
        self.fid = ([Fidelity("nn")] if net is not None else []) + [Fidelity("solver", n) for n in levels]
        self.L = len(self.fid) - 1
        self.ledger = Ledger(ledger)
        self.max_batch_bytes = max_batch_bytes
        self.max_steps = max_steps
        self.q = [dict(f=[], c=[], ok=[]) for _ in range(self.L + 1)]
        self.time = [0.0] * (self.L + 1)
        self.count = [0] * (self.L + 1)
        self.solve_seconds = 0.0

    # -- sampling -----------------------------------------------------------
    def _spec(self, n: int):
        cfg = dict(self.cfg)
        cfg["n"] = n
        return capi.make_spec(cfg, self.precision, t_end=self.t_end, n_steps=self.n_steps, max_steps=self.max_steps)

    def _state_bytes(self, n: int) -> float:
        d = self.cloud["ndim"]
        return 3.0 * (4 + d) * n ** d * (4 if self.precision == "f32" else 8)

    def _solve(self, ns: list, bubbles: list) -> list:
        """Batched solves, split so that one batch stays within max_batch_bytes."""
        out = [None] * len(ns)
        order = list(range(len(ns)))
        batch, size = [], 0.0
        t0 = time.perf_counter()

        def flush():
            if not batch:
                return
            qs = capi.ofm_solve_batch(self.ctx, [self._spec(ns[i]) for i in batch], [bubbles[i] for i in batch])
            for i, q in zip(batch, qs):
                out[i] = q
        for i in order:
            b = self._state_bytes(ns[i])
            if batch and size + b > self.max_batch_bytes:
                flush()
                batch, size = [], 0.0
            batch.append(i)
            size += b
        flush()
        self.solve_seconds += time.perf_counter() - t0
        return out

    def _net_qoi(self, bubbles: list) -> np.ndarray:
        import torch
        sets = len(bubbles)
        b = torch.tensor(np.concatenate(bubbles), dtype=torch.float64, device="cuda")
        x = torch.empty((b.shape[0], 4), dtype=torch.float32, device="cuda")
        capi.ofm_nn_features(self.cloud, b, x)
        sizes = [len(bb) for bb in bubbles]
        off = torch.tensor(np.concatenate([[0], np.cumsum(sizes)]), dtype=torch.int32, device="cuda")
        y = torch.empty((sets, 5), dtype=torch.float32, device="cuda")
        self.net.forward(x, off, y)
        torch.cuda.synchronize()
        return y[:, 0].double().cpu().numpy()

    def sample(self, k: int, m_new: int):
        """Run m_new fresh samples of term k."""
        if m_new <= 0:
            return
        start = self.count[k]
        idx = list(range(start, start + m_new))
        todo = [i for i in idx if self.ledger.have(k, i) is None]
        t0 = time.perf_counter()
        if todo:
            bubs = [capi.ofm_sample_cloud(self.cloud, self.seed, k, i) for i in todo]
            fine, coarse = self.fid[k], (self.fid[k - 1] if k >= 1 else None)
            res = {}
            for which, f in (("f", fine), ("c", coarse)):
                if f is None:
                    continue
                if f.kind == "nn":
                    vals = self._net_qoi(bubs)
                    res[which] = [dict(p_max=float(v), status=SAMPLE_OK, steps=0) for v in vals]
                else:
                    res[which] = self._solve([f.n] * len(todo), bubs)
            dt = (time.perf_counter() - t0) / len(todo)
            rows = []
            for j, i in enumerate(todo):
                qf = res["f"][j]
                qc = res["c"][j] if "c" in res else None
                ok = qf["status"] == SAMPLE_OK and (qc is None or qc["status"] == SAMPLE_OK)
                rows.append(dict(term=k, index=i, qf=qf["p_max"], qc=qc["p_max"] if qc else None, ok=bool(ok),
                                 status_f=qf["status"], status_c=qc["status"] if qc else None,
                                 xf=list(qf.get("x", ())), tf=qf.get("t_at_max"), seconds=dt))
            self.ledger.add(rows)
        for i in idx:
            r = self.ledger.have(k, i)
            self.q[k]["f"].append(r["qf"])
            self.q[k]["c"].append(r["qc"] if r["qc"] is not None else 0.0)
            self.q[k]["ok"].append(1 if r["ok"] else 0)
            self.time[k] += r["seconds"]
        self.count[k] += m_new

    # -- estimator (device kernels) -------------------------------------------
    def moments(self):
        import torch
        mom = torch.zeros((self.L + 1, 6), dtype=torch.float64, device="cuda")
        for k in range(self.L + 1):
            qf = torch.tensor(self.q[k]["f"], dtype=torch.float64, device="cuda")
            qc = torch.tensor(self.q[k]["c"], dtype=torch.float64, device="cuda") if k >= 1 else None
            ok = torch.tensor(self.q[k]["ok"], dtype=torch.int32, device="cuda")
            capi.ofm_mlmc_moments(self.ctx, qf, qc, ok, mom[k])
        return mom

    def work(self):
        """Measured seconds per sample of each term."""
        return [self.time[k] / max(self.count[k], 1) for k in range(self.L + 1)]

    def evaluate(self, W, classical: bool = False) -> dict:
        import torch
        L = self.L
        mom = self.moments()
        Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
        alpha = torch.ones(L + 1, dtype=torch.float64, device="cuda")
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        if not classical and L >= 1:
            capi.ofm_ofmlmc_coefficients(self.ctx, L, mom, Wd, alpha, flag)
        sig = torch.zeros(L + 1, dtype=torch.float64, device="cuda")
        eps2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        capi.ofm_ofmlmc_errors(self.ctx, L, mom, alpha, sig, eps2)
        E = torch.zeros(1, dtype=torch.float64, device="cuda")
        capi.ofm_ofmlmc_estimate(self.ctx, L, mom, alpha, E)
        torch.cuda.synchronize()
        m = mom.cpu().numpy()
        return dict(E=E.item(), eps=math.sqrt(max(eps2.item(), 0.0)), alpha=alpha.cpu().tolist(),
                    sigma_t2=sig.cpu().tolist(), singular=int(flag.item()), M=[int(v) for v in m[:, 0]],
                    mean_f=m[:, 1].tolist(), mean_c=m[:, 2].tolist(), var_f=m[:, 3].tolist(),
                    var_c=m[:, 4].tolist(), cov=m[:, 5].tolist(), W=list(W))

    def allocate(self, sig_t2, W, tau: float):
        import torch
        L = self.L
        have = torch.tensor(self.count, dtype=torch.int64, device="cuda")
        out = torch.zeros(L + 1, dtype=torch.int64, device="cuda")
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        capi.ofm_ofmlmc_optimal_M(self.ctx, L, torch.tensor(sig_t2, dtype=torch.float64, device="cuda"),
                                  torch.tensor(W, dtype=torch.float64, device="cuda"), have, capi.OFM_MODE_TOLERANCE,
                                  tau, out, flag)
        torch.cuda.synchronize()
        return out.cpu().tolist(), int(flag.item())

    def run(self, rel_tol: float = 0.01, warmup=None, W_model=None, max_iter: int = 10, min_samples: int = 2,
            max_new_finest: int | None = None, log=print) -> dict:
        """Adaptive loop to eps <= rel_tol |E|.  warmup: explicit counts, or
        eq. (warmup) from W_model (relative cost per term)."""
        L = self.L
        if warmup is None:
            W0 = W_model
            warmup = [max(min_samples, int(math.ceil(W0[L] / W0[k] / 2.0 ** (L - k)))) for k in range(L + 1)]
        history = []
        t_start = time.perf_counter()
        target = list(warmup)
        for it in range(max_iter):
            for k in range(L + 1):
                self.sample(k, max(0, target[k] - self.count[k]))
            W = self.work()
            res = self.evaluate(W)
            tau = rel_tol * abs(res["E"])
            res.update(iteration=it, tau=tau, counts=list(self.count), seconds=time.perf_counter() - t_start)
            history.append(res)
            log("iter %d: E=%.6e eps=%.3e tau=%.3e M=%s alpha=%s" % (it, res["E"], res["eps"], tau, self.count,
                                                                     [round(a, 4) for a in res["alpha"]]))
            if res["eps"] <= tau:
                break
            M, flag = self.allocate(res["sigma_t2"], W, tau)
            if max_new_finest is not None:
                M[L] = min(M[L], self.count[L] + max_new_finest)
            target = [max(m, c) for m, c in zip(M, self.count)]
            if target == self.count:
                break
        out = dict(history[-1])
        out["history"] = history
        out["wall_seconds"] = time.perf_counter() - t_start
        out["fidelities"] = [repr(f) for f in self.fid]
        return out
