"""Writes collapse_qoi.json: the oracle's QoIs of whole cloud-collapse solves
(to the end time) and how far those QoIs move when the oracle's own initial
state is perturbed at the level of its rounding.

    python tests/golden/make_collapse_golden.py [--jobs 6]

Calls only oracle/ and workloads/.  Solves (FP64, the serial oracle, Sec. 2.2
scheme on the Sec. 3.1 set-up, QoIs of Sec. 3.3):

  * 3-D clouds through the whole collapse and rebound: the 50-bubble cloud of
    the single-solve workload at 48^3 and 64^3, and the 500-bubble cloud at
    64^3 (the coarsest level of the batched and OF-MLMC workloads);
  * the same 50-bubble cloud at 48^3 with the third-order reconstruction,
    and with the characteristic far-field sides;
  * the 2-D two-level workload (16 clouds at 32^2, 4 pairs at 64^2 / 32^2),
    the samples of the end-to-end estimator test.

For each solve the file keeps the unperturbed QoIs and, for P perturbed
copies of the initial conserved state, their QoIs:
  * "ulp": every stored value moved by one unit in the last place of a
    double, in a seeded random direction;
  * "f32": every stored value scaled by (1 + s 2^-24), s = +-1 seeded (the
    rounding scale of a float state).
The spread of a QoI is the largest relative deviation of the perturbed runs
from the unperturbed one.  A violent collapse amplifies rounding
differences, and how much differs from sample to sample by orders of
magnitude (a sample whose peak is set by a near-tie between two collapsing
regions is far more sensitive than one with a single dominant peak), so a
GPU result is held to each sample's own spread, not to one bar for all.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle.flow as OF                          # noqa: E402
from oracle.sampler import sample_cloud           # noqa: E402
from workloads.configs import MASTER_SEED, cloud_spec, solver_config, t_end   # noqa: E402

OUT = os.path.join(HERE, "collapse_qoi.json")
QOIS = ("p_max", "t_at_max", "p_sensor", "gas_min", "c_max", "steps", "argmax", "status")
N_ULP = 3
N_F32 = 2

# (cloud, n, term, index, options of the scheme: "" = WENO5 with zero-gradient sides)
CASES_3D = [("cloud50", 48, 0, 0, ""), ("cloud50", 48, 0, 1, ""), ("cloud50", 64, 0, 0, ""),
            ("cloud500", 64, 0, 0, ""),
            ("cloud50", 48, 0, 0, "weno3"), ("cloud50", 48, 0, 0, "characteristic")]
CASES_2D = [("cloud2d", 32, 0, i, "") for i in range(16)] + [("cloud2d", 64, 1, i, "") for i in range(4)] + \
           [("cloud2d", 32, 1, i, "") for i in range(4)]


def options(opt: str) -> dict:
    """Solver options of a case: WENO3 (Sec. 2.2 allows third order) or the
    characteristic far-field sides (Sec. 3.1)."""
    return {"": {}, "weno3": {"weno_order": 3}, "characteristic": {"bc": "characteristic"}}[opt]


def perturb(U: np.ndarray, kind: str, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    s = rng.choice(np.array([-1.0, 1.0]), size=U.shape)
    if kind == "ulp":
        return np.nextafter(U, U + s * np.inf)
    return U * (1.0 + s * 2.0 ** -24)


def solve(job):
    cloud, n, term, index, opt, kind, seed = job
    cfg = solver_config(cloud, n, **options(opt))
    bub = sample_cloud(cloud_spec(cloud), MASTER_SEED, term, index)
    U0 = OF.init_state(cfg, bub)
    if kind != "base":
        U0 = perturb(U0, kind, seed)
    t0 = time.time()
    r = OF.solve(cfg, bub, t_end=t_end(cloud), U0=U0)
    q = {k: (int(r[k]) if k in ("steps", "argmax", "status") else float(r[k])) for k in QOIS}
    return job, q, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    jobs = []
    for cloud, n, term, index, opt in CASES_3D + CASES_2D:
        jobs.append((cloud, n, term, index, opt, "base", 0))
        jobs += [(cloud, n, term, index, opt, "ulp", 100 + k) for k in range(N_ULP)]
        jobs += [(cloud, n, term, index, opt, "f32", 200 + k) for k in range(N_F32)]
    # largest first, so the pool's tail is short
    jobs.sort(key=lambda j: -(j[1] ** (3 if j[0] != "cloud2d" else 2)))
    res = {}
    with ProcessPoolExecutor(a.jobs) as ex:
        for job, q, wall in ex.map(solve, jobs):
            print("%-9s n=%-3d term %d index %-2d %-14s %-4s seed %-3d  p_max %.9e steps %d  (%.0f s)"
                  % (job[0], job[1], job[2], job[3], job[4] or "-", job[5], job[6], q["p_max"], q["steps"], wall),
                  flush=True)
            res[job] = q
    cases = []
    for cloud, n, term, index, opt in CASES_3D + CASES_2D:
        base = res[(cloud, n, term, index, opt, "base", 0)]
        runs = {kind: [res[(cloud, n, term, index, opt, kind, s)] for s in seeds]
                for kind, seeds in (("ulp", range(100, 100 + N_ULP)), ("f32", range(200, 200 + N_F32)))}
        spread = {}
        for kind, rr in runs.items():
            spread[kind] = {k: max(abs(r[k] - base[k]) / max(abs(base[k]), 1e-300) for r in rr)
                            for k in ("p_max", "t_at_max", "p_sensor", "gas_min", "c_max")}
        cases.append(dict(cloud=cloud, ndim=cloud_spec(cloud)["ndim"], n=n, term=term, index=index,
                          options=options(opt), t_end=t_end(cloud), qoi=base, perturbed=runs, spread=spread))
    doc = dict(
        what="QoIs of whole solves to the end time by the FP64 oracle, and their spread under perturbations "
             "of the oracle's initial state at its rounding level",
        source="Sec. 2.2 scheme (oracle/flow_oracle.c), Sec. 3.1 cloud set-up, Sec. 3.3 QoIs; "
               "clouds from oracle/sampler.py with the master seed",
        generator="tests/golden/make_collapse_golden.py",
        master_seed=MASTER_SEED,
        perturbations=dict(ulp="every stored double moved by one ulp, seeded random direction",
                           f32="every stored value scaled by (1 + s 2^-24), s = +-1 seeded"),
        cases=cases)
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
