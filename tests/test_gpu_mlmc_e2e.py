"""End to end: the two-level 2-D FP64 MLMC of the plain method (8 bubbles,
32^2 with 16 samples, 64^2/32^2 with 4 coupled pairs, run to the end time)
through the driver and the library, against the same pipeline built from the
oracle (its sampler, its solver, its estimator).

The oracle's per-sample QoIs come from tests/golden/collapse_qoi.json
(written by tests/golden/make_collapse_golden.py with the oracle alone), with
how far each moves when the oracle's initial state is perturbed by one ulp.
Each sample's FP64 p_max is held to max(1e-10, 10 x its own spread): a
violent collapse amplifies rounding differences by a factor that differs
between samples by orders of magnitude."""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle.mlmc as OM
from workloads.configs import MASTER_SEED, cloud_spec, solver_config, t_end

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_two_level_2d_fp64_against_oracle_pipeline(tmp_path):
    from paper_1705_04374_amd import capi
    from paper_1705_04374_amd.driver import OFMLMC
    ctx = capi.Context(0)
    T = t_end("cloud2d")
    spec = cloud_spec("cloud2d")
    cfg = solver_config("cloud2d", 32)
    mc = OFMLMC(ctx, cfg, spec, [32, 64], "f64", t_end=T, seed=MASTER_SEED, ledger=str(tmp_path / "ledger.jsonl"))
    say("gpu mlmc")
    mc.sample(0, 16)
    mc.sample(1, 4)
    W = [1.0, 9.0]           # pair cost 64^3 + 32^3 in units of a 32^3 solve
    res = mc.evaluate(W)
    classical = mc.evaluate(W, classical=True)
    say("oracle pipeline (stored QoIs)")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "collapse_qoi.json")))
    cases = {(c["n"], c["term"], c["index"]): c for c in gold["cases"] if c["cloud"] == "cloud2d"}
    order = [(32, 0, i) for i in range(16)] + [(64, 1, i) for i in range(4)] + [(32, 1, i) for i in range(4)]
    assert all(cases[k]["t_end"] == T and cases[k]["qoi"]["status"] == 0 for k in order)
    ora = np.array([cases[k]["qoi"]["p_max"] for k in order])
    bars = np.array([max(1e-10, 10.0 * cases[k]["spread"]["ulp"]["p_max"]) for k in order])
    qf0, qf1, qc1 = list(ora[:16]), list(ora[16:20]), list(ora[20:])
    # per-sample QoIs through the whole collapse (FP64), each to its bar
    gpu = np.array(mc.q[0]["f"] + mc.q[1]["f"] + mc.q[1]["c"])
    d = np.abs(gpu / ora - 1)
    say("full-run QoI relative differences:", np.array2string(d, precision=2))
    say("per-sample bars:                  ", np.array2string(bars, precision=2))
    assert np.all(d <= bars), [(order[i], d[i], bars[i]) for i in np.nonzero(d > bars)[0]]
    assert all(mc.q[0]["ok"]) and all(mc.q[1]["ok"])
    # the estimator on identical QoIs: the estimator bar (1e-12)
    g0 = OM.term_moments(mc.q[0]["f"])
    g1 = OM.term_moments(mc.q[1]["f"], mc.q[1]["c"])
    ga = OM.coefficients([g0["Vf"], g1["Vf"]], [0.0, g1["Vc"]], [0.0, g1["C"]], W)
    gE = OM.estimate([g0["mean_f"], g1["mean_f"]], [0.0, g1["mean_c"]], ga)
    gs = OM.term_variances([g0["Vf"], g1["Vf"]], [0.0, g1["Vc"]], [0.0, g1["C"]], ga)
    assert math.isclose(res["alpha"][0], ga[0], rel_tol=1e-12)
    assert math.isclose(res["E"], gE, rel_tol=1e-12)
    assert math.isclose(res["eps"], math.sqrt(OM.error2(gs, [16, 4])), rel_tol=1e-12)
    # and the whole oracle pipeline
    def pipeline(q):
        m0 = OM.term_moments(list(q[:16]))
        m1 = OM.term_moments(list(q[16:20]), list(q[20:]))
        a = OM.coefficients([m0["Vf"], m1["Vf"]], [0.0, m1["Vc"]], [0.0, m1["C"]], W)
        return OM.estimate([m0["mean_f"], m1["mean_f"]], [0.0, m1["mean_c"]], a), a

    E, a = pipeline(ora)
    say("alpha", res["alpha"], a, "E", res["E"], E)
    # the estimate may differ from the oracle pipeline's by what the samples'
    # allowed differences move it (first order, each sample by its bar, the
    # estimator itself being exact to 1e-12)
    sens = sum(abs(pipeline(ora * np.where(np.arange(24) == i, 1.0 + bars[i], 1.0))[0] - E) for i in range(24))
    assert abs(res["E"] - E) <= 2.0 * sens + 1e-12 * abs(E), (res["E"], E, sens)
    # classical MLMC is the same estimator with alpha = 1
    assert math.isclose(classical["E"], np.mean(mc.q[0]["f"]) + np.mean(mc.q[1]["f"]) - np.mean(mc.q[1]["c"]),
                        rel_tol=1e-12)
    # the ledger lets a second driver resume without solving again
    mc2 = OFMLMC(ctx, cfg, spec, [32, 64], "f64", t_end=T, seed=MASTER_SEED, ledger=str(tmp_path / "ledger.jsonl"))
    mc2.sample(0, 16)
    mc2.sample(1, 4)
    assert mc2.solve_seconds == 0.0
    assert mc2.evaluate(W)["E"] == res["E"]
    ctx.close()


def test_indicator_fit_with_one_finest_warmup_sample(tmp_path):
    """App. A.1: one warm-up sample on the finest term, its variances inferred
    from the lower terms' fit (Sec. 2.4.4 step 3); the driver's estimate
    equals the oracle's fit + completion + estimator on the same QoIs."""
    from paper_1705_04374_amd import capi
    from paper_1705_04374_amd.driver import OFMLMC
    ctx = capi.Context(0)
    T = t_end("cloud2d")
    spec = cloud_spec("cloud2d")
    cfg = solver_config("cloud2d", 16)
    mc = OFMLMC(ctx, cfg, spec, [16, 32, 64, 128], "f32", t_end=T, seed=MASTER_SEED, log=say)
    say("fit warm-up")
    mc.sample_terms([32, 16, 8, 1])
    W = [1.0, 9.0, 72.0, 576.0]
    r = mc.evaluate(W, fit=True)
    assert r["fit_flag"] == 0 and r["M"] == [sum(mc.q[k]["ok"]) for k in range(4)] and r["M"][3] == 1
    mom = [OM.term_moments(mc.q[k]["f"], mc.q[k]["c"] if k else None, mc.q[k]["ok"]) for k in range(4)]
    v_ref, ok = OM.fit_indicators([m["M"] for m in mom], [m["Vf"] + m["Vc"] - 2 * m["C"] for m in mom], 1)
    assert ok
    np.testing.assert_allclose(r["v_hat"], v_ref, rtol=1e-12)
    OM.infer_missing_terms(mom, v_ref, 1)
    assert math.isclose(r["var_c"][3], mom[2]["Vf"], rel_tol=1e-12)
    assert math.isclose(r["var_f"][3], mom[3]["Vf"], rel_tol=1e-12)
    assert math.isclose(r["cov"][3], mom[3]["C"], rel_tol=1e-12)
    assert r["cov"][3] ** 2 <= r["var_f"][3] * r["var_c"][3] * (1 + 1e-12)
    a = OM.coefficients([m["Vf"] for m in mom], [m["Vc"] for m in mom], [m["C"] for m in mom], W)
    np.testing.assert_allclose(r["alpha"], a, rtol=1e-10)
    E = OM.estimate([m["mean_f"] for m in mom], [m["mean_c"] for m in mom], a)
    assert math.isclose(r["E"], E, rel_tol=1e-10)
    # without the fit the single finest sample has no variance
    assert mc.evaluate(W)["var_f"][3] == 0.0
    ctx.close()
