"""Whole cloud collapses in 3-D against the oracle: the Sec. 2.2 scheme run
through the collapse and rebound of the Sec. 3.1 set-up to the end time, the
QoIs of Sec. 3.3 compared with the FP64 oracle's (stored by
tests/golden/make_collapse_golden.py, which calls only the oracle), with
WENO5 and zero-gradient sides, and with the third-order reconstruction and
the characteristic far-field sides.

A collapse amplifies rounding differences, and by how much depends on the
sample.  The golden file keeps, per sample, how far the oracle's own QoIs
move when its initial state is perturbed by one ulp (and by float rounding).
The library's FP64 arithmetic differs from the oracle's at every operation
(contractions, reciprocal refinements, the stored energy Et), so each QoI is
held to max(FLOOR, K x that spread): K = 10 covers rounding differences at
every step rather than once at the start, FLOOR = 1e-10 is the bar of the
100-step field comparisons.  The FP32 stencil is held to p_max within 0.5 %
(or K x the oracle's spread under float-sized perturbations, where that is
larger)."""
import json
import math
import os
import sys

import numpy as np
import pytest

from workloads.configs import MASTER_SEED, cloud_spec, solver_config

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "collapse_qoi.json")))
CASES3 = [c for c in GOLD["cases"] if c["ndim"] == 3]
K, FLOOR = 10.0, 1e-10
QOIS = ("p_max", "t_at_max", "p_sensor", "gas_min", "c_max")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1705_04374_amd import capi
    c = capi.Context(0)
    yield c
    c.close()


def bar(case, kind, q):
    return max(FLOOR, K * case["spread"][kind][q])


def case_id(c):
    opt = "-".join("%s=%s" % kv for kv in sorted(c.get("options", {}).items()))
    return "%s-%d-%d%s" % (c["cloud"], c["n"], c["index"], "-" + opt if opt else "")


@pytest.mark.parametrize("case", CASES3, ids=case_id)
def test_fp64_collapse_qois_against_oracle(ctx, case):
    from paper_1705_04374_amd import capi
    say("3-D collapse, FP64:", case_id(case))
    cfg = solver_config(case["cloud"], case["n"], **case.get("options", {}))
    bub = capi.ofm_sample_cloud(cloud_spec(case["cloud"]), MASTER_SEED, case["term"], case["index"])
    q = capi.ofm_solve(ctx, capi.make_spec(cfg, "f64", t_end=case["t_end"]), bub)
    ref = case["qoi"]
    assert q["status"] == 0 and ref["status"] == 0
    assert q["steps"] == ref["steps"]
    assert q["t"] == pytest.approx(case["t_end"], rel=1e-15)
    for k in QOIS:
        d = abs(q[k] / ref[k] - 1)
        say("  %-9s gpu %.12e oracle %.12e  rel %.2e  bar %.2e" % (k, q[k], ref[k], d, bar(case, "ulp", k)))
        assert d <= bar(case, "ulp", k), (k, d)
    # the peak's cell: where the oracle's own perturbed runs agree on it, the
    # library must find the same cell
    if all(r["argmax"] == ref["argmax"] for r in case["perturbed"]["ulp"]):
        assert q["argmax"] == ref["argmax"]


@pytest.mark.parametrize("case", CASES3, ids=case_id)
def test_fp32_collapse_peak_pressure_against_oracle(ctx, case):
    from paper_1705_04374_amd import capi
    say("3-D collapse, FP32:", case_id(case))
    cfg = solver_config(case["cloud"], case["n"], **case.get("options", {}))
    bub = capi.ofm_sample_cloud(cloud_spec(case["cloud"]), MASTER_SEED, case["term"], case["index"])
    q = capi.ofm_solve(ctx, capi.make_spec(cfg, "f32", t_end=case["t_end"]), bub)
    ref = case["qoi"]
    assert q["status"] == 0
    d = abs(q["p_max"] / ref["p_max"] - 1)
    b = max(5e-3, K * case["spread"]["f32"]["p_max"])
    say("  p_max gpu %.9e oracle %.9e rel %.2e bar %.2e; steps %d / %d" % (q["p_max"], ref["p_max"], d, b,
                                                                         q["steps"], ref["steps"]))
    assert d <= b
    assert abs(q["steps"] - ref["steps"]) <= max(2, 0.01 * ref["steps"])
