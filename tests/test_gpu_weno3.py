"""The third-order reconstruction (Sec. 2.2 allows WENO3 or WENO5): GPU
parity with the oracle run at weno_order 3, to the same bars as WENO5
(FP64 <= 1e-10 per field after 100 steps; FP32 relative L1 <= 1e-4 and p_max
within 0.5 %), tiling invariance, and argument checks."""
import math
import sys

import numpy as np
import pytest

import oracle.flow as OF
from oracle.sampler import sample_cloud
from workloads.configs import BASE, EOS, MASTER_SEED, cloud_spec, riemann_primitives, solver_config
from helpers import alloc_state, max_rel_field, oracle_shape, read_state, rel_l1

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_04374_amd import capi
    assert torch.cuda.is_available()
    c = capi.Context(0)
    yield c
    c.close()


def run(ctx, cfg, precision, n_steps, bubbles=None, W=None, tune=None):
    import torch
    from paper_1705_04374_amd import capi
    if tune:
        capi.ofm_tune_set(ctx, capi.OFM_F64 if precision == "f64" else capi.OFM_F32, cfg["ndim"], cfg["n"], *tune)
    spec = capi.make_spec(cfg, precision, n_steps=n_steps)
    st, bufs = alloc_state(cfg, precision)
    if W is not None:
        w = torch.tensor(W.reshape(W.shape[0], -1), dtype=torch.float64, device="cuda").contiguous()
        capi.ofm_state_from_primitive(ctx, spec, w, st)
    else:
        capi.ofm_state_init(ctx, spec, bubbles, st)
    q, dts = capi.ofm_step(ctx, spec, st, n_steps)
    return read_state(ctx, spec, st), q, dts


def w3(cloud, n):
    cfg = solver_config(cloud, n)
    cfg["weno_order"] = 3
    return cfg


@pytest.mark.parametrize("cloud,n", [("cloud2d", 48), ("cloud50", 24)])
def test_weno3_fp64_cloud_100_steps(ctx, cloud, n):
    say("weno3 fp64 100 steps", cloud, n)
    cfg = w3(cloud, n)
    bub = sample_cloud(cloud_spec(cloud), MASTER_SEED, 0, 1)
    U, q, dts = run(ctx, cfg, "f64", 100, bubbles=bub)
    R, rdts = OF.run_steps(cfg, OF.init_state(cfg, bub), 100)
    np.testing.assert_allclose(dts, rdts, rtol=1e-12, atol=0)
    err = max_rel_field(oracle_shape(cfg, U), R)
    assert np.all(err <= 1e-10), err
    ref = OF.solve(cfg, bub, n_steps=100)
    assert q["status"] == 0 and math.isclose(q["p_max"], ref["p_max"], rel_tol=1e-10)
    assert q["argmax"] == ref["argmax"]
    # and it is a different scheme from WENO5 on the same cloud
    R5, _ = OF.run_steps(solver_config(cloud, n), OF.init_state(cfg, bub), 100)
    assert np.max(max_rel_field(R5, R)) > 1e-6


def test_weno3_fp64_shock_tube(ctx):
    say("weno3 sod")
    n = 200
    cfg = dict(BASE)
    cfg.update(ndim=1, n=n, eos=dict(EOS), weno_order=3)
    W = riemann_primitives(1, n, dict(a1r1=0.0, a2r2=1.0, u=0.0, p=1.0, a2=1.0),
                           dict(a1r1=0.0, a2r2=0.125, u=0.0, p=0.1, a2=1.0))
    U, _, dts = run(ctx, cfg, "f64", 100, W=W)
    R, rdts = OF.run_steps(cfg, OF.prim_to_cons(cfg, W), 100)
    np.testing.assert_allclose(dts, rdts, rtol=1e-12)
    assert np.all(max_rel_field(oracle_shape(cfg, U), R) <= 1e-10)


@pytest.mark.parametrize("cloud,n", [("cloud2d", 48), ("cloud500", 32)])
def test_weno3_fp32_cloud_100_steps(ctx, cloud, n):
    say("weno3 fp32 100 steps", cloud, n)
    cfg = w3(cloud, n)
    bub = sample_cloud(cloud_spec(cloud), MASTER_SEED, 0, 5)
    U, q, _ = run(ctx, cfg, "f32", 100, bubbles=bub)
    ref = OF.solve(cfg, bub, n_steps=100)
    err = rel_l1(oracle_shape(cfg, U), ref["U"])
    assert np.all(err <= 1e-4), err
    assert abs(q["p_max"] / ref["p_max"] - 1) <= 5e-3 and q["status"] == 0


def test_weno3_fp32_tiling_invariance_bitwise(ctx):
    say("weno3 fp32 tiling invariance")
    cfg = w3("cloud50", 40)
    bub = sample_cloud(cloud_spec("cloud50"), MASTER_SEED, 0, 5)
    outs = [run(ctx, cfg, "f32", 5, bubbles=bub, tune=t)[0] for t in [(16, 14, 16, 2), (16, 16, 7, 2), (16, 8, 3, 2)]]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_weno_order_is_checked(ctx):
    from paper_1705_04374_amd import capi
    cfg = solver_config("cloud2d", 16)
    bub = sample_cloud(cloud_spec("cloud2d"), MASTER_SEED, 0, 0)
    bad = capi.make_spec(cfg, "f64", n_steps=2)
    bad.weno_order = 4
    with pytest.raises(capi.OfmError) as e:
        capi.ofm_solve(ctx, bad, bub)
    assert e.value.code == capi.OFM_EINVAL and "weno_order" in str(e.value)
    a = capi.make_spec(cfg, "f64", n_steps=2)
    b = capi.make_spec(w3("cloud2d", 16), "f64", n_steps=2)
    with pytest.raises(capi.OfmError) as e:
        capi.ofm_solve_batch(ctx, [a, b], [bub, bub])
    assert e.value.code == capi.OFM_EINVAL
    # 0 means the default, WENO5
    z = capi.make_spec(cfg, "f64", n_steps=2)
    z.weno_order = 0
    assert capi.ofm_solve(ctx, z, bub) == capi.ofm_solve(ctx, a, bub)
