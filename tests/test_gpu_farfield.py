"""The characteristic far-field boundary (Sec. 3.1): GPU parity with the
oracle under OFM_BC_CHARACTERISTIC, to the bars of the zero-gradient runs
(FP64 <= 1e-10 per field after 100 steps; FP32 relative L1 <= 1e-4 and p_max
within 0.5 %), on grids where the waves reach the sides within the run, and
the same state for every tiling (the ghosts are built in the x-y halo of
each tile and in each thread's z column)."""
import math
import sys

import numpy as np
import pytest

import oracle.flow as OF
from oracle.sampler import sample_cloud
from workloads.configs import BASE, EOS, MASTER_SEED, cloud_spec, solver_config
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


def far(cloud, n):
    cfg = solver_config(cloud, n)
    cfg["bc"] = "characteristic"
    return cfg


@pytest.mark.parametrize("cloud,n", [("cloud2d", 48), ("cloud50", 24)])
def test_farfield_fp64_cloud_100_steps(ctx, cloud, n):
    say("far field fp64 100 steps", cloud, n)
    cfg = far(cloud, n)
    bub = sample_cloud(cloud_spec(cloud), MASTER_SEED, 0, 1)
    U, q, dts = run(ctx, cfg, "f64", 100, bubbles=bub)
    R, rdts = OF.run_steps(cfg, OF.init_state(cfg, bub), 100)
    np.testing.assert_allclose(dts, rdts, rtol=1e-12, atol=0)
    err = max_rel_field(oracle_shape(cfg, U), R)
    assert np.all(err <= 1e-10), err
    ref = OF.solve(cfg, bub, n_steps=100)
    assert q["status"] == 0 and math.isclose(q["p_max"], ref["p_max"], rel_tol=1e-10)
    for k in ("p_sensor", "gas_min", "c_max"):
        assert math.isclose(q[k], ref[k], rel_tol=1e-10, abs_tol=1e-300), k
    # the sides act within the run: the zero-gradient state differs
    Rz, _ = OF.run_steps(solver_config(cloud, n), OF.init_state(cfg, bub), 100)
    assert np.max(max_rel_field(Rz, R)) > 1e-8


def test_farfield_fp64_acoustic_pulse_1d(ctx):
    say("far field 1d pulse")
    n = 128
    cfg = dict(BASE)
    cfg.update(ndim=1, n=n, eos=dict(EOS), bc="characteristic")
    p_inf = cfg["p_inf"]
    Z = 1000.0 * math.sqrt(EOS["gamma1"] * (p_inf + EOS["pc1"]) / 1000.0)
    x = (np.arange(n) + 0.5) / n
    dp = 1e5 * np.exp(-((x - 0.8) / 0.05) ** 2)
    W = np.zeros((5, n))
    W[0], W[2], W[3] = 1000.0, dp / Z, p_inf + dp
    U, _, dts = run(ctx, cfg, "f64", 100, W=W)
    R, rdts = OF.run_steps(cfg, OF.prim_to_cons(cfg, W), 100)
    np.testing.assert_allclose(dts, rdts, rtol=1e-12)
    assert np.all(max_rel_field(oracle_shape(cfg, U), R) <= 1e-10)


def test_farfield_fp32_cloud500_100_steps(ctx):
    say("far field fp32 100 steps")
    cfg = far("cloud500", 32)
    bub = sample_cloud(cloud_spec("cloud500"), MASTER_SEED, 0, 5)
    U, q, _ = run(ctx, cfg, "f32", 100, bubbles=bub)
    ref = OF.solve(cfg, bub, n_steps=100)
    assert np.all(rel_l1(oracle_shape(cfg, U), ref["U"]) <= 1e-4)
    assert abs(q["p_max"] / ref["p_max"] - 1) <= 5e-3 and q["status"] == 0


def test_farfield_tiling_invariance_bitwise(ctx):
    """n = 20 leaves ragged tiles; every tile shape and z-chunk builds the
    same ghosts, bit for bit, in FP64 and FP32."""
    say("far field tiling invariance")
    cfg = far("cloud50", 20)
    bub = sample_cloud(cloud_spec("cloud50"), MASTER_SEED, 0, 2)
    outs = [run(ctx, cfg, "f64", 40, bubbles=bub, tune=t)[0] for t in [(16, 8, 16, 2), (16, 16, 7, 2), (16, 14, 3, 2)]]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    R, _ = OF.run_steps(cfg, OF.init_state(cfg, bub), 40)
    assert np.all(max_rel_field(oracle_shape(cfg, outs[0]), R) <= 1e-10)
    outs = [run(ctx, cfg, "f32", 10, bubbles=bub, tune=t)[0] for t in [(16, 14, 16, 2), (16, 8, 3, 2)]]
    assert np.array_equal(outs[0], outs[1])


def test_farfield_batch_needs_one_far_field_pressure(ctx):
    from paper_1705_04374_amd import capi
    cfg = far("cloud2d", 16)
    bub = sample_cloud(cloud_spec("cloud2d"), MASTER_SEED, 0, 0)
    a = capi.make_spec(cfg, "f64", n_steps=2)
    b = capi.make_spec(dict(cfg, p_inf=2.0e7), "f64", n_steps=2)
    with pytest.raises(capi.OfmError) as e:
        capi.ofm_solve_batch(ctx, [a, b], [bub, bub])
    assert e.value.code == capi.OFM_EINVAL
    qa = capi.ofm_solve_batch(ctx, [a, a], [bub, bub])
    assert qa[0] == qa[1] == capi.ofm_solve(ctx, a, bub)


def test_farfield_weno3_batch_equals_single_solves(ctx):
    """The options in the batched path: samples of different sizes with the
    far-field boundary and WENO3, advanced in the same launches, give the
    QoIs of their single solves bit for bit."""
    from paper_1705_04374_amd import capi
    say("far field + weno3 batch")
    T = 6.0e-4
    specs, bubs = [], []
    for i, n in enumerate([32, 16, 24, 32]):
        cfg = far("cloud2d", n)
        cfg["weno_order"] = 3
        specs.append(capi.make_spec(cfg, "f64", t_end=T))
        bubs.append(sample_cloud(cloud_spec("cloud2d"), MASTER_SEED, 2, i))
    qb = capi.ofm_solve_batch(ctx, specs, bubs)
    for s, b, q in zip(specs, bubs, qb):
        assert capi.ofm_solve(ctx, s, b) == q
    cfg = far("cloud2d", 24)
    cfg["weno_order"] = 3
    ref = OF.solve(cfg, bubs[2], t_end=T)
    assert math.isclose(qb[2]["p_max"], ref["p_max"], rel_tol=1e-9) and qb[2]["steps"] == ref["steps"]
