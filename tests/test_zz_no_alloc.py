"""The stepping entry point that allocates nothing (ofm_step_noalloc) against
ofm_step: the same kernels and launches, so the same state, step sizes and
QoI bit for bit; on calls in a row that share the fixed scratch, each after
the first with a smaller grid; a call whose scratch would not fit is
refused before any launch."""
import sys

import numpy as np
import pytest

from workloads.configs import MASTER_SEED, cloud_spec, solver_config

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1705_04374_amd import capi
    c = capi.Context(0)
    yield c
    c.close()


def run_pair(ctx, cloud, n, prec, steps):
    import torch
    from paper_1705_04374_amd import capi
    from paper_1705_04374_amd.state import alloc_state, current
    say("no-alloc vs ofm_step:", cloud, n, prec, steps)
    cfg = solver_config(cloud, n)
    bub = capi.ofm_sample_cloud(cloud_spec(cloud), MASTER_SEED, 0, 0)
    spec = capi.make_spec(cfg, prec, n_steps=steps)
    sa, ba = alloc_state(cfg, prec)
    sb, bb = alloc_state(cfg, prec)
    capi.ofm_state_init(ctx, spec, bub, sa)
    capi.ofm_state_init(ctx, spec, bub, sb)
    # the partner buffer and the RK register start as NaN in the second run:
    # a read before the first write would show
    bb[1].fill_(float("nan"))
    bb[2].fill_(float("nan"))
    torch.cuda.synchronize()
    qa, da = capi.ofm_step(ctx, spec, sa, steps)
    qb, db = capi.ofm_step_noalloc(ctx, spec, sb, steps)
    ua, ub = current(sa, ba), current(sb, bb)
    assert qa["status"] == 0 and qa["steps"] == steps
    assert torch.equal(ua, ub)
    assert np.array_equal(da, db)
    assert qa == qb
    # without the step-size log the result is the same
    capi.ofm_state_init(ctx, spec, bub, sb)
    qc, _ = capi.ofm_step_noalloc(ctx, spec, sb, steps, log_dts=False)
    assert qc == qa and torch.equal(current(sb, bb), ua)


def test_noalloc_equals_ofm_step_on_calls_in_a_row(ctx):
    run_pair(ctx, "cloud500", 64, "f32", 6)     # 3-D, 64 tiles of 16 x 16 x 16
    run_pair(ctx, "cloud50", 40, "f64", 4)      # smaller 3-D grid, double
    run_pair(ctx, "cloud2d", 32, "f64", 12)     # smaller still, 2-D


def test_noalloc_refuses_a_scratch_it_does_not_have(ctx):
    """A step-size log longer than the fixed scratch: OFM_EINVAL, state and
    pointers untouched."""
    import torch
    from paper_1705_04374_amd import capi
    from paper_1705_04374_amd.state import alloc_state
    cfg = solver_config("cloud50", 8)
    spec = capi.make_spec(cfg, "f32", n_steps=1)
    st, bufs = alloc_state(cfg, "f32")
    bub = capi.ofm_sample_cloud(cloud_spec("cloud50"), MASTER_SEED, 0, 0)
    capi.ofm_state_init(ctx, spec, bub, st)
    torch.cuda.synchronize()
    before = bufs[0].clone()
    u0 = st.u
    steps = capi.OFM_NOALLOC_SCRATCH_BYTES // 8 + 1
    with pytest.raises(capi.OfmError) as e:
        capi.ofm_step_noalloc(ctx, spec, st, steps)
    assert "scratch" in str(e.value) and "-1" in str(e.value)
    torch.cuda.synchronize()
    assert st.u == u0 and torch.equal(bufs[0], before)
    # the context still steps afterwards
    q, _ = capi.ofm_step_noalloc(ctx, spec, st, 2)
    assert q["status"] == 0 and q["steps"] == 2
