"""GPU parity of the set-network surrogate against the oracle fed the same
bf16-rounded operands (the oracle accumulates in double, the kernels in float
on the matrix cores).

Two bars on outputs and gradients:
  * whole tensor: relative L2 error <= 1e-3;
  * element by element: |gpu - ref| <= RTOL |ref| + ATOL max|ref| over the
    tensor.  The two sides round the same operands to bf16 except where an
    intermediate activation, accumulated in float on one side and in double
    on the other, lands on different sides of a bf16 rounding midpoint: that
    operand then differs by one bf16 ulp (2^-8 relative) and moves the
    entries it feeds by up to 2^-8 of that one term.  RTOL = 1e-3 and
    ATOL = 1e-4 leave room for flips of terms that do not dominate an entry
    (the largest deviation measured on these problems with the kernels'
    fixed summation orders is 4.6e-6 of a tensor's scale, in the W2
    gradient); a flip of a term that dominates an entry can exceed them (a
    64-row chunking of the pooling, with its float sums in another order,
    moved one W3 gradient entry by 3.5e-4 of the tensor's scale), so a
    change of a summation order is checked against these problems again.
    The largest element-wise deviations are printed."""
import sys

import numpy as np
import pytest

import oracle.setnet as N
from workloads.configs import MASTER_SEED, cloud_spec

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1705_04374_amd import capi
    c = capi.Context(0)
    yield c
    c.close()


def problem(seed, sizes):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = rng.normal(size=(int(off[-1]), 4)).astype(np.float32).astype(np.float64)
    p = N.he_uniform(seed)
    for k in p:
        p[k] = N.f32(p[k] if k.startswith("W") else rng.normal(0, 0.05, size=p[k].shape))
    t = rng.normal(size=(len(sizes), 5)).astype(np.float32).astype(np.float64)
    return p, x, off, t


def gpu_net(ctx, p, pool_scale):
    import torch
    from paper_1705_04374_amd import capi
    net = capi.SetNet(ctx, pool_scale)
    net.set_params(torch.tensor(N.flatten(p), dtype=torch.float32, device="cuda"))
    return net


def dev(a, dt=None):
    import torch
    a = np.asarray(a)
    if dt is None:
        dt = torch.int32 if a.dtype.kind in "iu" else torch.float32
    return torch.tensor(a, dtype=dt, device="cuda").contiguous()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-30))


RTOL, ATOL = 1e-3, 1e-4


def elementwise(name, got, ref, rtol=RTOL, atol=ATOL):
    """Element-wise bar |got - ref| <= rtol |ref| + atol max|ref|; reports the
    worst entry relative to its own magnitude and to the tensor's scale."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(np.abs(ref).max(), 1e-30)
    d = np.abs(got - ref)
    bound = rtol * np.abs(ref) + atol * scale
    worst = np.unravel_index(np.argmax(d / bound), d.shape)
    say("  %s: max |d|/scale %.2e, max |d|/(rtol|ref| + atol scale) %.3f at %s (ref %.3e, got %.3e), "
        "entries above 1e-4 of scale: %d of %d" % (name, d.max() / scale, (d / bound).max(), worst, ref[worst],
                                                   got[worst], int((d > 1e-4 * scale).sum()), d.size))
    assert np.all(d <= bound), name


SIZES = [500, 1, 127, 128, 129, 257, 3, 500, 64]


def test_forward_matches_oracle(ctx):
    import torch
    say("nn forward")
    p, x, off, _ = problem(1, SIZES)
    net = gpu_net(ctx, p, 1.0 / 500)
    y = torch.empty((len(SIZES), 5), dtype=torch.float32, device="cuda")
    net.forward(dev(x), dev(off), y)
    ref, _ = N.forward(p, x, off, 1.0 / 500, bf16_ops=True)
    got = y.cpu().numpy().astype(np.float64)
    assert rel(got, ref) <= 1e-3, rel(got, ref)
    elementwise("outputs", got, ref)
    # per set, too (a wrong segment would show here)
    for i in range(len(SIZES)):
        assert rel(got[i], ref[i]) <= 3e-3, (i, rel(got[i], ref[i]))
    # float vs the pure-double network: the bf16 operands cost < 1 %
    ref64, _ = N.forward(p, x, off, 1.0 / 500, bf16_ops=False)
    assert rel(got, ref64) <= 2e-2


def test_gradients_match_oracle(ctx):
    import torch
    say("nn grads")
    p, x, off, t = problem(2, SIZES)
    net = gpu_net(ctx, p, 1.0 / 500)
    g = torch.zeros(N.param_count(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.grads(dev(x), dev(off), dev(t), g, loss)
    lref, gref = N.loss_and_grads(p, x, off, 1.0 / 500, t, bf16_ops=True)
    assert abs(loss.item() / lref - 1) <= 1e-4
    gg = N.unflatten(g.cpu().numpy().astype(np.float64))
    for k in gref:
        assert rel(gg[k], gref[k]) <= 1e-3, (k, rel(gg[k], gref[k]))
        elementwise(k, gg[k], gref[k])


def test_deterministic(ctx):
    import torch
    p, x, off, t = problem(3, SIZES)
    net = gpu_net(ctx, p, 1.0 / 500)
    outs = []
    for _ in range(2):
        g = torch.zeros(N.param_count(), dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        net.grads(dev(x), dev(off), dev(t), g, loss)
        outs.append((g.cpu().numpy(), loss.item()))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


def test_adam_steps_match_oracle(ctx):
    """Five training steps: after each, the parameters equal the oracle's
    Adam (its moment recursions and bias correction pinned over several
    steps on the CPU) applied to the GPU's gradient at the same parameters
    (which isolates the update from the gradient's accumulation order)."""
    import torch
    say("nn adam")
    p, x, off, t = problem(4, SIZES)
    net = gpu_net(ctx, p, 1.0 / 500)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    pr = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    got = torch.zeros(N.param_count(), dtype=torch.float32, device="cuda")
    for step in range(1, 6):
        g = torch.zeros(N.param_count(), dtype=torch.float32, device="cuda")
        net.grads(dev(x), dev(off), dev(t), g, loss)
        net.train_step(dev(x), dev(off), dev(t), loss)
        net.get_params(got)
        gd = N.unflatten(g.cpu().numpy().astype(np.float64))
        N.adam_step(pr, gd, m, v, step)
        np.testing.assert_allclose(got.cpu().numpy(), N.flatten(pr), rtol=1e-5, atol=1e-7, err_msg="step %d" % step)


def test_features_match_oracle(ctx):
    import torch
    from paper_1705_04374_amd import capi
    spec = cloud_spec("cloud500")
    bub = capi.ofm_sample_cloud(spec, MASTER_SEED, 5, 0)
    x = torch.empty((bub.shape[0], 4), dtype=torch.float32, device="cuda")
    capi.ofm_nn_features(spec, torch.tensor(bub, device="cuda"), x)
    np.testing.assert_allclose(x.cpu().numpy(), N.features(bub, spec), rtol=1e-6, atol=1e-6)


def test_training_learns_a_set_function(ctx):
    """A permutation-invariant target (the mean of the inputs over the set
    and its spread) is learnt: the loss falls by 10x."""
    import torch
    from paper_1705_04374_amd import capi
    say("nn learning")
    rng = np.random.default_rng(7)
    S, B = 256, 50
    x = rng.normal(size=(S * B, 4))
    off = np.arange(S + 1) * B
    xm = x.reshape(S, B, 4)
    t = np.stack([xm[:, :, 0].mean(1) * 3, xm[:, :, 1].mean(1) * 3, (xm[:, :, 2] ** 2).mean(1),
                  np.abs(xm[:, :, 3]).mean(1), xm[:, :, 0].std(1)], axis=1)
    t = (t - t.mean(0)) / t.std(0)
    net = capi.SetNet(ctx, 1.0 / B, seed=11, lr=3e-3)
    xd, od, td = dev(x), dev(off), dev(t)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    first = None
    for it in range(300):
        net.train_step(xd, od, td, loss)
        if first is None:
            first = loss.item()
    last = loss.item()
    say("  loss", first, "->", last)
    assert last < 0.1 * first


def test_forward_of_many_sets_is_per_set(ctx):
    """More sets than workgroups (each workgroup then takes several sets):
    every set's output equals the one computed in a small batch, bit for
    bit, and a sample of them matches the oracle."""
    import torch
    say("nn forward, many sets")
    rng = np.random.default_rng(5)
    sizes = rng.integers(0, 300, size=9000)
    sizes[:3] = [500, 0, 129]
    p, x, off, _ = problem(2, list(sizes))
    net = gpu_net(ctx, p, 1.0 / 500)
    y = torch.empty((len(sizes), 5), dtype=torch.float32, device="cuda")
    net.forward(dev(x), dev(off), y)
    got = y.cpu().numpy()
    for lo in (0, 4096, 8990):
        hi = min(lo + 10, len(sizes))
        xs = x[off[lo]:off[hi]]
        offs = off[lo:hi + 1] - off[lo]
        ys = torch.empty((hi - lo, 5), dtype=torch.float32, device="cuda")
        net.forward(dev(xs), dev(offs), ys)
        assert np.array_equal(ys.cpu().numpy(), got[lo:hi]), lo
        ref, _ = N.forward(p, xs, offs, 1.0 / 500, bf16_ops=True)
        assert rel(got[lo:hi].astype(np.float64), ref) <= 1e-3
    assert np.all(np.isfinite(got))
