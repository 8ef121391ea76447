"""Pins of the set-network oracle: gradients against central differences,
permutation invariance, bf16 rounding against its definition, and the Adam
update against a closed form."""
import numpy as np

import oracle.setnet as N


def toy(seed, sets=(3, 5, 1, 4)):
    rng = np.random.default_rng(seed)
    offsets = np.concatenate([[0], np.cumsum(sets)])
    x = rng.normal(size=(offsets[-1], N.D_IN))
    p = N.he_uniform(seed)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.normal(0, 0.1, size=p[k].shape)
    t = rng.normal(size=(len(sets), N.D_OUT))
    return p, x, offsets, t


def test_gradients_match_central_differences():
    p, x, off, t = toy(1)
    loss, g = N.loss_and_grads(p, x, off, 0.3, t)
    rng = np.random.default_rng(2)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            e = 1e-6
            old = p[name][idx]
            p[name][idx] = old + e
            lp, _ = N.loss_and_grads(p, x, off, 0.3, t)
            p[name][idx] = old - e
            lm, _ = N.loss_and_grads(p, x, off, 0.3, t)
            p[name][idx] = old
            fd = (lp - lm) / (2 * e)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_permutation_invariance_and_set_independence():
    p, x, off, t = toy(3)
    y, _ = N.forward(p, x, off, 0.5)
    perm = np.concatenate([off[i] + np.random.default_rng(i).permutation(off[i + 1] - off[i])
                           for i in range(len(off) - 1)])
    y2, _ = N.forward(p, x[perm], off, 0.5)
    np.testing.assert_allclose(y2, y, rtol=1e-13, atol=1e-13)
    # a set's output does not depend on the other sets
    y3, _ = N.forward(p, x[off[1]:off[2]], np.array([0, off[2] - off[1]]), 0.5)
    np.testing.assert_allclose(y3[0], y[1], rtol=1e-13, atol=1e-13)


def test_bf16_rounding_definition():
    vals = np.array([1.0, 1.00390625, 1.001953125, 1.005859375, -3.140625, 1e-20, 65504.0], dtype=np.float64)
    r = N.bf16(vals)
    # 1 + 2^-8 is exactly halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert r[1] == 1.0
    # 1 + 2^-9 rounds down; 1 + 3 * 2^-9 (0.75 ulp) rounds up to 1 + 2^-7
    assert r[2] == 1.0 and r[3] == 1.0078125
    assert r[4] == -3.140625
    # every result has 8 significant bits
    f = r.astype(np.float32).view(np.uint32)
    assert np.all((f & 0xFFFF) == 0)


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -1e-3, 5.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    N.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> update lr * sign(g)
    np.testing.assert_allclose(p["w"], [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01], rtol=1e-14)


def test_param_count_and_flatten_round_trip():
    p, *_ = toy(4)
    f = N.flatten(p)
    assert f.size == N.param_count() == 128 * 4 + 128 + 128 * 128 + 128 + 128 * 128 + 128 + 5 * 128 + 5
    q = N.unflatten(f)
    for k in p:
        assert np.array_equal(q[k], p[k])


def test_adam_recursion_over_several_steps_closed_forms():
    """Adam beyond its first step, against closed forms of its moment
    recursions (geometric series), eps = 0:
      * constant gradient g: m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so
        the bias-corrected step is lr sign(g) at every t;
      * alternating gradient g_t = (-1)^(t+1) g:
        m_t = (1 - b1) g (-1)^(t+1) (1 - (-b1)^t) / (1 + b1), v_t = (1 - b2^t) g^2,
        so step t moves w by -lr (-1)^(t+1) sign(g) c_t with
        c_t = (1 - b1)(1 - (-b1)^t) / ((1 + b1)(1 - b1^t)) (v_hat = g^2).
    A bias correction with a shifted exponent (b^(t+1)) or a step counter
    that does not advance changes c_t from the second step on."""
    b1, b2, lr = 0.9, 0.999, 0.01
    g0 = np.array([0.3, -1e-3, 5.0])
    # constant gradient
    p = {"w": np.array([1.0, -2.0, 0.5])}
    m, v = {"w": np.zeros(3)}, {"w": np.zeros(3)}
    for t in range(1, 8):
        N.adam_step(p, {"w": g0.copy()}, m, v, t, lr=lr, b1=b1, b2=b2, eps=0.0)
        np.testing.assert_allclose(m["w"], (1 - b1 ** t) * g0, rtol=1e-13)
        np.testing.assert_allclose(v["w"], (1 - b2 ** t) * g0 ** 2, rtol=1e-13)
        np.testing.assert_allclose(p["w"], np.array([1.0, -2.0, 0.5]) - t * lr * np.sign(g0), rtol=1e-13)
    # alternating gradient
    w0 = np.array([1.0, -2.0, 0.5])
    p = {"w": w0.copy()}
    m, v = {"w": np.zeros(3)}, {"w": np.zeros(3)}
    expect = w0.copy()
    for t in range(1, 8):
        s = (-1.0) ** (t + 1)
        N.adam_step(p, {"w": s * g0}, m, v, t, lr=lr, b1=b1, b2=b2, eps=0.0)
        np.testing.assert_allclose(m["w"], (1 - b1) * g0 * s * (1 - (-b1) ** t) / (1 + b1), rtol=1e-13)
        np.testing.assert_allclose(v["w"], (1 - b2 ** t) * g0 ** 2, rtol=1e-13)
        c_t = (1 - b1) * (1 - (-b1) ** t) / ((1 + b1) * (1 - b1 ** t))
        expect = expect - lr * s * np.sign(g0) * c_t
        np.testing.assert_allclose(p["w"], expect, rtol=1e-13)
    # the second step of the alternating sequence is not a signed lr step
    assert abs((1 - b1) * (1 - b1 ** 2) / ((1 + b1) * (1 - b1 ** 2)) - 1) > 0.5
