"""Pins of the oracle solver against what the mathematics and the paper fix.

Each test checks the oracle against something other than itself: closed forms,
textbook exact Riemann solutions, invariants of the scheme (conservation on a
periodic domain, pressure/velocity equilibrium across an interface, mirror
symmetry) and exact rational properties of the Runge-Kutta coefficients.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle.flow as F
from oracle.riemann import ExactRiemann, Side
from oracle.sampler import sample_cloud
from workloads.configs import (BASE, EOS, interface_primitives, random_smooth_primitives,
                               cloud_spec, riemann_primitives, solver_config)

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def cfg1d(n, **kw):
    c = dict(BASE)
    c.update(ndim=1, n=n, eos=dict(EOS))
    c.update(kw)
    return c


def cfg_nd(ndim, n, **kw):
    c = dict(BASE)
    c.update(ndim=ndim, n=n, eos=dict(EOS))
    c.update(kw)
    return c


# --------------------------------------------------------------------------
# Equation of state (Sec. 2.1)
# --------------------------------------------------------------------------

def test_eos_round_trip_and_pure_phases():
    rng = np.random.default_rng(1)
    c = cfg_nd(3, 8)
    W = np.zeros((7, 50))
    W[6] = rng.uniform(0, 1, 50)
    W[0] = (1 - W[6]) * rng.uniform(500, 1500, 50)
    W[1] = W[6] * rng.uniform(0.5, 5, 50)
    W[2:5] = rng.normal(0, 50, (3, 50))
    W[5] = rng.uniform(1e3, 1e8, 50)
    Q = F.prim_to_cons(c, W)
    W2 = F.cons_to_prim(c, Q)
    np.testing.assert_allclose(W2, W, rtol=1e-9, atol=1e-12)
    # pure air with p_c = 0 is an ideal gas: p = (gamma - 1)(E - rho|u|^2/2)
    w = np.array([0.0, 1.2, 3.0, -4.0, 5.0, 1.0e5, 1.0])
    q = F.prim_to_cons(c, w.reshape(7, 1)).ravel()
    rho = 1.2
    ke = 0.5 * rho * (9 + 16 + 25)
    assert math.isclose(q[5], 1.0e5 / 0.4 + ke, rel_tol=1e-14)
    # pure water: stiffened gas p = (gamma - 1) rho e - gamma p_c
    w = np.array([998.0, 0.0, 1.0, 2.0, 3.0, 2.0e6, 0.0])
    q = F.prim_to_cons(c, w.reshape(7, 1)).ravel()
    rho_e = q[5] - 0.5 * 998.0 * 14.0
    assert math.isclose((6.12 - 1) * rho_e - 6.12 * 3.43e8, 2.0e6, rel_tol=1e-9)


def test_sound_speed_and_cfl_on_uniform_states():
    """Pure phases at rest: c^2 = gamma (p + p_c)/rho (textbook), and the CFL
    step is cfl h / (|u| + c)."""
    n = 16
    for a2, rho, p, g, pc in ((0.0, 1000.0, 1.0e7, 6.12, 3.43e8), (1.0, 1.0, 2340.0, 1.4, 0.0)):
        c = cfg1d(n)
        left = dict(a1r1=(1 - a2) * rho, a2r2=a2 * rho, u=7.0, p=p, a2=a2)
        U = F.prim_to_cons(c, riemann_primitives(1, n, left, left))
        r = F.reduce(c, U)
        cs = math.sqrt(g * (p + pc) / rho)
        assert math.isclose(r["s_max"], 7.0 + cs, rel_tol=1e-12)
        assert math.isclose(r["p_max"], p, rel_tol=1e-9)
        _, dts = F.run_steps(c, U, 1)
        assert math.isclose(dts[0], 0.3 / n / (7.0 + cs), rel_tol=1e-12)


def test_k_coefficient_matches_wood_form():
    """eq. (var_K) equals the Kapila form a1 a2 (1/(r2c2^2) - 1/(r1c1^2)) /
    (a1/(r1c1^2) + a2/(r2c2^2)); it vanishes in pure phases."""
    c = cfg1d(4)
    for a2 in (0.1, 0.5, 0.93):
        for p in (2340.0, 1e5, 1e8):
            r1 = 6.12 * (p + 3.43e8)
            r2 = 1.4 * p
            a1 = 1 - a2
            kap = a1 * a2 * (1 / r2 - 1 / r1) / (a1 / r1 + a2 / r2)
            assert math.isclose(F.k_coefficient(c, a2, p), kap, rel_tol=1e-12)
    assert F.k_coefficient(c, 0.0, 1e5) == 0.0
    assert F.k_coefficient(c, 1.0, 1e5) == 0.0


def test_k_coefficient_keeps_a2_plus_k_in_unit_interval():
    """a2 + K = a2 r1 / (a1 r2 + a2 r1) is the share of the mixture's volume
    change taken by the gas.  It lies in [0, 1] whenever both phases are in
    their stiffened-gas range; below it (a trace of gas in water under
    tension) the formula's denominator can vanish, and the reading keeps
    a2 + K in [0, 1] there by clamping (the formula itself is unchanged where
    its value is in range)."""
    c = cfg1d(4)
    rng = np.random.default_rng(5)
    for _ in range(4000):
        a2 = rng.uniform(1e-9, 1 - 1e-9)
        p = rng.uniform(-5e8, 1e9)
        s = a2 + F.k_coefficient(c, a2, p)
        assert -1e-12 <= s <= 1 + 1e-12, (a2, p, s)
    # the divergent case seen at a collapse rebound: a2 = 2e-4, p = -3.1e5
    a2, p = 2.0e-4, -3.1e5
    r1, r2 = 6.12 * (p + 3.43e8), 1.4 * p
    raw = a2 * r1 / ((1 - a2) * r2 + a2 * r1)
    assert raw < -10                                   # the unclamped share
    assert a2 + F.k_coefficient(c, a2, p) == 0.0
    # a share above 1 (denominator small and positive) is clamped to 1
    p = -2.9e5
    r1, r2 = 6.12 * (p + 3.43e8), 1.4 * p
    assert a2 * r1 / ((1 - a2) * r2 + a2 * r1) > 1
    assert math.isclose(a2 + F.k_coefficient(c, a2, p), 1.0, rel_tol=1e-12)
    # in range, the clamp changes nothing (bitwise against the plain formula)
    for a2, p in ((0.3, 1e5), (0.01, 2340.0), (0.999, 1e8)):
        r1, r2 = 6.12 * (p + 3.43e8), 1.4 * p
        k = (1 - a2) * a2 * (r1 - r2) / ((1 - a2) * r2 + a2 * r1)
        assert F.k_coefficient(c, a2, p) == k


# --------------------------------------------------------------------------
# WENO5 (Sec. 2.2)
# --------------------------------------------------------------------------

def test_weno5_exact_for_quadratics():
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, b, cc = rng.normal(size=3)
        h = 0.1
        # cell averages of f(x) = a + b x + c x^2 over [ (i-1/2)h, (i+1/2)h ]
        avg = lambda i: a + b * i * h + cc * ((i * h) ** 2 + h * h / 12.0)
        v = [avg(i) for i in range(-2, 3)]
        exact = a + b * 0.5 * h + cc * (0.5 * h) ** 2
        assert abs(F.weno5_right_edge(*v, 1e-6) - exact) < 1e-12 * (1 + abs(exact))


def test_weno5_fifth_order_on_smooth_data():
    def err(n):
        h = 1.0 / n
        x0 = 0.3
        f_avg = lambda i: (math.cos(2 * math.pi * (x0 + (i - 0.5) * h))
                           - math.cos(2 * math.pi * (x0 + (i + 0.5) * h))) / (2 * math.pi * h)
        v = [f_avg(i) for i in range(-2, 3)]
        return abs(F.weno5_right_edge(*v, 1e-12) - math.sin(2 * math.pi * (x0 + 0.5 * h)))
    order = math.log2(err(160) / err(320))
    assert order > 4.5


# --------------------------------------------------------------------------
# WENO3 (Sec. 2.2: the paper's third-order option)
# --------------------------------------------------------------------------

def test_weno3_exact_for_linear_data_and_mirrored_left_edge():
    rng = np.random.default_rng(12)
    for _ in range(20):
        a, b = rng.normal(size=2)
        h = 0.1
        v = [a + b * i * h for i in (-1, 0, 1)]       # cell averages of a + b x
        assert abs(F.weno3_right_edge(*v, 1e-6) - (a + 0.5 * b * h)) < 1e-13 * (1 + abs(a))
        assert abs(F.weno3_right_edge(*v[::-1], 1e-6) - (a - 0.5 * b * h)) < 1e-13 * (1 + abs(a))


def test_weno3_ideal_weights_give_the_third_order_linear_scheme():
    """With eps far above every indicator the weights are the ideal ones and
    the edge value is that of the parabola with the three cell averages: exact
    for quadratics."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        a, b, cc = rng.normal(size=3)
        h = 0.1
        avg = lambda i: a + b * i * h + cc * ((i * h) ** 2 + h * h / 12.0)
        v = [avg(i) for i in (-1, 0, 1)]
        exact = a + b * 0.5 * h + cc * (0.5 * h) ** 2
        assert abs(F.weno3_right_edge(*v, 1e30) - exact) < 1e-12 * (1 + abs(exact))


def test_weno3_third_order_on_smooth_data():
    def err(n):
        h = 1.0 / n
        x0 = 0.3
        f_avg = lambda i: (math.cos(2 * math.pi * (x0 + (i - 0.5) * h))
                           - math.cos(2 * math.pi * (x0 + (i + 0.5) * h))) / (2 * math.pi * h)
        v = [f_avg(i) for i in (-1, 0, 1)]
        return abs(F.weno3_right_edge(*v, 1e-12) - math.sin(2 * math.pi * (x0 + 0.5 * h)))
    assert math.log2(err(160) / err(320)) > 2.5


def test_weno3_essentially_non_oscillatory_at_a_step():
    """A jump between cells c and c+1: the right edge of c comes from the
    smooth stencil (c-1, c), up to eps^2."""
    assert abs(F.weno3_right_edge(0.0, 0.0, 1.0, 1e-6)) < 1e-11
    assert abs(F.weno3_right_edge(1.0, 1.0, 0.0, 1e-6) - 1.0) < 1e-11


def test_weno3_positivity_uses_the_simpson_point():
    """A narrow dip in a partial density: both WENO3 edges are positive, but
    with the cell mean they imply a negative value at the cell centre under
    Simpson's rule, so the variable falls back to the cell value."""
    c = cfg1d(8, weno_order=3)
    w = lambda r: np.array([r, 0.0, 0.0, 1e5, 0.0])
    st = [w(1.0), w(1.0), w(0.01), w(1.0), w(1.0)]
    hi3 = F.weno3_right_edge(1.0, 0.01, 1.0, 1e-6)
    assert hi3 > 0 and (6 * 0.01 - 2 * hi3) / 4 < 0        # edges > 0, Simpson point < 0
    lo, hi, replaced = F.cell_edges(c, st)
    assert replaced and lo[0] == 0.01 and hi[0] == 0.01
    # a smooth positive stencil keeps its reconstruction
    st = [w(1.0), w(1.1), w(1.2), w(1.3), w(1.4)]
    lo, hi, replaced = F.cell_edges(c, st)
    assert not replaced
    assert abs(hi[0] - 1.25) < 1e-12 and abs(lo[0] - 1.15) < 1e-12
    # the order follows the spec: curved data, WENO3 and WENO5 edges differ
    st = [w(1.0 + 0.1 * k + 0.05 * k * k) for k in range(5)]
    r = [x[0] for x in st]
    lo, _, _ = F.cell_edges(c, st)
    _, hi5, _ = F.cell_edges(cfg1d(8), st)
    assert lo[0] == F.weno3_right_edge(r[3], r[2], r[1], 1e-6)
    assert hi5[0] == F.weno5_right_edge(*r, 1e-6)
    assert abs(lo[0] - F.weno5_right_edge(*r[::-1], 1e-6)) > 1e-4


def test_weno3_shock_tube_converges_to_exact():
    left, right, T, sl, sr = CASES["sod_ideal_gas"]
    e1 = _tube(100, left, right, T, sl, sr, weno_order=3)
    e2 = _tube(400, left, right, T, sl, sr, weno_order=3)
    assert e2[0] < 0.6 * e1[0] and e2[1] < 0.6 * e1[1]
    assert e2[0] < 0.015 and e2[1] < 0.015


# --------------------------------------------------------------------------
# HLLC (Sec. 2.2)
# --------------------------------------------------------------------------

def physical_flux(w, direction, ndim, g1=6.12, pc1=3.43e8, g2=1.4, pc2=0.0):
    """Flux vectors F, G, H of eq. (system) for primitive state w."""
    a1r1, a2r2 = w[0], w[1]
    u = w[2:2 + ndim]
    p, a2 = w[2 + ndim], w[3 + ndim]
    rho = a1r1 + a2r2
    G = (1 - a2) / (g1 - 1) + a2 / (g2 - 1)
    P = (1 - a2) * g1 * pc1 / (g1 - 1) + a2 * g2 * pc2 / (g2 - 1)
    E = G * p + P + 0.5 * rho * np.dot(u, u)
    un = u[direction]
    f = [a1r1 * un, a2r2 * un]
    f += [rho * u[m] * un + (p if m == direction else 0.0) for m in range(ndim)]
    f += [(E + p) * un, a2 * un, un]
    return np.array(f)


@pytest.mark.parametrize("direction", [0, 1, 2])
def test_hllc_consistency(direction):
    c = cfg_nd(3, 4)
    rng = np.random.default_rng(3 + direction)
    for _ in range(10):
        a2 = rng.uniform(0, 1)
        w = np.array([(1 - a2) * 1000, a2 * 1.0, *rng.normal(0, 100, 3), rng.uniform(1e4, 1e7), a2])
        f = F.hllc(c, direction, w, w)
        np.testing.assert_allclose(f, physical_flux(w, direction, 3), rtol=1e-12, atol=1e-9)


def test_hllc_isolated_contact_is_upwind():
    """Equal p and u on both sides (a pure material contact): the HLLC flux is
    the upwind physical flux, and the face velocity is u."""
    c = cfg_nd(2, 4)
    for u in (40.0, -25.0):
        wl = np.array([1000.0, 0.0, u, 3.0, 1e6, 0.0])
        wr = np.array([0.0, 1.0, u, -2.0, 1e6, 1.0])
        f = F.hllc(c, 0, wl, wr)
        up = wl if u > 0 else wr
        np.testing.assert_allclose(f, physical_flux(up, 0, 2), rtol=1e-10, atol=1e-6)


# --------------------------------------------------------------------------
# Runge-Kutta (Sec. 2.2)
# --------------------------------------------------------------------------

def test_rk_coefficients_third_order_rational():
    A, B = F.rk_coefficients()
    fa = [Fraction(0), Fraction(-17, 32), Fraction(-32, 27)]
    fb = [Fraction(1, 4), Fraction(8, 9), Fraction(3, 4)]
    for k in range(3):
        assert abs(A[k] - float(fa[k])) < 1e-16 and abs(B[k] - float(fb[k])) < 1e-16
    # Butcher form of the 2N scheme dU <- A_k dU + dt L(U); U <- U + B_k dU:
    # the stage increments q_k = dt L(y_{k-1}) + A_k q_{k-1}, y_k = y_{k-1} + B_k q_k.
    s = 3
    Q = [[Fraction(0)] * s for _ in range(s)]   # q_k as combination of dt L(y_j)
    Y = [[Fraction(0)] * s for _ in range(s + 1)]  # y_k - y_0
    for k in range(s):
        Q[k] = [(fa[k] * Q[k - 1][j] if k else Fraction(0)) + (1 if j == k else 0) for j in range(s)]
        Y[k + 1] = [Y[k][j] + fb[k] * Q[k][j] for j in range(s)]
    b = Y[s]
    Amat = [Y[k] for k in range(s)]   # stage k is evaluated at y_k
    cvec = [sum(row) for row in Amat]
    assert sum(b) == 1
    assert sum(b[i] * cvec[i] for i in range(s)) == Fraction(1, 2)
    assert sum(b[i] * cvec[i] ** 2 for i in range(s)) == Fraction(1, 3)
    assert sum(b[i] * sum(Amat[i][j] * cvec[j] for j in range(s)) for i in range(s)) == Fraction(1, 6)


def test_rk_third_order_in_time():
    """Fixed grid, shrinking dt: successive differences shrink by about 2^3."""
    n = 32
    c = cfg1d(n, bc="periodic")
    W = random_smooth_primitives(1, n, seed=5, p_amp=1e5, u_amp=5.0, a2_amp=0.2)
    U0 = F.prim_to_cons(c, W)
    T = 2e-5
    sols = []
    for m in (4, 8, 16):
        U = U0.copy()
        for _ in range(m):
            U = F.step(c, U, T / m)
        sols.append(U)
    d1 = np.abs(sols[0] - sols[1]).max()
    d2 = np.abs(sols[1] - sols[2]).max()
    assert 6.0 < d1 / d2 < 10.0


# --------------------------------------------------------------------------
# Exact Riemann problems (Sec. 2.2: Godunov-type scheme)
# --------------------------------------------------------------------------

def test_exact_riemann_pinned_to_textbook():
    g = GOLD["sod_star"]
    ex = ExactRiemann(Side(1, 0, 1, 1.4, 0), Side(0.125, 0, 0.1, 1.4, 0))
    assert abs(ex.ps - g["p_star"]) < 1e-5
    assert abs(ex.us - g["u_star"]) < 1e-5


def _tube(n, left, right, T, sl, sr, **kw):
    c = cfg1d(n, **kw)
    U = F.prim_to_cons(c, riemann_primitives(1, n, left, right))
    h = 1.0 / n
    t = 0.0
    while t < T:
        dt = min(0.3 * h / F.reduce(c, U)["s_max"], T - t)
        U = F.step(c, U, dt)
        t += dt
    W = F.cons_to_prim(c, U)
    ex = ExactRiemann(sl, sr)
    x = (np.arange(n) + 0.5) / n
    rho, u, p, _ = ex.profile(x, 0.5, T)
    return (np.mean(np.abs((W[0] + W[1]).ravel() - rho)) / np.max(rho),
            np.mean(np.abs(W[3].ravel() - p)) / np.max(np.abs(p)))


CASES = {
    "sod_ideal_gas": (dict(a1r1=0.0, a2r2=1.0, u=0.0, p=1.0, a2=1.0),
                      dict(a1r1=0.0, a2r2=0.125, u=0.0, p=0.1, a2=1.0),
                      0.2, Side(1, 0, 1, 1.4, 0), Side(0.125, 0, 0.1, 1.4, 0)),
    "water_stiffened": (dict(a1r1=1000.0, a2r2=0.0, u=0.0, p=1e9, a2=0.0),
                        dict(a1r1=1000.0, a2r2=0.0, u=0.0, p=1e5, a2=0.0),
                        1.2e-4, Side(1000, 0, 1e9, 6.12, 3.43e8), Side(1000, 0, 1e5, 6.12, 3.43e8)),
    "water_air": (dict(a1r1=1000.0, a2r2=0.0, u=0.0, p=1e9, a2=0.0),
                  dict(a1r1=0.0, a2r2=50.0, u=0.0, p=1e5, a2=1.0),
                  2.4e-4, Side(1000, 0, 1e9, 6.12, 3.43e8), Side(50, 0, 1e5, 1.4, 0)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_shock_tube_converges_to_exact(case):
    left, right, T, sl, sr = CASES[case]
    e1 = _tube(100, left, right, T, sl, sr)
    e2 = _tube(400, left, right, T, sl, sr)
    assert e2[0] < 0.6 * e1[0] and e2[1] < 0.6 * e1[1]
    assert e2[0] < 0.01 and e2[1] < 0.01


# --------------------------------------------------------------------------
# Characteristic far-field boundary (Sec. 3.1, after Poinsot and Lele)
# --------------------------------------------------------------------------

def _water_impedance(p, rho=1000.0):
    """rho c of pure water from the textbook stiffened-gas sound speed."""
    return rho * math.sqrt(EOS["gamma1"] * (p + EOS["pc1"]) / rho)


def test_char_ghost_keeps_outgoing_and_relaxes_incoming_invariant():
    c = cfg1d(16, bc="characteristic")
    rng = np.random.default_rng(21)
    p_inf = c["p_inf"]
    for _ in range(20):
        p = rng.uniform(0.5, 2.0) * p_inf
        u = rng.normal(0, 20.0)
        w = np.array([1000.0, 0.0, u, p, 0.0])
        Z = _water_impedance(p)
        for side in (-1, 1):
            assert np.array_equal(F.char_ghost(c, 0, side, 0.0, w), w)       # beta = 0: zero gradient
            for beta in (0.3, 1.0):
                g = F.char_ghost(c, 0, side, beta, w)
                assert g[0] == w[0] and g[1] == w[1] and g[4] == w[4]
                rp, rm = p + side * Z * u, p - side * Z * u
                assert abs(g[3] + side * Z * g[2] - rp) <= 1e-12 * p_inf          # outgoing kept
                assert abs(g[3] - side * Z * g[2] - (rm + beta * (p_inf - rm))) <= 1e-12 * p_inf
    # the far field at rest is a fixed point; tangential velocity is copied
    c2 = cfg_nd(2, 16, bc="characteristic")
    w = np.array([1000.0, 0.0, 0.0, 3.0, p_inf, 0.0])
    g = F.char_ghost(c2, 0, 1, 0.7, w)
    assert g[2] == 0.0 and g[3] == 3.0 and g[4] == p_inf


def test_char_boundary_rate_matches_linear_acoustics():
    """Uniform water at rest with a small excess D over p_inf: only the two
    boundary cells move, at the rates of the acoustic Riemann problem against
    the ghost state: dp/dt = -c beta D / (2h), du/dt = s beta D / (2 rho h)
    (outwards: s = -1 on the low side, +1 on the high side)
    (beta = sigma h with sigma = 0.25), i.e. the incoming invariant relaxes at
    K = sigma c.  The WENO epsilon is taken far below the squared jumps (the
    ghost velocity is ~1e-6 m/s), so that the reconstruction keeps the two
    constant states apart and the face sees exactly this Riemann problem."""
    n = 32
    c = cfg1d(n, bc="characteristic", weno_eps=1e-30)
    p_inf = c["p_inf"]
    D = 1e-4 * p_inf
    W = np.zeros((5, n))
    W[0], W[3] = 1000.0, p_inf + D
    U = F.prim_to_cons(c, W)
    L, _ = F.rhs(c, U)
    h, beta = 1.0 / n, 0.25 / n
    cs = _water_impedance(p_inf + D) / 1000.0
    G = 1.0 / (EOS["gamma1"] - 1.0)
    dpdt = L[3] / G                               # at rest, pure water: p = (Et)/Gamma
    dudt = L[2] / 1000.0
    assert np.all(L[:, 3:-3] == 0.0)
    for i, side in ((0, -1), (n - 1, 1)):
        assert abs(dpdt[i] / (-cs * beta * D / (2 * h)) - 1) < 2e-3
        assert abs(dudt[i] / (side * beta * D / (2 * 1000.0 * h)) - 1) < 2e-3
        assert abs(L[0, i]) > 0                   # mass leaves / enters with the wave


def _run_to(c, W, T):
    U = F.prim_to_cons(c, W)
    t, h = 0.0, 1.0 / c["n"]
    while t < T:
        dt = min(0.3 * h / F.reduce(c, U)["s_max"], T - t)
        U = F.step(c, U, dt)
        t += dt
    return F.cons_to_prim(c, U)


def test_char_boundary_lets_an_acoustic_pulse_leave():
    """A right-running pressure pulse (p' = Z u') leaves through the far-field
    boundary: what stays in the domain after it has left is below 1.5 % of
    its amplitude."""
    n = 128
    c = cfg1d(n, bc="characteristic")
    p_inf = c["p_inf"]
    Z = _water_impedance(p_inf)
    x = (np.arange(n) + 0.5) / n
    A = 1e5
    dp = A * np.exp(-((x - 0.5) / 0.05) ** 2)
    W = np.zeros((5, n))
    W[0], W[2], W[3] = 1000.0, dp / Z, p_inf + dp
    Wt = _run_to(c, W, 0.9 / (Z / 1000.0))
    assert np.max(np.abs(Wt[3] - p_inf)) < 0.015 * A


def test_char_boundary_relaxes_the_pressure_to_the_far_field():
    """Water at rest 10 % above p_inf: the mean excess decays monotonically
    under the far-field condition (below half after 4 L/c), while with
    zero-gradient sides it stays."""
    n = 64
    W = np.zeros((5, n))
    W[0], W[3] = 1000.0, 1.1e7
    cl = _water_impedance(1.0e7) / 1000.0
    devs = []
    for T in (1.0, 2.0, 4.0):
        Wt = _run_to(cfg1d(n, bc="characteristic"), W, T / cl)
        devs.append(np.mean(Wt[3] - 1.0e7) / 1.0e6)
    assert 1.0 > devs[0] > devs[1] > devs[2] and devs[2] < 0.5
    Wz = _run_to(cfg1d(n), W, 1.0 / cl)
    assert np.max(np.abs(Wz[3] / 1.1e7 - 1)) < 1e-13


def test_char_boundary_keeps_mirror_symmetry():
    """A centred bubble in 2-D: the far-field sides keep the solution
    symmetric under x -> 1 - x and x <-> y."""
    n = 24
    c = cfg_nd(2, n, bc="characteristic", cloud_radius=0.2)
    bub = np.array([[0.5, 0.5, 0.0, 0.12]])
    U = F.init_state(c, bub)
    U, _ = F.run_steps(c, U, 30)
    W = F.cons_to_prim(c, U)
    p = W[4].reshape(n, n)
    assert np.max(np.abs(p - p[:, ::-1])) <= 1e-9 * np.max(np.abs(p))
    assert np.max(np.abs(p - p.T)) <= 1e-9 * np.max(np.abs(p))


# --------------------------------------------------------------------------
# Invariants of the scheme
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_conservation_periodic(ndim):
    n = 16 if ndim == 2 else 10
    c = cfg_nd(ndim, n, bc="periodic")
    U = F.prim_to_cons(c, random_smooth_primitives(ndim, n, seed=7))
    s0 = U.reshape(U.shape[0], -1).sum(axis=1)
    U, _ = F.run_steps(c, U, 20 if ndim == 2 else 10)
    s1 = U.reshape(U.shape[0], -1).sum(axis=1)
    for v in range(3 + ndim):        # a1r1, a2r2, momenta, E (a2 has a source)
        scale = np.abs(U[v]).sum()
        assert abs(s1[v] - s0[v]) <= 1e-13 * scale, v


@pytest.mark.parametrize("ndim", [1, 2])
def test_interface_pressure_velocity_equilibrium(ndim):
    """Uniform p and u across jumps of a2 between 0 and 1 stay uniform to
    round-off (Johnsen-Colonius adaptation of HLLC, Sec. 2.2; Abgrall's
    criterion).

    Two materials with different gamma (6.12 and 1.4), a 1000:1 density jump
    and no stiffness (pc1 = 0): p and u stay uniform to 1e-12 relative after
    40 steps.  With water's stiffness (pc1 = 3.43e8) the oracle recovers p
    from the stored E, which is dominated by Pi ~ 4e8 against Gamma p ~ 2e4,
    so the round-off of E (not the scheme) sets the pressure's error: it is
    held to 1e-12 of the energy's pressure scale max(E) / Gamma_water, and
    the velocity to 1e-10 relative."""
    n = 32
    W0 = interface_primitives(ndim, n, seed=11)
    # no stiffness: round-off of p itself
    c = cfg_nd(ndim, n, bc="periodic", eos=dict(EOS, pc1=0.0))
    U, _ = F.run_steps(c, F.prim_to_cons(c, W0), 40)
    W = F.cons_to_prim(c, U)
    assert np.abs(W[2 + ndim] / 1.0e5 - 1).max() <= 1e-12
    for m in range(ndim):
        assert np.abs(W[2 + m] / W0[2 + m][0, 0, 0] - 1).max() <= 1e-12
    # stiffened water: round-off of the stored energy
    c = cfg_nd(ndim, n, bc="periodic")
    U = F.prim_to_cons(c, W0)
    e_scale = np.abs(U[2 + ndim]).max() * (EOS["gamma1"] - 1.0)
    U, _ = F.run_steps(c, U, 40)
    W = F.cons_to_prim(c, U)
    assert np.abs(W[2 + ndim] - 1.0e5).max() <= 1e-12 * e_scale
    for m in range(ndim):
        assert np.abs(W[2 + m] / W0[2 + m][0, 0, 0] - 1).max() <= 1e-10
    # the material jump is still there (the test is not of a smeared field)
    assert W[3 + ndim].min() < 0.5 < W[3 + ndim].max()


def test_mirror_symmetry_single_bubble():
    n = 32
    c = solver_config("cloud2d", n)
    bub = np.array([[0.5, 0.5, 0.0, 0.1]])
    U = F.init_state(c, bub)
    U, _ = F.run_steps(c, U, 60)
    W = F.cons_to_prim(c, U)
    p = W[4, 0]
    scale = np.abs(p).max()
    assert np.abs(p - p[:, ::-1]).max() < 1e-9 * scale
    assert np.abs(p - p[::-1, :]).max() < 1e-9 * scale
    assert np.abs(p - p.T).max() < 1e-9 * scale
    # velocity is odd under the mirror
    u = W[2, 0]
    assert np.abs(u + u[:, ::-1]).max() < 1e-9 * np.abs(u).max()


# --------------------------------------------------------------------------
# Initial state (Sec. 3.1)
# --------------------------------------------------------------------------

def test_init_volume_fraction_brute_force():
    n, ns = 8, 4
    c = solver_config("cloud50", n, n_sub=ns)
    bub = np.array([[0.41, 0.52, 0.47, 0.13], [0.7, 0.3, 0.6, 0.08]])
    U = F.init_state(c, bub)
    a2 = U[6]
    for k in range(n):
        for j in range(n):
            for i in range(n):
                cnt = 0
                for sc in range(ns):
                    for sb in range(ns):
                        for sa in range(ns):
                            x = ((ns * i + sa) + 0.5) / (ns * n)
                            y = ((ns * j + sb) + 0.5) / (ns * n)
                            z = ((ns * k + sc) + 0.5) / (ns * n)
                            if any((x - b[0]) ** 2 + (y - b[1]) ** 2 + (z - b[2]) ** 2 < b[3] ** 2 for b in bub):
                                cnt += 1
                assert a2[k, j, i] == cnt / ns ** 3


def test_init_gas_volume_and_pressure_ramp():
    n = 128
    c = solver_config("cloud2d", n)
    r = 0.05
    U = F.init_state(c, np.array([[0.5, 0.5, 0.0, r]]))
    W = F.cons_to_prim(c, U)
    area = W[5].sum() / n ** 2
    assert abs(area - math.pi * r * r) < 2e-3 * math.pi * r * r
    # pressure: p_bubble inside the cloud, p_inf past the ramp
    p = W[4, 0]
    assert abs(p[n // 2, n // 2] - 2340.0) < 1e-6
    assert abs(p[0, 0] - 1.0e7) < 1e-3
    assert np.all(W[2:4] == 0.0)
    np.testing.assert_allclose(W[0] + W[1], (1 - W[5]) * 1000.0 + W[5] * 1.0, rtol=1e-14)


# --------------------------------------------------------------------------
# Time loop and QoI
# --------------------------------------------------------------------------

def test_solve_qoi_tracks_running_maximum():
    n = 32
    c = solver_config("cloud2d", n)
    bub = np.array([[0.5, 0.5, 0.0, 0.08], [0.3, 0.62, 0.0, 0.05]])
    nst = 40
    q = F.solve(c, bub, n_steps=nst)
    assert q["status"] == 0 and q["steps"] == nst
    # brute force over the time levels with single steps
    U = F.init_state(c, bub)
    best, where, when, t = -np.inf, -1, 0.0, 0.0
    for s in range(nst + 1):
        W = F.cons_to_prim(c, U)
        p = W[4].ravel()
        i = int(np.argmax(p))
        if p[i] > best:
            best, where, when = p[i], i, t
        if s < nst:
            U, dts = F.run_steps(c, U, 1)
            t += dts[0]
    assert q["p_max"] == best and q["argmax"] == where and q["t_at_max"] == when
    assert q["x"][0] == ((where % n) + 0.5) / n and q["x"][1] == ((where // n) + 0.5) / n


def _ball_cells(cfg, r2):
    n, d = cfg["n"], cfg["ndim"]
    axes = [(np.arange(n) + 0.5) / n - cfg["center"][a] for a in range(d)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")          # (z, y, x) order of the state
    d2 = sum(g * g for g in grids)
    return (d2 <= r2).ravel()


def test_sensor_qois_brute_force():
    """Sensor QoIs (eq. (sensor)) against a scan over the time levels: the
    ball averages of p and a2 are the means over the cells whose centres lie
    in the balls, maxima/minima are tracked over n = 0..steps (earliest time
    on ties), c_max over cells and levels, the peak distance from x."""
    n = 32
    c = solver_config("cloud2d", n)
    bub = np.array([[0.5, 0.5, 0.0, 0.08], [0.3, 0.62, 0.0, 0.05]])
    nst = 30
    q = F.solve(c, bub, n_steps=nst)
    rp = max(c["cloud_radius"] / 40.0, 1.01 * 0.5 * math.sqrt(2.0) / n)
    in_p = _ball_cells(c, rp * rp)
    in_a = _ball_cells(c, c["cloud_radius"] ** 2)
    U = F.init_state(c, bub)
    g1, g2 = c["eos"]["gamma1"], c["eos"]["gamma2"]
    P1 = g1 * c["eos"]["pc1"] / (g1 - 1)
    ps_best, ps_t, gs_best, gs_t, cmax, t = -np.inf, 0.0, np.inf, 0.0, 0.0, 0.0
    for st in range(nst + 1):
        W = F.cons_to_prim(c, U)
        rho = (W[0] + W[1]).ravel()
        p, a2 = W[4].ravel(), W[5].ravel()
        G = (1 - a2) / (g1 - 1) + a2 / (g2 - 1)
        Pi = (1 - a2) * P1
        cs = np.sqrt(((G + 1) * p + Pi) / (G * rho))
        ps, gs = p[in_p].mean(), a2[in_a].mean()
        if ps > ps_best:
            ps_best, ps_t = ps, t
        if gs < gs_best:
            gs_best, gs_t = gs, t
        cmax = max(cmax, cs.max())
        if st < nst:
            U, dts = F.run_steps(c, U, 1)
            t += dts[0]
    assert math.isclose(q["p_sensor"], ps_best, rel_tol=1e-13) and q["t_p_sensor"] == ps_t
    assert math.isclose(q["gas_min"], gs_best, rel_tol=1e-13) and q["t_gas_min"] == gs_t
    assert math.isclose(q["c_max"], cmax, rel_tol=1e-13)
    assert math.isclose(q["peak_distance"], math.hypot(q["x"][0] - 0.5, q["x"][1] - 0.5), rel_tol=1e-15)


def test_sensor_closed_forms_at_rest():
    """At t = 0 the sensor at the centre of the cloud reads the bubble
    pressure (the ramp starts beyond the cloud), the fastest sound is pure
    water's at p_inf, a coarse even grid's pressure ball is the 2^d cells
    around the centre, and the gas sensor counts the lattice points in the
    cloud's ball."""
    for cloud, n in (("cloud500", 64), ("cloud2d", 48)):
        c = solver_config(cloud, n)
        bub = sample_cloud(cloud_spec(cloud), 170504374, 0, 1)
        r = F.initial_reduction(c, bub)
        d = c["ndim"]
        assert r["n_ball_p"] == 2 ** d                     # R_c/40 is below half a cell diagonal here
        # cells of the pressure ball are not all water: the sensor reads the
        # cells' pressure, p_bubble in water and gas alike
        assert math.isclose(r["p_ball"] / r["n_ball_p"], c["p_bubble"], rel_tol=1e-12)
        cw = math.sqrt(c["eos"]["gamma1"] * (c["p_inf"] + c["eos"]["pc1"]) / c["rho1"])
        assert math.isclose(r["c_max"], cw, rel_tol=1e-12)
        assert r["n_ball_a"] == int(_ball_cells(c, c["cloud_radius"] ** 2).sum())
    # at 512^3 the pressure ball has radius R_c/40 = 3.84 cells: the oracle's
    # count on a box around the centre equals the half-integer lattice points
    # in that ball
    c = solver_config("cloud500", 512)
    rp = c["cloud_radius"] / 40.0
    m = np.arange(-6, 6) + 0.5
    lattice = int(((m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2) / 512 ** 2 <= rp * rp).sum())
    box = ((250, 250, 250), (12, 12, 12))
    bub = sample_cloud(cloud_spec("cloud500"), 170504374, 0, 1)
    r = F.reduce(c, F.init_state(c, bub, box), box)
    assert r["n_ball_p"] == lattice == 208


def test_solve_lands_on_end_time_and_caps_steps():
    c = solver_config("cloud2d", 16)
    bub = np.array([[0.5, 0.5, 0.0, 0.1]])
    q = F.solve(c, bub, t_end=1.0e-4)
    assert q["status"] == 0 and q["t"] == 1.0e-4
    q = F.solve(c, bub, t_end=1.0e-4, max_steps=3)
    assert q["status"] == 3 and q["steps"] == 3


def test_box_steps_match_full_domain_inside():
    """A sub-box advanced with the same steps equals the full solve away from
    its artificial sides (used to check single cells of large grids)."""
    n = 32
    c = solver_config("cloud50", n)
    bub = np.array([[0.45, 0.5, 0.55, 0.12]])
    U = F.init_state(c, bub)
    U1, dts = F.run_steps(c, U, 1)
    lo, ln = (3, 2, 5), (24, 26, 22)       # (x, y, z); every side is artificial
    B = F.box_steps(c, bub, (lo, ln), dts)
    m = 9                                  # 3 stages x 3 cells of stencil reach
    inner = (slice(None), slice(m, ln[2] - m), slice(m, ln[1] - m), slice(m, ln[0] - m))
    ref = U1[:, lo[2]:lo[2] + ln[2], lo[1]:lo[1] + ln[1], lo[0]:lo[0] + ln[0]]
    assert B[inner].size > 0
    assert np.array_equal(B[inner], ref[inner])
    # a box touching the domain sides is exact up to those sides
    lo2, ln2 = (0, 0, 0), (20, 20, 20)
    B2 = F.box_steps(c, bub, (lo2, ln2), dts)
    assert np.array_equal(B2[:, :11, :11, :11], U1[:, :11, :11, :11])


def test_stored_collapse_qois_are_the_oracles():
    """The golden file of whole-collapse QoIs (written by
    tests/golden/make_collapse_golden.py) matches the oracle as it stands:
    one 2-D sample recomputed to the end time, and the stored spreads are
    those of its stored perturbed runs."""
    from workloads.configs import MASTER_SEED, t_end
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "collapse_qoi.json")))
    case = [c for c in gold["cases"] if (c["cloud"], c["n"], c["term"], c["index"]) == ("cloud2d", 32, 0, 4)][0]
    cfg = solver_config("cloud2d", 32)
    bub = sample_cloud(cloud_spec("cloud2d"), MASTER_SEED, 0, 4)
    r = F.solve(cfg, bub, t_end=t_end("cloud2d"))
    assert case["t_end"] == t_end("cloud2d")
    for k in ("p_max", "t_at_max", "p_sensor", "gas_min", "c_max"):
        assert math.isclose(r[k], case["qoi"][k], rel_tol=1e-13), k
    assert r["steps"] == case["qoi"]["steps"] and r["argmax"] == case["qoi"]["argmax"]
    for c in gold["cases"]:
        for kind, runs in c["perturbed"].items():
            for k in ("p_max", "c_max"):
                s = max(abs(x[k] - c["qoi"][k]) / abs(c["qoi"][k]) for x in runs)
                assert s == c["spread"][kind][k]
