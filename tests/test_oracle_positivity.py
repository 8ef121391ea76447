"""Pins of the oracle's WENO5 positivity / bounds fallback (the reading of the
Sec. 2.2 scheme that keeps partial densities non-negative and a2 in [0, 1]).

Every stencil here holds the cell averages of a known quadratic
q(x) = A + B x + G x^2 (cell k covers [k - 1/2, k + 1/2], the centre cell is
k = 0).  Each of WENO5's three candidate stencils reconstructs a quadratic
exactly, so the edge values are q(-1/2) and q(1/2) whatever the nonlinear
weights are, and the test knows them without the reconstruction formula.

The four-point Gauss-Lobatto rule on the cell (nodes -1/2, -x1, x1, 1/2 with
x1 = 1/(2 sqrt 5), weights 1/12, 5/12, 5/12, 1/12) is exact up to degree 5, so
for the quadratic the cell mean is q(-1/2)/12 + 5/12 (q(-x1) + q(x1)) +
q(1/2)/12.  The interior value the check uses is the mean of the two interior
nodes; the tests compute it from the polynomial at those nodes, and check that
the mean identity holds, so that the pins do not restate the oracle's form
(12 mean - lo - hi) / 10.
"""
import math

import numpy as np
import pytest

import oracle.flow as F
from workloads.configs import BASE, EOS

X1 = 1.0 / (2.0 * math.sqrt(5.0))       # interior Gauss-Lobatto node of the unit cell
TOL = 1e-12                              # round-off allowance of the FP64 oracle


def cfg(ndim=1, **kw):
    c = dict(BASE)
    c.update(ndim=ndim, n=8, eos=dict(EOS))
    c.update(kw)
    return c


def quad(A, B, G):
    """(cell averages k = -2..2, left edge, right edge, interior GL value, mean)."""
    avg = [A + B * k + G * (k * k + 1.0 / 12.0) for k in range(-2, 3)]
    q = lambda x: A + B * x + G * x * x
    lo, hi = q(-0.5), q(0.5)
    mid = 0.5 * (q(-X1) + q(X1))
    mean = avg[2]
    # the rule is exact for the quadratic: the identity the check relies on
    assert math.isclose(lo / 12 + 5.0 / 6.0 * mid + hi / 12, mean, rel_tol=1e-13, abs_tol=1e-15)
    return avg, lo, hi, mid, mean


def stencil(ndim, cols):
    """Five primitive states [a1r1, a2r2, u_1..u_d, p, a2] from per-variable
    lists of five cell values (missing velocities are zero)."""
    nv = 4 + ndim
    st = np.zeros((5, nv))
    for v, vals in cols.items():
        st[:, v] = vals
    return st


# quiet companions: smooth positive data whose edges are exact quadratic values
Q_A2R2 = quad(0.5, 0.01, 0.002)
Q_U = quad(3.0, -0.5, 0.2)
Q_P = quad(1.0e5, 300.0, 40.0)
Q_A2 = quad(0.4, 0.05, 0.0)


def base_cols(ndim):
    cols = {1: Q_A2R2[0], 2: Q_U[0], 2 + ndim: Q_P[0], 3 + ndim: Q_A2[0]}
    return cols


def assert_kept(lo, hi, v, q, rel=1e-12):
    assert math.isclose(lo[v], q[1], rel_tol=rel, abs_tol=1e-14), (v, lo[v], q[1])
    assert math.isclose(hi[v], q[2], rel_tol=rel, abs_tol=1e-14), (v, hi[v], q[2])


@pytest.mark.parametrize("ndim", [1, 3])
def test_partial_density_interior_point_negative_falls_back_alone(ndim):
    """A convex dip in the water's partial density: every cell average and
    both edges are positive, the interior Gauss-Lobatto value is negative.
    Only that variable takes its cell value at both edges; the other
    variables keep their reconstructions."""
    q = quad(-3.3, 2.0, 60.0)
    avg, lo_e, hi_e, mid, mean = q
    assert min(avg) > 0 and lo_e > 0 and hi_e > 0 and mid < 0 and mean > 0
    cols = base_cols(ndim)
    cols[0] = avg
    lo, hi, replaced = F.cell_edges(cfg(ndim), stencil(ndim, cols))
    assert replaced
    assert lo[0] == avg[2] and hi[0] == avg[2]
    for v, qq in ((1, Q_A2R2), (2, Q_U), (2 + ndim, Q_P), (3 + ndim, Q_A2)):
        assert_kept(lo, hi, v, qq)


def test_partial_density_positive_interior_point_is_kept():
    """The same dip made shallower: the interior value is positive, the
    reconstruction is kept (edges of the quadratic)."""
    q = quad(-2.9, 2.0, 60.0)
    assert q[3] > 0
    cols = base_cols(1)
    cols[0] = q[0]
    lo, hi, replaced = F.cell_edges(cfg(1), stencil(1, cols))
    assert not replaced
    assert_kept(lo, hi, 0, q)


def test_gas_partial_density_interior_point_negative_falls_back_alone():
    q = quad(-0.033, 0.02, 0.6)
    assert min(q[0]) > 0 and q[1] > 0 and q[2] > 0 and q[3] < 0
    cols = base_cols(1)
    cols[1] = q[0]
    cols[0] = quad(900.0, 5.0, 1.0)[0]
    lo, hi, replaced = F.cell_edges(cfg(1), stencil(1, cols))
    assert replaced and lo[1] == q[0][2] and hi[1] == q[0][2]
    assert_kept(lo, hi, 0, quad(900.0, 5.0, 1.0))
    assert_kept(lo, hi, 3, Q_P)


def concave_peak_at_right_edge(mean, G):
    """Quadratic with its maximum at x = 1/2 and cell mean `mean`."""
    B = -G
    A = mean - G / 12.0
    return quad(A, B, G)


@pytest.mark.parametrize("ndim", [1, 3])
def test_a2_outside_unit_interval_at_one_edge_falls_back_alone(ndim):
    """a2 averages all in [0, 1] whose reconstruction overshoots 1 at the right
    edge (interior value inside): only a2 takes its cell value.  Had the
    c^2 check looked at the overshooting edge (Pi(a2 > 1) < 0 in water), the
    whole cell would have gone first order; the check follows the per-variable
    replacement, so the partial densities keep their reconstructions."""
    q = concave_peak_at_right_edge(0.98, -0.15)
    avg, lo_e, hi_e, mid, _ = q
    assert all(0.0 <= a <= 1.0 for a in avg) and hi_e > 1.0 and 0 <= lo_e <= 1 and 0 <= mid <= 1
    c = cfg(ndim)
    cols = base_cols(ndim)
    cols[3 + ndim] = avg
    cols[0] = quad(20.0, 1.0, 0.5)[0]
    lo, hi, replaced = F.cell_edges(c, stencil(ndim, cols))
    assert replaced
    assert lo[3 + ndim] == avg[2] and hi[3 + ndim] == avg[2]
    assert_kept(lo, hi, 0, quad(20.0, 1.0, 0.5))
    assert_kept(lo, hi, 1, Q_A2R2)
    assert_kept(lo, hi, 2 + ndim, Q_P)
    # the overshooting edge state itself has no positive c^2 in this EOS
    e = EOS
    a2 = hi_e
    G = (1 - a2) / (e["gamma1"] - 1) + a2 / (e["gamma2"] - 1)
    Pi = (1 - a2) * e["gamma1"] * e["pc1"] / (e["gamma1"] - 1)
    assert (G + 1) * Q_P[2] + Pi <= 0


def test_a2_interior_point_outside_unit_interval_falls_back():
    """a2 edges inside [0, 1], interior value below 0."""
    q = quad(-0.011, 0.0, 0.2)
    avg, lo_e, hi_e, mid, _ = q
    assert 0 <= lo_e <= 1 and 0 <= hi_e <= 1 and mid < 0 and all(a >= 0 for a in avg)
    cols = base_cols(1)
    cols[4] = avg
    lo, hi, replaced = F.cell_edges(cfg(1), stencil(1, cols))
    assert replaced and lo[4] == avg[2] and hi[4] == avg[2]
    assert_kept(lo, hi, 1, Q_A2R2)
    assert_kept(lo, hi, 3, Q_P)


@pytest.mark.parametrize("ndim", [1, 3])
def test_negative_c2_at_an_edge_makes_the_whole_cell_first_order(ndim):
    """Pure air (a2 = 1, pc2 = 0): (Gamma + 1) p + Pi = gamma2 p / (gamma2 - 1)
    is negative where p is.  Pressure averages all positive, left edge
    negative: after the per-variable checks (which keep everything here)
    every variable of both edges takes the cell value."""
    qp = quad(-3.3e3, 30.0e3, 60.0e3)
    avg_p, lo_p, hi_p, _, _ = qp
    assert min(avg_p) > 0 and lo_p < 0 < hi_p
    cols = {0: [0.0] * 5, 1: Q_A2R2[0], 2: Q_U[0], 2 + ndim: avg_p, 3 + ndim: [1.0] * 5}
    st = stencil(ndim, cols)
    lo, hi, replaced = F.cell_edges(cfg(ndim), st)
    assert replaced
    np.testing.assert_array_equal(lo, st[2])
    np.testing.assert_array_equal(hi, st[2])
    # the same stencil with the pressure dip removed keeps the reconstruction
    cols[2 + ndim] = Q_P[0]
    lo, hi, replaced = F.cell_edges(cfg(ndim), stencil(ndim, cols))
    assert not replaced
    assert_kept(lo, hi, 1, Q_A2R2)
    assert_kept(lo, hi, 2, Q_U)


def dip_with_interior(mid_target, G, B=0.0):
    """Convex quadratic whose interior Gauss-Lobatto value is mid_target."""
    A = mid_target - G / 20.0
    return quad(A, B, G)


@pytest.mark.parametrize("var,rho1,rho2", [(0, 10.0, 1.0), (1, 1000.0, 0.5)])
def test_roundoff_allowance_of_each_phase_scales_with_its_reference_density(var, rho1, rho2):
    """A partial density whose interior value is negative by less than
    ORC_ROUND_TOL x the phase's reference density (the initial rho_k of that
    phase, larger than every value in the stencil) is round-off and kept; by
    more than that, it falls back.  The pair 0.9 / 1.1 x the allowance also
    fixes the interior value's normalisation: (12 mean - lo - hi) / 12 would
    keep the 1.1 case."""
    ref = rho1 if var == 0 else rho2
    c = cfg(1, rho1=rho1, rho2=rho2)
    for factor, kept in ((0.9, True), (1.1, False)):
        q = dip_with_interior(-factor * TOL * ref, 0.06 * ref)
        avg = q[0]
        assert max(abs(a) for a in avg) < ref and q[3] < 0
        cols = base_cols(1)
        cols[var] = avg
        if var == 1:
            cols[0] = quad(900.0, 5.0, 1.0)[0]
        lo, hi, replaced = F.cell_edges(c, stencil(1, cols))
        if kept:
            assert not replaced, factor
            assert_kept(lo, hi, var, q, rel=1e-9)
        else:
            assert replaced and lo[var] == avg[2] and hi[var] == avg[2], factor


def test_roundoff_allowance_scales_with_the_stencil_when_it_exceeds_the_reference():
    """Where a stencil value exceeds the phase's reference density, the
    allowance is ORC_ROUND_TOL x the largest magnitude in the stencil."""
    c = cfg(1, rho1=1.0)
    for factor, kept in ((0.9, True), (1.1, False)):
        G = 50.0
        A = 0.0 - G / 20.0
        avg = [A + G * (k * k + 1.0 / 12.0) for k in range(-2, 3)]
        big = max(abs(a) for a in avg)
        q = dip_with_interior(-factor * TOL * big, G)
        avg = q[0]
        assert max(abs(a) for a in avg) > 1.0
        cols = base_cols(1)
        cols[0] = avg
        lo, hi, replaced = F.cell_edges(c, stencil(1, cols))
        assert replaced == (not kept), factor


@pytest.mark.parametrize("edge", ["hi_above", "lo_below"])
def test_a2_allowance_is_absolute(edge):
    """a2 edges beyond [0, 1] by less than ORC_ROUND_TOL are kept; by more,
    a2 falls back.  Linear a2 data: both edges exact."""
    for factor, kept in ((0.9, True), (1.1, False)):
        s = 0.1
        if edge == "hi_above":
            mean = 1.0 + factor * TOL - s / 2
        else:
            mean = -factor * TOL + s / 2
        avg = [mean + s * k for k in range(-2, 3)]
        cols = base_cols(1)
        cols[4] = avg
        lo, hi, replaced = F.cell_edges(cfg(1), stencil(1, cols))
        if kept:
            assert not replaced
            assert math.isclose(hi[4], mean + s / 2, rel_tol=1e-15, abs_tol=1e-16)
            assert math.isclose(lo[4], mean - s / 2, rel_tol=1e-15, abs_tol=1e-16)
        else:
            assert replaced and lo[4] == avg[2] and hi[4] == avg[2]
