"""Pins of the OF-MLMC estimator oracle (Sec. 2.4 of arXiv:1705.04374).

Closed-form toy: omega = (Y, Z) ~ N(0,1)^2, q_l = mu + s Y + b 2^-l Z, so
Var q_l = s^2 + b^2 4^-l and Cov(q_l, q_{l-1}) = s^2 + 2 b^2 4^-l.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle.mlmc as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def toy_moments(L, s=1.0, b=0.7):
    Vf = [s * s + b * b * 4.0 ** -l for l in range(L + 1)]
    Vc = [0.0] + [s * s + b * b * 4.0 ** -(l - 1) for l in range(1, L + 1)]
    C = [0.0] + [s * s + 2 * b * b * 4.0 ** -l for l in range(1, L + 1)]
    return Vf, Vc, C


def cost(alpha, Vf, Vc, C, W):
    """C(alpha) of eq. (cv-mlmc-var), written out term by term."""
    tot = alpha[0] ** 2 * Vf[0] * W[0]
    for l in range(1, len(W)):
        tot += (alpha[l] ** 2 * Vf[l] + alpha[l - 1] ** 2 * Vc[l]
                - 2 * alpha[l] * alpha[l - 1] * C[l]) * W[l]
    return tot


def test_two_level_closed_form():
    """L = 1 reduces to eq. (alpha-opt-works); W_0 = 0 gives Cov/Var
    (eq. (alpha-opt))."""
    Vf, Vc, C = toy_moments(1)
    W = [1.0, 9.0]
    a = O.coefficients(Vf, Vc, C, W)
    assert math.isclose(a[0], W[1] / (W[0] + W[1]) * C[1] / Vf[0], rel_tol=1e-14)
    assert a[1] == 1.0
    a0 = O.coefficients(Vf, Vc, C, [0.0, 9.0])
    assert math.isclose(a0[0], C[1] / Vc[1], rel_tol=1e-14)


@pytest.mark.parametrize("L", [2, 3, 5])
def test_coefficients_minimise_cost(L):
    rng = np.random.default_rng(L)
    # per-term sample estimates (they differ between terms, as in practice)
    Vf, Vc, C = [], [], []
    for l in range(L + 1):
        Y, Z = rng.normal(size=(2, 30))
        qf = Y + 0.7 * 2.0 ** -l * Z
        m = O.term_moments(qf, Y + 0.7 * 2.0 ** -(l - 1) * Z if l else None)
        Vf.append(m["Vf"]); Vc.append(m["Vc"]); C.append(m["C"])
    W = [16.0 ** l for l in range(L + 1)]
    a = O.coefficients(Vf, Vc, C, W)
    c0 = cost(a, Vf, Vc, C, W)
    for k in range(L):
        for d in (1e-4, -1e-4):
            ap = a.copy()
            ap[k] += d
            assert cost(ap, Vf, Vc, C, W) > c0
        # stationarity by central differences
        e = 1e-6
        ap, am = a.copy(), a.copy()
        ap[k] += e
        am[k] -= e
        g = (cost(ap, Vf, Vc, C, W) - cost(am, Vf, Vc, C, W)) / (2 * e)
        assert abs(g) < 1e-6 * c0


def test_matrix_is_paper_matrix_with_single_variances():
    """With one variance per level the system is eq. (alpha-matvec)."""
    L = 3
    sig2 = [2.0, 1.5, 1.2, 1.1]
    cov = [None, 1.4, 1.1, 1.0]
    W = [1.0, 16.0, 256.0, 4096.0]
    Vf = sig2
    Vc = [0.0] + sig2[:-1]
    A, b = O.coefficient_matrix(Vf, Vc, cov, W)
    for k in range(L):
        assert A[k, k] == sig2[k] * (W[k + 1] + W[k])
        if k + 1 < L:
            assert A[k, k + 1] == -cov[k + 1] * W[k + 1] == A[k + 1, k]
    assert b[L - 1] == cov[L] * W[L] and np.all(b[:L - 1] == 0)


def test_variance_reduction_identities():
    """eq. (cv-var-opt): at alpha = Cov/Var, Var q* = (1 - Cor^2) Var q_l;
    eq. (cv-var-0.5): with alpha = 1 and equal variances, Cor < 1/2 increases
    the variance."""
    V, Cv = 2.0, 1.2
    a = O.coefficients([V, V], [0, V], [0, Cv], [0.0, 1.0])
    st = O.term_variances([V, V], [0, V], [0, Cv], [a[0], 1.0])
    cor = Cv / V
    assert math.isclose(st[1], (1 - cor * cor) * V, rel_tol=1e-14)
    st1 = O.term_variances([V, V], [0, V], [0, 0.4 * V], [1.0, 1.0])
    assert st1[1] > V


def test_moments_exact_rational():
    rng = np.random.default_rng(3)
    qf = rng.normal(5, 2, 37)
    qc = qf + rng.normal(0, 0.3, 37)
    m = O.term_moments(qf, qc)
    F = [Fraction(float(x)) for x in qf]
    G = [Fraction(float(x)) for x in qc]
    M = len(F)
    mf, mc = sum(F) / M, sum(G) / M
    Vf = sum((x - mf) ** 2 for x in F) / (M - 1)
    Vc = sum((x - mc) ** 2 for x in G) / (M - 1)
    Cc = sum((x - mf) * (y - mc) for x, y in zip(F, G)) / (M - 1)
    for key, ex in (("mean_f", mf), ("mean_c", mc), ("Vf", Vf), ("Vc", Vc), ("C", Cc)):
        assert abs(m[key] - float(ex)) <= 1e-14 * abs(float(ex))


def test_failed_samples_are_excluded():
    qf = np.array([1.0, 2.0, np.nan, 4.0])
    qc = np.array([0.5, 1.5, 7.0, 3.0])
    ok = np.array([1, 1, 0, 1], bool)
    m = O.term_moments(qf, qc, ok)
    ref = O.term_moments(qf[ok], qc[ok])
    assert m == ref and m["M"] == 3


def test_sigma_tilde_is_sample_variance_of_weighted_difference():
    rng = np.random.default_rng(4)
    qf = rng.normal(0, 1, 200)
    qc = 0.8 * qf + rng.normal(0, 0.5, 200)
    m = O.term_moments(qf, qc)
    a = [0.83, 1.0]
    st = O.term_variances([0.0, m["Vf"]], [0.0, m["Vc"]], [0.0, m["C"]], a)
    direct = np.var(a[1] * qf - a[0] * qc, ddof=1)
    assert math.isclose(st[1], direct, rel_tol=1e-12)


def test_estimator_unbiased_on_toy():
    """E[q_L] = mu for every L; the OF-MLMC mean over many repetitions is
    within a CLT band of mu, and the error estimate matches the spread."""
    mu, L = 3.0, 2
    W = [1.0, 8.0, 64.0]
    rng = np.random.default_rng(5)
    Ms = [400, 60, 10]
    ests, errs = [], []
    for rep in range(200):
        means_f, means_c, Vf, Vc, Cs = [], [], [], [], []
        for l in range(L + 1):
            Y = rng.normal(size=Ms[l])
            Z = rng.normal(size=Ms[l])
            qf = mu + Y + 0.7 * 2.0 ** -l * Z
            qc = mu + Y + 0.7 * 2.0 ** -(l - 1) * Z if l else None
            m = O.term_moments(qf, qc)
            means_f.append(m["mean_f"]); means_c.append(m["mean_c"])
            Vf.append(m["Vf"]); Vc.append(m["Vc"]); Cs.append(m["C"])
        a = O.coefficients(Vf, Vc, Cs, W)
        ests.append(O.estimate(means_f, means_c, a))
        errs.append(O.error2(O.term_variances(Vf, Vc, Cs, a), Ms))
    ests = np.array(ests)
    rmse_est = math.sqrt(np.mean(errs))
    assert abs(ests.mean() - mu) < 4 * rmse_est / math.sqrt(len(ests))
    assert 0.7 < ests.std() / rmse_est < 1.3


def test_classical_mlmc_is_alpha_one():
    means_f = [1.0, 1.3, 1.35]
    means_c = [0.0, 1.1, 1.32]
    e = O.estimate(means_f, means_c, [1.0, 1.0, 1.0])
    assert math.isclose(e, 1.0 + (1.3 - 1.1) + (1.35 - 1.32), rel_tol=1e-15)


def test_warmup_counts_from_paper():
    g = GOLD["warmup_3d"]
    W = [g["W_ratio"] ** l for l in range(g["L"] + 1)]
    assert O.warmup_samples(W, floor=1) == g["M"]
    # the warm-up iteration costs less than 2 W_L
    assert sum(m * w for m, w in zip(g["M"], W)) < 2 * W[-1]
    assert O.warmup_samples(W) == [512, 64, 8, 2]


def test_table_budget_is_about_eight_finest_solves():
    """Pair costs (W_l = single(l) + single(l-1), Sec. 2.4.1) with single
    solve cost 16^l reproduce the paper's '8 times one finest solve'."""
    g = GOLD["ofmlmc_table"]
    single = [g["W_ratio"] ** l for l in range(4)]
    W = [single[0]] + [single[l] + single[l - 1] for l in range(1, 4)]
    total = sum(m * w for m, w in zip(g["M"], W)) / single[3]
    assert abs(total - g["total_over_finest_approx"]) < 0.1


def test_optimal_samples_tolerance_and_budget():
    sig = [4.0, 0.5, 0.06, 0.01]
    W = [1.0, 17.0, 272.0, 4352.0]
    tau = 0.01
    M = O.optimal_samples(sig, W, [2, 2, 2, 2], "tol", tau)
    assert O.error2(sig, M) <= tau * tau
    # before the ceiling the constraint is met with equality
    S = sum(math.sqrt(s * w) for s, w in zip(sig, W))
    Mr = [math.sqrt(s / w) * S / tau ** 2 for s, w in zip(sig, W)]
    assert math.isclose(O.error2(sig, Mr), tau * tau, rel_tol=1e-12)
    B = 1.0e6
    Mb = O.optimal_samples(sig, W, [0, 0, 0, 0], "budget", B)
    assert sum(m * w for m, w in zip(Mb, W)) <= B + sum(W)
    assert sum(m * w for m, w in zip(Mb, W)) >= B - 1e-9


def test_optimal_samples_keeps_computed_levels():
    sig = [4.0, 0.5, 0.06, 0.01]
    W = [1.0, 17.0, 272.0, 4352.0]
    have = [10, 5, 5000, 2]         # level 2 already over-sampled (optimum ~2300)
    M = O.optimal_samples(sig, W, have, "tol", 0.01)
    assert all(m >= h for m, h in zip(M, have))
    assert M[2] == 5000
    assert O.error2(sig, M) <= 0.01 ** 2
    # levels that keep more than their optimum leave a smaller share to the rest
    free = O.optimal_samples(sig, W, [2, 2, 2, 2], "tol", 0.01)
    assert M[0] <= free[0] and M[1] <= free[1] and M[3] <= free[3]


def test_mc_sample_count():
    assert O.mc_samples(4.0, 0.1) == 400


# --------------------------------------------------------------------------
# indicator fit (App. A.1)
# --------------------------------------------------------------------------

def test_fit_recovers_an_exact_exponential_decay():
    """Data exactly on V_l = c r^l: the fitted line goes through every point
    whatever the weights, and extrapolates to the unmeasured finest term."""
    c, r = 3.7e15, 0.31
    M = [0, 40, 9, 3, 1]
    V = [0.0] + [c * r ** l for l in range(1, 5)]
    V[4] = 0.0                                   # a single sample: no variance
    v_hat, ok = O.fit_indicators(M, V, first=1)
    assert ok
    for l in range(1, 5):
        assert math.isclose(v_hat[l], c * r ** l, rel_tol=1e-12)


def test_fit_two_points_is_the_line_through_them_and_minimises_weighted_residual():
    M = [0, 11, 5, 1]
    V = [0.0, 2.0e15, 5.0e14, 0.0]
    v_hat, ok = O.fit_indicators(M, V)
    assert ok and math.isclose(v_hat[1], 2.0e15, rel_tol=1e-13) and math.isclose(v_hat[2], 5.0e14, rel_tol=1e-13)
    assert math.isclose(v_hat[3], 1.25e14, rel_tol=1e-12)      # halving in the log per level
    # three noisy points: the fitted (a, b) zero the gradient of the weighted
    # squared residual sum_l w_l (ln V_l - a - b l)^2
    M = [0, 30, 12, 6]
    V = [0.0, 2.0e15, 7.0e14, 1.0e14]
    v_hat, ok = O.fit_indicators(M, V)
    b = math.log(v_hat[2] / v_hat[1])
    a = math.log(v_hat[1]) - b
    g_a = g_b = 0.0
    for l in (1, 2, 3):
        w = (M[l] - 1) / 2.0
        res = math.log(V[l]) - a - b * l
        g_a += w * res
        g_b += w * res * l
    assert abs(g_a) < 1e-9 and abs(g_b) < 1e-9
    # too few points
    _, ok = O.fit_indicators([0, 5, 1], [0.0, 1e14, 0.0])
    assert not ok


def test_inferred_finest_term_moments():
    """A single finest sample: the coarse member takes the measured variance
    of its level, the members' correlation is that of the term below, and
    the difference variance is the inferred one; the result is a valid
    covariance even when the inferred difference exceeds what equal member
    variances allow (variances growing with the level)."""
    for v in (8.0e14, 6.0e16):                         # small, and > 4 x 5e15
        mom = [dict(M=100, Vf=4.0e15, Vc=0.0, C=0.0), dict(M=20, Vf=5.0e15, Vc=4.1e15, C=4.3e15),
               dict(M=1, Vf=0.0, Vc=0.0, C=0.0)]
        v_hat = np.array([0.0, 5.0e14, v])
        O.infer_missing_terms(mom, v_hat, first=1)
        m = mom[2]
        assert m["Vc"] == 5.0e15
        assert math.isclose(m["Vf"] + m["Vc"] - 2 * m["C"], v, rel_tol=1e-12)
        rho_below = 4.3e15 / math.sqrt(5.0e15 * 4.1e15)
        assert math.isclose(m["C"] / math.sqrt(m["Vf"] * m["Vc"]), rho_below, rel_tol=1e-12)
        assert m["C"] ** 2 <= m["Vf"] * m["Vc"] * (1 + 1e-12)
        assert mom[1]["C"] == 4.3e15                   # measured terms untouched
    # below the smallest difference variance the correlation allows: the
    # fine member takes s = rho sqrt(Vc), the closest consistent value
    mom = [dict(M=100, Vf=4.0e15, Vc=0.0, C=0.0), dict(M=20, Vf=1.0, Vc=1.0, C=0.6),
           dict(M=1, Vf=0.0, Vc=0.0, C=0.0)]
    O.infer_missing_terms(mom, np.array([0.0, 0.8, 0.1]), first=1)
    m = mom[2]
    assert math.isclose(m["Vf"], 0.36, rel_tol=1e-12) and math.isclose(m["C"], 0.36, rel_tol=1e-12)
    assert math.isclose(m["Vf"] + m["Vc"] - 2 * m["C"], 1 - 0.36, rel_tol=1e-12)


def test_inferred_term_with_negative_correlation_below():
    """Completion when the term below has a negative correlation (rho < 0):
    the difference variance s^2 + Vc - 2 rho s sqrt(Vc) grows with s >= 0, so
    the smallest value it can take is Vc (s = 0), not (1 - rho^2) Vc.  Checked
    by brute force over a grid of s: the completed difference variance is
    max(v_hat, min_s D(s)), and the completed moments are a covariance with
    correlation rho wherever s > 0."""
    rho = -0.6
    for v in (0.1, 0.9, 3.0, 40.0):
        mom = [dict(M=100, Vf=4.0, Vc=0.0, C=0.0), dict(M=20, Vf=1.0, Vc=1.0, C=rho),
               dict(M=1, Vf=0.0, Vc=0.0, C=0.0)]
        O.infer_missing_terms(mom, np.array([0.0, 0.8, v]), first=1)
        m = mom[2]
        assert m["Vc"] == 1.0
        s_grid = np.linspace(0.0, 10.0, 200001)
        D = s_grid ** 2 + 1.0 - 2.0 * rho * s_grid
        diff = m["Vf"] + m["Vc"] - 2 * m["C"]
        assert math.isclose(diff, max(v, D.min()), rel_tol=1e-9), (v, diff)
        assert m["Vf"] >= 0 and m["C"] ** 2 <= m["Vf"] * m["Vc"] * (1 + 1e-12)
        if m["Vf"] > 0:
            assert math.isclose(m["C"] / math.sqrt(m["Vf"] * m["Vc"]), rho, rel_tol=1e-12)
        else:
            assert m["C"] == 0.0 and v < 1.0


def test_merged_shard_moments_equal_the_moments_of_the_union():
    """The pairwise update gives the two-pass moments of the concatenated
    samples (to round-off), whatever the split, including empty and
    single-sample shards; merging is commutative and associative."""
    rng = np.random.default_rng(31)
    qf = 5.0 + rng.normal(size=1000) * 3.0
    qc = qf * 0.8 + rng.normal(size=1000)
    whole = O.term_moments(qf, qc)
    for cuts in ([0, 1000], [1, 999], [0, 0, 1000], [137, 400, 463], [500, 1, 499]):
        edges = np.cumsum([0] + cuts)
        parts = [O.term_moments(qf[a:b], qc[a:b]) for a, b in zip(edges[:-1], edges[1:])]
        m = parts[0]
        for p in parts[1:]:
            m = O.merge_moments(m, p)
        assert m["M"] == whole["M"]
        for k in ("mean_f", "mean_c", "Vf", "Vc", "C"):
            assert abs(m[k] - whole[k]) <= 1e-13 * abs(whole[k]), (cuts, k)
    a, b, c = (O.term_moments(qf[i:j], qc[i:j]) for i, j in ((0, 300), (300, 310), (310, 1000)))
    ab_c = O.merge_moments(O.merge_moments(a, b), c)
    a_bc = O.merge_moments(a, O.merge_moments(b, c))
    ba = O.merge_moments(b, a)
    ab = O.merge_moments(a, b)
    for k in ("mean_f", "Vf", "C"):
        assert abs(ab_c[k] - a_bc[k]) <= 1e-13 * abs(whole[k])
        assert abs(ab[k] - ba[k]) <= 1e-13 * abs(whole[k])
    # two single samples: the variance of two values
    one = O.merge_moments(O.term_moments([1.0], [2.0]), O.term_moments([4.0], [0.0]))
    assert one["M"] == 2 and one["Vf"] == 4.5 and one["Vc"] == 2.0 and one["C"] == -3.0


def test_few_sample_terms_keep_the_inferred_variance_as_a_floor():
    """A term with 2 <= M < floor samples: its difference variance becomes
    max(measured, inferred) by lowering the members' covariance; a larger
    measured value, a term at the floor, or one below the fit's first term is
    left as measured; the covariance stays valid (|C| <= sqrt(Vf Vc))."""
    def terms():
        return [dict(M=100, Vf=4.0, Vc=0.0, C=0.0), dict(M=20, Vf=1.0, Vc=1.2, C=0.9),
                dict(M=3, Vf=2.0, Vc=1.0, C=1.3)]
    # measured V = 2 + 1 - 2.6 = 0.4 < 0.9 inferred: raised to 0.9
    mom = O.refine_few_sample_terms(terms(), [0.0, 0.5, 0.9], first=1, m_floor=8)
    m = mom[2]
    assert math.isclose(m["Vf"] + m["Vc"] - 2 * m["C"], 0.9, rel_tol=1e-15)
    assert (m["Vf"], m["Vc"]) == (2.0, 1.0) and m["C"] ** 2 <= m["Vf"] * m["Vc"]
    assert mom[1] == terms()[1]                              # 20 >= floor 8: untouched
    # an inferred value beyond what a covariance allows: the largest valid one
    mom = O.refine_few_sample_terms(terms(), [0.0, 0.5, 50.0], first=1, m_floor=8)
    assert math.isclose(mom[2]["C"], -math.sqrt(2.0), rel_tol=1e-15)
    assert math.isclose(mom[2]["Vf"] + mom[2]["Vc"] - 2 * mom[2]["C"], (math.sqrt(2.0) + 1.0) ** 2, rel_tol=1e-15)
    # measured above the inferred value, at the floor, or below `first`: unchanged
    assert O.refine_few_sample_terms(terms(), [0.0, 0.5, 0.1], 1, 8) == terms()
    assert O.refine_few_sample_terms(terms(), [0.0, 0.5, 0.9], 1, 3) == terms()
    assert O.refine_few_sample_terms(terms(), [0.0, 0.5, 0.9], 3, 8) == terms()
    # the brute-force minimiser of the error term agrees with the closed form
    # of V' (the difference variance is linear in C)
    for Vt in (0.9, 1.7):
        mom = O.refine_few_sample_terms(terms(), [0.0, 0.5, Vt], 1, 8)
        Cs = np.linspace(-math.sqrt(2.0), math.sqrt(2.0), 100001)
        best = Cs[np.argmin(np.abs(3.0 - 2 * Cs - Vt))]
        assert abs(mom[2]["C"] - best) <= 3e-5
