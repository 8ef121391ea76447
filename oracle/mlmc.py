"""Oracle of the OF-MLMC estimator (Sec. 2.4 of arXiv:1705.04374), NumPy FP64.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

Terms are indexed l = 0..L.  Term 0 holds M_0 single samples q_0^i; term l >= 1
holds M_l coupled pairs (q_l^i, q_{l-1}^i) drawn with the same omega
(eq. (mlmc), eq. (ocv-mlmc)).  W_l is the cost of one sample of term l: a
single solve for l = 0, a pair of solves for l >= 1 (Sec. 2.4.1).

Readings where the paper leaves a choice:
  * variances and covariances are the unbiased 1/(M-1) two-pass estimates of
    each term's own fine and coarse members; the coefficient system uses them
    row by row (which is the exact minimiser of the estimated cost
    C(alpha) = sum_l W_l Var(alpha_l q_l - alpha_{l-1} q_{l-1}),
    eq. (cv-mlmc-var)); with a single variance per level it is the matrix of
    eq. (alpha-matvec) verbatim;
  * the tolerance is on eps (eps^2 <= tau^2), as in eq. (M-tol);
  * samples with a failed status are left out of the moments (Sec. 2.5, FT-MLMC).
"""
from __future__ import annotations

import math

import numpy as np


def term_moments(qf, qc=None, ok=None) -> dict:
    """Two-pass moments of one term (step 3 of the adaptive algorithm)."""
    qf = np.asarray(qf, dtype=np.float64)
    if ok is not None:
        keep = np.asarray(ok, dtype=bool)
        qf = qf[keep]
        if qc is not None:
            qc = np.asarray(qc, dtype=np.float64)[keep]
    M = qf.size
    mf = float(np.sum(qf) / M) if M else 0.0
    out = dict(M=M, mean_f=mf, mean_c=0.0, Vf=0.0, Vc=0.0, C=0.0)
    if qc is not None:
        qc = np.asarray(qc, dtype=np.float64)
        out["mean_c"] = float(np.sum(qc) / M) if M else 0.0
    if M >= 2:
        df = qf - mf
        out["Vf"] = float(np.sum(df * df) / (M - 1))
        if qc is not None:
            dc = qc - out["mean_c"]
            out["Vc"] = float(np.sum(dc * dc) / (M - 1))
            out["C"] = float(np.sum(df * dc) / (M - 1))
    return out


def merge_moments(a: dict, b: dict) -> dict:
    """Moments of one term over the union of two disjoint sample sets, from
    each set's (M, means, unbiased variances and covariance): the pairwise
    update of Chan, Golub and LeVeque, which adds to the two sets' centred
    sums of squares (or products) the term M_a M_b / M delta_x delta_y of the
    difference of their means.  This is what an all-reduce of per-GPU moments
    would apply to combine sample shards."""
    na, nb = a["M"], b["M"]
    n = na + nb
    if na == 0:
        return dict(b)
    if nb == 0:
        return dict(a)
    df = b["mean_f"] - a["mean_f"]
    dc = b["mean_c"] - a["mean_c"]
    w = na * nb / n
    sff = a["Vf"] * (na - 1) + b["Vf"] * (nb - 1) + df * df * w
    scc = a["Vc"] * (na - 1) + b["Vc"] * (nb - 1) + dc * dc * w
    sfc = a["C"] * (na - 1) + b["C"] * (nb - 1) + df * dc * w
    out = dict(M=n, mean_f=a["mean_f"] + df * nb / n, mean_c=a["mean_c"] + dc * nb / n, Vf=0.0, Vc=0.0, C=0.0)
    if n >= 2:
        out.update(Vf=sff / (n - 1), Vc=scc / (n - 1), C=sfc / (n - 1))
    return out


def coefficient_matrix(Vf, Vc, C, W):
    """Tridiagonal system of eq. (alpha-matvec) for alpha_0..alpha_{L-1}
    (alpha_L = 1).  Row k is d C(alpha) / d alpha_k = 0."""
    L = len(W) - 1
    A = np.zeros((L, L))
    b = np.zeros(L)
    for k in range(L):
        A[k, k] = Vf[k] * W[k] + Vc[k + 1] * W[k + 1]
        if k >= 1:
            A[k, k - 1] = -C[k] * W[k]
        if k + 1 <= L - 1:
            A[k, k + 1] = -C[k + 1] * W[k + 1]
    b[L - 1] = C[L] * W[L]
    return A, b


def coefficients(Vf, Vc, C, W) -> np.ndarray:
    """Optimal control-variate coefficients alpha_0..alpha_L (alpha_L = 1),
    step 4 of the adaptive algorithm."""
    L = len(W) - 1
    alpha = np.ones(L + 1)
    if L == 0:
        return alpha
    A, b = coefficient_matrix(Vf, Vc, C, W)
    alpha[:L] = np.linalg.solve(A, b)
    return alpha


def term_variances(Vf, Vc, C, alpha) -> np.ndarray:
    """sigma~^2_l = Var(alpha_l q_l - alpha_{l-1} q_{l-1}) (eq. (ocv-mlmc-err))."""
    L = len(alpha) - 1
    s = np.zeros(L + 1)
    s[0] = alpha[0] ** 2 * Vf[0]
    for l in range(1, L + 1):
        s[l] = alpha[l] ** 2 * Vf[l] + alpha[l - 1] ** 2 * Vc[l] - 2.0 * alpha[l] * alpha[l - 1] * C[l]
    return s


def error2(sig_t2, M) -> float:
    """Estimated squared sampling error eps^2_OF = sum_l sigma~^2_l / M_l."""
    return float(sum(s / m for s, m in zip(sig_t2, M)))


def estimate(mean_f, mean_c, alpha) -> float:
    """OF-MLMC estimator eq. (ocv-mlmc)."""
    L = len(alpha) - 1
    e = alpha[0] * mean_f[0]
    for l in range(1, L + 1):
        e += alpha[l] * mean_f[l] - alpha[l - 1] * mean_c[l]
    return float(e)


def warmup_samples(W, floor: int = 2):
    """Warm-up sample counts eq. (warmup), then at least `floor` per term."""
    L = len(W) - 1
    return [max(floor, int(math.ceil(W[L] / W[l] / 2.0 ** (L - l)))) for l in range(L + 1)]


class InfeasibleTolerance(ValueError):
    pass


def optimal_samples(sig_t2, W, M_have, mode: str, target: float):
    """Sample counts by eq. (M-tol) (mode 'tol', target tau) or eq. (M-budget)
    (mode 'budget', target B), keeping samples already computed: levels whose
    optimum falls below what they hold are fixed at it, their error (or cost)
    is taken off the target, and the rest is optimised again, until no level
    falls below (step 7 of the adaptive algorithm)."""
    L = len(W) - 1
    free = set(range(L + 1))
    Mhat = [int(m) for m in M_have]
    while True:
        fixed = [l for l in range(L + 1) if l not in free]
        if mode == "tol":
            t2 = target * target - sum(sig_t2[l] / M_have[l] for l in fixed)
            if t2 <= 0.0:
                raise InfeasibleTolerance("tolerance exhausted by kept levels")
        else:
            B = target - sum(M_have[l] * W[l] for l in fixed)
        S = sum(math.sqrt(sig_t2[l] * W[l]) for l in free)
        changed = False
        for l in sorted(free):
            if mode == "tol":
                m = math.ceil(math.sqrt(sig_t2[l] / W[l]) * S / t2)
            else:
                m = math.ceil(B * math.sqrt(sig_t2[l] / W[l]) / S) if (B > 0 and S > 0) else 0
            Mhat[l] = int(m)
        for l in sorted(free):
            if Mhat[l] < M_have[l]:
                Mhat[l] = int(M_have[l])
                free.discard(l)
                changed = True
        if not changed or not free:
            break
    for l in range(L + 1):
        if l not in free:
            Mhat[l] = int(M_have[l])
    return Mhat


def fit_indicators(M, Vdiff, first: int = 1):
    """Inferred variances of level differences (step 3 of the adaptive
    algorithm, optional part; App. A.1): a least-squares line through
    y_l = ln V[q_l - q_{l-1}] against l, over the terms l = first..L that have
    at least 2 samples and V > 0, with Gaussian errors of variance
    2 / (M_l - 1) (Var[ln s^2] of a sample variance of M Gaussian values),
    i.e. weights w_l = (M_l - 1) / 2.  Returns (v_hat, ok): v_hat[l] =
    exp(a + b l) for l = first..L (0 below first); ok is False (v_hat all 0)
    when fewer than two terms qualify."""
    L = len(M) - 1
    pts = [(l, math.log(Vdiff[l]), (M[l] - 1) / 2.0) for l in range(first, L + 1) if M[l] >= 2 and Vdiff[l] > 0]
    v_hat = np.zeros(L + 1)
    if len(pts) < 2:
        return v_hat, False
    S = sum(w for _, _, w in pts)
    Sx = sum(w * l for l, _, w in pts)
    Sy = sum(w * y for _, y, w in pts)
    Sxx = sum(w * l * l for l, _, w in pts)
    Sxy = sum(w * l * y for l, y, w in pts)
    b = (S * Sxy - Sx * Sy) / (S * Sxx - Sx * Sx)
    a = (Sy - b * Sx) / S
    for l in range(first, L + 1):
        v_hat[l] = math.exp(a + b * l)
    return v_hat, True


def infer_missing_terms(mom: list, v_hat, first: int = 1):
    """Moments of the terms l >= max(first, 1) that have fewer than two
    samples (the single finest warm-up sample of App. A.1), from the fit.
    The coarse member is level l-1, whose variance term l-1 measured
    (Vc = its Vf); the correlation of the members is taken from term l-1
    (rho = C / sqrt(Vf Vc) there, 0 if undefined); the fine member's
    standard deviation s then solves s^2 + Vc - 2 rho s sqrt(Vc) = v_hat
    (V[a - b] = Va + Vb - 2 Cov), the larger root s >= 0, so that the
    completed moments are a valid covariance whose difference variance is
    v_hat.  Where v_hat is below the smallest difference variance that
    correlation allows, s takes its minimiser max(rho sqrt(Vc), 0): the
    completed difference variance is then (1 - rho^2) Vc for rho >= 0 and Vc
    (s = 0, no covariance) for rho < 0.
    mom: list of term_moments dicts, updated in place."""
    for l in range(max(first, 1), len(mom)):
        if mom[l]["M"] >= 2:
            continue
        a, b, c = mom[l - 1]["Vf"], mom[l - 1]["Vc"], mom[l - 1]["C"]
        rho = c / math.sqrt(a * b) if a > 0 and b > 0 else 0.0
        rho = min(max(rho, -1.0), 1.0)
        vc = a
        sc = math.sqrt(vc)
        s = max(rho * sc + math.sqrt(max(v_hat[l] - (1.0 - rho * rho) * vc, 0.0)), 0.0)
        mom[l]["Vc"] = vc
        mom[l]["Vf"] = s * s
        mom[l]["C"] = rho * s * sc
    return mom


def refine_few_sample_terms(mom: list, v_hat, first: int = 1, m_floor: int = 2):
    """Terms l >= max(first, 1) with at least two but fewer than m_floor
    samples keep the fit's inferred difference variance as a floor: their own
    estimate from so few samples refines the inferred value (App. A.1: further
    samples give a more accurate inference), it does not replace it.  The
    difference variance becomes max(measured, v_hat[l]) by lowering the
    covariance C of the two members (their variances Vf, Vc stay the measured
    ones), C' = (Vf + Vc - V') / 2, at least -sqrt(Vf Vc) (a valid
    covariance: V' at most (sqrt(Vf) + sqrt(Vc))^2).  mom: list of
    term_moments dicts, updated in place."""
    for l in range(max(first, 1), len(mom)):
        m = mom[l]
        if not (2 <= m["M"] < m_floor):
            continue
        v = m["Vf"] + m["Vc"] - 2.0 * m["C"]
        if not (v_hat[l] > v):
            continue
        c = 0.5 * (m["Vf"] + m["Vc"] - v_hat[l])
        m["C"] = max(c, -math.sqrt(m["Vf"] * m["Vc"]))
    return mom


def mc_samples(var_L: float, eps: float) -> int:
    """Plain Monte Carlo sample count for error eps at the finest level,
    eq. (speedup) with the square of the ratio (the error of a mean of M
    samples is sigma / sqrt(M))."""
    return int(math.ceil(var_L / (eps * eps)))
