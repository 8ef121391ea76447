// OF-MLMC estimator kernels (Sukys et al., arXiv:1705.04374, Sec. 2.4.3-2.4.4),
// all in double on the device.  The statistics are tiny next to the solves
// (Appendix A.3 notes the coefficient system is never a bottleneck), so each
// call is one workgroup; what matters is that the sums are deterministic
// (fixed-order strided partial sums, then a fixed tree) and stay on the GPU.
#include "flow_kernels.h"

#include <math.h>

namespace ofm {

constexpr int MT = 256;

// Fixed-order workgroup sum of one double per thread.
__device__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = MT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Moments of one term: (M_used, mean_f, mean_c, Var_f, Var_c, Cov), two-pass.
__global__ void __launch_bounds__(MT) moments_kernel(const double* qf, const double* qc, const int32_t* ok,
                                                     int64_t M, double* out)
{
    __shared__ double sh[MT];
    double cnt = 0.0, sf = 0.0, sc = 0.0;
    for (int64_t i = threadIdx.x; i < M; i += MT) {
        if (ok && ok[i] == 0) continue;
        cnt += 1.0;
        sf += qf[i];
        if (qc) sc += qc[i];
    }
    const double m = block_sum(cnt, sh);
    const double mf = m > 0.0 ? block_sum(sf, sh) / m : 0.0;
    const double mc = (m > 0.0 && qc) ? block_sum(sc, sh) / m : 0.0;
    double vf = 0.0, vc = 0.0, cv = 0.0;
    for (int64_t i = threadIdx.x; i < M; i += MT) {
        if (ok && ok[i] == 0) continue;
        const double df = qf[i] - mf;
        vf += df * df;
        if (qc) {
            const double dc = qc[i] - mc;
            vc += dc * dc;
            cv += df * dc;
        }
    }
    vf = block_sum(vf, sh);
    vc = block_sum(vc, sh);
    cv = block_sum(cv, sh);
    if (threadIdx.x == 0) {
        out[0] = m;
        out[1] = mf;
        out[2] = mc;
        const bool two = m >= 2.0;
        out[3] = two ? vf / (m - 1.0) : 0.0;
        out[4] = two && qc ? vc / (m - 1.0) : 0.0;
        out[5] = two && qc ? cv / (m - 1.0) : 0.0;
    }
}

// Tridiagonal system of eq. (alpha-matvec), generalised to per-term
// estimates: row k is the derivative of the estimated cost
// sum_l W_l Var(alpha_l q_f,l - alpha_{l-1} q_c,l) with respect to alpha_k.
// Thomas algorithm; a non-positive pivot means the estimates are not
// positive definite -> flag OFM_ESINGULAR and alpha = 1 (classical MLMC).
__global__ void coefficients_kernel(int L, const double* mom, const double* W, double* alpha, int32_t* flag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double cp[32], dp[32];
    int bad = 0;
    for (int k = 0; k < L; ++k) {
        const double diag = mom[6 * k + 3] * W[k] + mom[6 * (k + 1) + 4] * W[k + 1];
        const double low = k >= 1 ? -mom[6 * k + 5] * W[k] : 0.0;
        const double up = k + 1 <= L - 1 ? -mom[6 * (k + 1) + 5] * W[k + 1] : 0.0;
        const double rhs = k == L - 1 ? mom[6 * L + 5] * W[L] : 0.0;
        const double piv = diag - (k >= 1 ? low * cp[k - 1] : 0.0);
        if (!(piv > 0.0) || fabs(piv) < 1e-300) { bad = 1; break; }
        cp[k] = up / piv;
        dp[k] = (rhs - (k >= 1 ? low * dp[k - 1] : 0.0)) / piv;
    }
    alpha[L] = 1.0;
    if (bad) {
        for (int k = 0; k < L; ++k) alpha[k] = 1.0;
        *flag = OFM_ESINGULAR;
        return;
    }
    for (int k = L - 1; k >= 0; --k) alpha[k] = dp[k] - (k + 1 <= L - 1 ? cp[k] * alpha[k + 1] : 0.0);
    *flag = 0;
}

// eq. (ocv-mlmc-err): per-term variances of the weighted differences and
// the squared sampling error.
__global__ void errors_kernel(int L, const double* mom, const double* alpha, double* sig, double* eps2)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0;
    for (int l = 0; l <= L; ++l) {
        const double* m = mom + 6 * l;
        double s = alpha[l] * alpha[l] * m[3];
        if (l >= 1) s += alpha[l - 1] * alpha[l - 1] * m[4] - 2.0 * alpha[l] * alpha[l - 1] * m[5];
        sig[l] = s;
        e += s / m[0];
    }
    *eps2 = e;
}

// eq. (ocv-mlmc): the estimator.
__global__ void estimate_kernel(int L, const double* mom, const double* alpha, double* E)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = alpha[0] * mom[1];
    for (int l = 1; l <= L; ++l) e += alpha[l] * mom[6 * l + 1] - alpha[l - 1] * mom[6 * l + 2];
    *E = e;
}

// eq. (M-tol) / eq. (M-budget) with the keep-computed-samples loop of step 7.
__global__ void optimal_M_kernel(int L, const double* sig, const double* W, const int64_t* have, int mode,
                                 double target, int64_t* out, int32_t* flag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    bool fixed[32];
    int64_t M[32];
    for (int l = 0; l <= L; ++l) { fixed[l] = false; M[l] = have[l]; }
    *flag = 0;
    for (int it = 0; it <= L + 1; ++it) {
        double rest = mode == OFM_MODE_TOLERANCE ? target * target : target;
        double S = 0.0;
        for (int l = 0; l <= L; ++l) {
            if (fixed[l]) rest -= mode == OFM_MODE_TOLERANCE ? sig[l] / (double)have[l] : (double)have[l] * W[l];
            else S += sqrt(sig[l] * W[l]);
        }
        if (mode == OFM_MODE_TOLERANCE && !(rest > 0.0)) {
            *flag = OFM_EINFEASIBLE;
            for (int l = 0; l <= L; ++l) out[l] = have[l];
            return;
        }
        for (int l = 0; l <= L; ++l) {
            if (fixed[l]) continue;
            double m;
            if (mode == OFM_MODE_TOLERANCE) m = ceil(sqrt(sig[l] / W[l]) * S / rest);
            else m = (rest > 0.0 && S > 0.0) ? ceil(rest * sqrt(sig[l] / W[l]) / S) : 0.0;
            M[l] = (int64_t)m;
        }
        bool changed = false;
        for (int l = 0; l <= L; ++l) {
            if (!fixed[l] && M[l] < have[l]) { M[l] = have[l]; fixed[l] = true; changed = true; }
        }
        bool any_free = false;
        for (int l = 0; l <= L; ++l) any_free = any_free || !fixed[l];
        if (!changed || !any_free) break;
    }
    for (int l = 0; l <= L; ++l) out[l] = fixed[l] ? have[l] : M[l];
}

// Inferred variances of level differences (the optional part of step 3 of
// the adaptive algorithm, Sec. 2.4.4; App. A.1): a weighted least-squares
// line through ln V[q_l - q_{l-1}] against l over the terms l = first..L
// with at least two samples, weights (M_l - 1)/2 (Gaussian errors of a
// sample variance's logarithm).  Terms l >= max(first, 1) with fewer than
// two samples get their moments from the fit: the coarse member takes the
// variance of level l-1 (term l-1's fine variance Vc), the members'
// correlation rho is that of term l-1, and the fine member's deviation s
// gives the inferred difference variance s^2 + Vc - 2 rho s sqrt(Vc).  Terms
// with at least two but fewer than m_floor samples keep the inferred value as
// a floor of their difference variance (their few samples refine it, App.
// A.1): the covariance is lowered to (Vf + Vc - vhat) / 2, at least
// -sqrt(Vf Vc).  One thread: L is a handful of terms.
__global__ void fit_kernel(int L, int first, int m_floor, double* mom, double* vhat, int32_t* flag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double S = 0.0, Sx = 0.0, Sy = 0.0, Sxx = 0.0, Sxy = 0.0;
    int np = 0;
    for (int l = first; l <= L; ++l) {
        const double* m = mom + 6 * l;
        const double V = m[3] + m[4] - 2.0 * m[5];
        if (m[0] >= 2.0 && V > 0.0) {
            const double y = log(V), w = (m[0] - 1.0) / 2.0, x = (double)l;
            S += w;
            Sx += w * x;
            Sy += w * y;
            Sxx += w * x * x;
            Sxy += w * x * y;
            ++np;
        }
    }
    for (int l = 0; l <= L; ++l) vhat[l] = 0.0;
    if (np < 2) {
        *flag = OFM_ESINGULAR;
        return;
    }
    const double b = (S * Sxy - Sx * Sy) / (S * Sxx - Sx * Sx);
    const double a = (Sy - b * Sx) / S;
    for (int l = first; l <= L; ++l) vhat[l] = exp(a + b * (double)l);
    // terms with fewer than two samples: coarse member = level l-1 (term
    // l-1's fine variance), the members' correlation that of term l-1, and
    // the fine member's deviation s >= 0 from s^2 + Vc - 2 rho s sqrt(Vc) =
    // vhat (larger root).  Where vhat is below the smallest difference
    // variance that correlation allows, s takes the minimiser max(rho
    // sqrt(Vc), 0): (1 - rho^2) Vc for rho >= 0, Vc (s = 0) for rho < 0.
    for (int l = first > 1 ? first : 1; l <= L; ++l) {
        double* m = mom + 6 * l;
        if (m[0] >= 2.0) continue;
        const double* b = mom + 6 * (l - 1);
        double rho = (b[3] > 0.0 && b[4] > 0.0) ? b[5] / sqrt(b[3] * b[4]) : 0.0;
        rho = fmin(fmax(rho, -1.0), 1.0);
        const double vc = b[3], sc = sqrt(vc);
        const double s = fmax(rho * sc + sqrt(fmax(vhat[l] - (1.0 - rho * rho) * vc, 0.0)), 0.0);
        m[4] = vc;
        m[3] = s * s;
        m[5] = rho * s * sc;
    }
    // terms with 2 <= M < m_floor: the inferred value as a floor
    for (int l = first > 1 ? first : 1; l <= L; ++l) {
        double* m = mom + 6 * l;
        if (!(m[0] >= 2.0 && m[0] < (double)m_floor)) continue;
        const double v = m[3] + m[4] - 2.0 * m[5];
        if (!(vhat[l] > v)) continue;
        m[5] = fmax(0.5 * (m[3] + m[4] - vhat[l]), -sqrt(m[3] * m[4]));
    }
    *flag = 0;
}

// Moments of each term over the union of two disjoint sample sets
// (pairwise update: the centred sums add, plus Ma Mb / M times the product of
// the differences of the means); one thread per term.  out may be a or b.
__global__ void merge_kernel(int n_terms, const double* a, const double* b, double* out)
{
    const int t = threadIdx.x;
    if (t >= n_terms) return;
    const double* x = a + 6 * t;
    const double* y = b + 6 * t;
    const double na = x[0], nb = y[0];
    double r[6];
    if (na == 0.0 || nb == 0.0) {
        for (int k = 0; k < 6; ++k) r[k] = na == 0.0 ? y[k] : x[k];
    } else {
        const double n = na + nb;
        const double df = y[1] - x[1], dc = y[2] - x[2];
        const double w = na * nb / n;
        const double sff = x[3] * (na - 1.0) + y[3] * (nb - 1.0) + df * df * w;
        const double scc = x[4] * (na - 1.0) + y[4] * (nb - 1.0) + dc * dc * w;
        const double sfc = x[5] * (na - 1.0) + y[5] * (nb - 1.0) + df * dc * w;
        r[0] = n;
        r[1] = x[1] + df * nb / n;
        r[2] = x[2] + dc * nb / n;
        r[3] = n >= 2.0 ? sff / (n - 1.0) : 0.0;
        r[4] = n >= 2.0 ? scc / (n - 1.0) : 0.0;
        r[5] = n >= 2.0 ? sfc / (n - 1.0) : 0.0;
    }
    for (int k = 0; k < 6; ++k) out[6 * t + k] = r[k];
}

hipError_t launch_merge(int n_terms, const double* a, const double* b, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(merge_kernel, dim3(1), dim3(64), 0, s, n_terms, a, b, out);
    return hipGetLastError();
}

hipError_t launch_fit(int L, int first, int m_floor, double* mom, double* vhat, int32_t* flag, hipStream_t s)
{
    hipLaunchKernelGGL(fit_kernel, dim3(1), dim3(64), 0, s, L, first, m_floor, mom, vhat, flag);
    return hipGetLastError();
}

hipError_t launch_moments(const double* qf, const double* qc, const int32_t* ok, int64_t M, double* out,
                          hipStream_t s)
{
    hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(MT), 0, s, qf, qc, ok, M, out);
    return hipGetLastError();
}

hipError_t launch_coefficients(int L, const double* mom, const double* W, double* alpha, int32_t* flag, hipStream_t s)
{
    hipLaunchKernelGGL(coefficients_kernel, dim3(1), dim3(64), 0, s, L, mom, W, alpha, flag);
    return hipGetLastError();
}

hipError_t launch_errors(int L, const double* mom, const double* alpha, double* sig, double* eps2, hipStream_t s)
{
    hipLaunchKernelGGL(errors_kernel, dim3(1), dim3(64), 0, s, L, mom, alpha, sig, eps2);
    return hipGetLastError();
}

hipError_t launch_estimate(int L, const double* mom, const double* alpha, double* E, hipStream_t s)
{
    hipLaunchKernelGGL(estimate_kernel, dim3(1), dim3(64), 0, s, L, mom, alpha, E);
    return hipGetLastError();
}

hipError_t launch_optimal_M(int L, const double* sig, const double* W, const int64_t* have, int mode, double target,
                            int64_t* out, int32_t* flag, hipStream_t s)
{
    hipLaunchKernelGGL(optimal_M_kernel, dim3(1), dim3(64), 0, s, L, sig, W, have, mode, target, out, flag);
    return hipGetLastError();
}

}  // namespace ofm
