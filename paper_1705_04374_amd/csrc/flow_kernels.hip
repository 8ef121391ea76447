// HIP kernels of one level-l solve of the five-equation two-phase model
// (Sukys et al., arXiv:1705.04374, Sec. 2.1-2.3), written for gfx950.
//
// A time step is three launches of `stage_kernel` (one per stage of the
// low-storage third-order Runge-Kutta scheme) and one `finalize_kernel`
// launch.  The stage kernel fuses what the paper lists as the right-hand-side
// and Runge-Kutta-update kernels (Sec. 2.3); its third-stage epilogue also
// does the CFL / QoI reduction (the paper's first kernel), so a step reads
// and writes each state array the minimum number of times.
//
// Work decomposition: a workgroup owns an x-y tile of TX x TY cells of one
// sample and marches through a chunk of z-planes.  For each plane it stages
// the primitive variables of the tile plus a 3-cell halo in LDS, reconstructs
// every cell along x and y (WENO5, both edges at once, with the cell-wise
// positivity fallback), evaluates the HLLC face fluxes and the face
// velocities, and sums the x-y flux differences of its cell.  The z direction
// uses a per-thread register queue of the primitives of five planes of the
// thread's own column, read three planes ahead, so that each z face is
// computed once and a cell is finished in the iteration of its own plane.
//
// Layout in HBM: structure of arrays, one contiguous array per variable,
// x fastest; three arrays per sample (two ping-pong state buffers and the
// low-storage register dU).
//
// Energy variable: the state carries Et = E - Pi(a2) = Gamma(a2) p + rho|u|^2/2
// in place of the total energy E.  Since Pi(a2) = Pi_1 + a2 (Pi_2 - Pi_1) is
// linear in a2, the HLLC energy flux splits exactly into the flux of Et plus
// Pi(a2_K) u_f, and the update of Et is the one of E minus (Pi_2 - Pi_1) times
// the one of a2:  L(Et) = -sum_d dF(Et)/h - Pi(a2 + K) sum_d du_f/h.  This is
// the same scheme in exact arithmetic; in float it avoids recovering a
// pressure of a few kPa from E ~ 4e8 Pa (water's Pi), which would cost most
// of the significand.
#include "flow_kernels.h"

#include <math.h>

#include <type_traits>

namespace ofm {

// ---------------------------------------------------------------------------
// Arithmetic helpers: fast reciprocal/sqrt in float, IEEE in double.
// ---------------------------------------------------------------------------
template <typename T> struct Num;
template <> struct Num<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    // sqrt(a / b) for a, b > 0 with one transcendental: a / sqrt(a b)
    static __device__ __forceinline__ float sqrt_ratio(float a, float b) { return a * __builtin_amdgcn_rsqf(a * b); }
    // round-off allowance of the positivity checks, relative to the stencil
    static constexpr float round_tol = 1e-6f;
};
template <> struct Num<double> {
    // hardware reciprocal estimate refined by two Newton steps
    // r <- r + r (1 - x r): within an ulp or two of 1/x for the finite,
    // nonzero, normal x this code divides by
    static __device__ __forceinline__ double rcp(double x)
    {
        double r = __builtin_amdgcn_rcp(x);
        r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
        return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double sqrt_(double x) { return ::sqrt(x); }
    // sqrt(a / b) = a / sqrt(a b) for a, b > 0: reciprocal square root
    // estimate refined by two Newton steps y <- y (3/2 - (x/2) y^2)
    static __device__ __forceinline__ double sqrt_ratio(double a, double b)
    {
        const double x = a * b, h = 0.5 * x;
        double y = __builtin_amdgcn_rsq(x);
        y = y * __builtin_fma(-h, y * y, 1.5);
        y = y * __builtin_fma(-h, y * y, 1.5);
        return a * y;
    }
    static constexpr double round_tol = 1e-12;
};

// Device memory seen as the global address space.  The state arrays come
// from descriptors in memory, so the compiler cannot infer where they live
// and would use flat accesses; a flat load also counts against the LDS wait
// counter, so every LDS wait of the x-y work would wait for the column and
// cell loads issued ahead of it.
template <typename T> using glob = __attribute__((address_space(1))) T;

template <typename T> struct Phys {
    T g1inv, dginv, pi1, dpi;
    T eps;             // (12/13) x the WENO epsilon (the indicators' scale in weno5_cell)
    T eps3;            // the WENO epsilon (weno3_cell)
    T gam1, pc1, gam2, pc2;
    T rho1, rho2;      // reference phase densities (scale of the positivity checks)
    T pfar;            // far-field pressure of the characteristic boundary
    __device__ __forceinline__ explicit Phys(const PhysD& d)
        : g1inv((T)d.g1inv), dginv((T)(d.g2inv - d.g1inv)), pi1((T)d.pi1), dpi((T)(d.pi2 - d.pi1)),
          eps((T)(d.eps * (12.0 / 13.0))), eps3((T)d.eps), gam1((T)d.gamma1), pc1((T)d.pc1), gam2((T)d.gamma2), pc2((T)d.pc2),
          rho1((T)d.rho1), rho2((T)d.rho2), pfar((T)d.p_far) {}
    // mixture stiffened-gas coefficients under isobaric closure:
    // p = (E - rho|u|^2/2 - Pi(a2)) / Gamma(a2)
    __device__ __forceinline__ T gamma(T a2) const { return g1inv + a2 * dginv; }
    __device__ __forceinline__ T pinf(T a2) const { return pi1 + a2 * dpi; }
};

__device__ __forceinline__ int bc_map(int i, int n, int bc)
{
    if (bc == OFM_BC_PERIODIC) { i %= n; return i < 0 ? i + n : i; }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Characteristic far-field ghost (OFM_BC_CHARACTERISTIC): primitives w of
// the nearest cell become those of a ghost outside the domain side (axis,
// side = -1 low / +1 high).  The outgoing acoustic invariant p + side Z u_n
// (Z = rho c, frozen sound speed) is kept and the incoming one
// Rm = p - side Z u_n moves to Rm + beta (p_far - Rm), i.e. p += delta and
// u_n -= side delta / Z with delta = beta (p_far - Rm) / 2.  beta = sigma h
// with sigma = 0.25 on the unit domain relaxes the boundary towards p_far at
// the rate sigma c (Poinsot and Lele's penalty at low Mach number).  A state
// without a positive (rho c)^2 stays a zero-gradient copy.
constexpr double kFarFieldSigma = 0.25;

template <typename T, int ND>
__device__ __forceinline__ void char_ghost(const Phys<T>& ph, T (&w)[4 + ND], int axis, int side, T beta)
{
    const T rho = w[0] + w[1];
    const T a2 = w[3 + ND], p = w[2 + ND];
    const T g = ph.gamma(a2);
    const T a = rho * ((g + T(1)) * p + ph.pinf(a2));       // (rho c)^2 = a / g
    if (!(a > T(0))) return;
    const T Z = Num<T>::sqrt_ratio(a, g);
    const T sZ = side > 0 ? Z : -Z;
    T un = w[2];
#pragma unroll
    for (int m = 1; m < ND; ++m) un = axis == m ? w[2 + m] : un;
    const T delta = T(0.5) * beta * (ph.pfar - Num<T>::fma(-sZ, un, p));
    w[2 + ND] = p + delta;
    const T du = delta * Num<T>::rcp(sZ);
#pragma unroll
    for (int m = 0; m < ND; ++m) w[2 + m] = axis == m ? w[2 + m] - du : w[2 + m];
}

// State -> primitive (a1r1, a2r2, u_1..u_d, p, a2); the energy slot holds Et.
template <typename T, int ND>
__device__ __forceinline__ void to_prim(const Phys<T>& ph, const T* q, T* w)
{
    T rho = q[0] + q[1];
    T irho = Num<T>::rcp(rho);
    T ke = T(0);
    w[0] = q[0];
    w[1] = q[1];
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        w[2 + m] = q[2 + m] * irho;
        ke += q[2 + m] * w[2 + m];
    }
    T a2 = q[3 + ND];
    w[2 + ND] = (q[2 + ND] - T(0.5) * ke) * Num<T>::rcp(ph.gamma(a2));
    w[3 + ND] = a2;
}

// WENO5 (Jiang-Shu) edge values of the centre cell c of the stencil a..e:
// `lo` at its left edge, `hi` at its right edge.  The reconstruction is
// invariant under adding a constant to the stencil, so it is evaluated on the
// differences from the centre value (exact in exact arithmetic; in float it
// keeps the rounding of large offsets, such as 1e7 Pa, out of the weights and
// candidate values).  The two edges share the smoothness indicators.
//
// Arithmetic forms (each equal to the textbook one in exact arithmetic):
//  * the indicators are carried as (12/13) beta_k = t0^2 + (sqrt(3/13) t1)^2
//    with eps_s = (12/13) eps (Phys::eps holds eps_s), which leaves every
//    ratio (eps + beta_j) / (eps + beta_k), hence every weight, unchanged;
//  * the nonlinear weights are normalised by the smallest (eps + beta), so
//    that they cannot overflow, and the two weight sums, both in [0.1, 1],
//    share one reciprocal;
//  * the candidate values are carried times 6 and the 1/6 is applied with
//    that reciprocal.
template <typename T>
__device__ __forceinline__ void weno5_cell(T a, T b, T c, T d, T e, T eps_s, T& lo, T& hi)
{
    const T s3 = T(0.48038446141526137);     // sqrt(3/13)
    const T A = a - c, B = b - c, D = d - c, E = e - c;
    // stencils (a,b,c), (b,c,d), (c,d,e): t0 = A - 2B, t1 = A - 4B, ...
    T t0 = Num<T>::fma(B, T(-2), A);
    T u = Num<T>::fma(A, s3, B * (T(-4) * s3));
    const T e0 = Num<T>::fma(t0, t0, Num<T>::fma(u, u, eps_s));
    t0 = B + D;
    u = (B - D) * s3;
    const T e1 = Num<T>::fma(t0, t0, Num<T>::fma(u, u, eps_s));
    t0 = Num<T>::fma(D, T(-2), E);
    u = Num<T>::fma(E, s3, D * (T(-4) * s3));
    const T e2 = Num<T>::fma(t0, t0, Num<T>::fma(u, u, eps_s));
    const T m = fmin(fmin(e0, e1), e2);
    const T r0 = m * Num<T>::rcp(e0), r1 = m * Num<T>::rcp(e1), r2 = m * Num<T>::rcp(e2);
    const T q0 = r0 * r0, q2 = r2 * r2;
    // linear weights (1/10, 6/10, 3/10) at the right edge, mirrored at the left
    const T wh0 = T(0.1) * q0, w1 = T(0.6) * (r1 * r1), wh2 = T(0.3) * q2;
    const T wl0 = T(0.1) * q2, wl2 = T(0.3) * q0;
    // 6 x candidate values: right edge (2A - 7B, 2D - B, 5D - E), left edge mirrored
    const T ph0 = Num<T>::fma(A, T(2), B * T(-7)), ph1 = Num<T>::fma(D, T(2), -B), ph2 = Num<T>::fma(D, T(5), -E);
    const T pl0 = Num<T>::fma(E, T(2), D * T(-7)), pl1 = Num<T>::fma(B, T(2), -D), pl2 = Num<T>::fma(B, T(5), -A);
    const T nh = Num<T>::fma(wh0, ph0, Num<T>::fma(w1, ph1, wh2 * ph2));
    const T nl = Num<T>::fma(wl0, pl0, Num<T>::fma(w1, pl1, wl2 * pl2));
    const T sh = wh0 + w1 + wh2, sl = wl0 + w1 + wl2;
    const T r = Num<T>::rcp(sh * sl) * T(1.0 / 6.0);
    hi = Num<T>::fma(nh, sl * r, c);
    lo = Num<T>::fma(nl, sh * r, c);
}

// WENO3 (Jiang-Shu, candidate stencils (b, c) and (c, d), ideal weights 1/3
// and 2/3 at the right edge, mirrored at the left) edge values of the centre
// cell c, in the same difference form as weno5_cell: with B = b - c and
// D = d - c the indicators are B^2 and D^2, the candidates c - B/2 and
// c + D/2, the weights are normalised by the smaller (eps + beta) and the two
// weight sums (in [1, 3] after scaling by 3) share one reciprocal.
template <typename T>
__device__ __forceinline__ void weno3_cell(T b, T c, T d, T eps, T& lo, T& hi)
{
    const T B = b - c, D = d - c;
    const T eB = Num<T>::fma(B, B, eps), eD = Num<T>::fma(D, D, eps);
    const T m = fmin(eB, eD);
    const T rB = m * Num<T>::rcp(eB), rD = m * Num<T>::rcp(eD);
    const T qB = rB * rB, qD = rD * rD;
    // right edge: weights (qB, 2 qD) on (-B/2, D/2); left edge: (qD, 2 qB) on (-D/2, B/2)
    const T nh = Num<T>::fma(T(2) * D, qD, -(B * qB)), nl = Num<T>::fma(T(2) * B, qB, -(D * qD));
    const T sh = Num<T>::fma(T(2), qD, qB), sl = Num<T>::fma(T(2), qB, qD);
    const T r = Num<T>::rcp(sh * sl) * T(0.5);
    hi = Num<T>::fma(nh, sl * r, c);
    lo = Num<T>::fma(nl, sh * r, c);
}

// Edges of one cell along one axis with the positivity / bounds checks.
// Each partial density keeps its reconstruction only if it stays >= 0 at both
// edges and at the interior Gauss-Lobatto point that keeps the cell mean under
// the rule exact for the reconstruction (WENO5: four points, the interior
// value (12 mean - lo - hi)/10; WENO3: Simpson, (6 mean - lo - hi)/4)
// (up to round_tol times the phase's reference density
// or the largest magnitude of that partial density in the stencil);
// a2 keeps its reconstruction only if it stays in [0, 1] at the same three
// points (up to round_tol).  A variable that fails takes the cell value at
// both edges (first order for that variable alone, so that a decision taken
// on round-off moves the edges by round-off).  If then either edge state has
// (Gamma+1) p + Pi <= 0, the whole cell is first order.
//
// The gas's partial density and volume fraction are exactly zero in pure
// water, i.e. in most of a cloud's domain for the whole run.  WENO of a
// constant stencil returns the constant exactly, so where the stencils of a
// whole wavefront are constant in those two variables their reconstruction
// is skipped (same values, bit for bit).  ORD = 5 or 3 (WENO3 reads s[1..3]).
template <typename T, int ND, int ORD>
__device__ __forceinline__ void cell_edges(const Phys<T>& ph, const T (&s)[5][4 + ND],
                                           T (&lo)[4 + ND], T (&hi)[4 + ND])
{
    static_assert(ORD == 5 || ORD == 3, "WENO order");
    constexpr int NV = 4 + ND;
    constexpr int K0 = ORD == 5 ? 0 : 1, K1 = ORD == 5 ? 5 : 4;   // stencil cells read
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v == 1 || v == NV - 1) {
            // constant stencil across the wavefront: the edges are the cell
            // value, which every check below would keep as well
            const bool flat = (ORD == 3 || s[0][v] == s[2][v]) && s[1][v] == s[2][v] && s[3][v] == s[2][v] &&
                              (ORD == 3 || s[4][v] == s[2][v]);
            if (__all(flat)) {
                lo[v] = s[2][v];
                hi[v] = s[2][v];
                continue;
            }
        }
        if (ORD == 5)
            weno5_cell<T>(s[0][v], s[1][v], s[2][v], s[3][v], s[4][v], ph.eps, lo[v], hi[v]);
        else
            weno3_cell<T>(s[1][v], s[2][v], s[3][v], ph.eps3, lo[v], hi[v]);
        if (v < 2) {
            T big = v == 0 ? ph.rho1 : ph.rho2;
#pragma unroll
            for (int k = K0; k < K1; ++k) big = fmax(big, fabs(s[k][v]));
            const T tol = -Num<T>::round_tol * big;
            const T mid = ORD == 5 ? (T(12) * s[2][v] - lo[v] - hi[v]) * T(0.1)
                                   : (T(6) * s[2][v] - lo[v] - hi[v]) * T(0.25);
            const bool keep = (lo[v] >= tol) && (hi[v] >= tol) && (mid >= tol);
            lo[v] = keep ? lo[v] : s[2][v];
            hi[v] = keep ? hi[v] : s[2][v];
        } else if (v == NV - 1) {
            const T lb = -Num<T>::round_tol, ub = T(1) + Num<T>::round_tol;
            const T mid = ORD == 5 ? (T(12) * s[2][v] - lo[v] - hi[v]) * T(0.1)
                                   : (T(6) * s[2][v] - lo[v] - hi[v]) * T(0.25);
            const bool keep = (lo[v] >= lb) && (lo[v] <= ub) && (hi[v] >= lb) && (hi[v] <= ub) && (mid >= lb) && (mid <= ub);
            lo[v] = keep ? lo[v] : s[2][v];
            hi[v] = keep ? hi[v] : s[2][v];
        }
    }
    const T cl = (ph.gamma(lo[3 + ND]) + T(1)) * lo[2 + ND] + ph.pinf(lo[3 + ND]);
    const T ch = (ph.gamma(hi[3 + ND]) + T(1)) * hi[2 + ND] + ph.pinf(hi[3 + ND]);
    if (!((cl > T(0)) && (ch > T(0)))) {
#pragma unroll
        for (int v = 0; v < NV; ++v) { lo[v] = s[2][v]; hi[v] = s[2][v]; }
    }
}

// HLLC flux along axis DIR (Toro 1994) with Davis wave speeds; the a2 flux
// is a2_K u_f where u_f is the face velocity of the HLLC flux of a passive
// scalar (Johnsen-Colonius adaptation).  f[0..NV-2]: fluxes of (a1r1, a2r2,
// momenta, Et); f[NV-1]: a2 flux; f[NV]: u_f.  The flux of E is
// f[NV-2] + Pi(a2_K) u_f.
template <typename T, int ND, int DIR>
__device__ __forceinline__ void hllc(const Phys<T>& ph, const T (&wl)[4 + ND], const T (&wr)[4 + ND],
                                     T (&f)[5 + ND])
{
    constexpr int NV = 4 + ND;
    T rl = wl[0] + wl[1], rr = wr[0] + wr[1];
    T ul = wl[2 + DIR], ur = wr[2 + DIR];
    T pl = wl[2 + ND], pr = wr[2 + ND];
    T gl = ph.gamma(wl[3 + ND]), gr = ph.gamma(wr[3 + ND]);
    T Pl = ph.pinf(wl[3 + ND]), Pr = ph.pinf(wr[3 + ND]);
    T kel = T(0), ker = T(0);
#pragma unroll
    for (int m = 0; m < ND; ++m) { kel += wl[2 + m] * wl[2 + m]; ker += wr[2 + m] * wr[2 + m]; }
    // energies without Pi (its flux Pi(a2_K) u_f is added by the caller's source)
    T El = gl * pl + T(0.5) * rl * kel;
    T Er = gr * pr + T(0.5) * rr * ker;
    T cl = Num<T>::sqrt_ratio((gl + T(1)) * pl + Pl, gl * rl);
    T cr = Num<T>::sqrt_ratio((gr + T(1)) * pr + Pr, gr * rr);
    T sl = fmin(ul - cl, ur - cr);
    T sr = fmax(ul + cl, ur + cr);
    T ml = rl * (sl - ul), mr = rr * (sr - ur);
    T ss = (pr - pl + ml * ul - mr * ur) * Num<T>::rcp(ml - mr);
    // side whose (star) state enters: left if S_L >= 0 or S* >= 0
    const bool left = (sl >= T(0)) || (ss >= T(0));
    const T sK = left ? sl : sr;
    const T sk = left ? fmin(sl, T(0)) : fmax(sr, T(0));   // 0 for the upwind fluxes
    T w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = left ? wl[v] : wr[v];
    const T rho = left ? rl : rr;
    const T un = left ? ul : ur;
    const T p = left ? pl : pr;
    const T E = left ? El : Er;
    const bool star = sk != T(0);
    const T rs = star ? Num<T>::rcp(sK - ss) : T(0);
    const T chi = star ? (sK - un) * rs : T(1);
    f[0] = w[0] * un;
    f[1] = w[1] * un;
#pragma unroll
    for (int m = 0; m < ND; ++m) f[2 + m] = rho * w[2 + m] * un + (m == DIR ? p : T(0));
    f[2 + ND] = (E + p) * un;
    // star state minus state, times the wave speed of the jump
    f[0] += sk * (chi * w[0] - w[0]);
    f[1] += sk * (chi * w[1] - w[1]);
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        T qs = chi * rho * (m == DIR ? ss : w[2 + m]);
        f[2 + m] += sk * (qs - rho * w[2 + m]);
    }
    {
        // chi p / (S_K - u) = p / (S_K - S*)
        T Es = chi * (E + (ss - un) * rho * ss) + (ss - un) * p * rs;
        f[2 + ND] += sk * (Es - E);
    }
    T uf = un + sk * (chi - T(1));
    f[NV - 1] = w[3 + ND] * uf;
    f[NV] = uf;
}

// K of eq. (var_K) at a cell centre, a2 clamped to [0, 1], with a2 + K (the
// gas's share of the mixture's volume change) kept in [0, 1]: the formula
// leaves that range only when a phase is below its stiffened-gas range
// (p + pc_k < 0), where its denominator can vanish.
template <typename T>
__device__ __forceinline__ T k_coef(const Phys<T>& ph, T a2, T p)
{
    T a = fmin(fmax(a2, T(0)), T(1));
    T b = T(1) - a;
    T rc1 = ph.gam1 * (p + ph.pc1);
    T rc2 = ph.gam2 * (p + ph.pc2);
    T den = b * rc2 + a * rc1;
    T k = a * b * (rc1 - rc2) * Num<T>::rcp(den);
    k = a + k < T(0) ? -a : (a + k > T(1) ? T(1) - a : k);
    return (a == T(0) || a == T(1) || den == T(0)) ? T(0) : k;
}

// Running reduction of one thread (CFL speed, QoIs, failure counters).
struct Red {
    double s_max, p_max;
    int64_t argmax;
    int n_nf, n_c2;
    double c_max, p_ball, a_ball;   // sound speed; sums over the sensors' balls
    int n_p, n_a;                   // cells in the balls
    __device__ __forceinline__ void init()
    {
        s_max = 0.0; p_max = -INFINITY; argmax = INT64_MAX; n_nf = 0; n_c2 = 0;
        c_max = 0.0; p_ball = 0.0; a_ball = 0.0; n_p = 0; n_a = 0;
    }
    __device__ __forceinline__ void take(double s, double p, int64_t idx)
    {
        s_max = fmax(s_max, s);
        if (p > p_max || (p == p_max && idx < argmax)) { p_max = p; argmax = idx; }
    }
    __device__ __forceinline__ void merge(const Red& o)
    {
        s_max = fmax(s_max, o.s_max);
        if (o.p_max > p_max || (o.p_max == p_max && o.argmax < argmax)) { p_max = o.p_max; argmax = o.argmax; }
        n_nf += o.n_nf;
        n_c2 += o.n_c2;
        c_max = fmax(c_max, o.c_max);
        p_ball += o.p_ball;
        a_ball += o.a_ball;
        n_p += o.n_p;
        n_a += o.n_a;
    }
};

// Squared distance of a cell centre from the cloud centre, in the order
// x, then y, then z, without contraction (the sensors' ball membership).
__device__ __forceinline__ double axis_dist2(double centre, int i, double n)
{
#pragma clang fp contract(off)
    const double dx = ((double)i + 0.5) / n - centre;
    return dx * dx;
}
__device__ __forceinline__ double add_dist2(double a, double b)
{
#pragma clang fp contract(off)
    return a + b;
}

// Accumulate one cell of a new state into the reduction (all in double);
// d2: the cell centre's squared distance from the cloud centre.
template <typename T, int ND>
__device__ __forceinline__ void reduce_cell(const PhysD& ph, const SampleDesc& d, const T (&q)[4 + ND], int64_t idx,
                                            double d2, Red& r)
{
    constexpr int NV = 4 + ND;
    bool finite = true;
    double qd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { qd[v] = (double)q[v]; finite = finite && isfinite(qd[v]); }
    double rho = qd[0] + qd[1];
    const double irho = Num<double>::rcp(rho);
    double ke = 0.0, umax = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        double u = qd[2 + m] * irho;
        ke += qd[2 + m] * u;
        umax = fmax(umax, fabs(u));
    }
    double a2 = qd[3 + ND];
    double G = ph.g1inv + a2 * (ph.g2inv - ph.g1inv);
    double P = ph.pi1 + a2 * (ph.pi2 - ph.pi1);
    const double iG = Num<double>::rcp(G);
    double p = (qd[2 + ND] - 0.5 * ke) * iG;
    finite = finite && isfinite(p);
    if (!finite) { r.n_nf++; return; }
    double c2 = ((G + 1.0) * p + P) * iG * irho;
    if (!(rho > 0.0) || !(c2 > 0.0)) { r.n_c2++; return; }
    const double cs = sqrt(c2);
    r.take(umax + cs, p, idx);
    r.c_max = fmax(r.c_max, cs);
    if (d2 <= d.r2_p) { r.p_ball += p; r.n_p++; }
    if (d2 <= d.r2_a) { r.a_ball += a2; r.n_a++; }
}

// Workgroup-wide merge of the thread reductions; thread 0 writes the tile.
// Butterfly merge of the 64 lanes' reductions (fixed order: every lane ends
// with the same result).
__device__ __forceinline__ void wave_merge(Red& r)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Red o;
        o.s_max = __shfl_xor(r.s_max, off, 64);
        o.p_max = __shfl_xor(r.p_max, off, 64);
        o.argmax = __shfl_xor(r.argmax, off, 64);
        o.n_nf = __shfl_xor(r.n_nf, off, 64);
        o.n_c2 = __shfl_xor(r.n_c2, off, 64);
        o.c_max = __shfl_xor(r.c_max, off, 64);
        o.p_ball = __shfl_xor(r.p_ball, off, 64);
        o.a_ball = __shfl_xor(r.a_ball, off, 64);
        o.n_p = __shfl_xor(r.n_p, off, 64);
        o.n_a = __shfl_xor(r.n_a, off, 64);
        r.merge(o);
    }
}

// Workgroup-wide merge of the thread reductions (waves in order, through
// LDS); thread 0 returns the result.
template <int NT>
__device__ __forceinline__ Red block_merge(Red r)
{
    __shared__ Red s_r[NT / 64];
    wave_merge(r);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_r[wave] = r;
    __syncthreads();
    Red t;
    t.init();
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) t.merge(s_r[w]);
    return t;
}

// Workgroup-wide merge of the thread reductions; thread 0 writes the tile.
template <int NT>
__device__ __forceinline__ void write_partial(Red r, TilePartial* out)
{
    const Red t = block_merge<NT>(r);
    if (threadIdx.x == 0) {
        out->s_max = t.s_max;
        out->p_max = t.p_max;
        out->argmax = t.argmax;
        out->n_nonfinite = t.n_nf;
        out->n_negc2 = t.n_c2;
        out->c_max = t.c_max;
        out->p_ball = t.p_ball;
        out->a2_ball = t.a_ball;
        out->n_ball_p = t.n_p;
        out->n_ball_a = t.n_a;
    }
}

// Map the launch index to a work item so that consecutive tiles of a sample
// land on the same XCD (workgroups are dealt round-robin to the 8 XCDs; each
// XCD has its own L2, which then serves the halos of neighbouring tiles).
__device__ __forceinline__ int xcd_swizzle(int b, int G)
{
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__constant__ double c_rk_a[3] = { 0.0, -17.0 / 32.0, -32.0 / 27.0 };
__constant__ double c_rk_b[3] = { 0.25, 8.0 / 9.0, 0.75 };

// ---------------------------------------------------------------------------
// Fused right-hand side + low-storage RK stage (+ reduction at stage 3)
// ---------------------------------------------------------------------------
constexpr int round_up64(int x) { return (x + 63) / 64 * 64; }

// Threads per workgroup of a TX x TY tile: the cell count rounded up to whole
// wavefronts (threads past the last cell help with the x-y tasks only).
template <int TX, int TY> constexpr int stage_threads() { return round_up64(TX * TY); }

// Occupancy target of the stage kernel: three wavefronts per SIMD for the
// float kernels (at most 168 VGPRs), two for double (at most 256 VGPRs; the
// split x-y pass below keeps a 16 x 8 tile's LDS under a quarter of the CU's).
template <typename T> constexpr int stage_waves_per_eu() { return sizeof(T) == 4 ? 3 : 2; }

// The x-y part of a plane in one pass (float: the edges of both axes live in
// LDS at once, then all faces) or split by axis (double: the x edges, x faces
// and x sums, then the same for y, each axis's face fluxes written over its
// own edges after a barrier), which needs about half the LDS for the edges.
template <typename T> constexpr bool stage_split_xy() { return sizeof(T) == 8; }

// RK stage STAGE = 0, 1, 2 (compiled separately: only the last carries the
// reduction, only the first skips dU); WENO order ORD = 5 or 3.
template <typename T, int ND, int TX, int TY, int STAGE, int ORD>
__global__ void __launch_bounds__((stage_threads<TX, TY>()))
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<T>())))
stage_kernel(LaunchArgs a)
{
    constexpr int NV = 4 + ND;
    constexpr int NT = stage_threads<TX, TY>();
    constexpr int HX = TX + 6;
    constexpr int HY = ND >= 2 ? TY + 6 : 1;
    // Task lists of the x-y phases.  Edge tasks: x then y, contiguous (a
    // wavefront may hold both; they differ only in the gather stride).  Face
    // tasks: the x block is padded to whole wavefronts so that no wavefront
    // holds both x and y faces (the two HLLC variants would both run under a
    // split exec mask).
    constexpr int EXN = TY * (TX + 2);                         // x edge tasks
    constexpr int EYN = ND >= 2 ? (TY + 2) * TX : 0;           // y edge tasks
    constexpr int ES = EXN + EYN;
    constexpr int FXN = TY * (TX + 1);                         // x faces
    constexpr int FXP = ND >= 2 ? round_up64(FXN) : FXN;       // start of the y faces
    constexpr int FYN = ND >= 2 ? (TY + 1) * TX : 0;           // y faces
    constexpr int FS = FXP + FYN;
    constexpr int WSZ = NV * HX * HY;
    constexpr int FSZ = (NV + 1) * FS;
    constexpr int AL = WSZ > FSZ ? WSZ : FSZ;          // W plane and face fluxes share LDS
    // split pass: edge tasks of one axis at a time; an axis's face fluxes
    // ((NV+1) x its faces <= 2 NV x its edge tasks) overwrite its edges
    constexpr bool SPLIT = stage_split_xy<T>();
    constexpr int ESX = EXN > EYN ? EXN : EYN;
    constexpr int EST = SPLIT ? ESX : ES;              // stride of the edge arrays
    static_assert(!SPLIT || ((NV + 1) * FXN <= 2 * NV * ESX && (NV + 1) * FYN <= 2 * NV * ESX), "face alias");
    static_assert(!SPLIT || (FXN <= 2 * NT && FYN <= 2 * NT), "at most two faces per thread in the split pass");
    // a workgroup's LDS is kept below 64 KiB: the one stage-kernel variant
    // above it (a running reduction held in LDS) computed states that
    // differed between tilings, for a cause not found (the set network's
    // pooling kernel runs correctly with 73.2 KB); every variant that passed
    // the tiling-invariance test is below
    static_assert(sizeof(T) * (SPLIT ? WSZ + 2 * NV * ESX : AL + 2 * NV * ES) + sizeof(Red) * (NT / 64) <= 65536,
                  "stage kernel LDS above 64 KiB");
    __shared__ T smem[SPLIT ? WSZ + 2 * NV * ESX : AL + 2 * NV * ES];
    T* sW = smem;                                      // [NV][HY][HX]
    T* sEm = smem + (SPLIT ? WSZ : AL);                // left edges  [NV][EST]
    T* sEp = sEm + NV * EST;                           // right edges [NV][EST]
    T* sF = SPLIT ? sEm : smem;                        // face fluxes [NV+1][faces] (after the edges are read)

    const int wi = xcd_swizzle(blockIdx.x, gridDim.x);
    if (wi >= a.n_work) return;
    const WorkItem item = a.work[wi];
    const SampleDesc& d = a.desc[item.sample];
    SampleState* st = a.state + item.sample;
    if (st->done) return;

    const Phys<T> ph(a.ph);
    const int n = d.n;
    const int tid = threadIdx.x;
    // cell of this thread; threads past the tile shadow its last row
    const int tx = tid % TX, ty = min(tid / TX, TY - 1);
    const int ttx = item.tile % d.ntx;
    const int tty = (item.tile / d.ntx) % d.nty;
    const int tzc = item.tile / (d.ntx * d.nty);
    const int x0 = ttx * TX, y0 = tty * TY;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool mine = tid < TX * TY && gx < n && (ND < 2 || gy < n);
    const int64_t ncell = ND == 3 ? (int64_t)n * n * n : (ND == 2 ? (int64_t)n * n : (int64_t)n);
    const int64_t plane = ND >= 2 ? (int64_t)n * n : (int64_t)n;
    const glob<T>* __restrict__ ua = (const glob<T>*)d.buf[a.src];
    glob<T>* __restrict__ ub = (glob<T>*)d.buf[a.src ^ 1];
    glob<T>* __restrict__ du = (glob<T>*)d.du;
    const T dt = (T)st->dt;
    const T ih = (T)(1.0 / d.h);
    constexpr int stage = STAGE;
    const T rkA = (T)c_rk_a[stage], rkB = (T)c_rk_b[stage];
    const int bc = a.bc;

    Red red;
    red.init();

    const T beta = (T)(kFarFieldSigma * d.h);     // far-field relaxation fraction
    // load plane gz (with halo) into sW as primitives
    // A plane with its halo in two parts: the loads of this thread's cells of
    // it (at most PK) into registers, and their conversion into sW.  In
    // the 3-D float first stage the loads of plane p+1 are issued before the
    // x-y work of plane p and converted at plane p+1, so that their latency
    // hides under that work (the other stages and double have no registers
    // to spare: they would spill).
    constexpr int PK = (HX * HY + NT - 1) / NT;
    constexpr bool PREFETCH = ND == 3 && sizeof(T) == 4 && STAGE == 0;
    auto plane_fetch = [&](int gz, T (&pf)[PK][NV]) {
        const int64_t zoff = (int64_t)bc_map(gz, ND == 3 ? n : 1, bc) * plane;
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int e = tid + k * NT;
            if (e < HX * HY) {
                const int hy = e / HX, hx = e % HX;
                const int cx = bc_map(x0 + hx - 3, n, bc);
                const int cy = ND >= 2 ? bc_map(y0 + hy - 3, n, bc) : 0;
                const int64_t idx = zoff + (int64_t)cy * n + cx;
#pragma unroll
                for (int v = 0; v < NV; ++v) pf[k][v] = ua[v * ncell + idx];
            }
        }
    };
    auto plane_store = [&](const T (&pf)[PK][NV]) {
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int e = tid + k * NT;
            if (e < HX * HY) {
                const int hy = e / HX, hx = e % HX;
                const int rx = x0 + hx - 3, ry = ND >= 2 ? y0 + hy - 3 : 0;
                T w[NV];
                to_prim<T, ND>(ph, pf[k], w);
                if (bc == OFM_BC_CHARACTERISTIC) {
                    // ghosts outside one domain side (corner ghosts are never read)
                    const bool ox = rx < 0 || rx >= n, oy = ND >= 2 && (ry < 0 || ry >= n);
                    if (ox != oy) char_ghost<T, ND>(ph, w, ox ? 0 : 1, (ox ? rx : ry) < 0 ? -1 : 1, beta);
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) sW[(v * HY + hy) * HX + hx] = w[v];
            }
        }
    };
    // without prefetch: one cell at a time (fewer registers live at once)
    auto load_plane = [&](int gz) {
        const int64_t zoff = (int64_t)bc_map(gz, ND == 3 ? n : 1, bc) * plane;
        for (int e = tid; e < HX * HY; e += NT) {
            const int hy = e / HX, hx = e % HX;
            const int rx = x0 + hx - 3, ry = ND >= 2 ? y0 + hy - 3 : 0;
            const int cx = bc_map(rx, n, bc);
            const int cy = ND >= 2 ? bc_map(ry, n, bc) : 0;
            const int64_t idx = zoff + (int64_t)cy * n + cx;
            T q[NV], w[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) q[v] = ua[v * ncell + idx];
            to_prim<T, ND>(ph, q, w);
            if (bc == OFM_BC_CHARACTERISTIC) {
                // ghosts outside one domain side (corner ghosts are never read)
                const bool ox = rx < 0 || rx >= n, oy = ND >= 2 && (ry < 0 || ry >= n);
                if (ox != oy) char_ghost<T, ND>(ph, w, ox ? 0 : 1, (ox ? rx : ry) < 0 ? -1 : 1, beta);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) sW[(v * HY + hy) * HX + hx] = w[v];
        }
    };

    // split x-y pass, one axis (DIR = 0: x, 1: y): edges of the axis's tasks
    // into sEm/sEp, then its faces (at most two per thread, fluxes kept in
    // registers across the barrier that ends the edge reads), written over
    // the edges, and the cell's flux differences added to xy
    auto axis_xy = [&](auto dir_c, T (&xy)[NV + 1]) {
        constexpr int DIR = decltype(dir_c)::value;
        constexpr int NE = DIR == 0 ? EXN : EYN;
        constexpr int NF = DIR == 0 ? FXN : FYN;
        for (int e = tid; e < NE; e += NT) {
            int base, stride;
            if (DIR == 0) {
                const int row = e / (TX + 2), cx = e % (TX + 2) - 1;
                base = (row + (ND >= 2 ? 3 : 0)) * HX + cx + 1;
                stride = 1;
            } else {
                const int cy = e / TX - 1, col = e % TX;
                base = (cy + 1) * HX + col + 3;
                stride = HX;
            }
            T st[5][NV], lo[NV], hi[NV];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int v = 0; v < NV; ++v) st[k][v] = sW[v * HY * HX + base + k * stride];
            cell_edges<T, ND, ORD>(ph, st, lo, hi);
#pragma unroll
            for (int v = 0; v < NV; ++v) { sEm[v * EST + e] = lo[v]; sEp[v * EST + e] = hi[v]; }
        }
        __syncthreads();
        T fa[NV + 1], fb[NV + 1];
        auto face = [&](int f, T (&fl)[NV + 1]) {
            T wl[NV], wr[NV];
            int l, r;
            if (DIR == 0) {
                const int row = f / (TX + 1), i = f % (TX + 1);
                l = row * (TX + 2) + i;
                r = l + 1;
            } else {
                const int j = f / TX, col = f % TX;
                l = j * TX + col;
                r = l + TX;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) { wl[v] = sEp[v * EST + l]; wr[v] = sEm[v * EST + r]; }
            hllc<T, ND, (DIR < ND ? DIR : 0)>(ph, wl, wr, fl);
        };
        const bool ha = tid < NF, hb = tid + NT < NF;
        if (ha) face(tid, fa);
        if (hb) face(tid + NT, fb);
        __syncthreads();
#pragma unroll
        for (int v = 0; v <= NV; ++v) {
            if (ha) sF[v * NF + tid] = fa[v];
            if (hb) sF[v * NF + tid + NT] = fb[v];
        }
        __syncthreads();
        if (DIR == 0) {
            const int fx = ty * (TX + 1) + tx;
#pragma unroll
            for (int v = 0; v < NV; ++v) xy[v] = sF[v * NF + fx] - sF[v * NF + fx + 1];
            xy[NV] = sF[NV * NF + fx + 1] - sF[NV * NF + fx];
        } else {
            const int fy = ty * TX + tx;
#pragma unroll
            for (int v = 0; v < NV; ++v) xy[v] += sF[v * NF + fy] - sF[v * NF + fy + TX];
            xy[NV] += sF[NV * NF + fy + TX] - sF[NV * NF + fy];
        }
    };

    // x-y part of the plane now in sW: per-cell sums of the face-flux
    // differences (F_- - F_+) and of the face-velocity differences (u_+ - u_-)
    auto plane_xy_split = [&](T (&xy)[NV + 1]) {
        axis_xy(std::integral_constant<int, 0>{}, xy);
        if constexpr (ND >= 2) {
            __syncthreads();                 // the x sums are read before the y edges overwrite them
            axis_xy(std::integral_constant<int, 1>{}, xy);
        }
    };

    auto plane_xy_joint = [&](T (&xy)[NV + 1]) {
        // edges along x of cells -1..TX of every row, along y of rows -1..TY
        for (int e = tid; e < ES; e += NT) {
            // stencil of five cells through the centre cell, `stride` apart in sW
            const bool isx = e < EXN;
            const int f = e - EXN;
            const int row = e / (TX + 2), cx = e % (TX + 2) - 1;     // x task
            const int cy = f / TX - 1, col = f % TX;                  // y task
            const int base = isx ? (row + (ND >= 2 ? 3 : 0)) * HX + cx + 1 : (cy + 1) * HX + col + 3;
            const int stride = isx ? 1 : HX;
            T s[5][NV], lo[NV], hi[NV];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int v = 0; v < NV; ++v) s[k][v] = sW[v * HY * HX + base + k * stride];
            cell_edges<T, ND, ORD>(ph, s, lo, hi);
#pragma unroll
            for (int v = 0; v < NV; ++v) { sEm[v * ES + e] = lo[v]; sEp[v * ES + e] = hi[v]; }
        }
        __syncthreads();
        // faces: x faces i-1/2 (i = 0..TX) of every row, y faces j-1/2
        for (int f = tid; f < FS; f += NT) {
            if (f >= FXN && f < FXP) continue;             // padding of the x block
            T wl[NV], wr[NV], fl[NV + 1];
            if (f < FXP) {
                const int row = f / (TX + 1), i = f % (TX + 1);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    wl[v] = sEp[v * ES + row * (TX + 2) + i];
                    wr[v] = sEm[v * ES + row * (TX + 2) + i + 1];
                }
                hllc<T, ND, 0>(ph, wl, wr, fl);
            } else {
                if constexpr (ND >= 2) {
                    const int g = f - FXP;
                    const int j = g / TX, col = g % TX;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        wl[v] = sEp[v * ES + EXN + j * TX + col];
                        wr[v] = sEm[v * ES + EXN + (j + 1) * TX + col];
                    }
                    hllc<T, ND, 1 < ND ? 1 : 0>(ph, wl, wr, fl);
                }
            }
#pragma unroll
            for (int v = 0; v <= NV; ++v) sF[v * FS + f] = fl[v];
        }
        __syncthreads();
        const int fx = ty * (TX + 1) + tx;
#pragma unroll
        for (int v = 0; v < NV; ++v) xy[v] = sF[v * FS + fx] - sF[v * FS + fx + 1];
        xy[NV] = sF[NV * FS + fx + 1] - sF[NV * FS + fx];
        if constexpr (ND >= 2) {
            const int fy = FXP + ty * TX + tx;
#pragma unroll
            for (int v = 0; v < NV; ++v) xy[v] += sF[v * FS + fy] - sF[v * FS + fy + TX];
            xy[NV] += sF[NV * FS + fy + TX] - sF[NV * FS + fy];
        }
    };

    auto plane_xy = [&](T (&xy)[NV + 1]) {
        if constexpr (SPLIT)
            plane_xy_split(xy);
        else
            plane_xy_joint(xy);
    };

    // L(U) of one cell from its flux-difference sums and primitives
    auto rate = [&](const T (&sum)[NV + 1], const T (&wc)[NV], T (&L)[NV]) {
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] = sum[v] * ih;
        const T sk = wc[3 + ND] + k_coef<T>(ph, wc[3 + ND], wc[2 + ND]);
        const T divu = sum[NV] * ih;
        L[NV - 1] += sk * divu;              // R_7 = (a2 + K) div u
        L[NV - 2] -= ph.pinf(sk) * divu;     // Et = E - Pi(a2): -Pi(a2 + K) div u
    };
    // squared distances from the cloud centre (sensors): this thread's x-y
    // part, completed per plane in 3-D
    const double n_d = (double)n;
    double dxy2 = axis_dist2(d.centre[0], gx, n_d);
    if (ND >= 2) dxy2 = add_dist2(dxy2, axis_dist2(d.centre[1], gy, n_d));

    // the low-storage RK stage of one cell, given its U and dU
    auto update = [&](int64_t idx, const T (&L)[NV], const T (&uo)[NV], const T (&duo)[NV], double d2) {
        T qn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int64_t o = v * ncell + idx;
            T dv = dt * L[v];
            if constexpr (stage > 0) dv += rkA * duo[v];
            if constexpr (stage < 2) du[o] = dv;
            qn[v] = uo[v] + rkB * dv;
            ub[o] = qn[v];
        }
        if constexpr (stage == 2) reduce_cell<T, ND>(a.ph, d, qn, idx, d2, red);
    };

    if constexpr (ND <= 2) {
        load_plane(0);
        __syncthreads();
        T xy[NV + 1];
        T wc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) wc[v] = sW[(v * HY + ty + (ND >= 2 ? 3 : 0)) * HX + tx + 3];
        plane_xy(xy);
        if (mine) {
            const int64_t idx = (ND == 2 ? (int64_t)gy * n : 0) + gx;
            T L[NV], uo[NV], duo[NV];
            rate(xy, wc, L);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                uo[v] = ua[v * ncell + idx];
                duo[v] = stage > 0 ? du[v * ncell + idx] : T(0);
            }
            update(idx, L, uo, duo, dxy2);
        }
    } else {
        // z: each thread keeps the primitives of its own column, planes
        // p-1..p+3, in registers (read from HBM three planes ahead of the
        // x-y work), so that at plane p it knows the z edges of cell p+1 and
        // finishes cell p in the same iteration.
        const int z0 = tzc * a.zchunk;
        const int z1 = min(z0 + a.zchunk, n) - 1;      // last plane of the chunk
        const int cxg = min(gx, n - 1), cyg = min(gy, n - 1);
        const int64_t col = (int64_t)cyg * n + cxg;    // (clamped) column of this thread
        T q[5][NV];                                    // primitives of planes p-1..p+3
        T pf[PK][NV];                                  // this thread's cells of the next plane (prefetch)
        T ep[NV];                                      // upper z edge of cell p
        T fz_lo[NV + 1];                               // flux through face p-1/2
        // One loop body does all the work (so that every edge and face is
        // computed by the same code whatever the chunking, bit for bit):
        // p = z0-6..z0-3 only fill the queue, p = z0-2 adds the edges of
        // cell z0-1, p = z0-1 the face z0-1/2, and p >= z0 the x-y work of
        // plane p and the update of cell p.
        for (int p = z0 - 6; p <= z1; ++p) {
            const bool xy_work = p >= z0;
            // global loads issued before the x-y work: the column's plane
            // p+3 and this cell's U and dU
            const int64_t inext = (int64_t)bc_map(p + 3, n, bc) * plane + col;
            const int64_t icell = (int64_t)p * plane + col;
            // (in double, U and dU are loaded after the x-y work instead: 28
            // more registers across it would halve the occupancy)
            constexpr bool early = sizeof(T) == 4;
            T qn[NV], uo[NV], duo[NV];
            auto load_cell = [&]() {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    uo[v] = ua[v * ncell + icell];
                    duo[v] = stage > 0 ? du[v * ncell + icell] : T(0);
                }
            };
#pragma unroll
            for (int v = 0; v < NV; ++v) qn[v] = ua[v * ncell + inext];
            if (early && xy_work) load_cell();
            T xy[NV + 1];
            if (xy_work) {
                if constexpr (!SPLIT) __syncthreads();   // sW is the joint pass's face-flux area
                if constexpr (PREFETCH) {
                    plane_store(pf);                     // plane p, loaded one plane ahead
                    if (p < z1) plane_fetch(p + 1, pf);
                } else {
                    load_plane(p);
                }
                __syncthreads();
                plane_xy(xy);
                if (!early) load_cell();
            } else if (PREFETCH && p == z0 - 1) {
                plane_fetch(z0, pf);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int v = 0; v < NV; ++v) q[k][v] = q[k + 1][v];
            to_prim<T, ND>(ph, qn, q[4]);                          // planes p-1..p+3
            if (bc == OFM_BC_CHARACTERISTIC && (p + 3 < 0 || p + 3 >= n))
                char_ghost<T, ND>(ph, q[4], ND - 1, p + 3 < 0 ? -1 : 1, beta);
            if (p >= z0 - 2) {
                T lo[NV], hi[NV];
                cell_edges<T, ND, ORD>(ph, q, lo, hi);             // cell p+1
                if (p >= z0 - 1) {
                    T fz[NV + 1];
                    hllc<T, ND, ND - 1>(ph, ep, lo, fz);           // face p+1/2
                    if (xy_work && mine) {
                        T sum[NV + 1], L[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) sum[v] = xy[v] + (fz_lo[v] - fz[v]);
                        sum[NV] = xy[NV] + (fz[NV] - fz_lo[NV]);
                        rate(sum, q[1], L);
                        update(icell, L, uo, duo, stage == 2 ? add_dist2(dxy2, axis_dist2(d.centre[2], p, n_d)) : 0.0);
                    }
#pragma unroll
                    for (int v = 0; v <= NV; ++v) fz_lo[v] = fz[v];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) ep[v] = hi[v];
            }
        }
    }
    if constexpr (stage == 2) write_partial<NT>(red, a.part + d.tile0 + item.tile);
}

// ---------------------------------------------------------------------------
// Reduction of a state without stepping (initial level)
// ---------------------------------------------------------------------------
template <typename T, int ND, int TX, int TY>
__global__ void __launch_bounds__((stage_threads<TX, TY>())) reduce_kernel(LaunchArgs a)
{
    constexpr int NV = 4 + ND;
    constexpr int NT = stage_threads<TX, TY>();
    const int wi = xcd_swizzle(blockIdx.x, gridDim.x);
    if (wi >= a.n_work) return;
    const WorkItem item = a.work[wi];
    const SampleDesc& d = a.desc[item.sample];
    if (a.state[item.sample].done) return;
    const int n = d.n;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;   // ty >= TY: no cell
    const int ttx = item.tile % d.ntx, tty = (item.tile / d.ntx) % d.nty, tzc = item.tile / (d.ntx * d.nty);
    const int gx = ttx * TX + tx, gy = tty * TY + ty;
    const int64_t ncell = ND == 3 ? (int64_t)n * n * n : (ND == 2 ? (int64_t)n * n : (int64_t)n);
    const int64_t plane = ND >= 2 ? (int64_t)n * n : (int64_t)n;
    const glob<T>* u = (const glob<T>*)d.buf[a.src];
    Red red;
    red.init();
    if (ty < TY && gx < n && (ND < 2 || gy < n)) {
        const int z0 = ND == 3 ? tzc * a.zchunk : 0;
        const int z1 = ND == 3 ? min(z0 + a.zchunk, n) : 1;
        const double n_d = (double)n;
        double dxy2 = axis_dist2(d.centre[0], gx, n_d);
        if (ND >= 2) dxy2 = add_dist2(dxy2, axis_dist2(d.centre[1], gy, n_d));
        for (int z = z0; z < z1; ++z) {
            const int64_t idx = (int64_t)z * plane + (ND >= 2 ? (int64_t)gy * n : 0) + gx;
            T q[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) q[v] = u[v * ncell + idx];
            reduce_cell<T, ND>(a.ph, d, q, idx, ND == 3 ? add_dist2(dxy2, axis_dist2(d.centre[2], z, n_d)) : dxy2,
                               red);
        }
    }
    write_partial<NT>(red, a.part + d.tile0 + item.tile);
}

// ---------------------------------------------------------------------------
// Per-sample finalisation of a step: time, QoI, status, next dt
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) finalize_kernel(const SampleDesc* desc, SampleState* state,
                                                       const TilePartial* part, int initial, double* dt_log,
                                                       int64_t dt_log_len)
{
    const SampleDesc& d = desc[blockIdx.x];
    SampleState& st = state[blockIdx.x];
    if (st.done) return;
    Red r;
    r.init();
    for (int t = threadIdx.x; t < d.ntiles; t += 256) {
        const TilePartial& tp = part[d.tile0 + t];
        Red o;
        o.s_max = tp.s_max; o.p_max = tp.p_max; o.argmax = tp.argmax; o.n_nf = tp.n_nonfinite; o.n_c2 = tp.n_negc2;
        o.c_max = tp.c_max; o.p_ball = tp.p_ball; o.a_ball = tp.a2_ball; o.n_p = tp.n_ball_p; o.n_a = tp.n_ball_a;
        r.merge(o);
    }
    const Red t = block_merge<256>(r);
    if (threadIdx.x != 0) return;
    if (!initial) {
        st.t = st.last ? d.t_end : st.t + st.dt;
        st.steps += 1;
    }
    const double ps = t.n_p > 0 ? t.p_ball / (double)t.n_p : 0.0;
    const double gs = t.n_a > 0 ? t.a_ball / (double)t.n_a : 0.0;
    if (initial) {
        st.p_max = t.p_max;
        st.argmax = t.argmax;
        st.t_at_max = st.t;
        st.p_sensor = ps;
        st.t_p_sensor = st.t;
        st.gas_min = gs;
        st.t_gas_min = st.t;
        st.c_max = t.c_max;
    }
    if (t.n_nf > 0) { st.status = OFM_SAMPLE_NONFINITE; st.done = 1; return; }
    if (t.n_c2 > 0) { st.status = OFM_SAMPLE_NEGATIVE_C2; st.done = 1; return; }
    if (!initial) {
        if (t.p_max > st.p_max) {
            st.p_max = t.p_max;
            st.argmax = t.argmax;
            st.t_at_max = st.t;
        }
        if (ps > st.p_sensor) { st.p_sensor = ps; st.t_p_sensor = st.t; }
        if (gs < st.gas_min) { st.gas_min = gs; st.t_gas_min = st.t; }
        st.c_max = fmax(st.c_max, t.c_max);
    }
    const bool fin = d.n_steps > 0 ? st.steps >= d.n_steps : st.t >= d.t_end;
    if (fin) { st.done = 1; return; }
    if (st.steps >= d.max_steps) { st.status = OFM_SAMPLE_MAX_STEPS; st.done = 1; return; }
    double dt = d.cfl * d.h / t.s_max;
    st.last = 0;
    if (d.n_steps <= 0 && dt >= d.t_end - st.t) { dt = d.t_end - st.t; st.last = 1; }
    st.dt = dt;
    if (dt_log && st.steps < dt_log_len) dt_log[st.steps] = dt;
}

// ---------------------------------------------------------------------------
// Initial state of a cloud (one sample per launch)
// ---------------------------------------------------------------------------
struct InitArgs {
    PhysD ph;
    const double* bubbles;   // nb x 4
    int32_t nb;
    int32_t n, n_sub;
    double rho1, rho2, p_bubble, p_inf;
    double cx, cy, cz, radius, delta, width;
    void* u;
};

// Workgroup = 256 cells (8x8x4 in 3-D, 16x16 in 2-D, 256 in 1-D).  The
// bubbles are culled against the workgroup's box in chunks of 256 through
// LDS; each thread keeps a bit mask of its sub-samples found inside.  Inside
// tests are in double without contraction, as |x - c|^2 < r^2.
template <typename T, int ND>
__global__ void __launch_bounds__(256) init_kernel(InitArgs a)
{
#pragma clang fp contract(off)
    constexpr int BX = ND == 3 ? 8 : (ND == 2 ? 16 : 256);
    constexpr int BY = ND == 3 ? 8 : (ND == 2 ? 16 : 1);
    constexpr int BZ = ND == 3 ? 4 : 1;
    const int n = a.n;
    const int nbx = (n + BX - 1) / BX, nby = ND >= 2 ? (n + BY - 1) / BY : 1;
    const int b = blockIdx.x;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tid = threadIdx.x;
    const int i = bx * BX + tid % BX;
    const int j = ND >= 2 ? by * BY + (tid / BX) % BY : 0;
    const int k = ND == 3 ? bz * BZ + tid / (BX * BY) : 0;
    const double N = (double)n;
    // workgroup box with a margin, for culling
    const double m = 1e-9;
    const double lx = (double)(bx * BX) / N - m, hx = (double)(bx * BX + BX) / N + m;
    const double ly = (double)(by * BY) / N - m, hy = (double)(by * BY + BY) / N + m;
    const double lz = (double)(bz * BZ) / N - m, hz = (double)(bz * BZ + BZ) / N + m;
    __shared__ double sb[256][4];
    __shared__ int s_cnt;
    const int ns = a.n_sub;
    const int nsz = ND == 3 ? ns : 1, nsy = ND >= 2 ? ns : 1;
    uint64_t mask = 0;
    const double den = (double)((int64_t)ns * n);
    for (int c0 = 0; c0 < a.nb; c0 += 256) {
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        const int bi = c0 + tid;
        if (bi < a.nb) {
            const double* q = a.bubbles + 4 * bi;
            bool hit = q[0] + q[3] >= lx && q[0] - q[3] <= hx;
            if (ND >= 2) hit = hit && q[1] + q[3] >= ly && q[1] - q[3] <= hy;
            if (ND == 3) hit = hit && q[2] + q[3] >= lz && q[2] - q[3] <= hz;
            if (hit) {
                const int slot = atomicAdd(&s_cnt, 1);
                sb[slot][0] = q[0]; sb[slot][1] = q[1]; sb[slot][2] = q[2]; sb[slot][3] = q[3];
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (i < n && j < (ND >= 2 ? n : 1) && k < (ND == 3 ? n : 1)) {
            for (int t = 0; t < cnt; ++t) {
                const double bxc = sb[t][0], byc = sb[t][1], bzc = sb[t][2], r = sb[t][3];
                const double r2 = r * r;
                int bit = 0;
                for (int sc = 0; sc < nsz; ++sc)
                    for (int sbb = 0; sbb < nsy; ++sbb)
                        for (int sa = 0; sa < ns; ++sa, ++bit) {
                            const double px = ((double)((int64_t)ns * i + sa) + 0.5) / den;
                            const double dx = px - bxc;
                            double d2 = dx * dx;
                            if (ND >= 2) {
                                const double py = ((double)((int64_t)ns * j + sbb) + 0.5) / den;
                                const double dy = py - byc;
                                d2 = d2 + dy * dy;
                            }
                            if (ND == 3) {
                                const double pz = ((double)((int64_t)ns * k + sc) + 0.5) / den;
                                const double dz = pz - bzc;
                                d2 = d2 + dz * dz;
                            }
                            if (d2 < r2) mask |= (uint64_t)1 << bit;
                        }
            }
        }
        __syncthreads();
    }
    if (!(i < n && j < (ND >= 2 ? n : 1) && k < (ND == 3 ? n : 1))) return;
    const int ntot = ns * nsy * nsz;
    const double a2 = (double)__popcll(mask) / (double)ntot;
    double ccx = ((double)i + 0.5) / N - a.cx;
    double rr = ccx * ccx;
    if (ND >= 2) { const double ccy = ((double)j + 0.5) / N - a.cy; rr = rr + ccy * ccy; }
    if (ND == 3) { const double ccz = ((double)k + 0.5) / N - a.cz; rr = rr + ccz * ccz; }
    const double rad = sqrt(rr);
    double s = (rad - a.radius - a.delta) / a.width;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    const double p = a.p_bubble + (a.p_inf - a.p_bubble) * (s * s * (3.0 - 2.0 * s));
    const double G = a.ph.g1inv + a2 * (a.ph.g2inv - a.ph.g1inv);
    const int64_t ncell = ND == 3 ? (int64_t)n * n * n : (ND == 2 ? (int64_t)n * n : (int64_t)n);
    const int64_t idx = ((int64_t)k * (ND >= 2 ? n : 1) + j) * n + i;
    glob<T>* u = (glob<T>*)a.u;
    constexpr int NV = 4 + ND;
    u[0 * ncell + idx] = (T)((1.0 - a2) * a.rho1);
    u[1 * ncell + idx] = (T)(a2 * a.rho2);
#pragma unroll
    for (int mm = 0; mm < ND; ++mm) u[(2 + mm) * ncell + idx] = (T)0;
    u[(2 + ND) * ncell + idx] = (T)(G * p);   // Et at rest
    u[(NV - 1) * ncell + idx] = (T)a2;
}

// Primitive -> conserved (test states), element-wise.
template <typename T, int ND>
__global__ void __launch_bounds__(256) prim_to_cons_kernel(PhysD phd, const T* w, T* u, int64_t ncell)
{
    constexpr int NV = 4 + ND;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncell) return;
    const Phys<T> ph(phd);
    T wv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) wv[v] = w[v * ncell + c];
    const T rho = wv[0] + wv[1];
    T ke = T(0);
    u[c] = wv[0];
    u[ncell + c] = wv[1];
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        u[(2 + m) * ncell + c] = rho * wv[2 + m];
        ke += rho * wv[2 + m] * wv[2 + m];
    }
    const T a2 = wv[3 + ND];
    u[(2 + ND) * ncell + c] = ph.gamma(a2) * wv[2 + ND] + T(0.5) * ke;
    u[(3 + ND) * ncell + c] = a2;
}

// Library state -> the conserved vector Q of eq. (system) in double
// (E = Et + Pi(a2)), element-wise.
template <typename T, int ND>
__global__ void __launch_bounds__(256) to_conserved_kernel(PhysD ph, const T* u, double* q, int64_t ncell)
{
    constexpr int NV = 4 + ND;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncell) return;
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v * ncell + c] = (double)u[v * ncell + c];
    const double a2 = (double)u[(NV - 1) * ncell + c];
    q[(NV - 2) * ncell + c] += ph.pi1 + a2 * (ph.pi2 - ph.pi1);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T, int ND, int TX, int TY>
static hipError_t launch_stage_t(const LaunchArgs& a, int stage, hipStream_t s)
{
    const dim3 grid(a.n_work), block(stage_threads<TX, TY>());
    if (a.ph.order == 3) {
        if (stage == 0) hipLaunchKernelGGL((stage_kernel<T, ND, TX, TY, 0, 3>), grid, block, 0, s, a);
        else if (stage == 1) hipLaunchKernelGGL((stage_kernel<T, ND, TX, TY, 1, 3>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((stage_kernel<T, ND, TX, TY, 2, 3>), grid, block, 0, s, a);
    } else if (a.ph.order == 5) {
        if (stage == 0) hipLaunchKernelGGL((stage_kernel<T, ND, TX, TY, 0, 5>), grid, block, 0, s, a);
        else if (stage == 1) hipLaunchKernelGGL((stage_kernel<T, ND, TX, TY, 1, 5>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((stage_kernel<T, ND, TX, TY, 2, 5>), grid, block, 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int ND, int TX, int TY>
static hipError_t launch_reduce_t(const LaunchArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((reduce_kernel<T, ND, TX, TY>), dim3(a.n_work), dim3(stage_threads<TX, TY>()), 0, s, a);
    return hipGetLastError();
}

// Tile shapes compiled for each (precision, dimension).
#define OFM_FOR_TILES(X)                                                               \
    X(float, 3, 16, 14) X(float, 3, 16, 16) X(float, 3, 16, 8)                         \
    X(double, 3, 16, 8) X(double, 3, 16, 14) X(double, 3, 16, 16)                      \
    X(float, 2, 16, 14) X(float, 2, 16, 16) X(double, 2, 16, 14) X(double, 2, 16, 8)   \
    X(float, 1, 256, 1) X(double, 1, 256, 1) X(float, 1, 64, 1) X(double, 1, 64, 1)

bool tile_supported(int precision, int ndim, int tx, int ty)
{
#define X(T, ND, TX, TY) \
    if ((precision == OFM_F64) == (sizeof(T) == 8) && ndim == ND && tx == TX && ty == TY) return true;
    OFM_FOR_TILES(X)
#undef X
    return false;
}

int tile_list(int precision, int ndim, int (*out)[2], int cap)
{
    int k = 0;
#define X(T, ND, TX, TY)                                                                        \
    if ((precision == OFM_F64) == (sizeof(T) == 8) && ndim == ND) {                             \
        if (k < cap) { out[k][0] = TX; out[k][1] = TY; }                                        \
        ++k;                                                                                    \
    }
    OFM_FOR_TILES(X)
#undef X
    return k;
}

hipError_t launch_stage(int precision, int ndim, int tx, int ty, const LaunchArgs& a, int stage, hipStream_t s)
{
#define X(T, ND, TX, TY) \
    if ((precision == OFM_F64) == (sizeof(T) == 8) && ndim == ND && tx == TX && ty == TY) return launch_stage_t<T, ND, TX, TY>(a, stage, s);
    OFM_FOR_TILES(X)
#undef X
    return hipErrorInvalidValue;
}

template <typename T, int ND, int TX, int TY>
static int stage_blocks_per_cu_t(int order)
{
    int b = 0;
    const void* f = order == 3 ? reinterpret_cast<const void*>(&stage_kernel<T, ND, TX, TY, 2, 3>)
                               : reinterpret_cast<const void*>(&stage_kernel<T, ND, TX, TY, 2, 5>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, f, stage_threads<TX, TY>(), 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return b;
}

int stage_blocks_per_cu(int precision, int ndim, int tx, int ty, int order)
{
#define X(T, ND, TX, TY) \
    if ((precision == OFM_F64) == (sizeof(T) == 8) && ndim == ND && tx == TX && ty == TY) return stage_blocks_per_cu_t<T, ND, TX, TY>(order);
    OFM_FOR_TILES(X)
#undef X
    return 0;
}

hipError_t launch_reduce(int precision, int ndim, int tx, int ty, const LaunchArgs& a, hipStream_t s)
{
#define X(T, ND, TX, TY) \
    if ((precision == OFM_F64) == (sizeof(T) == 8) && ndim == ND && tx == TX && ty == TY) return launch_reduce_t<T, ND, TX, TY>(a, s);
    OFM_FOR_TILES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const SampleDesc* desc, SampleState* state, const TilePartial* part, int n_samples,
                           int initial, double* dt_log, int64_t dt_log_len, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(n_samples), dim3(256), 0, s, desc, state, part, initial, dt_log, dt_log_len);
    return hipGetLastError();
}

hipError_t launch_init(int precision, int ndim, const InitLaunch& L, hipStream_t s)
{
    InitArgs a;
    a.ph = L.ph;
    a.bubbles = L.bubbles;
    a.nb = L.nb;
    a.n = L.n;
    a.n_sub = L.n_sub;
    a.rho1 = L.rho1; a.rho2 = L.rho2; a.p_bubble = L.p_bubble; a.p_inf = L.p_inf;
    a.cx = L.center[0]; a.cy = L.center[1]; a.cz = L.center[2];
    a.radius = L.radius; a.delta = L.delta; a.width = L.width;
    a.u = L.u;
    const int n = L.n;
    int blocks;
    if (ndim == 3) blocks = ((n + 7) / 8) * ((n + 7) / 8) * ((n + 3) / 4);
    else if (ndim == 2) blocks = ((n + 15) / 16) * ((n + 15) / 16);
    else blocks = (n + 255) / 256;
#define IL(T, ND) hipLaunchKernelGGL((init_kernel<T, ND>), dim3(blocks), dim3(256), 0, s, a)
    if (precision == OFM_F64) {
        if (ndim == 3) IL(double, 3); else if (ndim == 2) IL(double, 2); else IL(double, 1);
    } else {
        if (ndim == 3) IL(float, 3); else if (ndim == 2) IL(float, 2); else IL(float, 1);
    }
#undef IL
    return hipGetLastError();
}

hipError_t launch_prim_to_cons(int precision, int ndim, const PhysD& ph, const void* w, void* u, int64_t ncell,
                               hipStream_t s)
{
    const int blocks = (int)((ncell + 255) / 256);
#define PL(T, ND) hipLaunchKernelGGL((prim_to_cons_kernel<T, ND>), dim3(blocks), dim3(256), 0, s, ph, (const T*)w, (T*)u, ncell)
    if (precision == OFM_F64) {
        if (ndim == 3) PL(double, 3); else if (ndim == 2) PL(double, 2); else PL(double, 1);
    } else {
        if (ndim == 3) PL(float, 3); else if (ndim == 2) PL(float, 2); else PL(float, 1);
    }
#undef PL
    return hipGetLastError();
}

}  // namespace ofm

namespace ofm {

hipError_t launch_to_conserved(int precision, int ndim, const PhysD& ph, const void* u, double* q, int64_t ncell,
                               hipStream_t s)
{
    const int blocks = (int)((ncell + 255) / 256);
#define CL(T, ND) hipLaunchKernelGGL((to_conserved_kernel<T, ND>), dim3(blocks), dim3(256), 0, s, ph, (const T*)u, q, ncell)
    if (precision == OFM_F64) {
        if (ndim == 3) CL(double, 3); else if (ndim == 2) CL(double, 2); else CL(double, 1);
    } else {
        if (ndim == 3) CL(float, 3); else if (ndim == 2) CL(float, 2); else CL(float, 1);
    }
#undef CL
    return hipGetLastError();
}

}  // namespace ofm
