/*
 * Oracle for the diffuse-interface two-phase solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, serial, FP64 CPU implementation
 * of what one level-l solve computes.  It exists so that tests, the smoke check
 * and the CPU baseline of the benchmark have something obviously correct to
 * compare the HIP library with.  It shares no code with the library, and the
 * product path never calls it.
 *
 * Passages followed (Sukys et al., "Optimal fidelity multi-level Monte Carlo
 * for quantification of uncertainty in simulations of cloud cavitation
 * collapse", arXiv:1705.04374):
 *   - Sec. 2.1, eqs. (mass_1)-(vol_frac), (var_K): the five-equation model and
 *     the K coefficient of the volume-fraction source.
 *   - Sec. 2.1, stiffened-gas EOS with isobaric closure; p_c = 0 is ideal gas.
 *   - Sec. 2.2, eq. (system): conserved vector Q = (a1r1, a2r2, rho u, E, a2),
 *     fluxes F, G, H and the source R_7 = a2 div u + K div u.
 *   - Sec. 2.2, eq. (ode): method of lines, finite volumes on a uniform grid;
 *     explicit third-order low-storage (2N) Runge-Kutta; HLLC fluxes; WENO
 *     reconstruction of primitive variables; HLLC adapted to the a2 equation;
 *     CFL-limited time step.
 *   - Sec. 3.1: cloud set-up (pressure equilibrium inside, smooth ramp to the
 *     ambient pressure starting just outside the cloud, constant phase
 *     densities, fluid at rest).
 *
 * Where the paper is silent the oracle takes these readings (the library takes
 * the same ones; each is listed with its reason in the design notes):
 *   mixture EOS  Gamma(a2) = (1-a2)/(g1-1) + a2/(g2-1),
 *                Pi(a2)    = (1-a2) g1 pc1/(g1-1) + a2 g2 pc2/(g2-1),
 *                p = (E - rho|u|^2/2 - Pi)/Gamma;
 *   sound speed  frozen mixture value c^2 = ((Gamma+1) p + Pi)/(Gamma rho);
 *   WENO         fifth-order Jiang-Shu (weno_order 5, the default) or
 *                third-order Jiang-Shu (weno_order 3; the paper allows
 *                either), eps = spec->weno_eps (absolute);
 *   positivity   each cell is reconstructed along each axis on its own
 *                (both edge values); a partial density that would be negative
 *                at an edge or at the interior Gauss-Lobatto point that keeps
 *                the cell mean (Zhang-Shu; four-point rule for WENO5, three-
 *                point (Simpson) rule for WENO3), or an a2 that would leave [0, 1]
 *                there, takes the cell value at both edges (first order for
 *                that variable); if an edge state then has (Gamma+1) p + Pi
 *                <= 0 the whole cell is first order;
 *   HLLC         Davis wave-speed estimates; the tie S* = 0 takes the left
 *                star state; the a2 flux is a2_K u_f with the face velocity
 *                u_f of the HLLC flux of a passive scalar;
 *   RK           2N-storage coefficients A = (0, -17/32, -32/27),
 *                B = (1/4, 8/9, 3/4);
 *   CFL          dt = cfl h / max_cells max_d (|u_d| + c), taken at the start
 *                of the step, kept for its three stages, clipped to land on T;
 *   boundary     zero-gradient (ghost = nearest cell of the box), periodic, or
 *                characteristic far field (Sec. 3.1, after Poinsot and Lele):
 *                ghost cells outside a domain side take the primitives of the
 *                nearest cell with the normal velocity and pressure changed
 *                so that the outgoing acoustic invariant p + s Z u_n
 *                (Z = rho c, s = +1 on the high side, -1 on the low side) is
 *                kept and the incoming one p - s Z u_n is moved a fraction
 *                beta = sigma h / L (sigma = 0.25, L = 1) towards its
 *                far-field value p_inf (fluid at rest); the upwind update of
 *                the boundary cell then relaxes its incoming invariant
 *                towards p_inf at the rate K = beta c / h = sigma c / L, the
 *                penalty rate of Poinsot and Lele at low Mach number;
 *   init         a2 = fraction of n_s^d midpoint sub-samples inside the union
 *                of bubbles; smoothstep pressure ramp from p_bubble to p_inf
 *                starting ramp_delta outside the cloud radius, width
 *                ramp_width;
 *   QoI          maximum cell pressure over the cells and over the time levels
 *                n = 0..steps, ties to the smallest flat index and then the
 *                earliest level.
 *
 * Built with -O2 -ffp-contract=off and no vector intrinsics.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>


typedef struct {
    int32_t ndim;      /* 1, 2 or 3 */
    int32_t n;         /* cells per side of the full unit domain */
    int32_t bc;        /* 0 = zero-gradient, 1 = periodic (box must be the domain),
                          2 = characteristic far field */
    int32_t n_sub;     /* sub-samples per axis for the initial volume fraction */
    double cfl;
    double gamma1, pc1, gamma2, pc2;   /* phase 1 = water, phase 2 = air */
    double rho1, rho2;                 /* initial phase densities */
    double p_bubble, p_inf;
    double center[3];
    double cloud_radius, ramp_delta, ramp_width;
    double weno_eps;
    int32_t weno_order; /* 5 (or 0) = WENO5, 3 = WENO3 */
    int32_t pad;
} orc_spec;

/* A box of cells [lo, lo+len) of the global grid, per axis. */
typedef struct {
    int32_t lo[3];
    int32_t len[3];
} orc_box;

typedef struct {
    double p_max;
    double x[3];
    double t_at_max;
    double t;          /* time reached */
    int64_t argmax;    /* flat global index (k*N + j)*N + i */
    int64_t steps;
    int32_t status;    /* 0 ok, 1 non-finite, 2 c^2 <= 0, 3 step cap */
    int32_t pad;
    /* the paper's other quantities of interest (Sec. 3.3) */
    double p_sensor;   /* max over time levels of the pressure sensor, eq. (sensor) */
    double t_p_sensor; /* its time */
    double gas_min;    /* min over time levels of the cloud gas-fraction sensor */
    double t_gas_min;  /* its time */
    double c_max;      /* max over time levels and cells of the sound speed */
    double peak_distance; /* distance of the p_max cell centre from the cloud centre */
} orc_qoi;

typedef struct {
    double s_max;      /* max_cells max_d(|u_d| + c) */
    double p_max;
    int64_t argmax;
    int64_t n_nonfinite;
    int64_t n_negc2;
    double c_max;      /* max_cells c */
    double p_ball;     /* sum of p over the cells of the pressure sensor's ball */
    double a2_ball;    /* sum of a2 over the cells of the gas sensor's ball */
    int64_t n_ball_p, n_ball_a;   /* their cell counts */
} orc_reduction;

/* ------------------------------------------------------------------ */
/* Equation of state (Sec. 2.1)                                        */
/* ------------------------------------------------------------------ */

static double mix_gamma(const orc_spec* s, double a2)
{
    return (1.0 - a2) / (s->gamma1 - 1.0) + a2 / (s->gamma2 - 1.0);
}

static double mix_pi(const orc_spec* s, double a2)
{
    return (1.0 - a2) * s->gamma1 * s->pc1 / (s->gamma1 - 1.0)
         + a2 * s->gamma2 * s->pc2 / (s->gamma2 - 1.0);
}

/* K of eq. (var_K), with rho_k c_k^2 = gamma_k (p + pc_k) for a stiffened
 * gas, evaluated at a cell centre with a2 clamped to [0, 1].
 * Reading where the paper is silent: a2 + K, the share of the mixture's
 * volume change taken by the gas (= a2 r1 / (a1 r2 + a2 r1)), is kept in
 * [0, 1].  The formula leaves that range only when a phase is below its
 * stiffened-gas range (p + pc_k < 0, e.g. a trace of gas in water under
 * tension), where its denominator a1 r2 + a2 r1 can vanish and K diverge;
 * there K is clamped so that a2 + K is 0 or 1.  K = 0 in pure phases and
 * where the denominator is exactly zero. */
double orc_k_coefficient(const orc_spec* s, double a2, double p)
{
    double a = a2 < 0.0 ? 0.0 : (a2 > 1.0 ? 1.0 : a2);
    double b = 1.0 - a;
    double rc1 = s->gamma1 * (p + s->pc1);
    double rc2 = s->gamma2 * (p + s->pc2);
    double den = b * rc2 + a * rc1;
    if (a == 0.0 || a == 1.0 || den == 0.0) return 0.0;
    double k = b * a * (rc1 - rc2) / den;
    if (a + k < 0.0) k = -a;
    else if (a + k > 1.0) k = 1.0 - a;
    return k;
}

/* Number of stored variables: a1r1, a2r2, ndim momenta, E, a2. */
static int nvars(int ndim) { return 4 + ndim; }

/* Primitive vector: a1r1, a2r2, u_1..u_d, p, a2 (same slot layout). */
void orc_cons_to_prim(const orc_spec* s, const double* q, double* w)
{
    int d = s->ndim;
    double rho = q[0] + q[1];
    double ke = 0.0;
    w[0] = q[0];
    w[1] = q[1];
    for (int m = 0; m < d; ++m) {
        w[2 + m] = q[2 + m] / rho;
        ke += q[2 + m] * w[2 + m];
    }
    double a2 = q[3 + d];
    w[2 + d] = (q[2 + d] - 0.5 * ke - mix_pi(s, a2)) / mix_gamma(s, a2);
    w[3 + d] = a2;
}

void orc_prim_to_cons(const orc_spec* s, const double* w, double* q)
{
    int d = s->ndim;
    double rho = w[0] + w[1];
    double ke = 0.0;
    q[0] = w[0];
    q[1] = w[1];
    for (int m = 0; m < d; ++m) {
        q[2 + m] = rho * w[2 + m];
        ke += rho * w[2 + m] * w[2 + m];
    }
    double a2 = w[3 + d];
    q[2 + d] = mix_gamma(s, a2) * w[2 + d] + mix_pi(s, a2) + 0.5 * ke;
    q[3 + d] = a2;
}

/* Frozen mixture sound speed squared. */
static double sound2(const orc_spec* s, double rho, double p, double a2)
{
    double g = mix_gamma(s, a2);
    return ((g + 1.0) * p + mix_pi(s, a2)) / (g * rho);
}

/* ------------------------------------------------------------------ */
/* WENO5 (Jiang-Shu) reconstruction of one primitive (Sec. 2.2)        */
/* ------------------------------------------------------------------ */

/* Value at the right edge of cell c from the cell averages a, b, c, d, e
 * (cells c-2 .. c+2).  The left-edge value of a cell is the same formula
 * applied to the mirrored stencil. */
double orc_weno5_right_edge(double a, double b, double c, double d, double e, double eps)
{
    double p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    double p1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    double p2 = (2.0 * c + 5.0 * d - e) / 6.0;
    double t;
    double b0, b1, b2;
    t = a - 2.0 * b + c;  b0 = 13.0 / 12.0 * t * t;
    t = a - 4.0 * b + 3.0 * c;  b0 += 0.25 * t * t;
    t = b - 2.0 * c + d;  b1 = 13.0 / 12.0 * t * t;
    t = b - d;  b1 += 0.25 * t * t;
    t = c - 2.0 * d + e;  b2 = 13.0 / 12.0 * t * t;
    t = 3.0 * c - 4.0 * d + e;  b2 += 0.25 * t * t;
    double w0 = 0.1 / ((eps + b0) * (eps + b0));
    double w1 = 0.6 / ((eps + b1) * (eps + b1));
    double w2 = 0.3 / ((eps + b2) * (eps + b2));
    return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

/* WENO3 (Jiang-Shu, two candidate stencils of two cells) value at the right
 * edge of cell c from the cell averages b, c, d (cells c-1 .. c+1): candidates
 * (3c - b)/2 and (c + d)/2 with ideal weights 1/3 and 2/3 and indicators
 * (c - b)^2 and (d - c)^2.  The left-edge value is the formula applied to the
 * mirrored stencil. */
double orc_weno3_right_edge(double b, double c, double d, double eps)
{
    double p0 = (3.0 * c - b) / 2.0;
    double p1 = (c + d) / 2.0;
    double b0 = (c - b) * (c - b);
    double b1 = (d - c) * (d - c);
    double w0 = (1.0 / 3.0) / ((eps + b0) * (eps + b0));
    double w1 = (2.0 / 3.0) / ((eps + b1) * (eps + b1));
    return (w0 * p0 + w1 * p1) / (w0 + w1);
}

/* ------------------------------------------------------------------ */
/* HLLC flux with the volume-fraction adaptation (Sec. 2.2)            */
/* ------------------------------------------------------------------ */

/* Face flux along axis `dir` between primitive states wl (left) and wr
 * (right).  Writes the nv-1 fluxes of the conserved components (a1r1, a2r2,
 * momenta, E) into f[0..nv-2], the a2 flux into f[nv-1] and the face velocity
 * into f[nv]. */
void orc_hllc(const orc_spec* s, int dir, const double* wl, const double* wr, double* f)
{
    int d = s->ndim;
    int nv = nvars(d);
    const double* w[2] = { wl, wr };
    double rho[2], un[2], p[2], a2[2], E[2], c[2];
    for (int k = 0; k < 2; ++k) {
        rho[k] = w[k][0] + w[k][1];
        un[k] = w[k][2 + dir];
        p[k] = w[k][2 + d];
        a2[k] = w[k][3 + d];
        double ke = 0.0;
        for (int m = 0; m < d; ++m) ke += w[k][2 + m] * w[k][2 + m];
        E[k] = mix_gamma(s, a2[k]) * p[k] + mix_pi(s, a2[k]) + 0.5 * rho[k] * ke;
        c[k] = sqrt(sound2(s, rho[k], p[k], a2[k]));
    }
    double sl = fmin(un[0] - c[0], un[1] - c[1]);
    double sr = fmax(un[0] + c[0], un[1] + c[1]);
    double ml = rho[0] * (sl - un[0]);
    double mr = rho[1] * (sr - un[1]);
    double ss = (p[1] - p[0] + ml * un[0] - mr * un[1]) / (ml - mr);

    /* physical flux of side k */
    double fk[2][8];
    for (int k = 0; k < 2; ++k) {
        fk[k][0] = w[k][0] * un[k];
        fk[k][1] = w[k][1] * un[k];
        for (int m = 0; m < d; ++m)
            fk[k][2 + m] = rho[k] * w[k][2 + m] * un[k] + (m == dir ? p[k] : 0.0);
        fk[k][2 + d] = (E[k] + p[k]) * un[k];
    }

    int side;          /* which side's state enters */
    double sk;         /* wave speed of the star jump taken, 0 for upwind */
    if (sl >= 0.0)      { side = 0; sk = 0.0; }
    else if (ss >= 0.0) { side = 0; sk = sl; }
    else if (sr >= 0.0) { side = 1; sk = sr; }
    else                { side = 1; sk = 0.0; }

    const double* ws = w[side];
    double Sk = side == 0 ? sl : sr;
    double chi = (Sk - un[side]) / (Sk - ss);
    for (int v = 0; v < nv - 1; ++v) f[v] = fk[side][v];
    if (sk != 0.0) {
        double qk[8], qs[8];
        qk[0] = ws[0];
        qk[1] = ws[1];
        for (int m = 0; m < d; ++m) qk[2 + m] = rho[side] * ws[2 + m];
        qk[2 + d] = E[side];
        qs[0] = chi * ws[0];
        qs[1] = chi * ws[1];
        for (int m = 0; m < d; ++m)
            qs[2 + m] = chi * rho[side] * (m == dir ? ss : ws[2 + m]);
        qs[2 + d] = chi * (E[side] + (ss - un[side]) * (rho[side] * ss + p[side] / (Sk - un[side])));
        for (int v = 0; v < nv - 1; ++v) f[v] = fk[side][v] + sk * (qs[v] - qk[v]);
        double uf = un[side] + sk * (chi - 1.0);
        f[nv - 1] = a2[side] * uf;
        f[nv] = uf;
    } else {
        f[nv - 1] = a2[side] * un[side];
        f[nv] = un[side];
    }
}

/* ------------------------------------------------------------------ */
/* Reconstruction of one cell along one axis with the positivity check */
/* ------------------------------------------------------------------ */

/* Relative size below which a negative partial density, or an excursion of
 * a2 outside [0, 1], is taken as round-off. */
#define ORC_ROUND_TOL 1e-12

/* Edge values of the centre cell c of the primitive stencil a, b, c, d, e
 * (cells c-2 .. c+2 along one axis; WENO3 reads b, c, d only): left edge into
 * wminus, right edge into wplus (either may be NULL).
 *   - each partial density keeps its reconstruction only if it is >= 0 at
 *     both edges and at the interior value that, with the two edges,
 *     reproduces the cell mean under the Gauss-Lobatto rule exact for the
 *     reconstruction's degree (Zhang-Shu positivity condition): the four-point
 *     rule for WENO5, (12 mean - left - right)/10, the three-point rule for
 *     WENO3, (6 mean - left - right)/4; up to round-off: ORC_ROUND_TOL times the
 *     phase's reference density (the initial rho_k) or the largest magnitude
 *     of that partial density in the stencil, whichever is larger; otherwise
 *     both its edges take the cell value;
 *   - a2 likewise keeps its reconstruction only if it lies in [0, 1] at the
 *     same three points, up to ORC_ROUND_TOL;
 *   - if an edge state then has (Gamma+1) p + Pi <= 0 (no positive c^2), all
 *     variables take the cell values (first order).
 * Replacing only the variable that fails keeps a decision taken on round-off
 * from moving the other edge values.  Returns 1 when any replacement was
 * made. */
int orc_cell_edges(const orc_spec* s, const double* a, const double* b, const double* c,
                   const double* d, const double* e, double eps, double* wminus, double* wplus)
{
    int nd = s->ndim;
    int nv = nvars(nd);
    double lm[8], lp[8];
    int third = s->weno_order == 3;
    for (int v = 0; v < nv; ++v) {
        if (third) {
            lp[v] = orc_weno3_right_edge(b[v], c[v], d[v], eps);
            lm[v] = orc_weno3_right_edge(d[v], c[v], b[v], eps);
        } else {
            lp[v] = orc_weno5_right_edge(a[v], b[v], c[v], d[v], e[v], eps);
            lm[v] = orc_weno5_right_edge(e[v], d[v], c[v], b[v], a[v], eps);
        }
    }
    int keep[8];
    for (int v = 0; v < nv; ++v) keep[v] = 1;
    /* each partial density on its own; round-off below the phase's scale
     * (its reference density, or the largest value in the stencil if that is
     * larger) does not count as negative */
    for (int v = 0; v < 2; ++v) {
        double big = v == 0 ? s->rho1 : s->rho2;
        big = fmax(big, fmax(fmax(fabs(a[v]), fabs(b[v])), fmax(fmax(fabs(c[v]), fabs(d[v])), fabs(e[v]))));
        double tol = -ORC_ROUND_TOL * big;
        double mid = third ? (6.0 * c[v] - lm[v] - lp[v]) / 4.0 : (12.0 * c[v] - lm[v] - lp[v]) / 10.0;
        if (!(lm[v] >= tol) || !(lp[v] >= tol) || !(mid >= tol)) keep[v] = 0;
    }
    /* the volume fraction */
    {
        int v = 3 + nd;
        double lo = -ORC_ROUND_TOL, hi = 1.0 + ORC_ROUND_TOL;
        double mid = third ? (6.0 * c[v] - lm[v] - lp[v]) / 4.0 : (12.0 * c[v] - lm[v] - lp[v]) / 10.0;
        if (!(lm[v] >= lo && lm[v] <= hi) || !(lp[v] >= lo && lp[v] <= hi) || !(mid >= lo && mid <= hi)) keep[v] = 0;
    }
    for (int v = 0; v < nv; ++v)
        if (!keep[v]) { lm[v] = c[v]; lp[v] = c[v]; }
    /* positive c^2 at both edges, else the whole cell is first order */
    int ok = 1;
    {
        const double* sides[2] = { lm, lp };
        for (int k = 0; k < 2; ++k) {
            double a2 = sides[k][3 + nd];
            double cc2 = (mix_gamma(s, a2) + 1.0) * sides[k][2 + nd] + mix_pi(s, a2);
            if (!(cc2 > 0.0)) ok = 0;
        }
    }
    for (int v = 0; v < nv; ++v) {
        if (wminus) wminus[v] = ok ? lm[v] : c[v];
        if (wplus) wplus[v] = ok ? lp[v] : c[v];
    }
    int nfb = 0;
    for (int v = 0; v < nv; ++v) nfb += !keep[v];
    return (nfb > 0) || !ok;
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    const orc_spec* s;
    orc_box box;
    int nv;
    int64_t ncell;
} grid;

static void grid_make(grid* g, const orc_spec* s, const orc_box* box)
{
    g->s = s;
    g->box = *box;
    for (int a = s->ndim; a < 3; ++a) { g->box.lo[a] = 0; g->box.len[a] = 1; }
    g->nv = nvars(s->ndim);
    g->ncell = (int64_t)g->box.len[0] * g->box.len[1] * g->box.len[2];
}

static int64_t cell_index(const grid* g, int i, int j, int k)
{
    return ((int64_t)k * g->box.len[1] + j) * g->box.len[0] + i;
}

/* Box-local index of a possibly out-of-box neighbour along one axis. */
static int ghost_map(const grid* g, int axis, int i)
{
    int n = g->box.len[axis];
    if (g->s->bc == 1) {
        i %= n;
        if (i < 0) i += n;
        return i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* ------------------------------------------------------------------ */
/* Characteristic far-field ghost state (Sec. 3.1)                     */
/* ------------------------------------------------------------------ */

#define ORC_NR_SIGMA 0.25

/* Ghost primitives g outside the domain side (axis, side = -1 low / +1 high)
 * from the primitives w of the nearest cell: the outgoing acoustic invariant
 * p + side Z u_n is kept and the incoming one Rm = p - side Z u_n moves to
 * Rm + beta (p_inf - Rm); solving the two for p and u_n gives
 * p_g = p + delta and u_n,g = u_n - side delta / Z with delta =
 * beta (p_inf - Rm) / 2.  Everything else is copied (zero gradient); so is
 * the whole state if (rho c)^2 is not positive. */
void orc_char_ghost(const orc_spec* s, int axis, int side, double beta, const double* w, double* g)
{
    int nd = s->ndim;
    int nv = nvars(nd);
    for (int v = 0; v < nv; ++v) g[v] = w[v];
    double rho = w[0] + w[1];
    double a2 = w[3 + nd];
    double p = w[2 + nd];
    double un = w[2 + axis];
    double G = mix_gamma(s, a2);
    double z2 = rho * ((G + 1.0) * p + mix_pi(s, a2)) / G;     /* (rho c)^2 */
    if (!(z2 > 0.0)) return;
    double Z = sqrt(z2);
    double Rm = p - side * Z * un;
    double delta = 0.5 * beta * (s->p_inf - Rm);
    g[2 + nd] = p + delta;
    g[2 + axis] = un - side * delta / Z;
}

/* beta of the characteristic boundary for this grid */
static double char_beta(const orc_spec* s)
{
    return ORC_NR_SIGMA / (double)s->n;
}

/* ------------------------------------------------------------------ */
/* Right-hand side L(U) (eq. (ode))                                    */
/* ------------------------------------------------------------------ */

/* U, Lout: [nv][ncell] for the box. */
void orc_rhs(const orc_spec* s, const orc_box* box, const double* U, double* Lout,
             int64_t* n_fallback)
{
    grid g;
    grid_make(&g, s, box);
    int d = s->ndim, nv = g.nv;
    int64_t nc = g.ncell;
    double eps = s->weno_eps;
    double h = 1.0 / (double)s->n;
    double* W = (double*)malloc(sizeof(double) * nv * nc);
    double* divu = (double*)calloc(nc, sizeof(double));
    int64_t nfb = 0;

    for (int64_t c = 0; c < nc; ++c) {
        double q[8], w[8];
        for (int v = 0; v < nv; ++v) q[v] = U[v * nc + c];
        orc_cons_to_prim(s, q, w);
        for (int v = 0; v < nv; ++v) W[v * nc + c] = w[v];
    }
    for (int64_t x = 0; x < (int64_t)nv * nc; ++x) Lout[x] = 0.0;

    int len[3] = { g.box.len[0], g.box.len[1], g.box.len[2] };
    for (int dir = 0; dir < d; ++dir) {
        int e[3] = { dir == 0, dir == 1, dir == 2 };
        /* faces i-1/2 for i = 0..len[dir], on every line along dir */
        int flen[3] = { len[0] + e[0], len[1] + e[1], len[2] + e[2] };
        for (int k = 0; k < flen[2]; ++k)
        for (int j = 0; j < flen[1]; ++j)
        for (int i = 0; i < flen[0]; ++i) {
            int pos[3] = { i, j, k };
            double st[7][8];    /* cells i-4 .. i+2 along dir */
            for (int o = 0; o < 7; ++o) {
                int cc[3] = { pos[0], pos[1], pos[2] };
                cc[dir] = ghost_map(&g, dir, pos[dir] - 4 + o);
                int64_t ci = cell_index(&g, cc[0], cc[1], cc[2]);
                for (int v = 0; v < nv; ++v) st[o][v] = W[v * nc + ci];
                /* a ghost outside a domain side under the far-field condition */
                int gi = g.box.lo[dir] + pos[dir] - 4 + o;
                if (s->bc == 2 && (gi < 0 || gi >= s->n)) {
                    double tmp[8];
                    orc_char_ghost(s, dir, gi < 0 ? -1 : 1, char_beta(s), st[o], tmp);
                    for (int v = 0; v < nv; ++v) st[o][v] = tmp[v];
                }
            }
            /* left state: right edge of cell i-1 (stencil slot 3);
             * right state: left edge of cell i (stencil slot 4) */
            double wl[8], wr[8];
            nfb += orc_cell_edges(s, st[1], st[2], st[3], st[4], st[5], eps, NULL, wl);
            nfb += orc_cell_edges(s, st[2], st[3], st[4], st[5], st[6], eps, wr, NULL);
            double f[9];
            orc_hllc(s, dir, wl, wr, f);
            /* scatter into the two adjacent cells inside the box */
            int lo[3] = { pos[0], pos[1], pos[2] };
            lo[dir] -= 1;
            if (lo[dir] >= 0) {
                int64_t ci = cell_index(&g, lo[0], lo[1], lo[2]);
                for (int v = 0; v < nv; ++v) Lout[v * nc + ci] -= f[v] / h;
                divu[ci] += f[nv] / h;
            }
            if (pos[dir] < len[dir]) {
                int64_t ci = cell_index(&g, pos[0], pos[1], pos[2]);
                for (int v = 0; v < nv; ++v) Lout[v * nc + ci] += f[v] / h;
                divu[ci] -= f[nv] / h;
            }
        }
    }
    /* volume-fraction source (a2 + K) div u, R_7 of eq. (system) */
    for (int64_t c = 0; c < nc; ++c) {
        double a2 = W[(3 + d) * nc + c];
        double p = W[(2 + d) * nc + c];
        Lout[(3 + d) * nc + c] += (a2 + orc_k_coefficient(s, a2, p)) * divu[c];
    }
    free(W);
    free(divu);
    if (n_fallback) *n_fallback = nfb;
}

/* ------------------------------------------------------------------ */
/* Low-storage RK3 step (Williamson 2N form, Gottlieb-Shu weights)     */
/* ------------------------------------------------------------------ */

static const double RK_A[3] = { 0.0, -17.0 / 32.0, -32.0 / 27.0 };
static const double RK_B[3] = { 0.25, 8.0 / 9.0, 0.75 };

void orc_rk_coefficients(double* a, double* b)
{
    for (int k = 0; k < 3; ++k) { a[k] = RK_A[k]; b[k] = RK_B[k]; }
}

/* One full time step of size dt; U is advanced in place. */
void orc_step(const orc_spec* s, const orc_box* box, double* U, double dt)
{
    grid g;
    grid_make(&g, s, box);
    int64_t n = (int64_t)g.nv * g.ncell;
    double* L = (double*)malloc(sizeof(double) * n);
    double* dU = (double*)calloc(n, sizeof(double));
    for (int k = 0; k < 3; ++k) {
        orc_rhs(s, box, U, L, NULL);
        for (int64_t x = 0; x < n; ++x) {
            dU[x] = RK_A[k] * dU[x] + dt * L[x];
            U[x] = U[x] + RK_B[k] * dU[x];
        }
    }
    free(L);
    free(dU);
}

/* ------------------------------------------------------------------ */
/* CFL / QoI reduction                                                 */
/* ------------------------------------------------------------------ */

/* Sensors (Sec. 3.3, eq. (sensor)): averages over the cells whose centres
 * lie in a ball around the cloud centre (midpoint rule for the ball
 * integral).  Reading: the pressure sensor's radius is the paper's 0.5 mm
 * against its 20 mm cloud, R_c / 40, but at least 1.01 half cell diagonals
 * (so that coarse grids average the 2^d cells around the centre instead of
 * none); the gas-fraction sensor's ball is the cloud's (radius R_c: the
 * paper's sensor containing the entire cloud). */
static double sensor_r2_p(const orc_spec* s)
{
    double h = 1.0 / (double)s->n;
    double r = s->cloud_radius / 40.0;
    double hd = 1.01 * 0.5 * h * sqrt((double)s->ndim);
    if (hd > r) r = hd;
    return r * r;
}

static double centre_dist2(const orc_spec* s, int64_t i, int64_t j, int64_t k)
{
    double N = (double)s->n;
    double dx = ((double)i + 0.5) / N - s->center[0];
    double d2 = dx * dx;
    if (s->ndim > 1) { double dy = ((double)j + 0.5) / N - s->center[1]; d2 = d2 + dy * dy; }
    if (s->ndim > 2) { double dz = ((double)k + 0.5) / N - s->center[2]; d2 = d2 + dz * dz; }
    return d2;
}

void orc_reduce(const orc_spec* s, const orc_box* box, const double* U, orc_reduction* r)
{
    grid g;
    grid_make(&g, s, box);
    int d = s->ndim, nv = g.nv;
    int64_t nc = g.ncell;
    int64_t N = s->n;
    r->s_max = 0.0;
    r->p_max = -INFINITY;
    r->argmax = -1;
    r->n_nonfinite = 0;
    r->n_negc2 = 0;
    r->c_max = 0.0;
    r->p_ball = 0.0;
    r->a2_ball = 0.0;
    r->n_ball_p = 0;
    r->n_ball_a = 0;
    const double r2p = sensor_r2_p(s), r2a = s->cloud_radius * s->cloud_radius;
    for (int k = 0; k < g.box.len[2]; ++k)
    for (int j = 0; j < g.box.len[1]; ++j)
    for (int i = 0; i < g.box.len[0]; ++i) {
        int64_t c = cell_index(&g, i, j, k);
        double q[8], w[8];
        int finite = 1;
        for (int v = 0; v < nv; ++v) {
            q[v] = U[v * nc + c];
            if (!isfinite(q[v])) finite = 0;
        }
        orc_cons_to_prim(s, q, w);
        double rho = q[0] + q[1];
        double p = w[2 + d];
        if (!isfinite(p)) finite = 0;
        if (!finite) { r->n_nonfinite++; continue; }
        double c2 = sound2(s, rho, p, w[3 + d]);
        if (!(rho > 0.0) || !(c2 > 0.0)) { r->n_negc2++; continue; }
        double cs = sqrt(c2);
        for (int m = 0; m < d; ++m) {
            double sp = fabs(w[2 + m]) + cs;
            if (sp > r->s_max) r->s_max = sp;
        }
        if (cs > r->c_max) r->c_max = cs;
        double d2 = centre_dist2(s, i + g.box.lo[0], j + g.box.lo[1], k + g.box.lo[2]);
        if (d2 <= r2p) { r->p_ball += p; r->n_ball_p++; }
        if (d2 <= r2a) { r->a2_ball += w[3 + d]; r->n_ball_a++; }
        int64_t gi = ((int64_t)(k + g.box.lo[2]) * N + (j + g.box.lo[1])) * N + (i + g.box.lo[0]);
        if (p > r->p_max || (p == r->p_max && gi < r->argmax)) {
            r->p_max = p;
            r->argmax = gi;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Initial state Q_0(x, omega) (Sec. 3.1)                              */
/* ------------------------------------------------------------------ */

/* bubbles: nb x 4 doubles (x, y, z, r); z ignored below 3-D. */
void orc_init(const orc_spec* s, const orc_box* box, const double* bubbles, int32_t nb, double* U)
{
    grid g;
    grid_make(&g, s, box);
    int d = s->ndim, nv = g.nv;
    int64_t nc = g.ncell;
    int64_t N = s->n;
    int ns = s->n_sub;
    int nsub_total = 1;
    for (int a = 0; a < d; ++a) nsub_total *= ns;
    double margin = 1e-9;
    int* list_k = (int*)malloc(sizeof(int) * (nb > 0 ? nb : 1));
    int* list_j = (int*)malloc(sizeof(int) * (nb > 0 ? nb : 1));
    int* list_i = (int*)malloc(sizeof(int) * (nb > 0 ? nb : 1));

    for (int k = 0; k < g.box.len[2]; ++k) {
        int gk = k + g.box.lo[2];
        /* bubbles whose z-extent touches this slab */
        int nk = 0;
        for (int b = 0; b < nb; ++b) {
            if (d < 3) { list_k[nk++] = b; continue; }
            double z0 = (double)gk / (double)N, z1 = (double)(gk + 1) / (double)N;
            const double* bb = bubbles + 4 * b;
            if (bb[2] + bb[3] < z0 - margin || bb[2] - bb[3] > z1 + margin) continue;
            list_k[nk++] = b;
        }
        for (int j = 0; j < g.box.len[1]; ++j) {
            int gj = j + g.box.lo[1];
            int nj = 0;
            for (int t = 0; t < nk; ++t) {
                int b = list_k[t];
                if (d < 2) { list_j[nj++] = b; continue; }
                double y0 = (double)gj / (double)N, y1 = (double)(gj + 1) / (double)N;
                const double* bb = bubbles + 4 * b;
                if (bb[1] + bb[3] < y0 - margin || bb[1] - bb[3] > y1 + margin) continue;
                list_j[nj++] = b;
            }
            for (int i = 0; i < g.box.len[0]; ++i) {
                int gi = i + g.box.lo[0];
                int ni = 0;
                double x0 = (double)gi / (double)N, x1 = (double)(gi + 1) / (double)N;
                for (int t = 0; t < nj; ++t) {
                    int b = list_j[t];
                    const double* bb = bubbles + 4 * b;
                    if (bb[0] + bb[3] < x0 - margin || bb[0] - bb[3] > x1 + margin) continue;
                    list_i[ni++] = b;
                }
                /* volume fraction by midpoint sub-sampling */
                int inside = 0;
                if (ni > 0) {
                    double den = (double)((int64_t)ns * N);
                    for (int sc = 0; sc < (d > 2 ? ns : 1); ++sc)
                    for (int sb = 0; sb < (d > 1 ? ns : 1); ++sb)
                    for (int sa = 0; sa < ns; ++sa) {
                        double px = ((double)((int64_t)ns * gi + sa) + 0.5) / den;
                        double py = ((double)((int64_t)ns * gj + sb) + 0.5) / den;
                        double pz = ((double)((int64_t)ns * gk + sc) + 0.5) / den;
                        for (int t = 0; t < ni; ++t) {
                            const double* bb = bubbles + 4 * list_i[t];
                            double dx = px - bb[0];
                            double r2 = dx * dx;
                            if (d > 1) { double dy = py - bb[1]; r2 = r2 + dy * dy; }
                            if (d > 2) { double dz = pz - bb[2]; r2 = r2 + dz * dz; }
                            if (r2 < bb[3] * bb[3]) { ++inside; break; }
                        }
                    }
                }
                double a2 = (double)inside / (double)nsub_total;
                /* pressure ramp around the cloud */
                double cx = ((double)gi + 0.5) / (double)N - s->center[0];
                double rr = cx * cx;
                if (d > 1) { double cy = ((double)gj + 0.5) / (double)N - s->center[1]; rr = rr + cy * cy; }
                if (d > 2) { double cz = ((double)gk + 0.5) / (double)N - s->center[2]; rr = rr + cz * cz; }
                double r = sqrt(rr);
                double sr = (r - s->cloud_radius - s->ramp_delta) / s->ramp_width;
                sr = sr < 0.0 ? 0.0 : (sr > 1.0 ? 1.0 : sr);
                double p = s->p_bubble + (s->p_inf - s->p_bubble) * (sr * sr * (3.0 - 2.0 * sr));
                double w[8];
                w[0] = (1.0 - a2) * s->rho1;
                w[1] = a2 * s->rho2;
                for (int m = 0; m < d; ++m) w[2 + m] = 0.0;
                w[2 + d] = p;
                w[3 + d] = a2;
                double q[8];
                orc_prim_to_cons(s, w, q);
                int64_t c = cell_index(&g, i, j, k);
                for (int v = 0; v < nv; ++v) U[v * nc + c] = q[v];
            }
        }
    }
    free(list_k);
    free(list_j);
    free(list_i);
}

/* ------------------------------------------------------------------ */
/* Time loop with QoI tracking                                         */
/* ------------------------------------------------------------------ */

static void cell_centre(const orc_spec* s, int64_t flat, double* x)
{
    int64_t N = s->n;
    int64_t i = flat % N, j = (flat / N) % N, k = flat / (N * N);
    x[0] = ((double)i + 0.5) / (double)N;
    x[1] = s->ndim > 1 ? ((double)j + 0.5) / (double)N : 0.0;
    x[2] = s->ndim > 2 ? ((double)k + 0.5) / (double)N : 0.0;
}

/* Advance U (box = whole domain) until t_end, or for exactly n_steps steps
 * when n_steps > 0.  max_steps caps the loop (status 3).  Returns the QoI. */
void orc_solve(const orc_spec* s, double* U, double t_end, int64_t n_steps,
               int64_t max_steps, orc_qoi* q)
{
    orc_box box = { { 0, 0, 0 }, { s->n, s->ndim > 1 ? s->n : 1, s->ndim > 2 ? s->n : 1 } };
    double h = 1.0 / (double)s->n;
    orc_reduction r;
    orc_reduce(s, &box, U, &r);
    q->status = 0;
    q->steps = 0;
    q->t = 0.0;
    q->p_max = r.p_max;
    q->argmax = r.argmax;
    q->t_at_max = 0.0;
    q->pad = 0;
    q->p_sensor = r.n_ball_p > 0 ? r.p_ball / (double)r.n_ball_p : 0.0;
    q->t_p_sensor = 0.0;
    q->gas_min = r.n_ball_a > 0 ? r.a2_ball / (double)r.n_ball_a : 0.0;
    q->t_gas_min = 0.0;
    q->c_max = r.c_max;
    if (r.n_nonfinite > 0) q->status = 1;
    else if (r.n_negc2 > 0) q->status = 2;
    double t = 0.0;
    while (q->status == 0) {
        if (n_steps > 0 ? q->steps >= n_steps : t >= t_end) break;
        if (q->steps >= max_steps) { q->status = 3; break; }
        double dt = s->cfl * h / r.s_max;
        int last = 0;
        if (n_steps <= 0 && dt >= t_end - t) { dt = t_end - t; last = 1; }
        orc_step(s, &box, U, dt);
        t = last ? t_end : t + dt;
        q->steps += 1;
        orc_reduce(s, &box, U, &r);
        if (r.n_nonfinite > 0) { q->status = 1; break; }
        if (r.n_negc2 > 0) { q->status = 2; break; }
        if (r.p_max > q->p_max) {
            q->p_max = r.p_max;
            q->argmax = r.argmax;
            q->t_at_max = t;
        }
        double ps = r.n_ball_p > 0 ? r.p_ball / (double)r.n_ball_p : 0.0;
        double gs = r.n_ball_a > 0 ? r.a2_ball / (double)r.n_ball_a : 0.0;
        if (ps > q->p_sensor) { q->p_sensor = ps; q->t_p_sensor = t; }
        if (gs < q->gas_min) { q->gas_min = gs; q->t_gas_min = t; }
        if (r.c_max > q->c_max) q->c_max = r.c_max;
    }
    q->t = t;
    cell_centre(s, q->argmax < 0 ? 0 : q->argmax, q->x);
    {
        double dd = 0.0;
        for (int a = 0; a < s->ndim; ++a) dd = dd + (q->x[a] - s->center[a]) * (q->x[a] - s->center[a]);
        q->peak_distance = sqrt(dd);
    }
}

/* Run exactly n_steps steps on the whole domain and report the time step
 * sizes used (dts[n_steps]); used by the parity tests of single steps. */
void orc_run_steps(const orc_spec* s, double* U, int64_t n_steps, double* dts)
{
    orc_box box = { { 0, 0, 0 }, { s->n, s->ndim > 1 ? s->n : 1, s->ndim > 2 ? s->n : 1 } };
    double h = 1.0 / (double)s->n;
    orc_reduction r;
    for (int64_t n = 0; n < n_steps; ++n) {
        orc_reduce(s, &box, U, &r);
        double dt = s->cfl * h / r.s_max;
        if (dts) dts[n] = dt;
        orc_step(s, &box, U, dt);
    }
}

/* Advance a sub-box with a prescribed sequence of time steps.  Cells within
 * 9*n_steps cells of a box side that is not a domain side are wrong (their
 * ghosts are not known); the rest is exact.  Used to check single cells of
 * large grids without solving the whole grid. */
void orc_box_steps(const orc_spec* s, const orc_box* box, const double* bubbles, int32_t nb,
                   int64_t n_steps, const double* dts, double* U)
{
    orc_init(s, box, bubbles, nb, U);
    for (int64_t n = 0; n < n_steps; ++n) orc_step(s, box, U, dts[n]);
}

/* Reduction over the whole domain of the initial state, without storing it
 * beyond one z-slab at a time (for grids too large to hold twice). */
void orc_initial_reduction(const orc_spec* s, const double* bubbles, int32_t nb, orc_reduction* r)
{
    int N = s->n;
    int nz = s->ndim > 2 ? N : 1;
    int ny = s->ndim > 1 ? N : 1;
    int nv = nvars(s->ndim);
    double* slab = (double*)malloc(sizeof(double) * nv * (int64_t)N * ny);
    r->s_max = 0.0;
    r->p_max = -INFINITY;
    r->argmax = -1;
    r->n_nonfinite = 0;
    r->n_negc2 = 0;
    r->c_max = 0.0;
    r->p_ball = 0.0;
    r->a2_ball = 0.0;
    r->n_ball_p = 0;
    r->n_ball_a = 0;
    for (int k = 0; k < nz; ++k) {
        orc_box b = { { 0, 0, k }, { N, ny, 1 } };
        orc_reduction rs;
        orc_init(s, &b, bubbles, nb, slab);
        orc_reduce(s, &b, slab, &rs);
        if (rs.s_max > r->s_max) r->s_max = rs.s_max;
        if (rs.p_max > r->p_max || (rs.p_max == r->p_max && rs.argmax < r->argmax)) {
            r->p_max = rs.p_max;
            r->argmax = rs.argmax;
        }
        r->n_nonfinite += rs.n_nonfinite;
        r->n_negc2 += rs.n_negc2;
        if (rs.c_max > r->c_max) r->c_max = rs.c_max;
        r->p_ball += rs.p_ball;
        r->a2_ball += rs.a2_ball;
        r->n_ball_p += rs.n_ball_p;
        r->n_ball_a += rs.n_ball_a;
    }
    free(slab);
}
