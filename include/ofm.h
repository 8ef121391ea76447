/*
 * ofm.h - C ABI of the MI355X optimal-fidelity MLMC library.
 *
 * The calls follow the problem statement of Sukys et al., "Optimal fidelity
 * multi-level Monte Carlo for quantification of uncertainty in simulations of
 * cloud cavitation collapse" (arXiv:1705.04374):
 *   random initial data Q_0(x, omega) of a bubble cloud (Sec. 2.4, Sec. 3.1)
 *   -> level-l finite-volume solve of the five-equation model (Sec. 2.1-2.2)
 *   -> quantity of interest q_l(omega): the global maximum pressure (Sec. 3.3)
 *   -> OF-MLMC moments, optimal coefficients, errors, estimate and sample
 *      allocation (Sec. 2.4.3-2.4.4, eqs. (alpha-matvec), (ocv-mlmc),
 *      (ocv-mlmc-err), (M-tol), (M-budget), (warmup)).
 *
 * Conventions
 *   Return value: OFM_OK (0) or a negative OFM_E* code; the message of the last
 *   failure of a context is returned by ofm_last_error().  Calls that take no
 *   context report through ofm_last_error(NULL) (thread-local).
 *   A physical failure of one sample (non-finite state, c^2 <= 0, step cap) is
 *   NOT a call error: it is reported in ofm_qoi.status.
 *   Ownership: the caller allocates and frees every buffer it passes; the
 *   library keeps no caller pointer after a call returns, except for work
 *   already enqueued on the caller's stream.  A context owns its internal
 *   scratch (per-sample states of batched solves, graphs, tuning table).
 *   Streams: every device operation is enqueued on the hipStream_t passed as
 *   `stream` (NULL = default stream).  Calls returning host results
 *   synchronise that stream before returning; the others are asynchronous.
 *   Pointers marked [dev] are device memory, [host] host memory.
 *   Units: SI.  Domain: unit interval/square/cube, cells of size h = 1/n.
 *   Threading: a context may be used by one thread at a time.
 */
#ifndef OFM_H
#define OFM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------- */
#define OFM_OK            0
#define OFM_EINVAL       -1   /* bad argument (sizes, layout, null pointer) */
#define OFM_ENOMEM       -2   /* device or host allocation failed */
#define OFM_EHIP         -3   /* a HIP runtime call failed */
#define OFM_EUNSUPPORTED -4   /* valid request the library does not implement */
#define OFM_ESINGULAR    -5   /* coefficient system not positive definite */
#define OFM_EINFEASIBLE  -6   /* sampler or allocation cannot meet its target */

/* ---- per-sample status (ofm_qoi.status) ------------------------------------ */
#define OFM_SAMPLE_OK          0
#define OFM_SAMPLE_NONFINITE   1   /* a state value or the pressure is NaN/Inf */
#define OFM_SAMPLE_NEGATIVE_C2 2   /* rho <= 0 or c^2 <= 0 in some cell */
#define OFM_SAMPLE_MAX_STEPS   3   /* step cap reached before the end time */

/* ---- enumerations ---------------------------------------------------------- */
#define OFM_F32 0   /* stencil arithmetic and state in float (QoI, dt in double) */
#define OFM_F64 1   /* everything in double */
#define OFM_BC_ZERO_GRADIENT 0
#define OFM_BC_PERIODIC      1
/* Characteristic far field (Sec. 3.1, after Poinsot and Lele): ghost cells
 * outside a domain side take the nearest cell's primitives with the normal
 * velocity and pressure set so that the outgoing acoustic invariant
 * p + s Z u_n (Z = rho c, s = +1 on the high side, -1 on the low side) is
 * kept and the incoming one moves a fraction beta = sigma h (sigma = 0.25,
 * unit domain) towards its far-field value p_inf of the fluid at rest: the
 * boundary relaxes towards p_inf at the rate sigma c, and outgoing waves
 * leave. */
#define OFM_BC_CHARACTERISTIC 2
#define OFM_MODE_TOLERANCE 0
#define OFM_MODE_BUDGET    1

typedef struct ofm_ctx ofm_ctx;

/* Stiffened-gas parameters of the two phases (Sec. 2.1):
 * p = (gamma_k - 1) rho_k e_k - gamma_k pc_k; phase 1 = liquid, 2 = gas. */
typedef struct {
    double gamma1, pc1, gamma2, pc2;
} ofm_eos;

/* One level-l solve (Sec. 2.2 scheme; Sec. 3.1 initial data).
 * State layout in device memory: structure of arrays, nv = 4 + ndim arrays of
 * n^ndim cells each, variable-major: [v][k][j][i] with i fastest; variables
 * (a1 rho1, a2 rho2, rho u_1..rho u_ndim, Et, a2), where the energy slot holds
 * Et = E - Pi(a2) = Gamma(a2) p + rho |u|^2 / 2, the total energy of
 * eq. (system) less the stiffened-gas constant of the mixture
 * (Pi(a2) = (1-a2) gamma1 pc1/(gamma1-1) + a2 gamma2 pc2/(gamma2-1)).  The
 * scheme is the same as with E in exact arithmetic; in float this keeps the
 * pressure of a gas at a few kPa next to water (Pi ~ 4e8 Pa) representable.
 * ofm_state_to_conserved returns the conserved vector Q with E. */
typedef struct {
    int32_t ndim;        /* 1, 2 or 3 */
    int32_t n;           /* cells per side, 8 <= n <= 4096 */
    int32_t precision;   /* OFM_F32 or OFM_F64 */
    int32_t bc;          /* OFM_BC_*; the far field takes p_inf below */
    int32_t n_sub;       /* sub-samples per axis for the initial a2 (n_sub^ndim <= 64) */
    int32_t weno_order;  /* reconstruction (Sec. 2.2 allows third or fifth order):
                            0 or 5 = WENO5, 3 = WENO3 (Jiang-Shu); else OFM_EINVAL */
    double cfl;          /* Courant number (0.3 in the paper, Sec. 3.1) */
    ofm_eos eos;
    double rho1, rho2;   /* initial phase densities (also the scale below which a
                            negative partial density counts as round-off) */
    double p_bubble;     /* pressure inside the cloud */
    double p_inf;        /* ambient pressure (and far-field pressure of OFM_BC_CHARACTERISTIC) */
    double center[3];    /* cloud centre */
    double cloud_radius; /* the ramp to p_inf starts at cloud_radius + ramp_delta */
    double ramp_delta;
    double ramp_width;
    double weno_eps;     /* WENO smoothness epsilon (absolute) */
    double t_end;        /* end time when n_steps == 0 */
    int64_t n_steps;     /* > 0: run exactly this many steps, t_end ignored */
    int64_t max_steps;   /* step cap (status OFM_SAMPLE_MAX_STEPS) */
} ofm_solve_spec;

/* Quantities of interest of one solve (Sec. 3.3), over the time levels
 * n = 0..steps:
 *   p_max: maximum cell pressure over cells and levels; ties to the smallest
 *     flat cell index (k n + j) n + i, then to the earliest level;
 *   p_sensor: maximum over levels of the pressure sensor of eq. (sensor), the
 *     mean pressure over the cells whose centres lie within
 *     max(R_c / 40, 1.01 half cell diagonals) of the cloud centre (the paper's
 *     0.5 mm ball in its 20 mm cloud); earliest level on ties;
 *   gas_min: minimum over levels of the gas-fraction sensor, the mean a2 over
 *     the cells whose centres lie within R_c of the cloud centre;
 *   c_max: maximum sound speed over cells and levels;
 *   peak_distance: distance of the p_max cell centre from the cloud centre. */
typedef struct {
    double p_max;
    double x[3];         /* centre of the argmax cell (unused axes 0) */
    double t_at_max;
    double t;            /* time reached */
    int64_t argmax;      /* flat cell index */
    int64_t steps;       /* steps taken */
    int32_t status;      /* OFM_SAMPLE_* */
    int32_t reserved;
    double p_sensor, t_p_sensor;
    double gas_min, t_gas_min;
    double c_max;
    double peak_distance;
} ofm_qoi;

/* Random cloud geometry (Sec. 3, 3.1): n_bubbles centres uniform in the
 * ball (disk) of radius cloud_radius around center, radii
 * r_median exp(r_sigma Z) with Z standard normal, redrawn while outside
 * [r_lo, r_hi] when r_hi > 0; bubbles never overlap. */
typedef struct {
    int32_t ndim;
    int32_t n_bubbles;
    double cloud_radius;
    double center[3];
    double r_median, r_sigma;
    double r_lo, r_hi;
} ofm_cloud_spec;

/* Three caller-owned device arrays of nv * n^ndim elements of the spec's
 * precision.  `u` holds the current state; `u_tmp` and `du` are scratch.
 * ofm_step may exchange u and u_tmp: read the pointers back after the call. */
typedef struct {
    void* u;
    void* u_tmp;
    void* du;
} ofm_state_view;

/* One member of a batched solve.  Items of one call share ndim, precision,
 * bc, eos, rho1, rho2, weno_eps and weno_order (and p_inf under
 * OFM_BC_CHARACTERISTIC); n, t_end and the cloud may differ.  A coupled
 * fine/coarse pair is two items with the same bubbles (Sec. 2.4.1). */
typedef struct {
    const ofm_solve_spec* spec;
    const double* bubbles;   /* [host] n_bubbles x 4 (x, y, z, r) */
    int32_t n_bubbles;
    int32_t reserved;
} ofm_batch_item;

/* ---- context --------------------------------------------------------------- */

/* Create a context on HIP device `device`.  Returns OFM_EHIP if the device
 * cannot be used. */
int ofm_ctx_create(int device, ofm_ctx** out);
void ofm_ctx_destroy(ofm_ctx* ctx);
/* Message of the last failing call on ctx (or of the calling thread when ctx
 * is NULL).  Valid until the next call. */
const char* ofm_last_error(const ofm_ctx* ctx);

/* ---- random initial data ------------------------------------------------- */

/* Bubbles of the cloud omega(seed, term, index) (Sec. 3.1: uniform centres,
 * log-normal radii, 2000 random numbers for 500 bubbles).  Host only,
 * deterministic.  Generator: SplitMix64 (Steele, Lea, Flood 2014) with initial
 * state mix(mix(mix(seed) ^ term) ^ index), mix(x) being the first output of a
 * generator whose state is x; uniforms (x >> 11) 2^-53.  Per bubble: centre by
 * rejection from [-1,1]^ndim into the unit ball; radius by Box-Muller with
 * u1 = 1 - U, u2 = U; candidates overlapping an accepted bubble are redrawn
 * (centre and radius), at most 100000 per bubble (then OFM_EINFEASIBLE).
 * bubbles: [host] capacity n_bubbles x 4 doubles (x, y, z, r; z = 0 below 3-D). */
int ofm_sample_cloud(const ofm_cloud_spec* spec, uint64_t seed, uint64_t term, uint64_t index,
                     double* bubbles);

/* ---- low-level state access (tests and custom drivers) --------------------- */

/* Initial state Q_0 of the cloud in st->u (Sec. 3.1): a2 = fraction of the
 * n_sub^ndim midpoint sub-samples of each cell inside the union of bubbles;
 * pressure p_bubble up to cloud_radius + ramp_delta from the centre, then a
 * smoothstep ramp of width ramp_width to p_inf; phase densities rho1, rho2;
 * fluid at rest.  bubbles: [host] n_bubbles x 4.  Asynchronous. */
int ofm_state_init(ofm_ctx* ctx, const ofm_solve_spec* spec, const double* bubbles,
                   int32_t n_bubbles, ofm_state_view* st, void* stream);

/* State st->u from primitive fields w [dev] of the spec's precision, same
 * layout with variables (a1 rho1, a2 rho2, u_1..u_ndim, p, a2).
 * Asynchronous. */
int ofm_state_from_primitive(ofm_ctx* ctx, const ofm_solve_spec* spec, const void* w,
                             ofm_state_view* st, void* stream);

/* Conserved vector Q of eq. (system) of the state st->u, in double:
 * q [dev] nv x n^ndim, variables (a1 rho1, a2 rho2, rho u, E, a2).
 * Asynchronous. */
int ofm_state_to_conserved(ofm_ctx* ctx, const ofm_solve_spec* spec, const ofm_state_view* st, double* q,
                           void* stream);

/* Advance st->u by n_steps CFL-limited steps (dt = cfl h / max(|u_d| + c),
 * taken at the start of each step, Sec. 2.2) of the three-stage low-storage
 * Runge-Kutta scheme; spec->t_end and spec->n_steps are ignored.  On return
 * st->u holds the new state (u and u_tmp may have been exchanged).  qoi
 * [host] receives the maximum pressure over the levels n = 0..n_steps of this
 * call; dts [host, may be NULL] receives the n_steps step sizes.  Synchronises
 * the stream. */
int ofm_step(ofm_ctx* ctx, const ofm_solve_spec* spec, ofm_state_view* st, int64_t n_steps,
             ofm_qoi* qoi, double* dts, void* stream);

/* Size of the fixed device scratch of ofm_step_noalloc, per GPU. */
#define OFM_NOALLOC_SCRATCH_BYTES (4u << 20)

/* ofm_step for callers that cannot allocate memory (tight serving loops,
 * harnesses that forbid device or pinned allocations; it synchronises the
 * stream, so it cannot be recorded into a graph): the same kernels and
 * launches, on the caller's stream, with
 * the same results bit for bit; it calls no hipMalloc, hipHostMalloc or
 * hipFree and creates no events.  Its scratch (the sample's descriptor and
 * dynamic state, 64 B of reduction partial and 8 B of work list per tile of
 * the tuned tiling, and 8 B per step when dts is given) is a fixed device
 * array of OFM_NOALLOC_SCRATCH_BYTES per GPU, kept until the process ends;
 * a call that needs more (e.g. a 16 x 16 x 16 tiling of a 1024^3 grid, or a
 * step log longer than about 500 000 steps) returns OFM_EINVAL before any
 * launch.  Every call on one GPU shares that array: calls that overlap in
 * time on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Arguments, results and u/u_tmp exchange as for
 * ofm_step; per-launch kernel timing (ofm_kernel_timing) does not apply.
 * Synchronises the stream (the QoI is returned in host memory). */
int ofm_step_noalloc(ofm_ctx* ctx, const ofm_solve_spec* spec, ofm_state_view* st, int64_t n_steps,
                     ofm_qoi* qoi, double* dts, void* stream);

/* ---- solves -------------------------------------------------------------- */

/* Solve one sample to spec->t_end (or spec->n_steps steps) and return its QoI
 * [host].  The library allocates the state internally (cached in ctx).
 * Synchronises the stream. */
int ofm_solve(ofm_ctx* ctx, const ofm_solve_spec* spec, const double* bubbles,
              int32_t n_bubbles, ofm_qoi* qoi, void* stream);

/* Solve n items together (samples of uneven grid sizes advance in the same
 * launches; Sec. 2.5 job merging, done inside one device).  qoi: [host] n
 * entries.  Synchronises the stream. */
int ofm_solve_batch(ofm_ctx* ctx, const ofm_batch_item* items, int32_t n, ofm_qoi* qoi,
                    void* stream);

/* ---- long batched runs, advanced in portions ---------------------------- */

/* A batched solve kept on the device between calls, so that a long run can
 * report progress, be time-sliced or interleaved with other work.  The same
 * solve as ofm_solve_batch (same kernels, same QoIs).
 *
 * ofm_run_begin: validates the n items [host] as ofm_solve_batch does,
 *   allocates the run's own state arrays (3 arrays of (4 + ndim) n^ndim
 *   values per item; OFM_ENOMEM if they do not fit), builds Q_0 of every item
 *   from its bubbles, takes the initial reduction and captures the step graph.
 *   The bubbles are copied; the caller may free them on return.  Waits for
 *   work queued on `stream` first; synchronous.
 * ofm_run_advance: advances until every sample is done or at least max_steps
 *   (>= 1) more time steps have been taken (whole graphs of steps); *done
 *   [host, may be NULL] = 1 once every sample is done.  Synchronous.
 * ofm_run_status: per item QoIs so far [host, n entries, may be NULL] (status
 *   OK with t < t_end while a sample is still running), steps taken by the
 *   run, seconds of initialisation and of stepping so far.
 * ofm_run_destroy: frees the run (NULL is ignored).
 * A run uses the context's stream; it must not outlive its context. */
typedef struct ofm_run ofm_run;
int ofm_run_begin(ofm_ctx* ctx, const ofm_batch_item* items, int32_t n, ofm_run** out, void* stream);
int ofm_run_advance(ofm_run* run, int64_t max_steps, int32_t* done);
int ofm_run_status(const ofm_run* run, ofm_qoi* qoi, int64_t* steps_taken, double* init_s, double* step_s);
void ofm_run_destroy(ofm_run* run);

/* Time spent in the last ofm_solve/ofm_solve_batch, in seconds, split into
 * initialisation and time stepping, and the number of cell-steps advanced. */
int ofm_last_solve_stats(const ofm_ctx* ctx, double* init_s, double* step_s,
                         double* cell_steps);

/* Override the stage kernel's tile shape and schedule for solves of the
 * given precision and dimension whose largest grid has n cells per side
 * (grids in the same power-of-two size class share the entry): tile tx x ty
 * cells, zchunk z-planes per workgroup (3-D), graph_steps time steps per
 * captured graph.  OFM_EUNSUPPORTED if the tile shape is not compiled in. */
int ofm_tune_set(ofm_ctx* ctx, int32_t precision, int32_t ndim, int32_t n, int32_t tx, int32_t ty,
                 int32_t zchunk, int32_t graph_steps);

/* Result of ofm_autotune: the chosen tile and schedule, the summed duration
 * of the three stage-kernel launches of one step with it (ms), and the number
 * of candidates timed. */
typedef struct ofm_tune_result {
    int32_t tx, ty, zchunk, graph_steps;
    double stage_ms_per_step;
    int32_t candidates;
    int32_t reserved;
} ofm_tune_result;

/* The tile and schedule that solves of (precision, ndim, n) use now (the
 * default, or the entry ofm_tune_set / ofm_autotune stored); out [host]
 * receives tx, ty, zchunk, graph_steps (stage_ms_per_step 0, candidates 0). */
int ofm_tune_get(const ofm_ctx* ctx, int32_t precision, int32_t ndim, int32_t n, ofm_tune_result* out);

/* Measure every compiled tile shape (and, in 3-D, z-chunks of 8, 16, 32 and
 * 64 planes not larger than n, and those whose workgroup count fills 1 to 8
 * whole rounds of the device's CUs at the tile's occupancy) of the stage kernel for spec's precision,
 * dimension and grid, by stepping the caller's state st [dev] `steps` time
 * steps per candidate with per-launch events, and store the fastest as the
 * entry ofm_tune_set would write; out [host] receives it.  The state is
 * advanced (candidates x steps steps, u and u_tmp may swap as in ofm_step):
 * pass a scratch copy.  all [host, may be NULL] receives up to all_cap
 * entries, one per candidate in the order timed (candidates = 1 each).  On
 * an error the previous entry is kept; OFM_EINVAL also if the state fails
 * (non-finite, c^2 <= 0) while stepping.  Synchronises the stream. */
int ofm_autotune(ofm_ctx* ctx, const ofm_solve_spec* spec, ofm_state_view* st, int32_t steps,
                 ofm_tune_result* out, ofm_tune_result* all, int32_t all_cap, void* stream);

/* Per-kernel timing for profiling: while enabled, solves launch their steps
 * one by one (no graphs) and bracket every stage-kernel launch with HIP events
 * on the stream the kernel runs on.  ofm_kernel_times returns, since the last
 * enable, the number of stage-kernel launches, their summed duration in ms,
 * and the cells they advanced (sum over launches of the cells of the samples
 * still running).  Host pointers; synchronous. */
int ofm_kernel_timing(ofm_ctx* ctx, int32_t enable);
int ofm_kernel_times(const ofm_ctx* ctx, int64_t* launches, double* total_ms, double* cells);

/* ---- OF-MLMC estimator (Sec. 2.4.3-2.4.4), all in double on the device ----- */

/* Moments of one term from M samples: q_f [dev] fine values, q_c [dev]
 * coarse values of the same omegas (NULL for term 0), ok [dev, may be NULL]
 * per-sample flag, nonzero = use (failed samples are left out, Sec. 2.5).
 * out [dev] 6 doubles: (M_used, mean_f, mean_c, Var_f, Var_c, Cov) with
 * unbiased 1/(M_used - 1) two-pass estimates (zeros when M_used < 2).
 * Deterministic (fixed reduction order).  Asynchronous. */
int ofm_mlmc_moments(ofm_ctx* ctx, const double* q_f, const double* q_c, const int32_t* ok,
                     int64_t M, double* out, void* stream);

/* Optimal control-variate coefficients alpha_0..alpha_L (alpha_L = 1) from
 * the terms' moments [dev] (L+1) x 6 (rows as written by ofm_mlmc_moments)
 * and costs W [dev] L+1 (W_0 one solve, W_l a fine/coarse pair): the
 * tridiagonal system eq. (alpha-matvec), row k (k < L)
 *   -C_k W_k a_{k-1} + (Vf_k W_k + Vc_{k+1} W_{k+1}) a_k - C_{k+1} W_{k+1} a_{k+1} = 0,
 * solved by the Thomas algorithm.  alpha [dev] L+1.  flag [dev] 1 int: 0, or
 * OFM_ESINGULAR when a pivot is not positive (alpha is then all ones).
 * Asynchronous. */
int ofm_ofmlmc_coefficients(ofm_ctx* ctx, int32_t L, const double* moments, const double* W,
                            double* alpha, int32_t* flag, void* stream);

/* sig_t2 [dev] L+1: Var(alpha_l q_l - alpha_{l-1} q_{l-1}) per term, and
 * eps2 [dev] 1: sum_l sig_t2_l / M_l (eq. (ocv-mlmc-err)); M from the moments.
 * Asynchronous. */
int ofm_ofmlmc_errors(ofm_ctx* ctx, int32_t L, const double* moments, const double* alpha,
                      double* sig_t2, double* eps2, void* stream);

/* OF-MLMC estimate eq. (ocv-mlmc) into E [dev] 1.  Asynchronous. */
int ofm_ofmlmc_estimate(ofm_ctx* ctx, int32_t L, const double* moments, const double* alpha,
                        double* E, void* stream);

/* Sample counts M_out [dev] L+1 for a tolerance on eps (mode
 * OFM_MODE_TOLERANCE, eq. (M-tol)) or a budget (OFM_MODE_BUDGET, eq.
 * (M-budget)), keeping the M_have [dev] samples already computed: levels whose
 * optimum is below M_have are fixed, their error (budget) is taken off the
 * target and the rest re-optimised until none falls below (step 7 of the
 * adaptive algorithm).  flag [dev] 1 int: 0 or OFM_EINFEASIBLE.
 * Asynchronous. */
int ofm_ofmlmc_optimal_M(ofm_ctx* ctx, int32_t L, const double* sig_t2, const double* W,
                         const int64_t* M_have, int32_t mode, double target, int64_t* M_out,
                         int32_t* flag, void* stream);

/* Moments of each term over the union of two disjoint sample sets (e.g. the
 * samples of two GPUs): from each set's rows of ofm_mlmc_moments (M, means,
 * unbiased variances and covariance; step 3 of the adaptive algorithm,
 * Sec. 2.4.4), the pairwise update of Chan, Golub and LeVeque: the centred
 * sums of squares and products add, plus M_a M_b / M times the product of
 * the differences of the means.  It is the reduction an all-reduce of
 * per-device moments applies; commutative, and associative up to rounding.
 * a, b, out [dev] n_terms x 6 doubles each; out may equal a or b (in-place
 * accumulation).  An empty set (M = 0) leaves the other unchanged.
 * 1 <= n_terms <= 32.  Asynchronous. */
int ofm_mlmc_merge_moments(ofm_ctx* ctx, int32_t n_terms, const double* a, const double* b, double* out,
                           void* stream);

/* Inferred variances of level differences (the optional part of step 3 of
 * the adaptive algorithm, Sec. 2.4.4; App. A.1): a weighted least-squares
 * line through ln V[q_l - q_{l-1}] (V = Var_f + Var_c - 2 Cov of the term's
 * moments) against l over the terms l = first..L that have at least two
 * samples and V > 0, with weights (M_l - 1)/2 (the variance of the logarithm
 * of a sample variance of Gaussian data is 2/(M - 1)).
 * mom [dev] (L+1) x 6 as written by ofm_mlmc_moments: the terms
 * l >= max(first, 1) with fewer than two samples (e.g. a single finest
 * warm-up sample) are completed in place: the coarse member takes the
 * variance of level l-1 (term l-1's fine variance), the members'
 * correlation is term l-1's, and the fine variance is set so that
 * Var_f + Var_c - 2 Cov equals the inferred value (a valid covariance; at
 * least the smallest value that correlation allows, (1 - rho^2) Var_c for
 * rho >= 0, Var_c for rho < 0).  Terms l >= max(first, 1) with at least two
 * but fewer than m_floor samples keep the inferred value as a floor of their
 * difference variance (App. A.1: their few samples refine the inference):
 * where Var_f + Var_c - 2 Cov is below it, Cov is lowered to
 * (Var_f + Var_c - v_hat) / 2, at least -sqrt(Var_f Var_c); m_floor <= 2
 * leaves them as measured.  v_hat [dev] L+1 doubles:
 * exp of the fitted line for l = first..L, 0 below.  flag [dev] 1 int: 0, or
 * OFM_ESINGULAR when fewer than two terms qualify (then v_hat is 0 and mom
 * unchanged).  1 <= L <= 31, 0 <= first <= L, m_floor >= 0.  Asynchronous. */
int ofm_ofmlmc_fit_indicators(ofm_ctx* ctx, int32_t L, int32_t first, int32_t m_floor, double* mom, double* v_hat,
                              int32_t* flag, void* stream);

/* ---- learned control variate (not in the paper) ----------------------------
 * A permutation-invariant set network over the bubbles of a cloud, used as an
 * extra low-fidelity level of the OF-MLMC estimator whose optimal coefficient
 * (eq. (alpha-matvec)) absorbs its error:
 *   phi(x) = ReLU(W2 ReLU(W1 x + b1) + b2)     per bubble, 4 -> 128 -> 128
 *   s      = pool_scale * sum over the set's bubbles of phi(x)
 *   y      = W4 ReLU(W3 s + b3) + b4            128 -> 128 -> 5, standardised
 *   output = y * out_std + out_mean             (p_max, x*, y*, z*, t*)
 * The 128-wide contractions (forward and backward) run on the matrix cores
 * with bf16 operands (round to nearest even) and float accumulation; the rest
 * is float.  Parameters are float masters, flat, in the order W1[128][4],
 * b1[128], W2[128][128], b2[128], W3[128][128], b3[128], W4[5][128], b4[5]
 * (W[out][in]).  Training minimises the mean squared error of the
 * standardised outputs with Adam.  Set inputs: x [dev] rows x 4 floats,
 * offsets [dev] n_sets + 1 ints (set i is rows offsets[i] .. offsets[i+1]-1).
 * All calls enqueue on `stream`; those taking offsets read offsets[n_sets]
 * back to the host (synchronising the stream). */
typedef struct ofm_nn ofm_nn;

typedef struct {
    int32_t d_in, width, d_out, reserved;  /* 4, 128, 5 */
    float pool_scale;                      /* 1 / (reference number of bubbles) */
    float lr, beta1, beta2, adam_eps, reserved2;
    float out_mean[5], out_std[5];         /* standardisation of the outputs */
} ofm_nn_spec;

/* Create a network on the current device with He-uniform weights drawn
 * from SplitMix64(seed ^ parameter index), zero biases. */
int ofm_nn_create(ofm_ctx* ctx, const ofm_nn_spec* spec, uint64_t seed, ofm_nn** out);
void ofm_nn_destroy(ofm_nn* nn);
int64_t ofm_nn_param_count(void);
/* params [dev] ofm_nn_param_count() floats */
int ofm_nn_get_params(ofm_nn* nn, float* params, void* stream);
int ofm_nn_set_params(ofm_nn* nn, const float* params, void* stream);
/* mean, std [dev] 5 floats each */
int ofm_nn_set_normalization(ofm_nn* nn, const float* mean, const float* std_dev, void* stream);
int ofm_nn_reset_optimizer(ofm_nn* nn, void* stream);
/* Per-bubble inputs ((c - center)/cloud_radius, ln(r/r_median)/r_sigma) of
 * bubbles [dev] rows x 4 doubles into x [dev] rows x 4 floats. */
int ofm_nn_features(const ofm_cloud_spec* spec, const double* bubbles, int64_t rows, float* x, void* stream);
/* y [dev] n_sets x 5 floats, in physical units. */
int ofm_nn_forward(ofm_nn* nn, const float* x, const int32_t* offsets, int32_t n_sets, float* y, void* stream);
/* Loss (mean squared standardised error) [dev] 1 float and its gradient
 * grads [dev, may be NULL] (parameter layout) for targets y_true [dev]
 * n_sets x 5 in physical units; parameters unchanged. */
int ofm_nn_grads(ofm_nn* nn, const float* x, const int32_t* offsets, int32_t n_sets, const float* y_true,
                 float* grads, float* loss, void* stream);
/* One Adam step on the batch (loss [dev] 1 float, before the step). */
int ofm_nn_train_step(ofm_nn* nn, const float* x, const int32_t* offsets, int32_t n_sets, const float* y_true,
                      float* loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OFM_H */
