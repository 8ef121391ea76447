// Launchers of the solver kernels (flow_kernels.hip).
#pragma once

#include "ofm_internal.h"

namespace ofm {

struct InitLaunch {
    PhysD ph;
    const double* bubbles;   // [dev] nb x 4
    int32_t nb;
    int32_t n, n_sub;
    double rho1, rho2, p_bubble, p_inf;
    double center[3];
    double radius, delta, width;
    void* u;                 // [dev] output state
};

bool tile_supported(int precision, int ndim, int tx, int ty);
// compiled tile shapes of (precision, ndim): up to cap (tx, ty) pairs; returns the count
int tile_list(int precision, int ndim, int (*out)[2], int cap);
hipError_t launch_stage(int precision, int ndim, int tx, int ty, const LaunchArgs& a, int stage, hipStream_t s);
// workgroups of the (third-stage) stage kernel of a tile that fit on one CU
// at once (0 if unknown)
int stage_blocks_per_cu(int precision, int ndim, int tx, int ty, int order);
hipError_t launch_reduce(int precision, int ndim, int tx, int ty, const LaunchArgs& a, hipStream_t s);
hipError_t launch_finalize(const SampleDesc* desc, SampleState* state, const TilePartial* part, int n_samples,
                           int initial, double* dt_log, int64_t dt_log_len, hipStream_t s);
hipError_t launch_init(int precision, int ndim, const InitLaunch& L, hipStream_t s);
hipError_t launch_to_conserved(int precision, int ndim, const PhysD& ph, const void* u, double* q, int64_t ncell,
                               hipStream_t s);
hipError_t launch_prim_to_cons(int precision, int ndim, const PhysD& ph, const void* w, void* u, int64_t ncell,
                               hipStream_t s);

// estimator (mlmc_kernels.hip)
hipError_t launch_moments(const double* qf, const double* qc, const int32_t* ok, int64_t M, double* out,
                          hipStream_t s);
hipError_t launch_coefficients(int L, const double* mom, const double* W, double* alpha, int32_t* flag,
                               hipStream_t s);
hipError_t launch_errors(int L, const double* mom, const double* alpha, double* sig, double* eps2, hipStream_t s);
hipError_t launch_estimate(int L, const double* mom, const double* alpha, double* E, hipStream_t s);
hipError_t launch_fit(int L, int first, int m_floor, double* mom, double* vhat, int32_t* flag, hipStream_t s);
hipError_t launch_merge(int n_terms, const double* a, const double* b, double* out, hipStream_t s);
hipError_t launch_optimal_M(int L, const double* sig, const double* W, const int64_t* have, int mode,
                            double target, int64_t* out, int32_t* flag, hipStream_t s);

}  // namespace ofm
