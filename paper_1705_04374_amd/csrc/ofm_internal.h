// Internal types shared by the library's host driver and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ofm.h"

namespace ofm {

// Physical constants of one launch, in double; kernels convert to their T.
struct PhysD {
    double g1inv;      // 1 / (gamma1 - 1)
    double g2inv;      // 1 / (gamma2 - 1)
    double pi1;        // gamma1 pc1 / (gamma1 - 1)
    double pi2;        // gamma2 pc2 / (gamma2 - 1)
    double gamma1, pc1, gamma2, pc2;
    double eps;        // WENO epsilon
    double rho1, rho2; // reference phase densities
    double p_far;      // far-field pressure of the characteristic boundary
    int32_t order;     // WENO order: 5 or 3
    int32_t pad;
};

// Static description of one sample in a launch.
struct SampleDesc {
    void* buf[2];      // state ping-pong buffers, [nv][n^d]
    void* du;          // low-storage RK register, [nv][n^d]
    int32_t n;         // cells per side
    int32_t ntx, nty;  // tiles along x and y
    int32_t nzc;       // z-chunks
    int32_t tile0;     // first index of this sample's tiles in the partial array
    int32_t ntiles;    // tiles of this sample
    double h;          // 1 / n
    double cfl;
    double t_end;
    int64_t n_steps;   // > 0: fixed step count
    int64_t max_steps;
    double centre[3];  // cloud centre (sensors)
    double r2_p;       // squared radius of the pressure sensor's ball
    double r2_a;       // squared radius of the gas-fraction sensor's ball
};

// Dynamic state of one sample, advanced on the device.
struct SampleState {
    double t;
    double dt;         // step size of the next step
    double p_max;      // running QoI
    double t_at_max;
    int64_t argmax;
    int64_t steps;
    int32_t status;
    int32_t done;
    int32_t last;      // next step lands on t_end
    int32_t pad;
    double p_sensor, t_p_sensor;   // running max of the pressure sensor
    double gas_min, t_gas_min;     // running min of the gas-fraction sensor
    double c_max;                  // running max of the sound speed
};

// Per-tile partial of the CFL / QoI reduction.
struct TilePartial {
    double s_max;
    double p_max;
    int64_t argmax;
    int32_t n_nonfinite;
    int32_t n_negc2;
    double c_max;
    double p_ball, a2_ball;        // sums over the sensors' cells
    int32_t n_ball_p, n_ball_a;    // and their counts
};

// One (sample, tile) work item of a batched launch.
struct WorkItem {
    int32_t sample;
    int32_t tile;      // tile index within the sample: (zc * nty + ty) * ntx + tx
};

struct LaunchArgs {
    PhysD ph;
    const WorkItem* work;
    int32_t n_work;
    int32_t zchunk;
    const SampleDesc* desc;
    SampleState* state;
    TilePartial* part;
    int32_t src;       // input buffer index
    int32_t bc;
};

}  // namespace ofm
