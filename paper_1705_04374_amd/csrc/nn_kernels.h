// Launchers of the set-network kernels (nn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace ofm {

// flat parameter layout (float): W1[128][4] b1[128] W2[128][128] b2[128]
// W3[128][128] b3[128] W4[5][128] b4[5]; W[out][in]
constexpr int NN_DIN = 4, NN_WIDTH = 128, NN_DOUT = 5;
constexpr int NN_W1 = 0;
constexpr int NN_B1 = NN_W1 + 128 * 4;
constexpr int NN_W2 = NN_B1 + 128;
constexpr int NN_B2 = NN_W2 + 128 * 128;
constexpr int NN_W3 = NN_B2 + 128;
constexpr int NN_B3 = NN_W3 + 128 * 128;
constexpr int NN_W4 = NN_B3 + 128;
constexpr int NN_B4 = NN_W4 + NN_DOUT * 128;
constexpr int NN_NPARAM = NN_B4 + NN_DOUT;

hipError_t nn_gemm(const uint16_t* A, bool a_km, const uint16_t* B, bool b_nk, float* C, int M, int N, int K, int lda,
                   int ldb, int splits, hipStream_t s);
int nn_gemm_splits(int K, int splits);
hipError_t nn_gemm_finish(const float* C, int splits, int64_t M, int N, int mode, const float* bias, const float* mask,
                          float* out, float* act, uint16_t* act_bf, hipStream_t s);
hipError_t nn_phi_pool(const float* x, const int32_t* offsets, int n_sets, const float* P, const uint16_t* W2bf,
                       float pool_scale, float* s_out, uint16_t* s_bf, uint16_t* h1_bf, float* z2, hipStream_t st);
hipError_t nn_head(const float* a3, const float* P, int n_sets, const float* mean, const float* stdv, float* y_phys,
                   const float* y_true, float* dy, float* sq, hipStream_t s);
hipError_t nn_head_back(const float* dy, const float* P, const float* z3, int n_sets, float* dz3, uint16_t* dz3_bf,
                        hipStream_t s);
hipError_t nn_dz2(const float* ds, const float* z2, const int32_t* offsets, int n_sets, int64_t rows, float pool_scale,
                  float* dz2, uint16_t* dz2_bf, hipStream_t s);
hipError_t nn_colsum(const float* in, int64_t rows, int cols, float* out, hipStream_t s);
hipError_t nn_dw4(const float* dy, const float* a3, int n_sets, float* g, hipStream_t s);
hipError_t nn_dw1(const float* dh1, const float* x, const float* P, int64_t rows, float* g, hipStream_t s);
hipError_t nn_loss(const float* sq, int n, float* loss, hipStream_t s);
hipError_t nn_adam(float* P, const float* G, float* m, float* v, float lr, float b1, float b2, float eps, int t,
                   uint16_t* W2bf, uint16_t* W3bf, hipStream_t s);
hipError_t nn_shadow(const float* P, uint16_t* W2bf, uint16_t* W3bf, hipStream_t s);
hipError_t nn_init_params(float* P, uint64_t seed, hipStream_t s);
hipError_t nn_features(const double* bub, int64_t rows, int ndim, const double* center, double R, double rmed,
                       double sigma, float* x, hipStream_t s);

}  // namespace ofm
