// C ABI of the learned control variate: parameters, Adam state and
// workspaces live in an ofm_nn; every computation is a kernel of
// nn_kernels.hip enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "nn_kernels.h"
#include "ofm.h"
#include "ofm_error.h"

struct ofm_nn {
    int device = 0;
    ofm_nn_spec spec;
    float* P = nullptr;       // parameters (float masters)
    float* G = nullptr;       // gradients
    float* m = nullptr;       // Adam moments
    float* v = nullptr;
    uint16_t* W2bf = nullptr; // bf16 shadows of the matrix-core operands
    uint16_t* W3bf = nullptr;
    float* norm = nullptr;    // out_mean[5], out_std[5]
    int t = 0;
    char* ws = nullptr;
    size_t ws_bytes = 0;
};

namespace {

using namespace ofm;

#define NNCHK(call)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(nullptr, OFM_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct WS {
    float *s, *z3, *a3, *y, *dy, *sq, *C, *z2, *dz2, *dh1, *dz3, *ds;
    uint16_t *s_bf, *h1_bf, *dz2_bf, *dz3_bf;
};

int workspace(ofm_nn* nn, int64_t rows, int sets, bool train, WS& w)
{
    size_t off = 0;
    size_t o_s = off; off += al(sizeof(float) * sets * 128);
    size_t o_sbf = off; off += al(2 * (size_t)sets * 128);
    size_t o_z3 = off; off += al(sizeof(float) * sets * 128);
    size_t o_a3 = off; off += al(sizeof(float) * sets * 128);
    size_t o_y = off; off += al(sizeof(float) * sets * NN_DOUT);
    size_t o_dy = off; off += al(sizeof(float) * sets * NN_DOUT);
    size_t o_sq = off; off += al(sizeof(float) * sets * NN_DOUT);
    const int sp_w = nn_gemm_splits((int)std::max<int64_t>(rows, sets), (int)std::max<int64_t>(1, std::max<int64_t>(rows, sets) / 4096));
    const size_t cN = std::max<size_t>({ (size_t)sets * 128, (size_t)sp_w * 128 * 128, train ? (size_t)rows * 128 : 0 });
    size_t o_C = off; off += al(sizeof(float) * cN);
    size_t o_z2 = off, o_dz2 = off, o_dh1 = off, o_dz3 = off, o_ds = off, o_h1 = off, o_dz2bf = off, o_dz3bf = off;
    if (train) {
        o_z2 = off; off += al(sizeof(float) * rows * 128);
        o_dz2 = off; off += al(sizeof(float) * rows * 128);
        o_dh1 = off; off += al(sizeof(float) * rows * 128);
        o_h1 = off; off += al(2 * (size_t)rows * 128);
        o_dz2bf = off; off += al(2 * (size_t)rows * 128);
        o_dz3 = off; off += al(sizeof(float) * sets * 128);
        o_ds = off; off += al(sizeof(float) * sets * 128);
        o_dz3bf = off; off += al(2 * (size_t)sets * 128);
    }
    if (off > nn->ws_bytes) {
        if (nn->ws) (void)hipFree(nn->ws);
        nn->ws = nullptr;
        nn->ws_bytes = 0;
        if (hipMalloc((void**)&nn->ws, off) != hipSuccess) {
            (void)hipGetLastError();
            return fail(nullptr, OFM_ENOMEM, "surrogate workspace of %zu bytes", off);
        }
        nn->ws_bytes = off;
    }
    char* b = nn->ws;
    w.s = (float*)(b + o_s); w.s_bf = (uint16_t*)(b + o_sbf); w.z3 = (float*)(b + o_z3); w.a3 = (float*)(b + o_a3);
    w.y = (float*)(b + o_y); w.dy = (float*)(b + o_dy); w.sq = (float*)(b + o_sq); w.C = (float*)(b + o_C);
    w.z2 = (float*)(b + o_z2); w.dz2 = (float*)(b + o_dz2); w.dh1 = (float*)(b + o_dh1); w.h1_bf = (uint16_t*)(b + o_h1);
    w.dz2_bf = (uint16_t*)(b + o_dz2bf); w.dz3 = (float*)(b + o_dz3); w.ds = (float*)(b + o_ds);
    w.dz3_bf = (uint16_t*)(b + o_dz3bf);
    return OFM_OK;
}

int check_sets(const float* x, const int32_t* off, int32_t n_sets, int64_t rows)
{
    if (!x || !off || n_sets < 1 || rows < 1) return fail(nullptr, OFM_EINVAL, "surrogate: bad inputs");
    return OFM_OK;
}

// forward through the head; train = also keep what the backward pass needs
int forward(ofm_nn* nn, const float* x, const int32_t* off, int32_t S, int64_t R, WS& w, bool train, hipStream_t s)
{
    NNCHK(nn_phi_pool(x, off, S, nn->P, nn->W2bf, nn->spec.pool_scale, w.s, w.s_bf, train ? w.h1_bf : nullptr,
                      train ? w.z2 : nullptr, s));
    NNCHK(nn_gemm(w.s_bf, false, nn->W3bf, true, w.C, S, 128, 128, 128, 128, 1, s));
    NNCHK(nn_gemm_finish(w.C, 1, S, 128, 1, nn->P + NN_B3, nullptr, w.z3, w.a3, nullptr, s));
    (void)R;
    return OFM_OK;
}

int backward(ofm_nn* nn, const float* x, const int32_t* off, int32_t S, int64_t R, const float* y_true, WS& w,
             float* loss, hipStream_t s)
{
    NNCHK(nn_head(w.a3, nn->P, S, nn->norm, nn->norm + 5, nullptr, y_true, w.dy, w.sq, s));
    NNCHK(nn_loss(w.sq, S * NN_DOUT, loss, s));
    NNCHK(nn_dw4(w.dy, w.a3, S, nn->G, s));
    NNCHK(nn_colsum(w.dy, S, NN_DOUT, nn->G + NN_B4, s));
    NNCHK(nn_head_back(w.dy, nn->P, w.z3, S, w.dz3, w.dz3_bf, s));
    NNCHK(nn_colsum(w.dz3, S, 128, nn->G + NN_B3, s));
    // dW3 = dz3^T s  (K = sets)
    int sp = nn_gemm_splits(S, std::max(1, S / 4096));
    NNCHK(nn_gemm(w.dz3_bf, true, w.s_bf, false, w.C, 128, 128, S, 128, 128, std::max(1, S / 4096), s));
    NNCHK(nn_gemm_finish(w.C, sp, 128, 128, 0, nullptr, nullptr, nn->G + NN_W3, nullptr, nullptr, s));
    // ds = dz3 W3
    NNCHK(nn_gemm(w.dz3_bf, false, nn->W3bf, false, w.C, S, 128, 128, 128, 128, 1, s));
    NNCHK(nn_gemm_finish(w.C, 1, S, 128, 0, nullptr, nullptr, w.ds, nullptr, nullptr, s));
    NNCHK(nn_dz2(w.ds, w.z2, off, S, R, nn->spec.pool_scale, w.dz2, w.dz2_bf, s));
    NNCHK(nn_colsum(w.dz2, R, 128, nn->G + NN_B2, s));
    // dW2 = dz2^T h1 (K = rows, split)
    const int want = (int)std::max<int64_t>(1, R / 4096);
    sp = nn_gemm_splits((int)R, want);
    NNCHK(nn_gemm(w.dz2_bf, true, w.h1_bf, false, w.C, 128, 128, (int)R, 128, 128, want, s));
    NNCHK(nn_gemm_finish(w.C, sp, 128, 128, 0, nullptr, nullptr, nn->G + NN_W2, nullptr, nullptr, s));
    // dh1 = dz2 W2
    NNCHK(nn_gemm(w.dz2_bf, false, nn->W2bf, false, w.C, (int)R, 128, 128, 128, 128, 1, s));
    NNCHK(nn_gemm_finish(w.C, 1, R, 128, 0, nullptr, nullptr, w.dh1, nullptr, nullptr, s));
    NNCHK(nn_dw1(w.dh1, x, nn->P, R, nn->G, s));
    return OFM_OK;
}

int64_t rows_of(const int32_t* off_dev, int32_t n_sets, hipStream_t s)
{
    int32_t last = 0;
    if (hipMemcpyAsync(&last, off_dev + n_sets, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    return last;
}

}  // namespace

extern "C" {

int ofm_nn_create(ofm_ctx* ctx, const ofm_nn_spec* spec, uint64_t seed, ofm_nn** out)
{
    if (!ctx || !spec || !out) return fail(nullptr, OFM_EINVAL, "ofm_nn_create: null argument");
    if (spec->d_in != 4 || spec->width != 128 || spec->d_out != 5)
        return fail(nullptr, OFM_EUNSUPPORTED, "ofm_nn_create: only the 4 -> 128 -> 128 / 128 -> 128 -> 5 network");
    *out = nullptr;
    ofm_nn* nn = new ofm_nn();
    nn->spec = *spec;
    (void)hipGetDevice(&nn->device);
    const size_t pb = sizeof(float) * NN_NPARAM;
    if (hipMalloc((void**)&nn->P, pb) != hipSuccess || hipMalloc((void**)&nn->G, pb) != hipSuccess ||
        hipMalloc((void**)&nn->m, pb) != hipSuccess || hipMalloc((void**)&nn->v, pb) != hipSuccess ||
        hipMalloc((void**)&nn->W2bf, 2 * 128 * 128) != hipSuccess ||
        hipMalloc((void**)&nn->W3bf, 2 * 128 * 128) != hipSuccess || hipMalloc((void**)&nn->norm, sizeof(float) * 10) != hipSuccess) {
        (void)hipGetLastError();
        ofm_nn_destroy(nn);
        return fail(nullptr, OFM_ENOMEM, "ofm_nn_create: allocation failed");
    }
    float nrm[10];
    for (int o = 0; o < 5; ++o) { nrm[o] = spec->out_mean[o]; nrm[5 + o] = spec->out_std[o] > 0.f ? spec->out_std[o] : 1.f; }
    if (hipMemcpy(nn->norm, nrm, sizeof nrm, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(nn->m, 0, pb) != hipSuccess || hipMemset(nn->v, 0, pb) != hipSuccess ||
        nn_init_params(nn->P, seed, nullptr) != hipSuccess || nn_shadow(nn->P, nn->W2bf, nn->W3bf, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        ofm_nn_destroy(nn);
        return fail(nullptr, OFM_EHIP, "ofm_nn_create: initialisation failed");
    }
    *out = nn;
    return OFM_OK;
}

void ofm_nn_destroy(ofm_nn* nn)
{
    if (!nn) return;
    (void)hipDeviceSynchronize();
    for (void* p : { (void*)nn->P, (void*)nn->G, (void*)nn->m, (void*)nn->v, (void*)nn->W2bf, (void*)nn->W3bf,
                     (void*)nn->norm, (void*)nn->ws })
        if (p) (void)hipFree(p);
    delete nn;
}

int64_t ofm_nn_param_count(void) { return NN_NPARAM; }

int ofm_nn_get_params(ofm_nn* nn, float* params, void* stream)
{
    if (!nn || !params) return fail(nullptr, OFM_EINVAL, "ofm_nn_get_params: null argument");
    NNCHK(hipMemcpyAsync(params, nn->P, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return OFM_OK;
}

int ofm_nn_set_params(ofm_nn* nn, const float* params, void* stream)
{
    if (!nn || !params) return fail(nullptr, OFM_EINVAL, "ofm_nn_set_params: null argument");
    hipStream_t s = (hipStream_t)stream;
    NNCHK(hipMemcpyAsync(nn->P, params, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToDevice, s));
    NNCHK(nn_shadow(nn->P, nn->W2bf, nn->W3bf, s));
    return OFM_OK;
}

int ofm_nn_set_normalization(ofm_nn* nn, const float* mean, const float* stdv, void* stream)
{
    if (!nn || !mean || !stdv) return fail(nullptr, OFM_EINVAL, "ofm_nn_set_normalization: null argument");
    hipStream_t s = (hipStream_t)stream;
    NNCHK(hipMemcpyAsync(nn->norm, mean, sizeof(float) * 5, hipMemcpyDeviceToDevice, s));
    NNCHK(hipMemcpyAsync(nn->norm + 5, stdv, sizeof(float) * 5, hipMemcpyDeviceToDevice, s));
    return OFM_OK;
}

int ofm_nn_reset_optimizer(ofm_nn* nn, void* stream)
{
    if (!nn) return fail(nullptr, OFM_EINVAL, "ofm_nn_reset_optimizer: null argument");
    hipStream_t s = (hipStream_t)stream;
    NNCHK(hipMemsetAsync(nn->m, 0, sizeof(float) * NN_NPARAM, s));
    NNCHK(hipMemsetAsync(nn->v, 0, sizeof(float) * NN_NPARAM, s));
    nn->t = 0;
    return OFM_OK;
}

int ofm_nn_features(const ofm_cloud_spec* spec, const double* bubbles, int64_t rows, float* x, void* stream)
{
    if (!spec || !bubbles || !x || rows < 1) return fail(nullptr, OFM_EINVAL, "ofm_nn_features: bad arguments");
    if (!(spec->cloud_radius > 0.0) || !(spec->r_median > 0.0) || !(spec->r_sigma > 0.0))
        return fail(nullptr, OFM_EINVAL, "ofm_nn_features: bad cloud spec");
    NNCHK(nn_features(bubbles, rows, spec->ndim, spec->center, spec->cloud_radius, spec->r_median, spec->r_sigma, x,
                      (hipStream_t)stream));
    return OFM_OK;
}

int ofm_nn_forward(ofm_nn* nn, const float* x, const int32_t* offsets, int32_t n_sets, float* y, void* stream)
{
    if (!nn || !y) return fail(nullptr, OFM_EINVAL, "ofm_nn_forward: null argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t R = rows_of(offsets, n_sets, s);
    int rc = check_sets(x, offsets, n_sets, R);
    if (rc) return rc;
    WS w;
    rc = workspace(nn, R, n_sets, false, w);
    if (rc) return rc;
    rc = forward(nn, x, offsets, n_sets, R, w, false, s);
    if (rc) return rc;
    NNCHK(nn_head(w.a3, nn->P, n_sets, nn->norm, nn->norm + 5, y, nullptr, nullptr, nullptr, s));
    return OFM_OK;
}

int ofm_nn_grads(ofm_nn* nn, const float* x, const int32_t* offsets, int32_t n_sets, const float* y_true,
                 float* grads, float* loss, void* stream)
{
    if (!nn || !y_true || !loss) return fail(nullptr, OFM_EINVAL, "ofm_nn_grads: null argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t R = rows_of(offsets, n_sets, s);
    int rc = check_sets(x, offsets, n_sets, R);
    if (rc) return rc;
    WS w;
    rc = workspace(nn, R, n_sets, true, w);
    if (rc) return rc;
    rc = forward(nn, x, offsets, n_sets, R, w, true, s);
    if (rc) return rc;
    rc = backward(nn, x, offsets, n_sets, R, y_true, w, loss, s);
    if (rc) return rc;
    if (grads) NNCHK(hipMemcpyAsync(grads, nn->G, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToDevice, s));
    return OFM_OK;
}

int ofm_nn_train_step(ofm_nn* nn, const float* x, const int32_t* offsets, int32_t n_sets, const float* y_true,
                      float* loss, void* stream)
{
    int rc = ofm_nn_grads(nn, x, offsets, n_sets, y_true, nullptr, loss, stream);
    if (rc) return rc;
    nn->t += 1;
    NNCHK(nn_adam(nn->P, nn->G, nn->m, nn->v, nn->spec.lr, nn->spec.beta1, nn->spec.beta2, nn->spec.adam_eps, nn->t,
                  nn->W2bf, nn->W3bf, (hipStream_t)stream));
    return OFM_OK;
}

}  // extern "C"
