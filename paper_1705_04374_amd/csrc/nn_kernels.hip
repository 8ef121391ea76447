// Learned low-fidelity level: a permutation-invariant set network
//   phi(x) = ReLU(W2 ReLU(W1 x + b1) + b2)     per bubble, 4 -> 128 -> 128
//   s      = pool_scale * sum_bubbles phi(x)
//   y      = W4 ReLU(W3 s + b3) + b4            128 -> 128 -> 5
// trained on the solver's QoIs and used as an extra control variate of the
// OF-MLMC estimator (its coefficient from eq. (alpha-matvec) absorbs its
// error).
//
// The three 128-wide contractions (and their backward products) run on the
// matrix cores: bf16 operands (round to nearest even from float), float
// accumulation, v_mfma_f32_32x32x16_bf16.  The 4-wide input layer, the
// 5-wide output layer, pooling, loss and Adam are plain vector code in float.
// Every reduction has a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "nn_kernels.h"

namespace ofm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
struct alignas(16) u16x8 { uint16_t v[8]; };

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 frag(const uint16_t* p)
{
    u16x8 t = *reinterpret_cast<const u16x8*>(p);
    return __builtin_bit_cast(bf16x8, t);
}

// Output element e (0..15) of a 32x32 MFMA block held by `lane`: column
// lane % 32, row (e / 4) * 8 + (lane / 32) * 4 + e % 4.
__device__ __forceinline__ int mfma_row(int e, int lane) { return (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3); }

// ---------------------------------------------------------------------------
// Generic bf16 GEMM, C[split][M][N] = A[M x Ksplit] B[Ksplit x N], float out.
// A(m, k) = A_KM ? A[k lda + m] : A[m lda + k];  B(k, n) = B_NK ? B[n ldb + k] : B[k ldb + n].
// Workgroup tile 128 x 128, k-step 32, four waves of 64 x 64 (2 x 2 MFMA blocks).
// ---------------------------------------------------------------------------
constexpr int GT = 128, GK = 32, GP = GK + 8;   // LDS row pitch keeps 16-byte fragments aligned

template <bool A_KM, bool B_NK>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                                                        float* __restrict__ C, int M, int N, int K, int lda, int ldb,
                                                        int k_per_split)
{
    __shared__ uint16_t sA[GT * GP];
    __shared__ uint16_t sB[GT * GP];
    const int tiles_n = (N + GT - 1) / GT;
    const int m0 = (blockIdx.x / tiles_n) * GT, n0 = (blockIdx.x % tiles_n) * GT;
    const int kb = blockIdx.y * k_per_split;
    const int ke = min(K, kb + k_per_split);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
    for (int k0 = kb; k0 < ke; k0 += GK) {
        __syncthreads();
        for (int e = tid; e < GT * GK; e += 256) {
            int ml, kl;
            if (A_KM) { kl = e / GT; ml = e % GT; } else { ml = e / GK; kl = e % GK; }
            const int m = m0 + ml, k = k0 + kl;
            uint16_t v = 0;
            if (m < M && k < ke) v = A_KM ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            sA[ml * GP + kl] = v;
        }
        for (int e = tid; e < GT * GK; e += 256) {
            int nl, kl;
            if (B_NK) { nl = e / GK; kl = e % GK; } else { kl = e / GT; nl = e % GT; }
            const int n = n0 + nl, k = k0 + kl;
            uint16_t v = 0;
            if (n < N && k < ke) v = B_NK ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
            sB[nl * GP + kl] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k16 = 0; k16 < GK; k16 += 16) {
            const int kk = k16 + (lane >> 5) * 8;
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = frag(&sA[(wr * 64 + i * 32 + (lane & 31)) * GP + kk]);
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = frag(&sB[(wc * 64 + j * 32 + (lane & 31)) * GP + kk]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    float* Cs = C + (int64_t)blockIdx.y * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wc * 64 + j * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int m = m0 + wr * 64 + i * 32 + mfma_row(e, lane);
                if (m < M && n < N) Cs[(int64_t)m * N + n] = acc[i][j][e];
            }
        }
}

// Sum of the splits in a fixed order, plus an epilogue:
//   mode 0: out = sum                          (float)
//   mode 1: z = sum + bias; out = z; act = ReLU(z) as float, act_bf = bf16(ReLU(z))
//   mode 2: out = sum * (mask > 0)             (ReLU derivative, mask = pre-activation)
__global__ void __launch_bounds__(256) gemm_finish_kernel(const float* __restrict__ C, int splits, int64_t MN, int N,
                                                         int mode, const float* __restrict__ bias,
                                                         const float* __restrict__ mask, float* __restrict__ out,
                                                         float* __restrict__ act, uint16_t* __restrict__ act_bf)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= MN) return;
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += C[(int64_t)k * MN + i];
    if (mode == 1) {
        s += bias[i % N];
        out[i] = s;
        const float a = fmaxf(s, 0.f);
        if (act) act[i] = a;
        if (act_bf) act_bf[i] = to_bf16(a);
    } else if (mode == 2) {
        out[i] = mask[i] > 0.f ? s : 0.f;
    } else {
        out[i] = s;
    }
}

// ---------------------------------------------------------------------------
// Fused per-set forward of phi and the sum pool.  A workgroup stages the
// weights in LDS once and then takes sets gridDim.x apart.  Rows of a set
// are processed 128 at a time: the input layer on the vector units into LDS
// (bf16), the 128 x 128 layer on the matrix cores, bias + ReLU, then column
// sums over the rows (fixed order, so a set's result does not depend on the
// grid).  In the input layer a thread owns one column (its four weights and
// bias in registers) for half of the chunk's rows, and the chunk's inputs
// are read from LDS one row at a time by the whole wavefront (a broadcast).
// ---------------------------------------------------------------------------
constexpr int HP = 128 + 8;

__global__ void __launch_bounds__(256) phi_pool_kernel(const float* __restrict__ x, const int32_t* __restrict__ offsets,
                                                       int n_sets,
                                                       const float* __restrict__ P, const uint16_t* __restrict__ W2bf,
                                                       float pool_scale, float* __restrict__ s_out,
                                                       uint16_t* __restrict__ s_bf, uint16_t* __restrict__ h1_bf,
                                                       float* __restrict__ z2_out)
{
    __shared__ uint16_t sW[128 * HP];   // W2 [n][k]
    __shared__ uint16_t sH[128 * HP];   // h1 chunk [row][k]
    __shared__ float4 sX[128];          // the chunk's input rows
    __shared__ float sb2[128];
    __shared__ float colsum[2][128];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    for (int e = tid; e < 128 * 128; e += 256) sW[(e >> 7) * HP + (e & 127)] = W2bf[e];
    if (tid < 128) sb2[tid] = P[NN_B2 + tid];
    // input layer: this thread's column and half of the rows
    const int ic = tid & 127, ih = (tid >> 7) * 64;
    const float ib = P[NN_B1 + ic];
    float iw[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) iw[k] = P[NN_W1 + ic * 4 + k];
    for (int set = blockIdx.x; set < n_sets; set += gridDim.x) {
        const int r0 = offsets[set], r1 = offsets[set + 1];
        float acc_col = 0.f;   // running column sum, thread tid < 128 owns column tid
        for (int c0 = r0; c0 < r1; c0 += 128) {
            __syncthreads();
            if (tid < 128) {
                const int r = c0 + tid;
                float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < r1) {
                    const float* xr = x + (int64_t)r * 4;
                    xv = make_float4(xr[0], xr[1], xr[2], xr[3]);
                }
                sX[tid] = xv;
            }
            __syncthreads();
            {
                const int nr = min(r1 - c0, 128);
                for (int rl = ih; rl < ih + 64; ++rl) {
                    uint16_t h = 0;
                    if (rl < nr) {
                        const float4 xv = sX[rl];
                        float z = ib;
                        z += xv.x * iw[0];
                        z += xv.y * iw[1];
                        z += xv.z * iw[2];
                        z += xv.w * iw[3];
                        h = to_bf16(fmaxf(z, 0.f));
                        if (h1_bf) h1_bf[(int64_t)(c0 + rl) * 128 + ic] = h;
                    }
                    sH[rl * HP + ic] = h;
                }
            }
            __syncthreads();
            floatx16 acc[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
#pragma unroll
            for (int k16 = 0; k16 < 128; k16 += 16) {
                const int kk = k16 + (lane >> 5) * 8;
                bf16x8 a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = frag(&sH[(wr * 64 + i * 32 + (lane & 31)) * HP + kk]);
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = frag(&sW[(wc * 64 + j * 32 + (lane & 31)) * HP + kk]);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
            // bias + ReLU + per-column partial sums of this wave's 64 rows
            // (a chunk of 128 rows needs no row check)
            const bool full = c0 + 128 <= r1;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = wc * 64 + j * 32 + (lane & 31);
                const float bb = sb2[col];
                float cs = 0.f;
                if (full && !z2_out) {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int e = 0; e < 16; ++e) cs += fmaxf(acc[i][j][e] + bb, 0.f);
                } else {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            const int rl = wr * 64 + i * 32 + mfma_row(e, lane);
                            const int r = c0 + rl;
                            const float z = acc[i][j][e] + bb;
                            if (r < r1) {
                                cs += fmaxf(z, 0.f);
                                if (z2_out) z2_out[(int64_t)r * 128 + col] = z;
                            }
                        }
                }
                cs += __shfl_xor(cs, 32, 64);
                if (lane < 32) colsum[wr][col] = cs;
            }
            __syncthreads();
            if (tid < 128) acc_col += colsum[0][tid] + colsum[1][tid];
        }
        if (tid < 128) {
            const float sv = pool_scale * acc_col;
            s_out[(int64_t)set * 128 + tid] = sv;
            s_bf[(int64_t)set * 128 + tid] = to_bf16(sv);
        }
    }
}

// Output layer, de-standardisation and (training) loss and its gradient.
// One thread per set; a3 [sets][128] after ReLU.
__global__ void __launch_bounds__(256) head_kernel(const float* __restrict__ a3, const float* __restrict__ P,
                                                   int n_sets, const float* __restrict__ mean,
                                                   const float* __restrict__ stdv, float* __restrict__ y_phys,
                                                   const float* __restrict__ y_true, float* __restrict__ dy,
                                                   float* __restrict__ sq)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_sets) return;
    const float* W4 = P + NN_W4;
    for (int o = 0; o < NN_DOUT; ++o) {
        float y = P[NN_B4 + o];
        for (int k = 0; k < 128; ++k) y += a3[(int64_t)s * 128 + k] * W4[o * 128 + k];
        if (y_phys) y_phys[s * NN_DOUT + o] = y * stdv[o] + mean[o];
        if (y_true) {
            const float t = (y_true[s * NN_DOUT + o] - mean[o]) / stdv[o];
            const float d = y - t;
            dy[s * NN_DOUT + o] = 2.f * d / (float)(n_sets * NN_DOUT);
            sq[s * NN_DOUT + o] = d * d;
        }
    }
}

// da3 = dy W4, dz3 = da3 * [z3 > 0] (float and bf16); one thread per (set, col).
__global__ void __launch_bounds__(256) head_back_kernel(const float* __restrict__ dy, const float* __restrict__ P,
                                                        const float* __restrict__ z3, int n_sets,
                                                        float* __restrict__ dz3, uint16_t* __restrict__ dz3_bf)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)n_sets * 128) return;
    const int s = (int)(i / 128), c = (int)(i % 128);
    float d = 0.f;
    for (int o = 0; o < NN_DOUT; ++o) d += dy[s * NN_DOUT + o] * P[NN_W4 + o * 128 + c];
    d = z3[i] > 0.f ? d : 0.f;
    dz3[i] = d;
    dz3_bf[i] = to_bf16(d);
}

// dz2 = pool_scale ds[set of row] * [z2 > 0] as bf16, plus its float copy for
// the bias gradient.  One thread per (row, col); row -> set by binary search.
__global__ void __launch_bounds__(256) dz2_kernel(const float* __restrict__ ds, const float* __restrict__ z2,
                                                  const int32_t* __restrict__ offsets, int n_sets, int64_t rows,
                                                  float pool_scale, float* __restrict__ dz2,
                                                  uint16_t* __restrict__ dz2_bf)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows * 128) return;
    const int64_t r = i / 128;
    const int c = (int)(i % 128);
    int lo = 0, hi = n_sets;   // offsets[lo] <= r < offsets[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offsets[mid] <= r) lo = mid; else hi = mid;
    }
    const float d = z2[i] > 0.f ? pool_scale * ds[(int64_t)lo * 128 + c] : 0.f;
    dz2[i] = d;
    dz2_bf[i] = to_bf16(d);
}

// Column sums out[c] = sum_r in[r][c] (fixed order), 128 columns, one
// workgroup per column block of 1 column, strided rows then a tree.
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ in, int64_t rows, int cols,
                                                     float* __restrict__ out)
{
    __shared__ float sh[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int64_t r = threadIdx.x; r < rows; r += 256) s += in[r * cols + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// dW4[o][k] = sum_s dy[s][o] a3[s][k]; one workgroup per (o, k).
__global__ void __launch_bounds__(256) dw4_kernel(const float* __restrict__ dy, const float* __restrict__ a3,
                                                  int n_sets, float* __restrict__ g)
{
    __shared__ float sh[256];
    const int o = blockIdx.x / 128, k = blockIdx.x % 128;
    float s = 0.f;
    for (int i = threadIdx.x; i < n_sets; i += 256) s += dy[i * NN_DOUT + o] * a3[(int64_t)i * 128 + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) g[NN_W4 + o * 128 + k] = sh[0];
}

// Input-layer gradients from dh1 (rows x 128): dz1 = dh1 [z1 > 0] with z1
// recomputed from x; dW1[c][k] = sum_r dz1[r][c] x[r][k], db1[c] = sum_r dz1.
// One workgroup per column c.
__global__ void __launch_bounds__(256) dw1_kernel(const float* __restrict__ dh1, const float* __restrict__ x,
                                                  const float* __restrict__ P, int64_t rows, float* __restrict__ g)
{
    __shared__ float sh[5][256];
    const int c = blockIdx.x;
    float w[4], b = P[NN_B1 + c];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = P[NN_W1 + c * 4 + k];
    float acc[5] = { 0.f, 0.f, 0.f, 0.f, 0.f };
    for (int64_t r = threadIdx.x; r < rows; r += 256) {
        float z = b;
#pragma unroll
        for (int k = 0; k < 4; ++k) z += x[r * 4 + k] * w[k];
        const float d = z > 0.f ? dh1[r * 128 + c] : 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += d * x[r * 4 + k];
        acc[4] += d;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int wdt = 128; wdt > 0; wdt >>= 1) {
        if ((int)threadIdx.x < wdt)
#pragma unroll
            for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + wdt];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) g[NN_W1 + c * 4 + k] = sh[k][0];
        g[NN_B1 + c] = sh[4][0];
    }
}

// sum of the squared errors -> loss (mean), fixed order, one workgroup.
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ sq, int n, float* __restrict__ loss)
{
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += sq[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] / (float)n;
}

// Adam (bias-corrected), float masters; refreshes the bf16 shadows.
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ P, const float* __restrict__ G,
                                                   float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2,
                                                   uint16_t* __restrict__ W2bf, uint16_t* __restrict__ W3bf)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    P[i] = p;
    if (i >= NN_W2 && i < NN_W2 + 128 * 128) W2bf[i - NN_W2] = to_bf16(p);
    if (i >= NN_W3 && i < NN_W3 + 128 * 128) W3bf[i - NN_W3] = to_bf16(p);
}

__global__ void __launch_bounds__(256) shadow_kernel(const float* __restrict__ P, uint16_t* __restrict__ W2bf,
                                                     uint16_t* __restrict__ W3bf)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 128 * 128) return;
    W2bf[i] = to_bf16(P[NN_W2 + i]);
    W3bf[i] = to_bf16(P[NN_W3 + i]);
}

// He-uniform initialisation from a counter-based generator (SplitMix64 of
// seed ^ index); biases zero.
__device__ __forceinline__ uint64_t sm64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) init_params_kernel(float* __restrict__ P, uint64_t seed)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NN_NPARAM) return;
    int fan_in = 0;
    if (i < NN_B1) fan_in = 4;
    else if (i >= NN_W2 && i < NN_B2) fan_in = 128;
    else if (i >= NN_W3 && i < NN_B3) fan_in = 128;
    else if (i >= NN_W4 && i < NN_B4) fan_in = 128;
    if (fan_in == 0) { P[i] = 0.f; return; }
    const double u = (double)(sm64(seed ^ (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    const double lim = sqrt(6.0 / fan_in);
    P[i] = (float)((2.0 * u - 1.0) * lim);
}

// Per-bubble inputs ((c - centre)/R, ln(r/r_median)/sigma).
__global__ void __launch_bounds__(256) features_kernel(const double* __restrict__ bub, int64_t rows, int ndim,
                                                       double cx, double cy, double cz, double R, double rmed,
                                                       double sigma, float* __restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    const double* b = bub + 4 * i;
    x[4 * i + 0] = (float)((b[0] - cx) / R);
    x[4 * i + 1] = (float)(ndim > 1 ? (b[1] - cy) / R : 0.0);
    x[4 * i + 2] = (float)(ndim > 2 ? (b[2] - cz) / R : 0.0);
    x[4 * i + 3] = (float)(log(b[3] / rmed) / sigma);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

hipError_t nn_gemm(const uint16_t* A, bool a_km, const uint16_t* B, bool b_nk, float* C, int M, int N, int K, int lda,
                   int ldb, int splits, hipStream_t s)
{
    const int kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    const int sp = (K + kps - 1) / kps;
    dim3 grid(cdiv64(M, GT) * cdiv64(N, GT), sp);
    if (!a_km && !b_nk) hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
    else if (!a_km && b_nk) hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
    else if (a_km && !b_nk) hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
    else hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
    return hipGetLastError();
}

int nn_gemm_splits(int K, int splits)
{
    const int kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    return (K + kps - 1) / kps;
}

hipError_t nn_gemm_finish(const float* C, int splits, int64_t M, int N, int mode, const float* bias, const float* mask,
                          float* out, float* act, uint16_t* act_bf, hipStream_t s)
{
    const int64_t MN = M * N;
    hipLaunchKernelGGL(gemm_finish_kernel, dim3(cdiv64(MN, 256)), dim3(256), 0, s, C, splits, MN, N, mode, bias, mask,
                       out, act, act_bf);
    return hipGetLastError();
}

hipError_t nn_phi_pool(const float* x, const int32_t* offsets, int n_sets, const float* P, const uint16_t* W2bf,
                       float pool_scale, float* s_out, uint16_t* s_bf, uint16_t* h1_bf, float* z2, hipStream_t st)
{
    // two resident workgroups per CU (73.2 KB of LDS each): a few rounds of
    // them, each taking sets gridDim.x apart
    const int grid = n_sets < 4096 ? n_sets : 4096;
    hipLaunchKernelGGL(phi_pool_kernel, dim3(grid), dim3(256), 0, st, x, offsets, n_sets, P, W2bf, pool_scale, s_out,
                       s_bf, h1_bf, z2);
    return hipGetLastError();
}

hipError_t nn_head(const float* a3, const float* P, int n_sets, const float* mean, const float* stdv, float* y_phys,
                   const float* y_true, float* dy, float* sq, hipStream_t s)
{
    hipLaunchKernelGGL(head_kernel, dim3(cdiv64(n_sets, 256)), dim3(256), 0, s, a3, P, n_sets, mean, stdv, y_phys,
                       y_true, dy, sq);
    return hipGetLastError();
}

hipError_t nn_head_back(const float* dy, const float* P, const float* z3, int n_sets, float* dz3, uint16_t* dz3_bf,
                        hipStream_t s)
{
    hipLaunchKernelGGL(head_back_kernel, dim3(cdiv64((int64_t)n_sets * 128, 256)), dim3(256), 0, s, dy, P, z3, n_sets,
                       dz3, dz3_bf);
    return hipGetLastError();
}

hipError_t nn_dz2(const float* ds, const float* z2, const int32_t* offsets, int n_sets, int64_t rows, float pool_scale,
                  float* dz2, uint16_t* dz2_bf, hipStream_t s)
{
    hipLaunchKernelGGL(dz2_kernel, dim3(cdiv64(rows * 128, 256)), dim3(256), 0, s, ds, z2, offsets, n_sets, rows,
                       pool_scale, dz2, dz2_bf);
    return hipGetLastError();
}

hipError_t nn_colsum(const float* in, int64_t rows, int cols, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3(cols), dim3(256), 0, s, in, rows, cols, out);
    return hipGetLastError();
}

hipError_t nn_dw4(const float* dy, const float* a3, int n_sets, float* g, hipStream_t s)
{
    hipLaunchKernelGGL(dw4_kernel, dim3(NN_DOUT * 128), dim3(256), 0, s, dy, a3, n_sets, g);
    return hipGetLastError();
}

hipError_t nn_dw1(const float* dh1, const float* x, const float* P, int64_t rows, float* g, hipStream_t s)
{
    hipLaunchKernelGGL(dw1_kernel, dim3(128), dim3(256), 0, s, dh1, x, P, rows, g);
    return hipGetLastError();
}

hipError_t nn_loss(const float* sq, int n, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, sq, n, loss);
    return hipGetLastError();
}

hipError_t nn_adam(float* P, const float* G, float* m, float* v, float lr, float b1, float b2, float eps, int t,
                   uint16_t* W2bf, uint16_t* W3bf, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(cdiv64(NN_NPARAM, 256)), dim3(256), 0, s, P, G, m, v, NN_NPARAM, lr, b1, b2,
                       eps, c1, c2, W2bf, W3bf);
    return hipGetLastError();
}

hipError_t nn_shadow(const float* P, uint16_t* W2bf, uint16_t* W3bf, hipStream_t s)
{
    hipLaunchKernelGGL(shadow_kernel, dim3(64), dim3(256), 0, s, P, W2bf, W3bf);
    return hipGetLastError();
}

hipError_t nn_init_params(float* P, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(init_params_kernel, dim3(cdiv64(NN_NPARAM, 256)), dim3(256), 0, s, P, seed);
    return hipGetLastError();
}

hipError_t nn_features(const double* bub, int64_t rows, int ndim, const double* center, double R, double rmed,
                       double sigma, float* x, hipStream_t s)
{
    hipLaunchKernelGGL(features_kernel, dim3(cdiv64(rows, 256)), dim3(256), 0, s, bub, rows, ndim, center[0], center[1],
                       center[2], R, rmed, sigma, x);
    return hipGetLastError();
}

}  // namespace ofm
