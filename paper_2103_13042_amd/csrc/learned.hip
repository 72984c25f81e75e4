// Kernels of the learned threshold: tile-norm histogram features, norm
// product bounds, FP64 sums of squares (for relative errors), and the
// training and inference kernels of the 129-128-128-1 GELU network.
//
// All reductions run in a fixed order, so every result is bitwise
// reproducible from run to run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace spamm {

// --------------------------------------------------------------------------
// Features: per matrix a 64-bin histogram of log10 of the positive leaf norms
// over [-46, 3) (norms outside the range in the first or last bin), as tiles
// per tile row (count / bdim) capped at kHistCap; zero norms are not
// counted.  Then log10(target).

constexpr int kHistBins = 64;
constexpr double kLogLo = -46.0, kLogHi = 3.0;
constexpr double kHistCap = 4.0;
constexpr int kFeatThreads = 1024;

__global__ __launch_bounds__(kFeatThreads) void tau_features_kernel(const double* __restrict__ pyr_a,
                                                                    const double* __restrict__ pyr_b, int64_t bdim,
                                                                    int lv, float log_target,
                                                                    float* __restrict__ out) {
    __shared__ int hist[2][kHistBins];
    if (threadIdx.x < 2 * kHistBins) hist[threadIdx.x / kHistBins][threadIdx.x % kHistBins] = 0;
    __syncthreads();
    const int64_t side = int64_t(1) << lv;
    const int64_t tiles = bdim * bdim;
    for (int m = 0; m < 2; ++m) {
        const double* leaf = (m == 0 ? pyr_a : pyr_b) + level_offset(lv);
        for (int64_t t = threadIdx.x; t < tiles; t += kFeatThreads) {
            const double x = leaf[(t / bdim) * side + t % bdim];
            if (x > 0.0) {
                const double pos = (log10(x) - kLogLo) * (double(kHistBins) / (kLogHi - kLogLo));
                const double f = floor(pos);
                const int bin = f < 0.0 ? 0 : (f > kHistBins - 1 ? kHistBins - 1 : int(f));
                atomicAdd(&hist[m][bin], 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kHistBins) {
        const double per_row = double(hist[threadIdx.x / kHistBins][threadIdx.x % kHistBins]) / double(bdim);
        out[threadIdx.x] = float(per_row < kHistCap ? per_row : kHistCap);
    }
    if (threadIdx.x == 0) out[2 * kHistBins] = log_target;
}

hipError_t launch_tau_features(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, float log_target,
                               float* out, hipStream_t s) {
    tau_features_kernel<<<1, kFeatThreads, 0, s>>>(pyr_a, pyr_b, bdim, lv, log_target, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Norm product bounds over the real bdim^3 triples, with products formed as in
// the plan (fl64(nA[i,k] * nB[k,j])):  out[0] = the smallest product >= lo,
// out[1] = the largest product, both as the bit patterns of non-negative
// doubles (which order like unsigned integers), +inf bits when no product is
// >= lo.  out must hold the initial values {+inf bits, 0} (bounds_init).

__global__ void bounds_init_kernel(unsigned long long* out) {
    if (threadIdx.x == 0) {
        out[0] = 0x7FF0000000000000ull;
        out[1] = 0ull;
    }
}

constexpr int kBoundThreads = 256;

__global__ __launch_bounds__(kBoundThreads) void product_bounds_kernel(const double* __restrict__ pyr_a,
                                                                       const double* __restrict__ pyr_b, int64_t bdim,
                                                                       int lv, double lo,
                                                                       unsigned long long* __restrict__ out) {
    const int64_t side = int64_t(1) << lv;
    const double* la = pyr_a + level_offset(lv);
    const double* lb = pyr_b + level_offset(lv);
    const int64_t i = blockIdx.x;
    double vmin = INFINITY, vmax = 0.0;
    const int64_t kj = bdim * bdim;
    for (int64_t e = threadIdx.x; e < kj; e += kBoundThreads) {
        const int64_t k = e / bdim, j = e - k * bdim;
        const double p = la[i * side + k] * lb[k * side + j];
        if (p >= lo && p < vmin) vmin = p;
        if (p > vmax) vmax = p;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        vmin = fmin(vmin, __shfl_xor(vmin, o));
        vmax = fmax(vmax, __shfl_xor(vmax, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&out[0], static_cast<unsigned long long>(__double_as_longlong(vmin)));
        atomicMax(&out[1], static_cast<unsigned long long>(__double_as_longlong(vmax)));
    }
}

hipError_t launch_product_bounds(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double lo,
                                 unsigned long long* out, hipStream_t s) {
    bounds_init_kernel<<<1, 64, 0, s>>>(out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    product_bounds_kernel<<<unsigned(bdim), kBoundThreads, 0, s>>>(pyr_a, pyr_b, bdim, lv, lo, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Sum of squares of an FP32 array in FP64 (squares are exact in FP64): a fixed
// grid of kSumBlocks blocks writes one partial each, then one block adds them
// in a fixed tree order.

constexpr int kSumThreads = 256;

template <int T>
__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < T / 64; ++w) tot += red[w];
    return tot;
}

__global__ __launch_bounds__(kSumThreads) void sumsq_partial_kernel(const float* __restrict__ x, int64_t count,
                                                                    double* __restrict__ partials) {
    __shared__ double red[kSumThreads / 64];
    const int64_t stride = int64_t(gridDim.x) * kSumThreads;
    double acc = 0.0;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15u) == 0;
    if (vec) {
        const int64_t n4 = count / 4;
        const float4* x4 = reinterpret_cast<const float4*>(x);
        for (int64_t q = int64_t(blockIdx.x) * kSumThreads + threadIdx.x; q < n4; q += stride) {
            const float4 v = x4[q];
            acc += double(v.x) * v.x + double(v.y) * v.y + double(v.z) * v.z + double(v.w) * v.w;
        }
        for (int64_t q = n4 * 4 + int64_t(blockIdx.x) * kSumThreads + threadIdx.x; q < count; q += stride)
            acc += double(x[q]) * x[q];
    } else {
        for (int64_t q = int64_t(blockIdx.x) * kSumThreads + threadIdx.x; q < count; q += stride)
            acc += double(x[q]) * x[q];
    }
    const double tot = block_sum<kSumThreads>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kSumThreads) void sum_partials_kernel(const double* __restrict__ partials, int np,
                                                                   double* __restrict__ out) {
    __shared__ double red[kSumThreads / 64];
    double acc = 0.0;
    for (int q = threadIdx.x; q < np; q += kSumThreads) acc += partials[q];
    const double tot = block_sum<kSumThreads>(acc, red);
    if (threadIdx.x == 0) *out = tot;
}

hipError_t launch_sumsq(const float* x, int64_t count, double* partials, double* out, hipStream_t s) {
    sumsq_partial_kernel<<<kSumBlocks, kSumThreads, 0, s>>>(x, count, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_partials_kernel<<<1, kSumThreads, 0, s>>>(partials, kSumBlocks, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// The network, FP32.  Parameters flat: W1 [128][129], b1 [128], W2 [128][128],
// b2 [128], w3 [128], b3 [1].  Layer l maps X [B][I] to Z = X W^T + b and
// H = gelu(Z) (erf form) for the hidden layers; the output layer has no
// activation.  Sums run over the input index in ascending order.

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

constexpr int kMaxIn = 132;

// block b = one sample; thread o = one output unit (O <= blockDim.x)
__global__ __launch_bounds__(128) void dense_fwd_kernel(const float* __restrict__ x, int in, const float* __restrict__ w,
                                                        const float* __restrict__ bias, int out_units,
                                                        float* __restrict__ z, float* __restrict__ h) {
    __shared__ float xs[kMaxIn];
    const int b = blockIdx.x, o = threadIdx.x;
    for (int i = threadIdx.x; i < in; i += blockDim.x) xs[i] = x[int64_t(b) * in + i];
    __syncthreads();
    if (o >= out_units) return;
    const float* wr = w + int64_t(o) * in;
    float acc = bias[o];
    for (int i = 0; i < in; ++i) acc = fmaf(xs[i], wr[i], acc);
    z[int64_t(b) * out_units + o] = acc;
    if (h) h[int64_t(b) * out_units + o] = gelu_f(acc);
}

// loss = mean (y - t)^2, dy = 2 (y - t) / B  (one block)
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int batch,
                                                  float* __restrict__ dy, float* __restrict__ loss) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int q = threadIdx.x; q < batch; q += 256) {
        const float r = y[q] - t[q];
        dy[q] = 2.0f * r / float(batch);
        acc += double(r) * r;
    }
    const double tot = block_sum<256>(acc, red);
    if (threadIdx.x == 0 && loss) *loss = float(tot / batch);
}

// dZ = dH * gelu'(Z) elementwise (dh and dz may be the same array)
__global__ void gelu_bwd_kernel(const float* dh, const float* __restrict__ z, int64_t count, float* dz) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < count) dz[q] = dh[q] * gelu_grad_f(z[q]);
}

// dW[o][i] = sum_b dZ[b][o] X[b][i] (i < I); db[o] = sum_b dZ[b][o] (i == I).
// Thread per (o, i); b ascending.
__global__ void dense_bwd_weight_kernel(const float* __restrict__ dz, const float* __restrict__ x, int batch, int in,
                                        int out_units, float* __restrict__ dw, float* __restrict__ db) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= int64_t(out_units) * (in + 1)) return;
    const int o = int(q / (in + 1)), i = int(q % (in + 1));
    float acc = 0.0f;
    if (i < in) {
        for (int b = 0; b < batch; ++b) acc = fmaf(dz[int64_t(b) * out_units + o], x[int64_t(b) * in + i], acc);
        dw[int64_t(o) * in + i] = acc;
    } else {
        for (int b = 0; b < batch; ++b) acc += dz[int64_t(b) * out_units + o];
        db[o] = acc;
    }
}

// dX[b][i] = sum_o dZ[b][o] W[o][i]; thread per (b, i); o ascending
__global__ void dense_bwd_input_kernel(const float* __restrict__ dz, const float* __restrict__ w, int batch, int in,
                                       int out_units, float* __restrict__ dx) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= int64_t(batch) * in) return;
    const int b = int(q / in), i = int(q % in);
    float acc = 0.0f;
    for (int o = 0; o < out_units; ++o) acc = fmaf(dz[int64_t(b) * out_units + o], w[int64_t(o) * in + i], acc);
    dx[q] = acc;
}

// Adam with bias correction: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

namespace {
unsigned blocks_for(int64_t count, int threads) { return unsigned((count + threads - 1) / threads); }
}  // namespace

hipError_t launch_mlp_forward(const float* params, const float* x, int batch, float* acts, float* y, hipStream_t s) {
    const MlpLayout P{}, A = MlpLayout::acts(batch);
    dense_fwd_kernel<<<batch, 128, 0, s>>>(x, kMlpIn, params + P.w1, params + P.b1, kMlpHid, acts + A.z1, acts + A.h1);
    dense_fwd_kernel<<<batch, 128, 0, s>>>(acts + A.h1, kMlpHid, params + P.w2, params + P.b2, kMlpHid, acts + A.z2,
                                            acts + A.h2);
    dense_fwd_kernel<<<batch, 128, 0, s>>>(acts + A.h2, kMlpHid, params + P.w3, params + P.b3, 1, y, nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* params, const float* x, const float* t, int batch, float* acts,
                                float* grad, float* loss, hipStream_t s) {
    const MlpLayout P{}, A = MlpLayout::acts(batch);
    hipError_t e = launch_mlp_forward(params, x, batch, acts, acts + A.y, s);
    if (e != hipSuccess) return e;
    float* dy = acts + A.dy;
    mse_kernel<<<1, 256, 0, s>>>(acts + A.y, t, batch, dy, loss);
    const int64_t bh = int64_t(batch) * kMlpHid;
    // output layer: dw3, db3; dH2 = dy w3^T; dZ2 = dH2 gelu'(Z2)
    dense_bwd_weight_kernel<<<blocks_for(kMlpHid + 1, 256), 256, 0, s>>>(dy, acts + A.h2, batch, kMlpHid, 1,
                                                                          grad + P.w3, grad + P.b3);
    dense_bwd_input_kernel<<<blocks_for(bh, 256), 256, 0, s>>>(dy, params + P.w3, batch, kMlpHid, 1, acts + A.d2);
    gelu_bwd_kernel<<<blocks_for(bh, 256), 256, 0, s>>>(acts + A.d2, acts + A.z2, bh, acts + A.d2);
    // hidden layer 2: dW2, db2; dH1 = dZ2 W2; dZ1 = dH1 gelu'(Z1)
    dense_bwd_weight_kernel<<<blocks_for(int64_t(kMlpHid) * (kMlpHid + 1), 256), 256, 0, s>>>(
        acts + A.d2, acts + A.h1, batch, kMlpHid, kMlpHid, grad + P.w2, grad + P.b2);
    dense_bwd_input_kernel<<<blocks_for(bh, 256), 256, 0, s>>>(acts + A.d2, params + P.w2, batch, kMlpHid, kMlpHid,
                                                                 acts + A.d1);
    gelu_bwd_kernel<<<blocks_for(bh, 256), 256, 0, s>>>(acts + A.d1, acts + A.z1, bh, acts + A.d1);
    // hidden layer 1: dW1, db1
    dense_bwd_weight_kernel<<<blocks_for(int64_t(kMlpHid) * (kMlpIn + 1), 256), 256, 0, s>>>(
        acts + A.d1, x, batch, kMlpIn, kMlpHid, grad + P.w1, grad + P.b1);
    return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int64_t count, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
    adam_kernel<<<blocks_for(count, 256), 256, 0, s>>>(params, grad, m, v, count, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace spamm
