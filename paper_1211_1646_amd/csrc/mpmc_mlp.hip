// Move-size network of the learned controller (FP32, gfx950): a 3 -> 32 ->
// 32 -> 1 perceptron with tanh hidden layers that maps a replica's packing
// fraction, mean cell occupancy and recent acceptance to the maximum trial
// displacement delta (the free parameter d of Sec. 3.3).  It acts only
// between equilibration windows; production runs use a frozen delta, so the
// sampled chain is the paper's.
//
// Kernels: inference (one lane per sample, weights broadcast from LDS),
// backpropagation with per-workgroup gradient partials reduced in a fixed
// order (reproducible), the squared-error gradient, Adam (Kingma and Ba,
// ICLR 2015, Alg. 1), and the in-chain controller that updates every
// replica's delta from its control block.  None is a dense contraction large
// enough to pay for MFMA: a training step on 1e5 samples is ~2e8 FLOP.
//
// Parameter vector (row-major, rows are outputs): W1[32][3] b1[32]
// W2[32][32] b2[32] W3[1][32] b3[1] -- 1217 floats.
#include <mutex>

#include "mpmc_internal.h"

#pragma clang fp contract(off)

namespace mpmc {
namespace {

constexpr int kH = 32;
constexpr int oW1 = 0, oB1 = 96, oW2 = 128, oB2 = 1152, oW3 = 1184, oB3 = 1216;
constexpr int kBwdBlock = 64;   // samples per backward workgroup
constexpr int kNoAllocMaxSamples = 65536;   // largest n of the no-allocation backward
constexpr int kRow = kBwdBlock + 1;

__device__ __forceinline__ void stage_params(const float *__restrict__ W, float *P)
{
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) P[i] = W[i];
    __syncthreads();
}

// y of one sample; h1, h2 receive the hidden activations.  Each
// pre-activation starts from its bias and adds the terms in input order.
__device__ __forceinline__ float net_forward(const float *P, float x0, float x1, float x2,
                                             float (&h1)[kH], float (&h2)[kH])
{
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float z = P[oB1 + j];
        z = z + P[oW1 + 3 * j] * x0;
        z = z + P[oW1 + 3 * j + 1] * x1;
        z = z + P[oW1 + 3 * j + 2] * x2;
        h1[j] = tanhf(z);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float z = P[oB2 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) z = z + P[oW2 + kH * j + k] * h1[k];
        h2[j] = tanhf(z);
    }
    float y = P[oB3];
#pragma unroll
    for (int k = 0; k < kH; ++k) y = y + P[oW3 + k] * h2[k];
    return y;
}

__global__ void __launch_bounds__(256)
k_mlp_forward(const float *__restrict__ W, const float *__restrict__ X, int n,
              float *__restrict__ Y, float *__restrict__ cache)
{
    __shared__ float P[kMlpParams];
    stage_params(W, P);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float h1[kH], h2[kH];
    const float y = net_forward(P, X[3 * i], X[3 * i + 1], X[3 * i + 2], h1, h2);
    Y[i] = y;
    if (cache) {   // feature-major: lanes write consecutive addresses
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            cache[(size_t)j * n + i] = h1[j];
            cache[(size_t)(kH + j) * n + i] = h2[j];
        }
    }
}

// One workgroup of 64 samples: per-sample backpropagation in registers, then
// the workgroup's sum of every parameter's per-sample terms, summed in
// sample order, into partial row blockIdx.x.
__global__ void __launch_bounds__(kBwdBlock)
k_mlp_backward(const float *__restrict__ W, const float *__restrict__ X,
               const float *__restrict__ cache, const float *__restrict__ dY, int n,
               float *__restrict__ dX, float *__restrict__ part)
{
    __shared__ float P[kMlpParams];
    __shared__ float s_h1[kH][kRow], s_h2[kH][kRow], s_dz1[kH][kRow], s_dz2[kH][kRow];
    __shared__ float s_x[3][kRow], s_dy[kRow];
    stage_params(W, P);
    const int t = threadIdx.x;
    const int i = blockIdx.x * kBwdBlock + t;
    const bool valid = i < n;
    float h1[kH], h2[kH], dz2[kH], dz1[kH];
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f, dy = 0.0f;
    if (valid) {
        x0 = X[3 * i];
        x1 = X[3 * i + 1];
        x2 = X[3 * i + 2];
        dy = dY[i];
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        h1[j] = valid ? cache[(size_t)j * n + i] : 0.0f;
        h2[j] = valid ? cache[(size_t)(kH + j) * n + i] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) dz2[j] = (dy * P[oW3 + j]) * (1.0f - h2[j] * h2[j]);
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) s = s + P[oW2 + kH * j + k] * dz2[j];
        dz1[k] = s * (1.0f - h1[k] * h1[k]);
    }
    if (valid && dX) {
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            g0 = g0 + P[oW1 + 3 * k] * dz1[k];
            g1 = g1 + P[oW1 + 3 * k + 1] * dz1[k];
            g2 = g2 + P[oW1 + 3 * k + 2] * dz1[k];
        }
        dX[3 * i] = g0;
        dX[3 * i + 1] = g1;
        dX[3 * i + 2] = g2;
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        s_h1[j][t] = h1[j];
        s_h2[j][t] = h2[j];
        s_dz1[j][t] = dz1[j];
        s_dz2[j][t] = dz2[j];
    }
    s_x[0][t] = x0;
    s_x[1][t] = x1;
    s_x[2][t] = x2;
    s_dy[t] = dy;
    __syncthreads();
    for (int p = t; p < kMlpParams; p += kBwdBlock) {
        const float *a;
        const float *b = nullptr;   // nullptr: the bias, factor 1
        if (p < oB1) {
            a = s_dz1[(p - oW1) / 3];
            b = s_x[(p - oW1) % 3];
        } else if (p < oW2) {
            a = s_dz1[p - oB1];
        } else if (p < oB2) {
            a = s_dz2[(p - oW2) / kH];
            b = s_h1[(p - oW2) % kH];
        } else if (p < oW3) {
            a = s_dz2[p - oB2];
        } else if (p < oB3) {
            a = s_dy;
            b = s_h2[p - oW3];
        } else {
            a = s_dy;
        }
        float acc = 0.0f;
        if (b) {
            for (int s = 0; s < kBwdBlock; ++s) acc = acc + a[s] * b[s];
        } else {
            for (int s = 0; s < kBwdBlock; ++s) acc = acc + a[s];
        }
        part[(size_t)blockIdx.x * kMlpParams + p] = acc;
    }
}

// dW[p] = sum of the partial rows in row order.
__global__ void __launch_bounds__(256)
k_mlp_reduce(const float *__restrict__ part, int rows, float *__restrict__ dW)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float acc = 0.0f;
    for (int r = 0; r < rows; ++r) acc = acc + part[(size_t)r * kMlpParams + p];
    dW[p] = acc;
}

// Squared error 1/(2n) sum (Y - T)^2: dY = (Y - T) / n, per-workgroup FP64
// partial sums of the squares in a fixed tree, then one workgroup totals them.
constexpr int kMseBlock = 256;

__global__ void __launch_bounds__(kMseBlock)
k_mse_grad(const float *__restrict__ Y, const float *__restrict__ T, int n,
           float *__restrict__ dY, double *__restrict__ part)
{
    __shared__ double sh[kMseBlock];
    const int i = blockIdx.x * kMseBlock + threadIdx.x;
    double sq = 0.0;
    if (i < n) {
        const float r = Y[i] - T[i];
        dY[i] = r / (float)n;
        sq = (double)r * (double)r;
    }
    sh[threadIdx.x] = sq;
    __syncthreads();
    for (int o = kMseBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kMseBlock)
k_mse_total(const double *__restrict__ part, int rows, int n, double *__restrict__ loss)
{
    __shared__ double sh[kMseBlock];
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += kMseBlock) s += part[r];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kMseBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = n > 0 ? 0.5 * sh[0] / (double)n : 0.0;
}

// Adam with bias correction; c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t).
__global__ void __launch_bounds__(256)
k_adam(float *__restrict__ W, float *__restrict__ m, float *__restrict__ v,
       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
       float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float mh = mi * c1;
    const float vh = vi * c2;
    W[i] = W[i] - lr * mh / (sqrtf(vh) + eps);
}

// Controller step for every replica (one lane each): with a the acceptance
// of the window since the last step, the network's inputs are
// 20 (phi - 0.7), mean disks per cell - 1.5 and 4 (a - 0.3), and
// delta = 0.1 exp(y), clamped to [1e-3, min(w)/2].  Opens the next window.
__global__ void __launch_bounds__(64) k_control(Tables t, const float *__restrict__ W, int apply)
{
    __shared__ float P[kMlpParams];
    stage_params(W, P);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= t.R) return;
    Ctl *ctl = t.ctls + r;
    const Geom g = t.reps[r].g;
    const unsigned long long tr = ctl->trials - ctl->win_trials;
    const unsigned long long ac = ctl->accepts - ctl->win_accepts;
    if (apply && tr > 0) {
        const double box = ((double)g.mx * (double)g.wx) * ((double)g.my * (double)g.wy);
        const double phi = (double)g.N * 3.14159265358979323846 / (4.0 * box);
        const double occ = (double)g.N / (double)g.C;
        const double a = (double)ac / (double)tr;
        const float x0 = (float)(20.0 * (phi - 0.7));
        const float x1 = (float)(occ - 1.5);
        const float x2 = (float)(4.0 * (a - 0.3));
        float h1[kH], h2[kH];
        const float y = net_forward(P, x0, x1, x2, h1, h2);
        double d = 0.1 * exp((double)y);
        const double hi = 0.5 * (double)(g.wx < g.wy ? g.wx : g.wy);
        if (d < 1e-3) d = 1e-3;
        if (d > hi) d = hi;
        ctl->delta = (float)d;
    }
    ctl->win_trials = ctl->trials;
    ctl->win_accepts = ctl->accepts;
}

}  // namespace

size_t mlp_work_bytes(int n)
{
    const size_t rows = (size_t)(n + kBwdBlock - 1) / kBwdBlock;
    const size_t mse = (size_t)(n + kMseBlock - 1) / kMseBlock;
    return ((rows * kMlpParams * sizeof(float) + 255) & ~(size_t)255) + mse * sizeof(double) + 256;
}

hipError_t launch_mlp_forward(const float *W, const float *X, int n, float *Y, float *cache,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, st, W, X, n, Y, cache);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *W, const float *X, const float *cache,
                               const float *dY, int n, float *dW, float *dX, void *work,
                               hipStream_t st)
{
    const int rows = (n + kBwdBlock - 1) / kBwdBlock;
    float *part = (float *)work;
    if (rows > 0)
        hipLaunchKernelGGL(k_mlp_backward, dim3(rows), dim3(kBwdBlock), 0, st, W, X, cache, dY, n,
                           dX, part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, part, rows, dW);
    return hipGetLastError();
}

namespace {

// ------------------------------------------------- no-allocation backward
// The backward pass's per-workgroup gradient rows in a device array of this
// library, for callers that cannot allocate (code under graph capture, tight
// serving loops): at most kNoAllocMaxSamples samples, kNoAllocMaxSamples /
// kBwdBlock rows of kMlpParams floats (4.6 MiB), held by every GPU the
// library runs on until the process ends.  Every call on one GPU shares that
// GPU's copy: calls that overlap on one GPU race.  Each row is written in
// full before the reduction reads it, so nothing needs clearing.
constexpr int kNoAllocMaxRows = kNoAllocMaxSamples / kBwdBlock;
static __device__ __align__(256) float scratch[(size_t)kNoAllocMaxRows * kMlpParams];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices];   // device address of scratch on each GPU

// The device address of the current GPU's copy of scratch, looked up once
// per device (the array's name is only a host-side stand-in).
hipError_t scratch_of_current_device(float **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t launch_mlp_backward_noalloc(const float *W, const float *X, const float *cache,
                                       const float *dY, int n, float *dW, float *dX,
                                       hipStream_t st)
{
    if (n < 0 || n > kNoAllocMaxSamples) return hipErrorInvalidValue;
    float *part = nullptr;
    const hipError_t e = scratch_of_current_device(&part);
    if (e != hipSuccess) return e;
    const int rows = (n + kBwdBlock - 1) / kBwdBlock;
    if (rows > 0)
        hipLaunchKernelGGL(k_mlp_backward, dim3(rows), dim3(kBwdBlock), 0, st, W, X, cache, dY, n,
                           dX, part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, part, rows, dW);
    return hipGetLastError();
}

hipError_t launch_mse(const float *Y, const float *T, int n, float *dY, double *loss, void *work,
                      hipStream_t st)
{
    const int rows = (n + kMseBlock - 1) / kMseBlock;
    const size_t off = ((size_t)((n + kBwdBlock - 1) / kBwdBlock) * kMlpParams * sizeof(float) + 255) &
                       ~(size_t)255;
    double *part = (double *)((char *)work + off);
    if (rows > 0)
        hipLaunchKernelGGL(k_mse_grad, dim3(rows), dim3(kMseBlock), 0, st, Y, T, n, dY, part);
    hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(kMseBlock), 0, st, part, rows, n, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *W, float *m, float *v, const float *g, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, W, m, v, g, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_control(const Tables &t, const float *W, int apply, hipStream_t st)
{
    hipLaunchKernelGGL(k_control, dim3((t.R + 63) / 64), dim3(64), 0, st, t, W, apply);
    return hipGetLastError();
}

}  // namespace mpmc
