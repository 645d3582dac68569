// Small multilayer perceptron that predicts the chemical potential and the
// expansion order from cheap Chebyshev data (stochastic moments, spectral
// interval, beta, filling).  FP32 weights and activations; affine layers
// with tanh between them and a linear output; mean-squared-error loss; Adam.
// The sizes are tiny (widths <= 256, batches of a few hundred), so each
// kernel maps one thread to one output element.
#include <cmath>

#include "dm_common.hpp"

namespace dm {
namespace {

// Y[b, o] = act(sum_i X[b, i] W[o, i] + bias[o]); act = tanh if use_tanh.
__global__ void linear_fwd_kernel(int B, int nin, int nout, const float* __restrict__ X,
                                  const float* __restrict__ W, const float* __restrict__ bias,
                                  int use_tanh, float* __restrict__ Y) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * nout) return;
    const int b = idx / nout, o = idx % nout;
    const float* x = X + (long)b * nin;
    const float* w = W + (long)o * nin;
    float s = bias[o];
    for (int i = 0; i < nin; ++i) s = fmaf(x[i], w[i], s);
    Y[idx] = use_tanh ? tanhf(s) : s;
}

// G = 2 (Y - T) / (B nout), loss partial sums per block
__global__ void mse_grad_kernel(int n, float inv_n, const float* __restrict__ Y,
                                const float* __restrict__ T, float* __restrict__ G,
                                float* __restrict__ loss_partial) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    float d = 0.f;
    if (idx < n) {
        d = Y[idx] - T[idx];
        G[idx] = 2.f * d * inv_n;
    }
    float sq = d * d;
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) loss_partial[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv_n;
}

__global__ void sum_kernel(int n, const float* __restrict__ x, float* __restrict__ out) {
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

// dW[o, i] = sum_b G[b, o] H[b, i];  db[o] = sum_b G[b, o]
__global__ void linear_wgrad_kernel(int B, int nin, int nout, const float* __restrict__ G,
                                    const float* __restrict__ H, float* __restrict__ dW,
                                    float* __restrict__ db) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < nout * nin) {
        const int o = idx / nin, i = idx % nin;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s = fmaf(G[(long)b * nout + o], H[(long)b * nin + i], s);
        dW[idx] = s;
    } else if (idx < nout * nin + nout) {
        const int o = idx - nout * nin;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += G[(long)b * nout + o];
        db[o] = s;
    }
}

// Gin[b, i] = (sum_o G[b, o] W[o, i]) (1 - H[b, i]^2)   (H = tanh output of the previous layer)
__global__ void linear_igrad_kernel(int B, int nin, int nout, const float* __restrict__ G,
                                    const float* __restrict__ W, const float* __restrict__ H,
                                    float* __restrict__ Gin) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * nin) return;
    const int b = idx / nin, i = idx % nin;
    float s = 0.f;
    for (int o = 0; o < nout; ++o) s = fmaf(G[(long)b * nout + o], W[(long)o * nin + i], s);
    const float h = H[idx];
    Gin[idx] = s * (1.f - h * h);
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void adam_kernel(long n, float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__device__ inline unsigned long long mix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// W ~ U(-1/sqrt(nin), 1/sqrt(nin)) from a counter-based hash, bias = 0
__global__ void init_layer_kernel(int nin, int nout, unsigned long long seed, float* W, float* b) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const float lim = 1.f / sqrtf((float)nin);
    if (idx < nin * nout) {
        const unsigned long long h = mix64(seed ^ mix64((unsigned long long)idx + 1));
        const float u = (float)((h >> 40) * (1.0 / 16777216.0));  // [0, 1)
        W[idx] = (2.f * u - 1.f) * lim;
    } else if (idx < nin * nout + nout) {
        b[idx - nin * nout] = 0.f;
    }
}

// Features of one problem (row of X):
//   x[0..n_mom-1] = m~_l / K            (stochastic moments per basis function)
//   x[n_mom + 0]  = Ebar / dE           (where zero energy sits in the interval)
//   x[n_mom + 1]  = log10(dE)
//   x[n_mom + 2]  = log10(beta dE) / 4  (sharpness of f_FD on the interval)
//   x[n_mom + 3]  = 4 n_e / (g K) - 2   (filling)
__global__ void features_kernel(int n_mom, const double* m, double emin, double emax, double beta,
                                double n_e, double spin, double K, float* x) {
    const int l = threadIdx.x;
    const double ebar = 0.5 * (emax + emin), de = 0.5 * (emax - emin);
    if (l < n_mom) x[l] = (float)(m[l] / K);
    if (l == 0) {
        x[n_mom + 0] = (float)(ebar / de);
        x[n_mom + 1] = (float)log10(de);
        x[n_mom + 2] = (float)(0.25 * log10(beta * de));
        x[n_mom + 3] = (float)(4.0 * n_e / (spin * K) - 2.0);
    }
}

}  // namespace

hipError_t mlp_linear_fwd(int B, int nin, int nout, const float* X, const float* W, const float* b,
                          bool use_tanh, float* Y, hipStream_t s) {
    const int n = B * nout;
    hipLaunchKernelGGL(linear_fwd_kernel, dim3((n + 255) / 256), dim3(256), 0, s, B, nin, nout, X, W,
                       b, (int)use_tanh, Y);
    return hipGetLastError();
}

hipError_t mlp_mse_grad(int n, const float* Y, const float* T, float* G, float* partial,
                        float* loss, hipStream_t s) {
    const int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks), dim3(256), 0, s, n, 1.f / n, Y, T, G, partial);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, blocks, partial, loss);
    return hipGetLastError();
}

hipError_t mlp_linear_bwd(int B, int nin, int nout, const float* G, const float* H, const float* W,
                          float* dW, float* db, float* Gin, hipStream_t s) {
    const int nw = nout * nin + nout;
    hipLaunchKernelGGL(linear_wgrad_kernel, dim3((nw + 255) / 256), dim3(256), 0, s, B, nin, nout, G,
                       H, dW, db);
    if (Gin) {
        const int n = B * nin;
        hipLaunchKernelGGL(linear_igrad_kernel, dim3((n + 255) / 256), dim3(256), 0, s, B, nin, nout,
                           G, W, H, Gin);
    }
    return hipGetLastError();
}

hipError_t mlp_adam(long n, float* w, const float* g, float* m, float* v, float lr, int t,
                    hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, w, g, m, v,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_init_layer(int nin, int nout, unsigned long long seed, float* W, float* b,
                          hipStream_t s) {
    const int n = nin * nout + nout;
    hipLaunchKernelGGL(init_layer_kernel, dim3((n + 255) / 256), dim3(256), 0, s, nin, nout, seed, W, b);
    return hipGetLastError();
}

hipError_t mlp_features(int n_mom, const double* m, double emin, double emax, double beta,
                        double n_e, double spin, double K, float* x, hipStream_t s) {
    hipLaunchKernelGGL(features_kernel, dim3(1), dim3(n_mom < 64 ? 64 : ((n_mom + 63) / 64) * 64), 0,
                       s, n_mom, m, emin, emax, beta, n_e, spin, K, x);
    return hipGetLastError();
}

}  // namespace dm
