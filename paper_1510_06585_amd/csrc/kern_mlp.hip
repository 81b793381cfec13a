// gfx950 kernels of the cost-model MLP (24 -> 64 -> 64 -> 1, ReLU), the
// learned replacement of the paper's configuration derivation by scattered
// data interpolation (Sec. 3.2).  The network is tiny (5825 parameters), so
// the kernels are organised for fixed summation order rather than peak rate:
//  forward   one thread per sample, weights staged once per work-group in LDS
//            and read as broadcasts;
//  deltas    one thread per sample, back-propagates dL/dz through both layers;
//  wgrad     one thread per parameter, sums its per-sample terms over the
//            batch in sample order (deterministic, no atomics);
//  adam      one thread per parameter.
// Parameter layout: W1 [64][24], b1 [64], W2 [64][64], b2 [64], W3 [64], b3.
#include "kern_common.h"
#include "kern.h"

namespace skel {

constexpr int kIn = 24, kH1 = 64, kH2 = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH1 * kIn, oW2 = oB1 + kH1, oB2 = oW2 + kH2 * kH1, oW3 = oB2 + kH2,
              oB3 = oW3 + kH2, kNP = oB3 + 1;
static_assert(kNP == 5825, "parameter count");
constexpr int kRec = kH1 + kH2 + 1;   // per-sample record: z1, z2, y  (or dz1, dz2, dy)

// Forward pass; when rec != null also stores z1, z2 and y per sample.
__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* __restrict__ params,
                                                          const float* __restrict__ X,
                                                          const int* __restrict__ idx, int n,
                                                          float* __restrict__ y, float* __restrict__ rec) {
    __shared__ float P[kNP];
    for (int k = threadIdx.x; k < kNP; k += blockDim.x) P[k] = params[k];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int row = idx ? idx[b] : b;
    float x[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i] = X[(size_t)row * kIn + i];
    float h1[kH1];
#pragma unroll
    for (int o = 0; o < kH1; ++o) {
        float z = P[oB1 + o];
#pragma unroll
        for (int i = 0; i < kIn; ++i) z = __builtin_fmaf(P[oW1 + o * kIn + i], x[i], z);
        if (rec) rec[(size_t)b * kRec + o] = z;
        h1[o] = z > 0.0f ? z : 0.0f;
    }
    float out = P[oB3];
    for (int o = 0; o < kH2; ++o) {
        float z = P[oB2 + o];
#pragma unroll
        for (int i = 0; i < kH1; ++i) z = __builtin_fmaf(P[oW2 + o * kH1 + i], h1[i], z);
        if (rec) rec[(size_t)b * kRec + kH1 + o] = z;
        out = __builtin_fmaf(P[oW3 + o], z > 0.0f ? z : 0.0f, out);
    }
    if (rec) rec[(size_t)b * kRec + kH1 + kH2] = out;
    if (y) y[b] = out;
}

// dL/dz for the MSE loss L = mean (y - t)^2 over the n samples.
__global__ void __launch_bounds__(256) mlp_delta_kernel(const float* __restrict__ params,
                                                        const float* __restrict__ rec,
                                                        const float* __restrict__ t,
                                                        const int* __restrict__ idx, int n,
                                                        float* __restrict__ del) {
    __shared__ float W2[kH2 * kH1];
    __shared__ float W3[kH2];
    for (int k = threadIdx.x; k < kH2 * kH1; k += blockDim.x) W2[k] = params[oW2 + k];
    for (int k = threadIdx.x; k < kH2; k += blockDim.x) W3[k] = params[oW3 + k];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const float* r = rec + (size_t)b * kRec;
    float* d = del + (size_t)b * kRec;
    const int row = idx ? idx[b] : b;
    const float dy = (2.0f / (float)n) * (r[kH1 + kH2] - t[row]);
    d[kH1 + kH2] = dy;
    float dz2[kH2];
#pragma unroll
    for (int o = 0; o < kH2; ++o) {
        dz2[o] = r[kH1 + o] > 0.0f ? dy * W3[o] : 0.0f;
        d[kH1 + o] = dz2[o];
    }
    for (int i = 0; i < kH1; ++i) {
        float g = 0.0f;
#pragma unroll
        for (int o = 0; o < kH2; ++o) g = __builtin_fmaf(dz2[o], W2[o * kH1 + i], g);
        d[i] = r[i] > 0.0f ? g : 0.0f;
    }
}

// grad[p] = sum over samples of that parameter's term, in sample order; the
// extra thread p == kNP writes the loss.
__global__ void __launch_bounds__(256) mlp_wgrad_kernel(const float* __restrict__ X,
                                                        const float* __restrict__ rec,
                                                        const float* __restrict__ del,
                                                        const float* __restrict__ t,
                                                        const int* __restrict__ idx, int n,
                                                        float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNP) return;
    float g = 0.0f;
    if (p == kNP) {
        for (int b = 0; b < n; ++b) {
            const int row = idx ? idx[b] : b;
            const float e = rec[(size_t)b * kRec + kH1 + kH2] - t[row];
            g = __builtin_fmaf(e, e, g);
        }
        if (loss) *loss = g / (float)n;
        return;
    }
    if (p < oB1) {
        const int o = p / kIn, i = p % kIn;
        for (int b = 0; b < n; ++b) {
            const int row = idx ? idx[b] : b;
            g = __builtin_fmaf(del[(size_t)b * kRec + o], X[(size_t)row * kIn + i], g);
        }
    } else if (p < oW2) {
        const int o = p - oB1;
        for (int b = 0; b < n; ++b) g += del[(size_t)b * kRec + o];
    } else if (p < oB2) {
        const int o = (p - oW2) / kH1, i = (p - oW2) % kH1;
        for (int b = 0; b < n; ++b) {
            const float z1 = rec[(size_t)b * kRec + i];
            g = __builtin_fmaf(del[(size_t)b * kRec + kH1 + o], z1 > 0.0f ? z1 : 0.0f, g);
        }
    } else if (p < oW3) {
        const int o = p - oB2;
        for (int b = 0; b < n; ++b) g += del[(size_t)b * kRec + kH1 + o];
    } else if (p < oB3) {
        const int i = p - oW3;
        for (int b = 0; b < n; ++b) {
            const float z2 = rec[(size_t)b * kRec + kH1 + i];
            g = __builtin_fmaf(del[(size_t)b * kRec + kH1 + kH2], z2 > 0.0f ? z2 : 0.0f, g);
        }
    } else {
        for (int b = 0; b < n; ++b) g += del[(size_t)b * kRec + kH1 + kH2];
    }
    grad[p] = g;
}

__global__ void mlp_adam_kernel(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, float c1, float c2, float lr, float b1, float b2,
                                float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float mh = mp / c1, vh = vp / c2;
    th[p] -= lr * mh / (sqrtf(vh) + eps);
}

size_t mlp_grad_work_floats(int n) { return (size_t)2 * (size_t)n * kRec; }

hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, s, params, X,
                       (const int*)nullptr, n, y, (float*)nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_grad_idx(const float* params, const float* X, const float* t, const int* idx, int n,
                               float* grad, float* loss, float* work, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    float* rec = work;
    float* del = work + (size_t)n * kRec;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, s, params, X, idx, n,
                       (float*)nullptr, rec);
    hipLaunchKernelGGL(mlp_delta_kernel, dim3((n + 255) / 256), dim3(256), 0, s, params, (const float*)rec, t,
                       idx, n, del);
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, X, (const float*)rec,
                       (const float*)del, t, idx, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* X, const float* t, int n, float* grad, float* loss,
                           float* work, hipStream_t s) {
    return launch_mlp_grad_idx(params, X, t, nullptr, n, grad, loss, work, s);
}

hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr, float b1,
                           float b2, float eps, hipStream_t s) {
    const float c1 = 1.0f - (float)pow((double)b1, (double)step);
    const float c2 = 1.0f - (float)pow((double)b2, (double)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNP + 255) / 256), dim3(256), 0, s, params, grad, m, v, c1, c2, lr,
                       b1, b2, eps);
    return hipGetLastError();
}

}  // namespace skel
