// gfx950 kernels of the cost-model MLP (24 -> 64 -> 64 -> 1, ReLU), the
// learned replacement of the paper's configuration derivation by scattered
// data interpolation (Sec. 3.2).  The layer products run on the matrix cores
// (fp32 MFMA, 16 x 16 x 4), one wavefront per 16 samples:
//  forward   the two hidden layers as 16 x 24 x 64 and 16 x 64 x 64 products,
//            the output unit as a cross-lane dot product;
//  grad      forward, then dh1 = dz2 W2 and the weight gradients
//            dW2 = dz2^T h1 and dW1 = dz1^T x as products over the
//            wavefront's samples, written as one row per wavefront;
//  reduce    one thread per parameter adds the rows in order (deterministic,
//            no atomics);
//  adam      one thread per parameter.
// Parameter layout: W1 [64][24], b1 [64], W2 [64][64], b2 [64], W3 [64], b3.
#include "kern_common.h"
#include "kern.h"

#include <algorithm>

namespace skel {

constexpr int kIn = 24, kH1 = 64, kH2 = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH1 * kIn, oW2 = oB1 + kH1, oB2 = oW2 + kH2 * kH1, oW3 = oB2 + kH2,
              oB3 = oW3 + kH2, kNP = oB3 + 1;
static_assert(kNP == 5825, "parameter count");

// Matrix-core formulation.  v_mfma_f32_16x16x4f32 computes D[16x16] +=
// A[16x4] B[4x16] over a wavefront: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4(l/16)+r][l%16] in accumulator register r.  One
// wavefront owns 16 samples; a 16 x K by K x 64 product is 4 output tiles of
// K/4 steps.  Activations are turned from the D layout into the A layout
// through a 16 x 64 LDS tile per wavefront.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Orders a wavefront's LDS writes before its following LDS reads by other
// lanes of the same wavefront.
static __device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static __device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Parameters in LDS (the same layout as in memory) plus two 16 x 64 tiles per
// wavefront.
constexpr int kWaves = 4;
struct MlpSmem {
    float P[kNP];
    float T[kWaves][2][16 * 64];
};

static __device__ __forceinline__ void load_params(MlpSmem& S, const float* params) {
    for (int k = threadIdx.x; k < kNP; k += blockDim.x) S.P[k] = params[k];
}

// Forward pass of the wavefront's 16 samples (rows of X given by `row`, valid
// when row >= 0).  Returns z1 and z2 (pre-activations, D layout, 4 tiles of
// 64 outputs) and y for samples 4(l/16) + r; leaves h1 = relu(z1) as a
// [sample][unit] tile in H.
static __device__ __forceinline__ void forward16(const MlpSmem& S, const float* X, int row, float* H,
                                                 f32x4 (&z1)[4], f32x4 (&z2)[4], float (&y)[4]) {
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
    const float* W1 = S.P + oW1;
    const float* W2 = S.P + oW2;
    float xa[kIn / 4];
#pragma unroll
    for (int s = 0; s < kIn / 4; ++s) xa[s] = row >= 0 ? X[(size_t)row * kIn + 4 * s + g] : 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < kIn / 4; ++s) acc = mfma4(xa[s], W1[(16 * t + c) * kIn + 4 * s + g], acc);
        const float b = S.P[oB1 + 16 * t + c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            acc[r] += b;
            H[(4 * g + r) * 64 + 16 * t + c] = acc[r] > 0.0f ? acc[r] : 0.0f;
        }
        z1[t] = acc;
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < kH1 / 4; ++s) acc = mfma4(H[c * 64 + 4 * s + g], W2[(16 * t + c) * kH1 + 4 * s + g], acc);
        const float b = S.P[oB2 + 16 * t + c];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += b;
        z2[t] = acc;
    }
    // y = b3 + sum_o relu(z2) W3[o]: per lane over its 4 columns, then across
    // the 16 lanes of its row group (fixed butterfly order).
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float p = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) p = __builtin_fmaf(z2[t][r] > 0.0f ? z2[t][r] : 0.0f, S.P[oW3 + 16 * t + c], p);
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) p += __shfl_xor(p, off, 64);
        y[r] = p + S.P[oB3];
    }
}

__global__ void __launch_bounds__(64 * kWaves) mlp_forward_kernel(const float* __restrict__ params,
                                                                  const float* __restrict__ X, int n,
                                                                  float* __restrict__ y) {
    __shared__ MlpSmem S;
    load_params(S, params);
    __syncthreads();
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4, w = threadIdx.x >> 6;
    const int base = (blockIdx.x * kWaves + w) * 16;
    if (base >= n) return;
    const int row = base + c < n ? base + c : -1;
    f32x4 z1[4], z2[4];
    float yy[4];
    forward16(S, X, row, S.T[w][0], z1, z2, yy);
    if (c == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (base + 4 * g + r < n) y[base + 4 * g + r] = yy[r];
}

// Gradient of L = mean over the n samples of (y - t)^2 for the wavefront's 16
// samples (X rows idx[b] or b): writes one row of kNP + 1 floats (the
// parameter gradient terms, then the sum of squared errors) to
// part[wavefront index].  The rows are summed in order by mlp_grad_reduce.
__global__ void __launch_bounds__(64 * kWaves) mlp_grad_kernel(const float* __restrict__ params,
                                                               const float* __restrict__ X,
                                                               const float* __restrict__ tgt,
                                                               const int* __restrict__ idx, int n,
                                                               float* __restrict__ part) {
    __shared__ MlpSmem S;
    load_params(S, params);
    __syncthreads();
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4, w = threadIdx.x >> 6;
    const int wave = blockIdx.x * kWaves + w;
    const int base = wave * 16;
    if (base >= n) return;
    float* H = S.T[w][0];   // h1 [sample][unit]
    float* D = S.T[w][1];   // dz2, then dz1 [sample][unit]
    const int row = base + c < n ? (idx ? idx[base + c] : base + c) : -1;
    f32x4 z1[4], z2[4];
    float y[4];
    forward16(S, X, row, H, z1, z2, y);
    float* out = part + (size_t)wave * (kNP + 1);
    // dy for samples 4g + r (0 outside the batch) and the squared errors.
    float dy[4], sq = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int b = base + 4 * g + r;
        const float e = b < n ? y[r] - tgt[idx ? idx[b] : b] : 0.0f;
        dy[r] = (2.0f / (float)n) * e;
        sq = __builtin_fmaf(e, e, sq);
    }
    // dz2 = dy W3 where z2 > 0; db3, dW3 and db2 reduce over the samples.
    float gW3[4], gB2[4], gB3 = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) gB3 += dy[r];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gW3[t] = 0.0f;
        gB2[t] = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float h2 = z2[t][r] > 0.0f ? z2[t][r] : 0.0f;
            const float d = z2[t][r] > 0.0f ? dy[r] * S.P[oW3 + 16 * t + c] : 0.0f;
            gW3[t] = __builtin_fmaf(dy[r], h2, gW3[t]);
            gB2[t] += d;
            D[(4 * g + r) * 64 + 16 * t + c] = d;
        }
    }
    wave_lds_sync();
    // dh1 = dz2 W2 (W2 [o][i]: B[k = o][n = i]); dz1 = dh1 where z1 > 0.
    f32x4 dz1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < kH2 / 4; ++s) acc = mfma4(D[c * 64 + 4 * s + g], S.P[oW2 + (4 * s + g) * kH1 + 16 * t + c], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = z1[t][r] > 0.0f ? acc[r] : 0.0f;
        dz1[t] = acc;
    }
    // dW2[o][i] = sum_s dz2[s][o] h1[s][i]: A[m = o][k = s] = D[s][o], B[k = s][n = i] = H[s][i].
#pragma unroll
    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc = mfma4(D[(4 * s + g) * 64 + 16 * tm + c], H[(4 * s + g) * 64 + 16 * tn + c], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) out[oW2 + (16 * tm + 4 * g + r) * kH1 + 16 * tn + c] = acc[r];
        }
    wave_lds_sync();   // every lane has read D before it is overwritten
    float gB1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gB1[t] = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            gB1[t] += dz1[t][r];
            D[(4 * g + r) * 64 + 16 * t + c] = dz1[t][r];
        }
    }
    // X tile of the 16 samples into H (h1 is no longer needed): [sample][feature].
    {
        const int xr = base + c < n ? (idx ? idx[base + c] : base + c) : -1;
        for (int k = g; k < kIn; k += 4) H[c * 64 + k] = xr >= 0 ? X[(size_t)xr * kIn + k] : 0.0f;
    }
    wave_lds_sync();
    // dW1[o][k] = sum_s dz1[s][o] x[s][k]: A = D[s][o], B = H[s][k] (k < 24).
#pragma unroll
    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            const int k = 16 * tn + c;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc = mfma4(D[(4 * s + g) * 64 + 16 * tm + c], k < kIn ? H[(4 * s + g) * 64 + k] : 0.0f, acc);
            if (k < kIn)
#pragma unroll
                for (int r = 0; r < 4; ++r) out[oW1 + (16 * tm + 4 * g + r) * kIn + k] = acc[r];
        }
    // Column sums over the 4 row groups (lanes c, c+16, c+32, c+48), fixed order.
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gB1[t] += __shfl_xor(gB1[t], 16, 64);
        gB1[t] += __shfl_xor(gB1[t], 32, 64);
        gB2[t] += __shfl_xor(gB2[t], 16, 64);
        gB2[t] += __shfl_xor(gB2[t], 32, 64);
        gW3[t] += __shfl_xor(gW3[t], 16, 64);
        gW3[t] += __shfl_xor(gW3[t], 32, 64);
    }
    gB3 += __shfl_xor(gB3, 16, 64);
    gB3 += __shfl_xor(gB3, 32, 64);
    sq += __shfl_xor(sq, 16, 64);
    sq += __shfl_xor(sq, 32, 64);
    if (g == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            out[oB1 + 16 * t + c] = gB1[t];
            out[oB2 + 16 * t + c] = gB2[t];
            out[oW3 + 16 * t + c] = gW3[t];
        }
        if (c == 0) {
            out[oB3] = gB3;
            out[kNP] = sq;
        }
    }
}

// grad[p] = sum of the wavefront rows' entry p in row order; the loss is the
// sum of their squared errors over n.
__global__ void __launch_bounds__(256) mlp_grad_reduce_kernel(const float* __restrict__ part, int rows, int n,
                                                              float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNP) return;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    int r = 0;
    for (; r + 4 <= rows; r += 4) {
        a0 += part[(size_t)r * (kNP + 1) + p];
        a1 += part[(size_t)(r + 1) * (kNP + 1) + p];
        a2 += part[(size_t)(r + 2) * (kNP + 1) + p];
        a3 += part[(size_t)(r + 3) * (kNP + 1) + p];
    }
    for (; r < rows; ++r) a0 += part[(size_t)r * (kNP + 1) + p];
    const float v = (a0 + a1) + (a2 + a3);
    if (p == kNP) {
        if (loss) *loss = v / (float)n;
    } else {
        grad[p] = v;
    }
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

static int mlp_waves(int n) { return (n + 15) / 16; }

size_t mlp_grad_work_floats(int n) { return (size_t)std::max(1, mlp_waves(n)) * (kNP + 1); }

hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int wgs = (mlp_waves(n) + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(wgs), dim3(64 * kWaves), 0, s, params, X, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad_idx(const float* params, const float* X, const float* t, const int* idx, int n,
                               float* grad, float* loss, float* work, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    const int rows = mlp_waves(n);
    const int wgs = (rows + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(wgs), dim3(64 * kWaves), 0, s, params, X, t, idx, n, work);
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, (const float*)work,
                       rows, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* X, const float* t, int n, float* grad, float* loss,
                           float* work, hipStream_t s) {
    return launch_mlp_grad_idx(params, X, t, nullptr, n, grad, loss, work, s);
}

hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr, float b1,
                           float b2, float eps, hipStream_t s) {
    // Bias corrections 1 - beta^t in double, rounded once: for beta2 = 0.999
    // and small t the difference cancels, and rounding beta^t to fp32 before
    // subtracting would cost ~1.5e-5 relative in 1 - beta2^2.
    const float c1 = (float)(1.0 - pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)step));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNP + 255) / 256), dim3(256), 0, s, params, grad, m, v, c1, c2, lr,
                       b1, b2, eps);
    return hipGetLastError();
}

}  // namespace skel
