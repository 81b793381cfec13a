// gfx950 kernels for the N-body Loop body (Sec. 4 N-Body: direct sum, every
// body reads every position -- the COPY transfer mode of Sec. 3.4).
//
// A work-group owns 64 bodies (one per lane) and `jsplit` wavefronts; wave w
// sums the interactions with bodies j in its slice of [0, N).  The j loop is
// wave-uniform, so body j's position and mass come in through scalar loads
// and each pair costs ~12 VALU ops plus one reciprocal square root, with no
// LDS traffic and no barrier inside the loop.  Interactions are accumulated
// in fp32 tiles of 256 j's and the tile partials are added into fp32 running
// sums; the slices are merged in a fixed order through LDS.  The fused kernel
// then applies the kick-drift update to its own bodies, so force and
// integration never round-trip through HBM.
#include "kern_common.h"
#include "kern.h"

namespace skel {

constexpr int kJTile = 256;
constexpr int kMaxJSplit = 16;

template <bool FUSED>
__global__ void __launch_bounds__(1024) nbody_force_kernel(const NBodyArgs A) {
    __shared__ float part[kMaxJSplit][3][64];
    const int lane = threadIdx.x & 63;
    const int w = wave_uniform(threadIdx.x >> 6);
    const int N = A.N;
    const int i = blockIdx.x * 64 + lane;
    const float4* __restrict__ P = A.pos_in;
    const float4 pi = P[i < N ? i : N - 1];
    const int chunk = (N + A.jsplit - 1) / A.jsplit;
    const int jb = w * chunk;
    const int je = min(jb + chunk, N);
    const float eps2 = A.eps2;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    for (int t0 = jb; t0 < je; t0 += kJTile) {
        const int t1 = min(t0 + kJTile, je);
        float tx = 0.0f, ty = 0.0f, tz = 0.0f;
#pragma unroll 8
        for (int j = t0; j < t1; ++j) {
            const float4 pj = P[j];
            const float dx = pj.x - pi.x;
            const float dy = pj.y - pi.y;
            const float dz = pj.z - pi.z;
            const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
            // d2 >= eps^2 > 0 is never denormal: the bare v_rsq_f32 instruction.
            const float inv = __builtin_amdgcn_rsqf(d2);
            const float s = (pj.w * inv) * (inv * inv);
            tx = __builtin_fmaf(s, dx, tx);
            ty = __builtin_fmaf(s, dy, ty);
            tz = __builtin_fmaf(s, dz, tz);
        }
        ax += tx;
        ay += ty;
        az += tz;
    }
    part[w][0][lane] = ax;
    part[w][1][lane] = ay;
    part[w][2][lane] = az;
    __syncthreads();
    if (w != 0 || i >= N) return;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    for (int k = 0; k < A.jsplit; ++k) {
        sx += part[k][0][lane];
        sy += part[k][1][lane];
        sz += part[k][2][lane];
    }
    sx *= A.G;
    sy *= A.G;
    sz *= A.G;
    if constexpr (FUSED) {
        // kick-drift: v += dt a; r += dt v
        float4 v = A.vel[i];
        v.x = __builtin_fmaf(A.dt, sx, v.x);
        v.y = __builtin_fmaf(A.dt, sy, v.y);
        v.z = __builtin_fmaf(A.dt, sz, v.z);
        A.vel[i] = v;
        float4 r = pi;
        r.x = __builtin_fmaf(A.dt, v.x, r.x);
        r.y = __builtin_fmaf(A.dt, v.y, r.y);
        r.z = __builtin_fmaf(A.dt, v.z, r.z);
        A.pos_out[i] = r;
    } else {
        A.acc[i] = make_float4(sx, sy, sz, 0.0f);
    }
}

__global__ void nbody_integrate_kernel(const NBodyArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.N) return;
    const float4 a = A.acc[i];
    float4 v = A.vel[i];
    v.x = __builtin_fmaf(A.dt, a.x, v.x);
    v.y = __builtin_fmaf(A.dt, a.y, v.y);
    v.z = __builtin_fmaf(A.dt, a.z, v.z);
    A.vel[i] = v;
    float4 r = A.pos_in[i];
    r.x = __builtin_fmaf(A.dt, v.x, r.x);
    r.y = __builtin_fmaf(A.dt, v.y, r.y);
    r.z = __builtin_fmaf(A.dt, v.z, r.z);
    A.pos_out[i] = r;
}

__global__ void copy_f32x4_kernel(const float4* src, float4* dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_nbody_force(const NBodyArgs& a, bool fused, hipStream_t s, const char** kname) {
    if (a.jsplit < 1 || a.jsplit > kMaxJSplit) return hipErrorInvalidValue;
    if (kname) *kname = fused ? "nbody_force_kick_drift" : "nbody_force";
    if (a.N <= 0) return hipSuccess;
    const int grid = (a.N + 63) / 64;
    if (fused)
        hipLaunchKernelGGL(nbody_force_kernel<true>, dim3(grid), dim3(64 * a.jsplit), 0, s, a);
    else
        hipLaunchKernelGGL(nbody_force_kernel<false>, dim3(grid), dim3(64 * a.jsplit), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_nbody_integrate(const NBodyArgs& a, hipStream_t s, const char** kname) {
    if (kname) *kname = "nbody_kick_drift";
    if (a.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(nbody_integrate_kernel, dim3((a.N + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy_f32x4(const float4* src, float4* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(copy_f32x4_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace skel
