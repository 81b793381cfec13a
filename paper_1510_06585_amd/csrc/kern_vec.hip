// gfx950 kernels for fp32 vector skeletons: fused saxpy / reversal chains
// (Sec. 4 Saxpy: single-precision a*x + y, here one fused multiply-add per
// stage) with an optional sum-reduce epilogue (MapReduce, Sec. 2.1).
//
// Each lane moves 16 bytes per access; a chain of k stages reads the input
// and k side vectors once and writes the output once.  A reversal is an
// address remap: stage inputs are read at u or n-1-u of the kernel's
// iteration coordinate u.  The sum is formed per thread, per wavefront
// (cross-lane adds) and per work-group (LDS); a second kernel adds the
// work-group partials in a fixed order in fp64.
#include "kern_common.h"
#include "kern.h"

namespace skel {

static __device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(1024) vec_chain_kernel(const VecGroupArgs A) {
    __shared__ float wsum[16];
    const int64_t n = A.n;
    const uint32_t nbytes = (uint32_t)(n * 4);
    const __amdgpu_buffer_rsrc_t rin = mk_rsrc(A.in, nbytes);
    const __amdgpu_buffer_rsrc_t rout = mk_rsrc(A.out, nbytes);
    const int64_t nvec = (n + 3) / 4;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    float acc = 0.0f;
    for (int e = 0; e < A.ept; ++e) {
        const int64_t v = (int64_t)e * nthreads + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (v >= nvec) break;
        const int64_t u0 = v * 4;
        float x[4];
        const bool fullv = (u0 + 4 <= n);
        if (fullv) {
            const u32x4 r = ld128(rin, (uint32_t)(u0 * 4));
            x[0] = __uint_as_float(r.x); x[1] = __uint_as_float(r.y);
            x[2] = __uint_as_float(r.z); x[3] = __uint_as_float(r.w);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = __uint_as_float(ld32(rin, (uint32_t)((u0 + i) * 4)));
        }
        for (int k = 0; k < A.nops; ++k) {
            const __amdgpu_buffer_rsrc_t rs = mk_rsrc(A.side[k], nbytes);
            const float a = A.a[k];
            float w[4];
            if (A.flip[k]) {
                if (fullv) {
                    const u32x4 r = ld128(rs, (uint32_t)((n - 4 - u0) * 4));
                    w[0] = __uint_as_float(r.w); w[1] = __uint_as_float(r.z);
                    w[2] = __uint_as_float(r.y); w[3] = __uint_as_float(r.x);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t src = n - 1 - (u0 + i);
                        w[i] = src >= 0 ? __uint_as_float(ld32(rs, (uint32_t)(src * 4))) : 0.0f;
                    }
                }
            } else {
                if (fullv) {
                    const u32x4 r = ld128(rs, (uint32_t)(u0 * 4));
                    w[0] = __uint_as_float(r.x); w[1] = __uint_as_float(r.y);
                    w[2] = __uint_as_float(r.z); w[3] = __uint_as_float(r.w);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) w[i] = __uint_as_float(ld32(rs, (uint32_t)((u0 + i) * 4)));
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = __builtin_fmaf(a, x[i], w[i]);
        }
        if (fullv) {
            acc += (x[0] + x[1]) + (x[2] + x[3]);
            if (A.write_out) {
                u32x4 r;
                if (A.out_flip) {
                    r.x = __float_as_uint(x[3]); r.y = __float_as_uint(x[2]);
                    r.z = __float_as_uint(x[1]); r.w = __float_as_uint(x[0]);
                    st128(r, rout, (uint32_t)((n - 4 - u0) * 4));
                } else {
                    r.x = __float_as_uint(x[0]); r.y = __float_as_uint(x[1]);
                    r.z = __float_as_uint(x[2]); r.w = __float_as_uint(x[3]);
                    st128(r, rout, (uint32_t)(u0 * 4));
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (u0 + i < n) {
                    acc += x[i];
                    if (A.write_out) {
                        const int64_t dst = A.out_flip ? (n - 1 - (u0 + i)) : (u0 + i);
                        st32(__float_as_uint(x[i]), rout, (uint32_t)(dst * 4));
                    }
                }
            }
        }
    }
    if (A.partials == nullptr) return;
    // Reduce: wavefront, then work-group (fixed order); the work-group's
    // partial is stored, and vec_sum_merge_kernel adds the partials.
    acc = wave_sum_f32(acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += wsum[w];
        A.partials[blockIdx.x] = s;
    }
}

// One 1024-thread work-group adds the n work-group partials in fp64 in a fixed
// order (thread t: partials t, t + 1024, ...; then a tree over the threads)
// and stores the rounded sum.  Launched after vec_chain_kernel on the same
// stream, so no inter-work-group synchronisation is needed.
constexpr int kMergeThreads = 1024;
__global__ void __launch_bounds__(kMergeThreads) vec_sum_merge_kernel(const float* partials, int n, float* out) {
    __shared__ double red[kMergeThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kMergeThreads) s += (double)partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kMergeThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)red[0];
}

hipError_t launch_vec_group(const VecGroupArgs& a, int grid, int wg, hipStream_t s, const char** kname) {
    if (kname) *kname = "vec_chain";
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(vec_chain_kernel, dim3(grid), dim3(wg), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.partials) return e;
    hipLaunchKernelGGL(vec_sum_merge_kernel, dim3(1), dim3(kMergeThreads), 0, s, (const float*)a.partials, grid,
                       a.sum_out);
    return hipGetLastError();
}

}  // namespace skel
