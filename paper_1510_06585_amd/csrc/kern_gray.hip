// gfx950 kernel for chains of Segmentation stages over a gray uint8 volume
// (Sec. 4 Segmentation: every voxel becomes black, gray or white; the stage is
// voxel-wise, so a chain of them is one pass over the bytes).
//
// Each lane moves 16 bytes per access through a raw buffer resource (the
// tail beyond n reads 0 and its stores are dropped by the range check).
//
// A stage's output takes only the values 0, 128 and 255, so a chain of k
// stages equals its first stage's split into three classes followed by the
// image of each class under stages 2..k: out = c0, c1 or c2 for v < lo1,
// lo1 <= v < hi1, v >= hi1.  Every wavefront folds the chain into
// (lo1, hi1, c0, c1, c2) once with uniform (scalar) arithmetic, so a voxel
// costs the same for any chain length.  A word's four bytes are split into
// two u16 pairs, bytes {0, 2} and {1, 3}; per pair, ge(v, t) =
// min(sat(v + 1 - t), 1) is 1 when v >= t, and the class value is
// c0 + ge(v, lo1) (c1 - c0) + ge(v, hi1) (c2 - c1) in 16-bit modular
// arithmetic (ge(v, hi1) = 1 implies ge(v, lo1) = 1, as lo1 <= hi1).
#include "kern_common.h"
#include "kern.h"

namespace skel {

constexpr int kGrayBatch = 4;   // 16-byte loads in flight per lane

struct GrayFold {
    uint32_t lo, hi;     // first stage's thresholds
    uint32_t c0, d1, d2; // class 0 value, class 1 - class 0, class 2 - class 1 (mod 2^16)
};

static __device__ __forceinline__ uint32_t seg_scalar(uint32_t v, uint32_t lo, uint32_t hi) {
    return v < lo ? 0u : (v < hi ? 128u : 255u);
}

static __device__ __forceinline__ GrayFold fold_chain(const GrayArgs& A) {
    uint32_t c[3] = {0u, 128u, 255u};
    for (int k = 1; k < A.nops; ++k)
        for (int j = 0; j < 3; ++j) c[j] = seg_scalar(c[j], A.lo[k], A.hi[k]);
    return {A.lo[0], A.hi[0], c[0], (c[1] - c[0]) & 0xFFFFu, (c[2] - c[1]) & 0xFFFFu};
}

static __device__ __forceinline__ u16x2 ge_pair(u16x2 v1, uint32_t t) {
    // v1 = v + 1; sat(v + 1 - t) capped at 1
    return __builtin_elementwise_min(__builtin_elementwise_sub_sat(v1, (u16x2)(unsigned short)t), (u16x2)1);
}

static __device__ __forceinline__ u16x2 classify_pair(u16x2 v, const GrayFold& F) {
    const u16x2 v1 = v + (u16x2)1;
    return (u16x2)(unsigned short)F.c0 + ge_pair(v1, F.lo) * (u16x2)(unsigned short)F.d1 +
           ge_pair(v1, F.hi) * (u16x2)(unsigned short)F.d2;
}

static __device__ __forceinline__ uint32_t segment_word(uint32_t w, const GrayFold& F) {
    const u16x2 e = as16(w & 0x00FF00FFu), o = as16(__builtin_amdgcn_perm(0u, w, 0x0C030C01u));
    return as32(classify_pair(e, F)) | (as32(classify_pair(o, F)) << 8);
}

__global__ void __launch_bounds__(1024) gray_chain_kernel(const GrayArgs A) {
    const uint32_t nbytes = (uint32_t)A.n;
    const __amdgpu_buffer_rsrc_t rin = mk_rsrc(A.in, nbytes);
    const __amdgpu_buffer_rsrc_t rout = mk_rsrc(A.out, nbytes);
    const GrayFold F = fold_chain(A);
    const int64_t nvec = (A.n + 15) / 16;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // Vectors e, e + 1, .. e + 3 of the thread are loaded before any is
    // stored, so four loads per lane are in flight.
    for (int e0 = 0; e0 < A.ept; e0 += kGrayBatch) {
        u32x4 r[kGrayBatch];
#pragma unroll
        for (int j = 0; j < kGrayBatch; ++j) {
            const int64_t v = (int64_t)(e0 + j) * nthreads + first;
            if (e0 + j < A.ept && v < nvec) r[j] = ld128(rin, (uint32_t)(v * 16));
        }
#pragma unroll
        for (int j = 0; j < kGrayBatch; ++j) {
            const int64_t v = (int64_t)(e0 + j) * nthreads + first;
            if (e0 + j >= A.ept || v >= nvec) break;
            const uint32_t off = (uint32_t)(v * 16);
            if (off + 16 <= nbytes) {
                r[j].x = segment_word(r[j].x, F);
                r[j].y = segment_word(r[j].y, F);
                r[j].z = segment_word(r[j].z, F);
                r[j].w = segment_word(r[j].w, F);
                st128(r[j], rout, off);
            } else {
                // ragged tail: byte by byte (n is not a multiple of 16)
                for (uint32_t b = off; b < nbytes; ++b) A.out[b] = (uint8_t)(segment_word(A.in[b], F) & 0xFFu);
            }
        }
    }
}

hipError_t launch_gray_chain(const GrayArgs& a, int grid, int wg, hipStream_t s) {
    if (a.n <= 0 || grid <= 0) return hipSuccess;
    if (a.n >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gray_chain_kernel, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}

}  // namespace skel
