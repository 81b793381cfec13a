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
// costs the same for any chain length.
//
// The four voxels of a 32-bit word are classified together, one byte per
// voxel.  v_lerp_u8 gives (a + b + 1) >> 1 for every byte; with b = 255 - t
// the sum reaches 256, i.e. bit 7 of the byte is set, exactly when v >= t.
// Two of them give the byte selector s = [v >= lo1] + 2 [v >= hi1] in
// {0, 1, 3}, and one byte permute of the word {c0, c1, -, c(255)} by s gives
// the four outputs: 7 instructions per word for any thresholds.  A threshold
// of 256 is clamped to 255, which only changes the selector of v = 255;
// entry 3 is therefore the class of 255 itself (c2, or c1 when hi1 = 256, or
// c0 when lo1 = 256).
#include "kern_common.h"
#include "kern.h"

namespace skel {

constexpr int kGrayBatch = 4;   // 16-byte loads in flight per lane

struct GrayFold {
    uint32_t blo, bhi;   // (255 - min(lo1, 255)) and (255 - min(hi1, 255)) in every byte
    uint32_t lut;        // bytes: c0, c1, 0, class of 255
};

static __device__ __forceinline__ uint32_t seg_scalar(uint32_t v, uint32_t lo, uint32_t hi) {
    return v < lo ? 0u : (v < hi ? 128u : 255u);
}

static __device__ __forceinline__ GrayFold fold_chain(const GrayArgs& A) {
    uint32_t c[3] = {0u, 128u, 255u};
    for (int k = 1; k < A.nops; ++k)
        for (int j = 0; j < 3; ++j) c[j] = seg_scalar(c[j], A.lo[k], A.hi[k]);
    const uint32_t lo = A.lo[0], hi = A.hi[0];
    const uint32_t top = 255u < lo ? c[0] : (255u < hi ? c[1] : c[2]);
    return {(255u - min(lo, 255u)) * 0x01010101u, (255u - min(hi, 255u)) * 0x01010101u,
            c[0] | (c[1] << 8) | (top << 24)};
}

static __device__ __forceinline__ uint32_t segment_word(uint32_t w, const GrayFold& F) {
    const uint32_t glo = __builtin_amdgcn_lerp(w, F.blo, 0x01010101u);   // bit 7 of byte i: v_i >= lo1
    const uint32_t ghi = __builtin_amdgcn_lerp(w, F.bhi, 0x01010101u);   // bit 7 of byte i: v_i >= hi1
    const uint32_t sel = ((glo >> 7) & 0x01010101u) | ((ghi >> 6) & 0x02020202u);
    return __builtin_amdgcn_perm(0u, F.lut, sel);
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
