// Launch interface between the host runtime (plan/executor) and the gfx950
// kernels.  Plain structs passed by value as kernel arguments.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace skel {

constexpr int kMaxOps = 8;          // value stages per side of a fused image kernel
constexpr int kBandOut = 252;       // output pixels per wavefront band (stencil kernels)
constexpr int kBandPx = 256;        // pixels a wavefront loads per row (64 lanes x 4)

// Value (non-moving) image stages inside a fused kernel.
enum : uint8_t { IOP_NONE = 0, IOP_NOISE = 1, IOP_SOL = 2 };

// A run of value stages.  flip[k] = 1 when stage k sees the mirrored
// coordinate W-1-u of the kernel's iteration coordinate u.
struct OpList {
    int32_t n;
    uint8_t op[kMaxOps];
    uint8_t flip[kMaxOps];
    uint32_t seed[kMaxOps];
};

// One fused image kernel: pre-stages, an optional 5x5 blur, post-stages, an
// optional histogram/sum epilogue.  The kernel iterates over coordinates u of
// the blur's frame (or of its input, without a blur); it reads the input at
// in_flip ? W-1-u : u and writes the output at out_flip ? W-1-u : u.
struct ImgGroupArgs {
    const uint8_t* in;
    uint8_t* out;
    uint32_t* part;      // histogram epilogue: one row of 4 x bins counts per work-group
    uint32_t* hist;      // reduce outputs cleared by work-group 0 (may be null)
    uint64_t* sum;
    int32_t bins;        // values emitted are < bins (128 or 256)
    int32_t W, H;
    int32_t tile_h;      // rows per tile
    int32_t nbands;      // tiles across a row
    int32_t ntiles;      // nbands * ceil(H / tile_h)
    int32_t in_flip, out_flip;
    int32_t write_out;   // 0 for a reduce-only kernel
    int32_t hist_ks;     // log2 of the histogram copies per bin (see hist_copies_log2)
    const uint32_t* guard;   // while Loop: the launch does nothing when *guard == 0 (null: always runs)
    OpList pre, post;
};

// Output values of a kernel are < bins (128 when the chain's last value stage
// is a solarise, else 256); the LDS histogram keeps copies = words / bins
// counters per bin, one per lane class, so equal values in neighbouring lanes
// hit different words and banks.  Returns log2(copies) for a per-channel
// region of `words` counters.
int hist_copies_log2(int bins, int words);
constexpr int kHistWgWords = 2048;     // per channel, one histogram per work-group

// Compile-time encoding of a value-stage run for specialised kernels:
// sum of op_k * 4^k; -1 selects the generic stage interpreter.
constexpr int kGeneric = -1;
int encode_ops(const OpList& l);

// Launches one fused image kernel with `wg` threads per work-group (64, 128
// or 256).  variant 1 forces the generic interpreter.  *kname receives the
// kernel's name.  t0 / t1 (may be null): events timestamped by the kernel's
// own dispatch (start and end of its execution).
hipError_t launch_img_group(const ImgGroupArgs& a, bool blur, bool hist, int wg, int variant,
                            hipStream_t s, const char** kname, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

const char* img_kernel_name(const ImgGroupArgs& a, bool blur, bool hist, int variant);
// Resident wavefronts per CU of the kernel launch_img_group would pick (16
// when the occupancy query is unavailable, e.g. without a device).
int img_waves_per_cu(const ImgGroupArgs& a, bool blur, bool hist, int wg, int variant);

// Merge of histogram rows (the reduce's merge function, Sec. 3.4): a segment
// owns rows [row_begin, row_begin + nrows) of 4 x bins counts, summed in
// chunks of crows rows by one 1024-thread work-group each, which adds its
// non-zero counts (and the channel sums they imply) to the segment's
// [4][256] histogram (may be null) and [4] sums with device-scope atomics.
// The outputs must be cleared before (hist_zero, or work-group 0 of the image
// kernel that writes the rows).
struct HistSeg {
    uint32_t* hist;
    uint64_t* sum;
    int32_t row_begin, nrows;
    int32_t crows, chunk_begin;
};
struct HistFinArgs {
    const uint32_t* part;
    const uint32_t* guard;   // as ImgGroupArgs::guard
    const HistSeg* segs;   // device array of nseg segments, or null for `one`
    HistSeg one;
    int32_t nseg;
    int32_t nchunks;       // chunks over all segments
    int32_t bins;
    int32_t pad;
};
// Rows per chunk for rows of 4 x bins words: 8 rows per thread of a
// 1024-thread work-group.
int hist_chunk_rows(int bins);
inline int hist_chunks(int n, int crows) { return n > 0 ? (n + crows - 1) / crows : 0; }
hipError_t launch_hist_merge(const HistFinArgs& a, hipStream_t s);
hipError_t launch_hist_zero(const HistFinArgs& a, hipStream_t s);

// While Loop on the device.  state[0] = 1 while the loop runs, state[1] =
// iterations run, state[2..3] = the previous iteration's tested channel sum
// (uint64).  init sets {1, 0}; step (after each iteration's merge) merges the
// iteration's carried reduce outputs into their accumulators, counts the
// iteration, stores the count to *count_out and clears the flag when
// count == max or the condition fails (kind 0: sum[channel] cmp threshold;
// kind 1: |sum[channel] - previous| cmp threshold, always true after the
// first iteration); copy moves `bytes` from src to dst when max - count is
// odd (the last iteration wrote src).
struct WhileCond {
    int32_t channel, cmp;
    uint64_t threshold;
    int32_t max, kind;
};
// Carried reduce outputs: acc += the iteration's result (null: not carried).
struct WhileMerge {
    const uint32_t* it_hist;
    uint32_t* acc_hist;     // [4][256]
    const uint64_t* it_sum;
    uint64_t* acc_sum;      // [4]
};
hipError_t launch_while_init(uint32_t* state, hipStream_t s);
hipError_t launch_while_step(uint32_t* state, const uint64_t* sum, const WhileCond& c, const WhileMerge& m,
                             uint32_t* count_out, hipStream_t s);
hipError_t launch_while_copy(const uint32_t* state, const void* src, void* dst, uint64_t bytes, uint32_t max,
                             hipStream_t s);

// Work list entry of the batched persistent kernel (one per request).
struct BatchReq {
    const uint8_t* in;
    uint8_t* out;
    uint32_t* hist;
    uint64_t* sum;
    int32_t W, H;
    int32_t nbands, nchunks;
    int32_t tile_begin;  // first global tile index of this request (a multiple of the wavefronts per group)
    int32_t tile_h;      // rows per tile of this request
};
struct BatchArgs {
    const BatchReq* reqs;
    const uint16_t* tile_req;   // request index of every tile
    int32_t nreq;
    int32_t ntiles;
    int32_t has_blur;
    int32_t in_flip, out_flip;
    int32_t has_hist;
    int32_t hist_ks;     // log2 copies per bin of the work-group histograms
    int32_t bins;        // values emitted are < bins
    int32_t pad;
    uint32_t* part;      // histogram rows, one per tile group (ticket)
    uint32_t* counter;   // work-queue ticket counter (zeroed before launch)
    OpList pre, post;
};
hipError_t launch_img_batch(const BatchArgs& a, int grid, int wg, hipStream_t s, const char** kname);
// Resident work-groups per CU of the persistent kernel for this chain.
int img_batch_blocks_per_cu(const BatchArgs& a, int wg);

// Fill kernel (graph-safe replacement of memset): n 32-bit words of `value`.
hipError_t launch_fill_u32(void* p, uint64_t nwords, uint32_t value, hipStream_t s);

// ---------------------------------------------------------------- fp32 chains
constexpr int kMaxVecOps = 8;
struct VecGroupArgs {
    const float* in;
    float* out;
    int64_t n;
    int32_t nops;
    int32_t in_flip, out_flip;
    int32_t ept;              // 4-float vectors per thread
    float* partials;          // per work-group partial sums (reduce) or null
    float* sum_out;           // final sum (with partials)
    int32_t write_out;
    int32_t pad;
    const float* side[kMaxVecOps];
    float a[kMaxVecOps];
    uint8_t flip[kMaxVecOps];
};
// Launches the chain kernel and, when a.partials is set, the kernel that adds
// the work-group partials into a.sum_out.
hipError_t launch_vec_group(const VecGroupArgs& a, int grid, int wg, hipStream_t s, const char** kname);

// ------------------------------------------------------------ gray volumes
// Fused chain of SEGMENT stages over n voxels (bytes): stage k maps v to
// v < lo[k] ? 0 : (v < hi[k] ? 128 : 255).  in may equal out.
struct GrayArgs {
    const uint8_t* in;
    uint8_t* out;
    int64_t n;
    int32_t nops;
    int32_t ept;          // 16-byte vectors per thread
    uint16_t lo[kMaxOps], hi[kMaxOps];   // 0 <= lo <= hi <= 256
};
hipError_t launch_gray_chain(const GrayArgs& a, int grid, int wg, hipStream_t s);

// --------------------------------------------------------------- complex FFT
// Batched 65536-point complex fp32 transforms (interleaved re, im), four-step
// 256 x 256.  mode 0: pass A (natural order in, transposed out), mode 1:
// pass B of a stage fused with pass A of the next, mode 2: pass B
// (transposed in, natural order out).  in and out must not overlap.
struct FftArgs {
    const void* in;
    void* out;
    const float2* tw;    // 65536 roots of unity (cos, sin)(2 pi m / 65536)
    int32_t nfft;        // transforms in the batch
    int32_t dir1, dir2;  // -1 forward, +1 inverse
    float scale1;        // applied to a stage's pass-B result (1/65536 after an inverse)
};
constexpr int kFftPoints = 65536;
// Row stride, in complex elements, of the transposed layout T[k2][n1] that
// passes exchange through plan scratch: 256 + 16 keeps every row on a 128-byte
// line boundary while breaking the power-of-two stride of the column runs.
constexpr int kFftTRow = 256 + 16;
hipError_t launch_fft_pass(const FftArgs& a, int mode, hipStream_t s);
const char* fft_pass_name(int mode);

// -------------------------------------------------------------------- N-body
struct NBodyArgs {
    const float4* pos_in;   // [N] x,y,z,m
    float4* pos_out;        // [N]
    float4* vel;            // [N] (w unused), updated in place
    float4* acc;            // [N] accelerations (unfused force kernel) or null
    int32_t N;
    int32_t jsplit;         // wavefronts sharing one group of 64 bodies
    float eps2, G, dt;
    int32_t pad;
};
// Fused force + kick-drift (fused = true) or force only into acc.
hipError_t launch_nbody_force(const NBodyArgs& a, bool fused, hipStream_t s, const char** kname);
hipError_t launch_nbody_integrate(const NBodyArgs& a, hipStream_t s, const char** kname);
hipError_t launch_copy_f32x4(const float4* src, float4* dst, int64_t n, hipStream_t s);

// ------------------------------------------------------------------- MLP
hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* y, hipStream_t s);
hipError_t launch_mlp_grad(const float* params, const float* X, const float* t, int n, float* grad,
                           float* loss, float* work, hipStream_t s);
// As launch_mlp_grad over the samples idx[0..n) of X / t (idx may be null).
hipError_t launch_mlp_grad_idx(const float* params, const float* X, const float* t, const int* idx, int n,
                               float* grad, float* loss, float* work, hipStream_t s);
hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s);
size_t mlp_grad_work_floats(int n);

}  // namespace skel
