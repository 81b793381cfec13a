// C-ABI entry points: SCT construction, plan compilation and execution
// requests (Table 1 of the paper), the device-resident Loop driver and the
// batched executor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

using namespace skel;

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(e_ == hipErrorOutOfMemory ? SKEL_ENOMEM : SKEL_EDEVICE, "%s: %s", \
                             #expr, hipGetErrorString(e_));                                    \
    } while (0)

namespace {

void node_addref(skel_node_s* n) {
    if (n) n->refs.fetch_add(1);
}

void node_release(skel_node_s* n) {
    if (!n) return;
    if (n->refs.fetch_sub(1) == 1) {
        for (skel_node_s* k : n->kids) node_release(k);
        delete n;
    }
}

skel_status new_node(skel_node* out, skel_node_s** n) {
    if (!out) return set_error(SKEL_EINVAL, "null output handle");
    *out = nullptr;
    *n = new (std::nothrow) skel_node_s();
    if (!*n) return set_error(SKEL_ENOMEM, "host allocation failed");
    return SKEL_OK;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// Byte range of a buffer, for overlap checks.
struct Range {
    uintptr_t lo, hi;
};
Range range_of(const skel_buffer& b) {
    int64_t bytes = b.ndim > 0 ? 1 : 0;
    for (int d = 0; d < b.ndim; ++d) bytes *= b.shape[d];
    const int64_t es = (b.dtype == SKEL_U8) ? 1 : ((b.dtype == SKEL_U64 || b.dtype == SKEL_F64) ? 8 : 4);
    return Range{(uintptr_t)b.data, (uintptr_t)b.data + (uintptr_t)(bytes * es)};
}
bool overlap(const skel_buffer& a, const skel_buffer& b) {
    const Range x = range_of(a), y = range_of(b);
    return x.lo < y.hi && y.lo < x.hi && x.hi > x.lo && y.hi > y.lo;
}

skel_status check_args(skel_plan p, const skel_buffer* args, int32_t nargs) {
    if (!p) return set_error(SKEL_EINVAL, "null plan");
    if (nargs != (int32_t)p->proto.size())
        return set_error(SKEL_EINVAL, "plan takes %d arguments, got %d", (int)p->proto.size(), nargs);
    if (nargs && !args) return set_error(SKEL_EINVAL, "null argument array");
    for (int k = 0; k < nargs; ++k) {
        const skel_buffer& a = args[k];
        const skel_buffer& q = p->proto[k];
        if (a.dtype != q.dtype) return set_error(SKEL_ETYPE, "argument %d: dtype differs from the compiled plan", k);
        if (a.ndim != q.ndim) return set_error(SKEL_ESHAPE, "argument %d: rank differs from the compiled plan", k);
        for (int d = 0; d < a.ndim; ++d)
            if (a.shape[d] != q.shape[d])
                return set_error(SKEL_ESHAPE, "argument %d: shape differs from the compiled plan (recompile for new shapes)", k);
        const int64_t es = (a.dtype == SKEL_U8) ? 1 : ((a.dtype == SKEL_U64 || a.dtype == SKEL_F64) ? 8 : 4);
        if (!dense_strides(a, es)) return set_error(SKEL_ESHAPE, "argument %d: not dense row-major", k);
        if (!a.data && range_of(a).hi != range_of(a).lo) return set_error(SKEL_EINVAL, "argument %d: null data", k);
    }
    return SKEL_OK;
}

skel_status check_aliasing(skel_plan p, const skel_buffer* args) {
    const Linear& L = p->lin;
    if (L.dom == DOM_U8 && L.is_while) {
        const int n = (int)p->proto.size();
        for (int a = 0; a < n; ++a)
            for (int b = a + 1; b < n; ++b)
                if (overlap(args[a], args[b])) return set_error(SKEL_EINVAL, "while Loop arguments must not overlap");
        return SKEL_OK;
    }
    if (L.dom == DOM_U8) {
        const bool same = args[0].data == args[1].data && range_of(args[0]).hi > range_of(args[0]).lo;
        if (overlap(args[0], args[1]) && !same) return set_error(SKEL_EINVAL, "input and output overlap partially");
        if (same) {
            for (const Kernel& k : p->kernels)
                if (k.src == -1 && k.dst == -2 && (k.blur || k.img.in_flip || k.img.out_flip))
                    return set_error(SKEL_EINVAL, "in-place run of a kernel with a stencil or a mirror");
        }
        for (int k = 2; k < (int)p->proto.size(); ++k)
            for (int j = 0; j < 2; ++j)
                if (overlap(args[k], args[j])) return set_error(SKEL_EINVAL, "reduce output overlaps an image");
        if (p->proto.size() == 4 && overlap(args[2], args[3])) return set_error(SKEL_EINVAL, "hist and sum overlap");
    } else if (L.dom == DOM_F32) {
        const int out = 1 + (int)std::count_if(L.st.begin(), L.st.end(), [](const Stage& s) { return s.op == SKEL_OP_SAXPY; });
        for (int k = 0; k < (int)p->proto.size(); ++k) {
            if (k == out) continue;
            if (!overlap(args[k], args[out])) continue;
            if (k == 0 && args[0].data == args[out].data) {
                for (const Kernel& kk : p->kernels)
                    if (kk.src == -1 && kk.dst == -2 && (kk.vec.out_flip || kk.vec.in_flip))
                        return set_error(SKEL_EINVAL, "in-place run of a kernel with a reversal");
                continue;
            }
            return set_error(SKEL_EINVAL, "argument %d overlaps the output", k);
        }
    } else if (L.dom == DOM_C32) {
        if (overlap(args[0], args[1])) return set_error(SKEL_EINVAL, "FFT input and output must not overlap");
    } else if (L.dom == DOM_GRAY) {
        if (overlap(args[0], args[1]) && args[0].data != args[1].data)
            return set_error(SKEL_EINVAL, "input and output overlap partially");
    } else if (L.dom == DOM_NBODY) {
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                if (overlap(args[a], args[b])) return set_error(SKEL_EINVAL, "N-body buffers must not overlap");
    }
    return SKEL_OK;
}

void* resolve_img(skel_plan p, const skel_buffer* args, int id) {
    if (id == -1) return args[0].data;
    if (id == -2) return args[1].data;
    if (id == 0 || id == 1) return p->scratch[id];
    return nullptr;
}

skel_status run_image(skel_plan p, const skel_buffer* args, hipStream_t s) {
    const Linear& L = p->lin;
    for (size_t ki = 0; ki < p->kernels.size(); ++ki) {
        Kernel& k = p->kernels[ki];
        ImgGroupArgs A = k.img;
        A.in = (const uint8_t*)resolve_img(p, args, k.src);
        A.out = (uint8_t*)resolve_img(p, args, k.dst);
        if (k.reduce) {
            A.part = p->hrows;
            A.hist = L.red == SKEL_RED_HIST256_SUM ? (uint32_t*)args[2].data : nullptr;
            A.sum = L.red == SKEL_RED_HIST256_SUM ? (uint64_t*)args[3].data : (uint64_t*)args[2].data;
        }
        const bool prof = (int)ki == p->prof_kernel;
        HIP_TRY(launch_img_group(A, k.blur, k.reduce, k.wg, p->cfg.variant, s, &k.name, prof ? p->prof_start : nullptr,
                                 prof ? p->prof_end : nullptr));
        if (k.reduce) {
            // Add the work-groups' histogram rows to the outputs, which
            // work-group 0 of the kernel cleared (or clear them: no tiles).
            HistFinArgs F;
            memset(&F, 0, sizeof(F));
            F.part = p->hrows;
            F.one.hist = A.hist;
            F.one.sum = A.sum;
            F.one.nrows = k.grid;
            F.one.crows = hist_chunk_rows(k.bins);
            F.nseg = 1;
            F.nchunks = hist_chunks(k.grid, F.one.crows);
            F.bins = k.bins;
            HIP_TRY(A.ntiles > 0 ? launch_hist_merge(F, s) : launch_hist_zero(F, s));
        }
    }
    return SKEL_OK;
}

// While Loop (skel_loop_while): iteration i (from 0) reads the previous
// iteration's image (the input for i = 0) and writes out when max - 1 - i is
// even, the plan's second image otherwise, so a loop that runs to its limit
// ends in out; every kernel of an iteration is guarded by the device flag,
// which the step kernel clears when the condition fails or the limit is
// reached.  The host enqueues blocks of check_every iterations; after each
// block it enqueues a 4-byte copy of the flag into a pinned slot and records
// an event, then waits for the previous block's event and reads that block's
// flag.  The GPU thus always has the newest block queued while the host
// waits, and a block enqueued after the condition failed runs only guarded
// no-op kernels.  A final guarded copy moves a result that ended in the
// second image.
//
// Carried reduce outputs (a carried_mask bit on hist or sum): the iteration's
// kernels write that output into the plan's iteration buffer instead, and the
// step kernel adds it to the caller's buffer, which is never cleared, so the
// result is the caller's initial content plus every iteration's partial
// result (the merge by addition of Sec. 3.4).  The condition always reads the
// iteration's own sums.  check_every < 0: the whole limit is enqueued with no
// host read-back, so the run is as asynchronous as any other.
skel_status run_image_while(skel_plan p, const skel_buffer* args, hipStream_t s) {
    const Linear& L = p->lin;
    const int nargs = (int)p->proto.size();
    const int sum_arg = L.red == SKEL_RED_HIST256_SUM ? 3 : 2;
    uint32_t* hist = L.red == SKEL_RED_HIST256_SUM ? (uint32_t*)args[2].data : nullptr;
    uint64_t* sum = (uint64_t*)args[sum_arg].data;
    uint32_t* count = (uint32_t*)args[nargs - 1].data;
    const bool carry_hist = hist && ((L.loop_carried >> 2) & 1u);
    const bool carry_sum = (L.loop_carried >> sum_arg) & 1u;
    uint32_t* it_hist = carry_hist ? p->witer_hist : hist;
    uint64_t* it_sum = carry_sum ? p->witer_sum : sum;
    WhileMerge M;
    memset(&M, 0, sizeof(M));
    if (carry_hist) {
        M.it_hist = it_hist;
        M.acc_hist = hist;
    }
    if (carry_sum) {
        M.it_sum = it_sum;
        M.acc_sum = sum;
    }
    WhileCond wc;
    memset(&wc, 0, sizeof(wc));
    wc.channel = L.wcond.channel;
    wc.cmp = L.wcond.cmp;
    wc.threshold = L.wcond.threshold;
    wc.max = L.while_max;
    wc.kind = L.wcond.kind;
    const bool async = L.wcond.check_every < 0;
    const int every = async ? L.while_max : (L.wcond.check_every > 0 ? L.wcond.check_every : 8);
    HIP_TRY(launch_while_init(p->wstate, s));
    int it = 0;
    for (int block = 0; it < L.while_max; ++block) {
        for (int j = 0; j < every && it < L.while_max; ++j, ++it) {
            auto dst_of = [&](int i) { return (L.while_max - 1 - i) % 2 == 0 ? args[1].data : p->wbuf; };
            void* src = it == 0 ? args[0].data : dst_of(it - 1);
            void* dst = dst_of(it);
            for (size_t ki = 0; ki < p->kernels.size(); ++ki) {
                Kernel& k = p->kernels[ki];
                ImgGroupArgs A = k.img;
                A.in = (const uint8_t*)(k.src == -1 ? src : (k.src == -2 ? dst : p->scratch[k.src]));
                A.out = (uint8_t*)(k.dst == -2 ? dst : (k.dst >= 0 ? p->scratch[k.dst] : nullptr));
                A.guard = p->wstate;
                if (k.reduce) {
                    A.part = p->hrows;
                    A.hist = it_hist;
                    A.sum = it_sum;
                }
                HIP_TRY(launch_img_group(A, k.blur, k.reduce, k.wg, p->cfg.variant, s, &k.name));
                if (k.reduce) {
                    HistFinArgs F;
                    memset(&F, 0, sizeof(F));
                    F.part = p->hrows;
                    F.guard = p->wstate;
                    F.one.hist = it_hist;
                    F.one.sum = it_sum;
                    F.one.nrows = k.grid;
                    F.one.crows = hist_chunk_rows(k.bins);
                    F.nseg = 1;
                    F.nchunks = hist_chunks(k.grid, F.one.crows);
                    F.bins = k.bins;
                    HIP_TRY(A.ntiles > 0 ? launch_hist_merge(F, s) : launch_hist_zero(F, s));
                }
            }
            HIP_TRY(launch_while_step(p->wstate, it_sum, wc, M, count, s));
        }
        if (it >= L.while_max || async) break;
        HIP_TRY(hipMemcpyAsync(p->h_flag + block % 2, p->wstate, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(p->wev[block % 2], s));
        if (block > 0) {
            HIP_TRY(hipEventSynchronize(p->wev[(block - 1) % 2]));
            if (p->h_flag[(block - 1) % 2] == 0) break;
        }
    }
    HIP_TRY(launch_while_copy(p->wstate, p->wbuf, args[1].data, (uint64_t)p->sh.W * p->sh.H * 4,
                              (uint32_t)L.while_max, s));
    return SKEL_OK;
}

skel_status run_gray(skel_plan p, const skel_buffer* args, hipStream_t s) {
    for (size_t ki = 0; ki < p->kernels.size(); ++ki) {
        Kernel& k = p->kernels[ki];
        GrayArgs A = k.gray;
        auto res = [&](int id) -> void* {
            if (id == -1) return args[0].data;
            if (id == -2) return args[1].data;
            return p->scratch[id];
        };
        A.in = (const uint8_t*)res(k.src);
        A.out = (uint8_t*)res(k.dst);
        const bool prof = (int)ki == p->prof_kernel;
        if (prof) HIP_TRY(hipEventRecord(p->prof_start, s));
        HIP_TRY(launch_gray_chain(A, k.grid, k.wg, s));
        if (prof) HIP_TRY(hipEventRecord(p->prof_end, s));
    }
    return SKEL_OK;
}

skel_status run_fft(skel_plan p, const skel_buffer* args, hipStream_t s) {
    for (size_t ki = 0; ki < p->kernels.size(); ++ki) {
        Kernel& k = p->kernels[ki];
        FftArgs A = k.fft;
        auto res = [&](int id) -> void* {
            if (id == -1) return args[0].data;
            if (id == -2) return args[1].data;
            return p->scratch[id];
        };
        A.in = res(k.src);
        A.out = res(k.dst);
        A.tw = p->fft_tw;
        A.nfft = (int32_t)p->sh.n;
        const bool prof = (int)ki == p->prof_kernel;
        if (prof) HIP_TRY(hipEventRecord(p->prof_start, s));
        HIP_TRY(launch_fft_pass(A, k.fft_mode, s));
        if (prof) HIP_TRY(hipEventRecord(p->prof_end, s));
    }
    return SKEL_OK;
}

skel_status run_vector(skel_plan p, const skel_buffer* args, hipStream_t s) {
    const Linear& L = p->lin;
    const int nargs = (int)p->proto.size();
    const int out = nargs - 1 - (L.red >= 0 ? 1 : 0);
    float* sum_out = L.red >= 0 ? (float*)args[nargs - 1].data : nullptr;
    if (L.red >= 0 && p->sh.n == 0) HIP_TRY(launch_fill_u32(sum_out, 1, 0, s));
    for (size_t ki = 0; ki < p->kernels.size(); ++ki) {
        Kernel& k = p->kernels[ki];
        VecGroupArgs A = k.vec;
        auto res = [&](int id) -> float* {
            if (id == -1) return (float*)args[0].data;
            if (id == -2) return (float*)args[out].data;
            if (id == 0 || id == 1) return (float*)p->scratch[id];
            return nullptr;
        };
        A.in = res(k.src);
        A.out = res(k.dst);
        for (size_t j = 0; j < k.side_args.size(); ++j) A.side[j] = (const float*)args[k.side_args[j]].data;
        if (k.reduce && p->sh.n > 0) {
            A.partials = p->partials;
            A.sum_out = sum_out;
        }
        const bool prof = (int)ki == p->prof_kernel;
        if (prof) HIP_TRY(hipEventRecord(p->prof_start, s));
        HIP_TRY(launch_vec_group(A, k.grid, k.wg, s, &k.name));
        if (prof) HIP_TRY(hipEventRecord(p->prof_end, s));
    }
    return SKEL_OK;
}

skel_status nbody_iterations(skel_plan p, float4* pos, float4* vel, float4* scr, hipStream_t s) {
    const Linear& L = p->lin;
    NBodyArgs A{};
    A.vel = vel;
    A.acc = p->nb_acc;
    A.N = (int32_t)p->sh.N;
    A.jsplit = p->cfg.tile_h;
    A.eps2 = L.nbody_prm.eps * L.nbody_prm.eps;
    A.G = L.nbody_prm.G;
    A.dt = L.nbody_prm.dt;
    const bool fused = p->cfg.fusion != SKEL_FUSE_OFF;
    for (int t = 0; t < L.nbody_iters; ++t) {
        A.pos_in = (t % 2 == 0) ? pos : scr;
        A.pos_out = (t % 2 == 0) ? scr : pos;
        HIP_TRY(launch_nbody_force(A, fused, s, &p->kernels[0].name));
        if (!fused) HIP_TRY(launch_nbody_integrate(A, s, &p->kernels[1].name));
    }
    if (L.nbody_iters % 2 == 1) HIP_TRY(launch_copy_f32x4(scr, pos, p->sh.N, s));
    return SKEL_OK;
}

// Loop driver: the whole counted loop is captured once into a HIP graph (per
// set of buffers) and replayed, so the loop state never leaves the device and
// no host round trip separates iterations (the paper runs the condition and
// state update on the host, Sec. 3.1).
skel_status run_nbody(skel_plan p, const skel_buffer* args, hipStream_t s) {
    float4* pos = (float4*)args[0].data;
    float4* vel = (float4*)args[1].data;
    float4* scr = (float4*)args[2].data;
    if (p->sh.N == 0 || p->lin.nbody_iters == 0) return SKEL_OK;
    if (p->cfg.variant == 1) return nbody_iterations(p, pos, vel, scr, s);
    std::vector<const void*> key = {pos, vel, scr};
    if (!p->gexec || key != p->gkey) {
        if (p->gexec) {
            HIP_TRY(hipGraphExecDestroy(p->gexec));
            p->gexec = nullptr;
        }
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        skel_status st = nbody_iterations(p, pos, vel, scr, p->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return set_error(SKEL_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return set_error(SKEL_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        p->gkey = key;
    }
    HIP_TRY(hipGraphLaunch(p->gexec, s));
    return SKEL_OK;
}

// Device resources of a plan are allocated on its first run, so compiling a
// plan is a host-only step: intermediate images/vectors between unfused
// kernels, reduce partials and the unfused N-body acceleration buffer.
skel_status ensure_resources(skel_plan p) {
    if (p->resources_ready) return SKEL_OK;
    int nscr = 0;
    for (const Kernel& k : p->kernels) nscr = std::max(nscr, k.dst >= 0 ? k.dst + 1 : 0);
    size_t bytes = 0;
    if (p->lin.dom == DOM_U8) bytes = (size_t)(p->sh.W * p->sh.H * 4);
    if (p->lin.dom == DOM_F32) bytes = (size_t)(p->sh.n * 4);
    // transposed intermediates take 256 rows of kFftTRow per transform (natural
    // order between unfused stages takes less)
    if (p->lin.dom == DOM_C32) bytes = (size_t)p->sh.n * 256 * kFftTRow * 8;
    if (p->lin.dom == DOM_GRAY) bytes = (size_t)p->sh.n;
    for (int k = 0; k < nscr; ++k)
        if (!p->scratch[k]) HIP_TRY(hipMalloc(&p->scratch[k], std::max<size_t>(bytes, 16)));
    if (p->lin.dom == DOM_F32 && p->lin.red >= 0 && !p->partials) {
        int g = 1;
        for (const Kernel& k : p->kernels)
            if (k.reduce) g = std::max(g, k.grid);
        HIP_TRY(hipMalloc(&p->partials, sizeof(float) * g));
    }
    if (p->lin.dom == DOM_U8 && p->lin.red >= 0 && !p->hrows) {
        for (const Kernel& k : p->kernels)
            if (k.reduce) {
                const size_t words = 4 * (size_t)k.bins;
                const size_t rows = std::max(1, k.grid);
                HIP_TRY(hipMalloc(&p->hrows, sizeof(uint32_t) * words * rows));
            }
    }
    if (p->lin.dom == DOM_C32 && !p->fft_tw) {
        // Roots of unity (cos, sin)(2 pi m / N) in double precision, rounded once.
        std::vector<float2> tw(kFftPoints);
        for (int m = 0; m < kFftPoints; ++m) {
            const double a = 2.0 * 3.14159265358979323846 * (double)m / (double)kFftPoints;
            tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
        HIP_TRY(hipMalloc(&p->fft_tw, sizeof(float2) * kFftPoints));
        HIP_TRY(hipMemcpy(p->fft_tw, tw.data(), sizeof(float2) * kFftPoints, hipMemcpyHostToDevice));
    }
    if (p->lin.dom == DOM_U8 && p->lin.is_while && !p->wstate) {
        HIP_TRY(hipMalloc(&p->wbuf, std::max<size_t>(bytes, 16)));
        HIP_TRY(hipMalloc(&p->wstate, 256));
        HIP_TRY(hipMalloc(&p->witer_hist, sizeof(uint32_t) * 1024 + sizeof(uint64_t) * 4));
        p->witer_sum = reinterpret_cast<uint64_t*>(p->witer_hist + 1024);
        HIP_TRY(hipHostMalloc((void**)&p->h_flag, 256, hipHostMallocDefault));
        for (hipEvent_t& e : p->wev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    if (p->lin.dom == DOM_NBODY && p->cfg.fusion == SKEL_FUSE_OFF && !p->nb_acc)
        HIP_TRY(hipMalloc(&p->nb_acc, sizeof(float4) * std::max<int64_t>(p->sh.N, 1)));
    p->resources_ready = true;
    return SKEL_OK;
}

}  // namespace

skel_status skel_ensure_resources(skel_plan p) { return ensure_resources(p); }

// Runs from caller-provided device scratch (the allocation-free entry point):
// the buffers ensure_resources would allocate -- intermediate images, vectors
// or volumes between unfused kernels, fp32 reduce partials and image histogram
// rows -- are carved out of one region in 256-byte aligned pieces.  Plans that
// need anything else (an N-body graph, FFT twiddles uploaded from the host, a
// while Loop's pinned flag and events) are SKEL_EUNSUPPORTED.
namespace {
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

skel_status noalloc_prepare(skel_plan p, const skel_buffer* args, int32_t nargs, size_t cap, NoallocLayout& L) {
    skel_status st = check_args(p, args, nargs);
    if (st) return st;
    if ((st = check_aliasing(p, args))) return st;
    const Domain dom = p->lin.dom;
    if (dom == DOM_NBODY || dom == DOM_C32 || (dom == DOM_U8 && p->lin.is_while) ||
        (dom != DOM_U8 && dom != DOM_F32 && dom != DOM_GRAY))
        return set_error(SKEL_EUNSUPPORTED,
                         "allocation-free runs cover image, fp32 and gray chains (not N-body loops, FFT chains or "
                         "while Loops)");
    L = NoallocLayout{};
    int nscr = 0;
    for (const Kernel& k : p->kernels) nscr = std::max(nscr, k.dst >= 0 ? k.dst + 1 : 0);
    size_t bytes = 0;
    if (dom == DOM_U8) bytes = (size_t)(p->sh.W * p->sh.H * 4);
    if (dom == DOM_F32) bytes = (size_t)(p->sh.n * 4);
    if (dom == DOM_GRAY) bytes = (size_t)p->sh.n;
    size_t off = 0;
    L.nimg = nscr;
    for (int k = 0; k < nscr; ++k) {
        L.off_img[k] = off;
        off += align256(std::max<size_t>(bytes, 16));
    }
    if (dom == DOM_F32 && p->lin.red >= 0) {
        int g = 1;
        for (const Kernel& k : p->kernels)
            if (k.reduce) g = std::max(g, k.grid);
        L.off_partials = off;
        L.has_partials = true;
        off += align256(sizeof(float) * g);
    }
    if (dom == DOM_U8 && p->lin.red >= 0) {
        for (const Kernel& k : p->kernels)
            if (k.reduce) {
                L.off_hrows = off;
                L.has_hrows = true;
                off += align256(sizeof(uint32_t) * 4 * (size_t)k.bins * (size_t)std::max(1, k.grid));
            }
    }
    L.total = off;
    if (off > cap)
        return set_error(SKEL_EUNSUPPORTED,
                         "this plan needs %zu bytes of device scratch; the allocation-free entry point holds %zu "
                         "(fuse the chain or use skel_plan_run)",
                         off, cap);
    return SKEL_OK;
}

skel_status noalloc_run(skel_plan p, const skel_buffer* args, void* stream, char* region, const NoallocLayout& L) {
    void* saved_scr[2] = {p->scratch[0], p->scratch[1]};
    float* saved_partials = p->partials;
    uint32_t* saved_hrows = p->hrows;
    for (int k = 0; k < L.nimg; ++k) p->scratch[k] = region + L.off_img[k];
    if (L.has_partials) p->partials = (float*)(region + L.off_partials);
    if (L.has_hrows) p->hrows = (uint32_t*)(region + L.off_hrows);
    const hipStream_t s = S(stream);
    skel_status st = SKEL_OK;
    switch (p->lin.dom) {
        case DOM_U8: st = run_image(p, args, s); break;
        case DOM_F32: st = run_vector(p, args, s); break;
        case DOM_GRAY: st = run_gray(p, args, s); break;
        default: st = set_error(SKEL_EUNSUPPORTED, "plan domain not covered by the allocation-free entry point");
    }
    p->scratch[0] = saved_scr[0];
    p->scratch[1] = saved_scr[1];
    p->partials = saved_partials;
    p->hrows = saved_hrows;
    return st;
}

extern "C" {

skel_status skel_init(int32_t device) {
    clear_error();
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return set_error(SKEL_EINVAL, "device %d of %d", device, n);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(SKEL_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    return noalloc_setup(device);
}

skel_status skel_map(int32_t op, const skel_params* p, skel_node* out) {
    clear_error();
    if (op < SKEL_OP_NOISE || op > SKEL_OP_SEGMENT) return set_error(SKEL_EINVAL, "unknown stage op %d", op);
    if (op == SKEL_OP_SEGMENT && p && (p->lo || p->hi) && (p->lo > p->hi || p->hi > 256))
        return set_error(SKEL_EINVAL, "SEGMENT thresholds need lo <= hi <= 256");
    skel_node_s* n;
    skel_status st = new_node(out, &n);
    if (st) return st;
    n->kind = NK_MAP;
    n->op = op;
    if (p) n->prm = *p;
    *out = n;
    return SKEL_OK;
}

skel_status skel_pipeline(const skel_node* stages, int32_t count, skel_node* out) {
    clear_error();
    if (count < 1 || !stages) return set_error(SKEL_EINVAL, "a pipeline needs at least one stage");
    for (int k = 0; k < count; ++k)
        if (!stages[k]) return set_error(SKEL_EINVAL, "pipeline stage %d is null", k);
    skel_node_s* n;
    skel_status st = new_node(out, &n);
    if (st) return st;
    n->kind = NK_PIPE;
    for (int k = 0; k < count; ++k) {
        node_addref(stages[k]);
        n->kids.push_back(stages[k]);
    }
    *out = n;
    return SKEL_OK;
}

skel_status skel_mapreduce(skel_node map, int32_t red, skel_node* out) {
    clear_error();
    if (!map) return set_error(SKEL_EINVAL, "null map node");
    if (red != SKEL_RED_HIST256_SUM && red != SKEL_RED_SUM) return set_error(SKEL_EINVAL, "unknown reduce %d", red);
    if (map->kind == NK_MAPRED) return set_error(SKEL_EINVAL, "nested MapReduce");
    skel_node_s* n;
    skel_status st = new_node(out, &n);
    if (st) return st;
    n->kind = NK_MAPRED;
    n->red = red;
    node_addref(map);
    n->kids.push_back(map);
    *out = n;
    return SKEL_OK;
}

skel_status skel_loop(skel_node body, const skel_loop_state* ls, skel_node* out) {
    clear_error();
    if (!body || !ls) return set_error(SKEL_EINVAL, "null loop body or state");
    if (ls->iterations < 0) return set_error(SKEL_EINVAL, "negative iteration count");
    if (body->kind == NK_MAPRED) return set_error(SKEL_EINVAL, "MapReduce is only valid at the root of a plan");
    skel_node_s* n;
    skel_status st = new_node(out, &n);
    if (st) return st;
    n->kind = NK_LOOP;
    n->loop = *ls;
    node_addref(body);
    n->kids.push_back(body);
    *out = n;
    return SKEL_OK;
}

skel_status skel_loop_while(skel_node body, const skel_loop_state* ls, const skel_loop_cond* cond,
                            skel_node* out) {
    clear_error();
    if (!body || !ls || !cond) return set_error(SKEL_EINVAL, "null loop body, state or condition");
    if (ls->iterations < 1) return set_error(SKEL_EINVAL, "a while Loop needs an iteration limit >= 1");
    if (body->kind != NK_MAPRED) return set_error(SKEL_EINVAL, "a while Loop's body must be a MapReduce");
    if (cond->channel < 0 || cond->channel > 3) return set_error(SKEL_EINVAL, "condition channel must be 0..3");
    if (cond->cmp < SKEL_CMP_GT || cond->cmp > SKEL_CMP_LE) return set_error(SKEL_EINVAL, "unknown comparison");
    if (cond->kind != SKEL_COND_VALUE && cond->kind != SKEL_COND_DELTA)
        return set_error(SKEL_EINVAL, "unknown condition kind %d", cond->kind);
    // Plan arguments: in, out, [hist,] sum, count.  The images are carried by
    // construction; reduce outputs may be; the count may not.
    const int nargs = body->red == SKEL_RED_HIST256_SUM ? 5 : 4;
    if (ls->carried_mask >> nargs)
        return set_error(SKEL_EINVAL, "carried_mask 0x%x names arguments beyond the %d of this while Loop",
                         ls->carried_mask, nargs);
    if ((ls->carried_mask >> (nargs - 1)) & 1u)
        return set_error(SKEL_EINVAL, "a while Loop's iteration count cannot be carried");
    skel_node_s* n;
    skel_status st = new_node(out, &n);
    if (st) return st;
    n->kind = NK_WHILE;
    n->loop = *ls;
    n->cond = *cond;
    node_addref(body);
    n->kids.push_back(body);
    *out = n;
    return SKEL_OK;
}

skel_status skel_node_release(skel_node node) {
    clear_error();
    node_release(node);
    return SKEL_OK;
}

skel_status skel_plan_compile(skel_node root, const skel_buffer* proto, int32_t nargs, const skel_plan_opts* opts,
                              skel_plan* out) {
    clear_error();
    if (!out) return set_error(SKEL_EINVAL, "null output handle");
    *out = nullptr;
    if (!root) return set_error(SKEL_EINVAL, "null root node");
    if (nargs < 0 || (nargs > 0 && !proto)) return set_error(SKEL_EINVAL, "bad prototype arguments");
    skel_plan_s* p = new (std::nothrow) skel_plan_s();
    if (!p) return set_error(SKEL_ENOMEM, "host allocation failed");
    skel_status st = linearize(root, p->lin);
    if (!st && p->lin.dom == DOM_NONE) {
        p->lin.dom = (nargs > 0 && proto[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
        if (p->lin.dom == DOM_F32 && p->lin.red == SKEL_RED_HIST256_SUM)
            st = set_error(SKEL_ETYPE, "the histogram reduce applies to RGBA uint8 images only");
    }
    if (!st) st = derive_shape(p->lin, proto, nargs, p->sh);
    if (!st) st = resolve_config(p->lin, p->sh, opts, p->cfg);
    if (!st) st = build_kernels(p->lin, p->sh, p->cfg, p->kernels);
    if (st) {
        delete p;
        return st;
    }
    p->proto.assign(proto, proto + nargs);
    for (auto& b : p->proto) b.data = nullptr;
    node_addref(root);
    p->root = root;
    // Compiling needs no device (describe() and the structure queries work
    // without one); with none, device 0 is recorded and the first run reports
    // the device error.  The failed query's error state is cleared so that it
    // is not taken for a later launch's.
    if (hipGetDevice(&p->device) != hipSuccess) {
        p->device = 0;
        (void)hipGetLastError();
    }
    *out = p;
    return SKEL_OK;
}

skel_status skel_plan_run(skel_plan p, const skel_buffer* args, int32_t nargs, void* stream) {
    clear_error();
    skel_status st = check_args(p, args, nargs);
    if (st) return st;
    if ((st = check_aliasing(p, args))) return st;
    if ((st = ensure_resources(p))) return st;
    const hipStream_t s = S(stream);
    switch (p->lin.dom) {
        case DOM_U8: return p->lin.is_while ? run_image_while(p, args, s) : run_image(p, args, s);
        case DOM_F32: return run_vector(p, args, s);
        case DOM_NBODY: return run_nbody(p, args, s);
        case DOM_C32: return run_fft(p, args, s);
        case DOM_GRAY: return run_gray(p, args, s);
        default: return set_error(SKEL_EINVAL, "plan has no domain");
    }
}

skel_status skel_plan_run_event(skel_plan p, const skel_buffer* args, int32_t nargs, void* stream, void* done) {
    skel_status st = skel_plan_run(p, args, nargs, stream);
    if (st) return st;
    if (done) HIP_TRY(hipEventRecord((hipEvent_t)done, S(stream)));
    return SKEL_OK;
}

skel_status skel_plan_describe(skel_plan p, char* buf, size_t len) {
    clear_error();
    if (!p || !buf || len == 0) return set_error(SKEL_EINVAL, "null plan or buffer");
    std::string s = "{\"sct\":\"" + p->lin.sct + "\",\"domain\":\"";
    s += p->lin.dom == DOM_U8    ? "u8"
         : p->lin.dom == DOM_F32 ? "f32"
         : p->lin.dom == DOM_C32 ? "c32"
         : p->lin.dom == DOM_GRAY ? "gray"
                                  : "nbody";
    s += "\",\"stages\":[";
    for (size_t i = 0; i < p->lin.st.size(); ++i) {
        static const char* nm[] = {"noise", "solarise", "mirror", "blur5", "saxpy", "nbody_force", "leapfrog",
                                   "fft", "ifft", "segment"};
        s += (i ? ",\"" : "\"") + std::string(nm[p->lin.st[i].op]) + "\"";
    }
    s += "],\"reduce\":";
    s += p->lin.red < 0 ? "null" : (p->lin.red == SKEL_RED_HIST256_SUM ? "\"hist256_sum\"" : "\"sum\"");
    char tmp[256];
    snprintf(tmp, sizeof(tmp), ",\"iterations\":%d,\"loop_carried\":%u,\"loop_sync\":%d",
             p->lin.nbody_iters, p->lin.loop_carried, p->lin.loop_sync);
    s += tmp;
    if (p->lin.is_while)
        snprintf(tmp, sizeof(tmp),
                 ",\"while\":{\"max\":%d,\"channel\":%d,\"cmp\":%d,\"threshold\":%llu,\"check_every\":%d,"
                 "\"kind\":\"%s\"}",
                 p->lin.while_max, p->lin.wcond.channel, p->lin.wcond.cmp,
                 (unsigned long long)p->lin.wcond.threshold, p->lin.wcond.check_every,
                 p->lin.wcond.kind == SKEL_COND_DELTA ? "delta" : "value");
    else
        snprintf(tmp, sizeof(tmp), ",\"while\":null");
    s += tmp;
    s += ",\"kernels\":[";
    for (size_t i = 0; i < p->kernels.size(); ++i) {
        const Kernel& k = p->kernels[i];
        snprintf(tmp, sizeof(tmp),
                 "%s{\"name\":\"%s\",\"stages\":[%d,%d],\"blur\":%s,\"reduce\":%s,\"grid\":%d,\"wg\":%d,"
                 "\"tile_h\":%d}",
                 i ? "," : "", k.name, k.first, k.last, k.blur ? "true" : "false", k.reduce ? "true" : "false",
                 k.grid, k.wg, p->lin.dom == DOM_U8 ? k.img.tile_h : p->cfg.tile_h);
        s += tmp;
    }
    snprintf(tmp, sizeof(tmp),
             "],\"batch_grid\":%d,\"config\":{\"fusion\":%d,\"split_mask\":%u,\"tile_h\":%d,\"wg\":%d,\"ept\":%d,"
             "\"variant\":%d}}",
             p->batch_grid, p->cfg.fusion, p->cfg.split_mask, p->cfg.tile_h, p->cfg.wg, p->cfg.ept, p->cfg.variant);
    s += tmp;
    strncpy(buf, s.c_str(), len - 1);
    buf[len - 1] = 0;
    return SKEL_OK;
}

skel_status skel_plan_kernel_events(skel_plan p, int32_t kernel, void* start, void* end) {
    clear_error();
    if (!p) return set_error(SKEL_EINVAL, "null plan");
    if (kernel >= (int32_t)p->kernels.size()) return set_error(SKEL_EINVAL, "plan has %d kernels", (int)p->kernels.size());
    if (kernel < 0 || !start || !end) {
        p->prof_kernel = -1;
        p->prof_start = p->prof_end = nullptr;
        return SKEL_OK;
    }
    p->prof_kernel = kernel;
    p->prof_start = (hipEvent_t)start;
    p->prof_end = (hipEvent_t)end;
    return SKEL_OK;
}

skel_status skel_plan_destroy(skel_plan p) {
    clear_error();
    if (!p) return SKEL_OK;
    for (void* q : p->scratch)
        if (q) (void)hipFree(q);
    if (p->partials) (void)hipFree(p->partials);
    if (p->fft_tw) (void)hipFree(p->fft_tw);
    if (p->hrows) (void)hipFree(p->hrows);
    if (p->wbuf) (void)hipFree(p->wbuf);
    if (p->wstate) (void)hipFree(p->wstate);
    if (p->witer_hist) (void)hipFree(p->witer_hist);
    if (p->h_flag) (void)hipHostFree(p->h_flag);
    for (hipEvent_t e : p->wev)
        if (e) (void)hipEventDestroy(e);
    if (p->d_segs) (void)hipFree(p->d_segs);
    if (p->h_segs) (void)hipHostFree(p->h_segs);
    if (p->b_rows) (void)hipFree(p->b_rows);
    if (p->d_tile_req) (void)hipFree(p->d_tile_req);
    if (p->nb_acc) (void)hipFree(p->nb_acc);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->bexec) (void)hipGraphExecDestroy(p->bexec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_reqs) (void)hipFree(p->d_reqs);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->h_reqs) (void)hipHostFree(p->h_reqs);
    node_release(p->root);
    delete p;
    return SKEL_OK;
}

skel_status skel_sync(void* stream) {
    clear_error();
    HIP_TRY(hipStreamSynchronize(S(stream)));
    HIP_TRY(hipGetLastError());
    return SKEL_OK;
}

}  // extern "C"
