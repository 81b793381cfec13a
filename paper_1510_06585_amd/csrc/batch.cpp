// Batched execution: many execution requests over data sets that differ in
// content and size (the batch model of Sec. 2) run as one persistent kernel.
// The host lays out a work list of wavefront tiles, largest requests first
// (longest-processing-time order, so the tail of the launch is made of small
// tiles), and captures [reset ticket, clear outputs, persistent kernel,
// histogram merge] into a HIP graph that is replayed while the same buffers
// and shapes come back.  Every group of tiles (one per wavefront of a
// work-group, all of one request) stores its work-group histogram as a row;
// the merge sums each request's rows in chunks and adds them to its outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>

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

// Byte range [lo, hi) of a dense buffer of esize-byte elements.
struct Span {
    uintptr_t lo, hi;
};
Span span_of(const skel_buffer& b, int64_t esize) {
    int64_t n = b.ndim > 0 ? 1 : 0;
    for (int d = 0; d < b.ndim; ++d) n *= b.shape[d] > 0 ? b.shape[d] : 0;
    return Span{(uintptr_t)b.data, (uintptr_t)b.data + (uintptr_t)(n * esize)};
}
bool spans_overlap(const Span& x, const Span& y) { return x.hi > x.lo && y.hi > y.lo && x.lo < y.hi && y.lo < x.hi; }

skel_status check_req(const skel_buffer* a, int nargs, int red, int r, bool inplace_ok) {
    auto esize = [&](int k) -> int64_t { return k < 2 ? 1 : (k == 2 && red == SKEL_RED_HIST256_SUM ? 4 : 8); };
    for (int k = 0; k < nargs; ++k)
        if (!dense_strides(a[k], esize(k)))
            return set_error(SKEL_ESHAPE, "request %d argument %d: not dense row-major", r, k);
    const skel_buffer &in = a[0], &out = a[1];
    if (in.dtype != SKEL_U8 || out.dtype != SKEL_U8 || in.ndim != 3 || out.ndim != 3 || in.shape[2] != 4 ||
        out.shape[0] != in.shape[0] || out.shape[1] != in.shape[1] || out.shape[2] != 4)
        return set_error(SKEL_ESHAPE, "request %d: images must be uint8 [H, W, 4] of equal shape", r);
    const int64_t H = in.shape[0], W = in.shape[1];
    if (H < 0 || W < 0 || H > kMaxDim || W > kMaxDim || W * H * 4 >= ((int64_t)1 << 31))
        return set_error(SKEL_EUNSUPPORTED, "request %d: image of %lld x %lld is out of range", r, (long long)H,
                         (long long)W);
    if (W * H > 0 && (!in.data || !out.data)) return set_error(SKEL_EINVAL, "request %d: null image", r);
    // A request's in and out are either the same buffer (pointwise chains
    // only) or disjoint: a partial overlap would race with the stencil's halo
    // reads of other tiles of the same persistent launch.
    const Span si = span_of(in, 1), so = span_of(out, 1);
    if (in.data == out.data && W * H > 0 && !inplace_ok)
        return set_error(SKEL_EINVAL, "request %d: in-place run of a kernel with a stencil or a mirror", r);
    if (in.data != out.data && spans_overlap(si, so))
        return set_error(SKEL_EINVAL, "request %d: input and output overlap partially", r);
    for (int k = 2; k < nargs; ++k) {
        const Span sk = span_of(a[k], esize(k));
        if (spans_overlap(sk, si) || spans_overlap(sk, so))
            return set_error(SKEL_EINVAL, "request %d: reduce output %d overlaps an image", r, k);
        for (int j = k + 1; j < nargs; ++j)
            if (spans_overlap(sk, span_of(a[j], esize(j))))
                return set_error(SKEL_EINVAL, "request %d: reduce outputs overlap", r);
    }
    if (red == SKEL_RED_HIST256_SUM) {
        if (a[2].dtype != SKEL_U32 || a[2].ndim != 2 || a[2].shape[0] != 4 || a[2].shape[1] != 256 || !a[2].data)
            return set_error(SKEL_ESHAPE, "request %d: hist must be uint32 [4, 256]", r);
        if (a[3].dtype != SKEL_U64 || a[3].ndim != 1 || a[3].shape[0] != 4 || !a[3].data)
            return set_error(SKEL_ESHAPE, "request %d: sum must be uint64 [4]", r);
    } else if (red == SKEL_RED_SUM) {
        if (a[2].dtype != SKEL_U64 || a[2].ndim != 1 || a[2].shape[0] != 4 || !a[2].data)
            return set_error(SKEL_ESHAPE, "request %d: sum must be uint64 [4]", r);
    }
    return SKEL_OK;
}

// Requests of one batch run in the same launch, in no particular order, so no
// buffer a request writes (image out, hist, sum) may overlap any other
// request's buffers; inputs may be shared.  Sweep over the spans sorted by
// start: every overlapping pair involving a write is found through the span
// reaching furthest so far (an in-place request's in == out counts as one
// written span).
skel_status check_disjoint(const skel_buffer* args, int nargs, int nreq, int red) {
    struct Item {
        Span sp;
        int req;
        bool write;
    };
    std::vector<Item> it;
    it.reserve((size_t)nreq * nargs);
    for (int r = 0; r < nreq; ++r) {
        const skel_buffer* a = args + (size_t)r * nargs;
        for (int k = 0; k < nargs; ++k) {
            if (k == 0 && a[0].data == a[1].data) continue;   // in place: the output span covers it
            const int64_t es = k < 2 ? 1 : (k == 2 && red == SKEL_RED_HIST256_SUM ? 4 : 8);
            const Span sp = span_of(a[k], es);
            if (sp.hi > sp.lo) it.push_back(Item{sp, r, k > 0});
        }
    }
    std::sort(it.begin(), it.end(), [](const Item& x, const Item& y) { return x.sp.lo < y.sp.lo; });
    const Item* far = nullptr;
    for (const Item& c : it) {
        if (far && c.sp.lo < far->sp.hi && (c.write || far->write))
            return set_error(SKEL_EINVAL, "requests %d and %d: a written buffer overlaps another buffer", far->req,
                             c.req);
        if (!far || c.sp.hi > far->sp.hi) far = &c;
    }
    return SKEL_OK;
}

}  // namespace

namespace {

// The plan and every request on their own (no device work).
skel_status check_requests(skel_plan p, const skel_buffer* args, int32_t nargs, int32_t nreq) {
    if (!p) return set_error(SKEL_EINVAL, "null plan");
    if (p->lin.dom != DOM_U8 || p->kernels.size() != 1)
        return set_error(SKEL_EUNSUPPORTED, "batched runs need a fully fused image plan (one kernel)");
    if (nargs != (int32_t)p->proto.size()) return set_error(SKEL_EINVAL, "expected %d arguments per request", (int)p->proto.size());
    if (nreq < 0 || (nreq > 0 && !args)) return set_error(SKEL_EINVAL, "bad request array");
    if (nreq > 65535) return set_error(SKEL_EUNSUPPORTED, "at most 65535 requests per batch");
    const Kernel& K = p->kernels[0];
    const bool inplace_ok = !(K.blur || K.img.in_flip || K.img.out_flip);
    for (int r = 0; r < nreq; ++r) {
        skel_status st = check_req(args + (size_t)r * nargs, nargs, p->lin.red, r, inplace_ok);
        if (st) return st;
    }
    return SKEL_OK;
}

}  // namespace

skel_status batch_validate(skel_plan p, const skel_buffer* args, int32_t nargs, int32_t nreq) {
    skel_status st = check_requests(p, args, nargs, nreq);
    if (st || nreq == 0) return st;
    return check_disjoint(args, nargs, nreq, p->lin.red);
}

extern "C" skel_status skel_batch_run(skel_plan p, const skel_buffer* args, int32_t nargs, int32_t nreq,
                                      void* stream) {
    clear_error();
    if (skel_status st = check_requests(p, args, nargs, nreq)) return st;
    if (nreq == 0) return SKEL_OK;
    const Kernel& K = p->kernels[0];
    const int red = p->lin.red;
    const hipStream_t s = (hipStream_t)stream;
    // Rows per tile: the plan's tile_h when it was given, else kBatchTileRows
    // for every request.  With work-groups taking groups of adjacent tiles,
    // short tiles keep the tail of the work list fine-grained for the cost
    // of some halo recompute: on the 256-request benchmark batch, 31-34 rows
    // measured best (1.735-1.744 ms), 23 or 48 rows 1.76 ms, 64 rows 1.79 ms,
    // and the former per-request rule (ceil(H / 32) in [32, 128]) 1.78 ms.
    constexpr int kBatchTileRows = 31;
    auto tile_rows = [&](int64_t) -> int { return p->cfg.auto_tile ? kBatchTileRows : p->cfg.tile_h; };
    const int bw = K.blur ? kBandOut : kBandPx;

    std::vector<int64_t> key;
    key.reserve((size_t)nreq * 6);
    for (int r = 0; r < nreq; ++r) {
        const skel_buffer* a = args + (size_t)r * nargs;
        key.push_back((int64_t)(uintptr_t)a[0].data);
        key.push_back((int64_t)(uintptr_t)a[1].data);
        key.push_back(nargs > 2 ? (int64_t)(uintptr_t)a[2].data : 0);
        key.push_back(nargs > 3 ? (int64_t)(uintptr_t)a[3].data : 0);
        key.push_back(a[0].shape[0]);
        key.push_back(a[0].shape[1]);
    }
    if (p->bexec && key == p->bkey) {
        HIP_TRY(hipGraphLaunch(p->bexec, s));
        return SKEL_OK;
    }
    // New request set (a replayed key was checked when it was laid out).
    if (skel_status st = check_disjoint(args, nargs, nreq, red)) return st;
    // Lay out the work list, largest requests first.
    std::vector<int> order(nreq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const skel_buffer* a = args + (size_t)x * nargs;
        const skel_buffer* b = args + (size_t)y * nargs;
        return a[0].shape[0] * a[0].shape[1] > b[0].shape[0] * b[0].shape[1];
    });
    // Queued replays of the previous graph may still read the work list and
    // the histogram rows: wait for them before anything is rewritten.
    HIP_TRY(hipStreamSynchronize(s));
    if ((size_t)nreq > p->d_reqs_cap) {
        if (p->d_reqs) (void)hipFree(p->d_reqs);
        if (p->h_reqs) (void)hipHostFree(p->h_reqs);
        if (p->d_segs) (void)hipFree(p->d_segs);
        if (p->h_segs) (void)hipHostFree(p->h_segs);
        p->d_reqs = nullptr;
        p->h_reqs = nullptr;
        p->d_segs = nullptr;
        p->h_segs = nullptr;
        p->d_reqs_cap = 0;
        HIP_TRY(hipMalloc(&p->d_reqs, sizeof(BatchReq) * nreq));
        HIP_TRY(hipHostMalloc((void**)&p->h_reqs, sizeof(BatchReq) * nreq, hipHostMallocDefault));
        HIP_TRY(hipMalloc(&p->d_segs, sizeof(HistSeg) * nreq));
        HIP_TRY(hipHostMalloc((void**)&p->h_segs, sizeof(HistSeg) * nreq, hipHostMallocDefault));
        p->d_reqs_cap = nreq;
    }
    if (!p->d_counter) HIP_TRY(hipMalloc(&p->d_counter, 256));
    // Tiles are handed out in groups of one per wavefront of a work-group;
    // every request's tile range is padded to whole groups, so a group (and
    // its histogram row) belongs to one request.
    const int gw = K.wg / 64;
    int64_t tiles = 0, chunks = 0;
    for (int k = 0; k < nreq; ++k) {
        const skel_buffer* a = args + (size_t)order[k] * nargs;
        BatchReq& R = p->h_reqs[k];
        memset(&R, 0, sizeof(R));
        R.in = (const uint8_t*)a[0].data;
        R.out = (uint8_t*)a[1].data;
        R.hist = red == SKEL_RED_HIST256_SUM ? (uint32_t*)a[2].data : nullptr;
        R.sum = red == SKEL_RED_HIST256_SUM ? (uint64_t*)a[3].data : (red == SKEL_RED_SUM ? (uint64_t*)a[2].data : nullptr);
        R.H = (int32_t)a[0].shape[0];
        R.W = (int32_t)a[0].shape[1];
        R.nbands = (R.W + bw - 1) / bw;
        R.tile_h = tile_rows(R.H);
        R.nchunks = (R.H + R.tile_h - 1) / R.tile_h;
        R.tile_begin = (int32_t)tiles;
        const int64_t nt = (R.W > 0 && R.H > 0) ? (int64_t)R.nbands * R.nchunks : 0;
        const int64_t ngroups = (nt + gw - 1) / gw;
        tiles += ngroups * gw;
        if (tiles >= ((int64_t)1 << 31)) return set_error(SKEL_EUNSUPPORTED, "batch has too many tiles");
        HistSeg& G = p->h_segs[k];
        memset(&G, 0, sizeof(G));
        G.hist = R.hist;
        G.sum = R.sum;
        G.row_begin = R.tile_begin / gw;
        G.nrows = (int32_t)ngroups;
        G.crows = hist_chunk_rows(K.bins);
        G.chunk_begin = (int32_t)chunks;
        chunks += hist_chunks((int)ngroups, G.crows);
    }
    const size_t words = 4 * (size_t)K.bins;
    const size_t rows = (size_t)(tiles / gw);
    if (red >= 0 && rows * words > p->b_rows_cap) {
        if (p->b_rows) (void)hipFree(p->b_rows);
        p->b_rows = nullptr;
        p->b_rows_cap = 0;
        HIP_TRY(hipMalloc(&p->b_rows, sizeof(uint32_t) * rows * words));
        p->b_rows_cap = rows * words;
    }
    // Tile -> request table (tiles are numbered request by request).
    std::vector<uint16_t> tile_req((size_t)tiles);
    for (int k = 0; k < nreq; ++k) {
        const int64_t end = k + 1 < nreq ? p->h_reqs[k + 1].tile_begin : tiles;
        for (int64_t t = p->h_reqs[k].tile_begin; t < end; ++t) tile_req[(size_t)t] = (uint16_t)k;
    }
    if ((size_t)tiles > p->tile_req_cap) {
        if (p->d_tile_req) (void)hipFree(p->d_tile_req);
        p->d_tile_req = nullptr;
        p->tile_req_cap = 0;
        HIP_TRY(hipMalloc(&p->d_tile_req, sizeof(uint16_t) * tiles));
        p->tile_req_cap = (size_t)tiles;
    }
    if (tiles > 0)
        HIP_TRY(hipMemcpy(p->d_tile_req, tile_req.data(), sizeof(uint16_t) * tiles, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_reqs, p->h_reqs, sizeof(BatchReq) * nreq, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_segs, p->h_segs, sizeof(HistSeg) * nreq, hipMemcpyHostToDevice));

    BatchArgs A;
    memset(&A, 0, sizeof(A));
    A.reqs = p->d_reqs;
    A.tile_req = p->d_tile_req;
    A.nreq = nreq;
    A.ntiles = (int32_t)tiles;
    A.has_blur = K.blur;
    A.in_flip = K.img.in_flip;
    A.out_flip = K.img.out_flip;
    A.has_hist = red >= 0;
    A.hist_ks = hist_copies_log2(K.bins, kHistWgWords);
    A.bins = K.bins;
    A.part = p->b_rows;
    A.counter = p->d_counter;
    A.pre = K.img.pre;
    A.post = K.img.post;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, p->device));
    const int wg = K.wg;
    int per_cu = img_batch_blocks_per_cu(A, wg);
    if (per_cu < 1) per_cu = 1;
    int grid = per_cu * prop.multiProcessorCount;
    const int need = (int)(tiles / gw);
    grid = std::max(1, std::min(grid, need));
    p->batch_grid = grid;

    if (p->bexec) {
        (void)hipGraphExecDestroy(p->bexec);
        p->bexec = nullptr;
    }
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const char* kname = nullptr;
    HistFinArgs F;
    memset(&F, 0, sizeof(F));
    F.part = p->b_rows;
    F.segs = p->d_segs;
    F.nseg = nreq;
    F.nchunks = (int32_t)chunks;
    F.bins = K.bins;
    hipError_t e1 = launch_fill_u32(p->d_counter, 1, 0, p->cap_stream);
    if (e1 == hipSuccess && red >= 0) e1 = launch_hist_zero(F, p->cap_stream);
    hipError_t e2 = tiles > 0 ? launch_img_batch(A, grid, wg, p->cap_stream, &kname) : hipSuccess;
    hipError_t e3 = red >= 0 ? launch_hist_merge(F, p->cap_stream) : hipSuccess;
    hipGraph_t g = nullptr;
    hipError_t e4 = hipStreamEndCapture(p->cap_stream, &g);
    if (e1 || e2 || e3 || e4) {
        if (g) (void)hipGraphDestroy(g);
        return set_error(SKEL_EDEVICE, "batch graph capture failed: %s",
                         hipGetErrorString(e1 ? e1 : (e2 ? e2 : (e3 ? e3 : e4))));
    }
    hipError_t e = hipGraphInstantiate(&p->bexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(SKEL_EDEVICE, "batch graph instantiate failed: %s", hipGetErrorString(e));
    p->bkey = key;
    HIP_TRY(hipGraphLaunch(p->bexec, s));
    return SKEL_OK;
}
