// Plan compiler: linearises a skeleton tree, checks its typing, resolves the
// execution configuration and groups adjacent Map stages into fused kernels.
//
// Fusion follows the paper's locality-aware decomposition (Sec. 3.1): kernels
// that pass data to each other must see the same partitioning so the data can
// stay where it is.  On one GPU the strongest form of that rule is to run the
// communicating stages in one kernel over one tile, so intermediates never
// leave registers.  A mirror is a pixel permutation within a line; inside a
// fused kernel it becomes a coordinate flip of the stages around it.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include <algorithm>
#include <cmath>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace skel {

static thread_local std::string g_err;

skel_status set_error(skel_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
void clear_error() { g_err.clear(); }
const char* last_error_str() { return g_err.c_str(); }

static const char* op_name(int op) {
    switch (op) {
        case SKEL_OP_NOISE: return "noise";
        case SKEL_OP_SOLARISE: return "solarise";
        case SKEL_OP_MIRROR: return "mirror";
        case SKEL_OP_BLUR5: return "blur5";
        case SKEL_OP_SAXPY: return "saxpy";
        case SKEL_OP_NBODY_FORCE: return "nbody_force";
        case SKEL_OP_LEAPFROG: return "leapfrog";
        case SKEL_OP_FFT: return "fft";
        case SKEL_OP_IFFT: return "ifft";
        case SKEL_OP_SEGMENT: return "segment";
    }
    return "?";
}

static skel_status lin_rec(const skel_node_s* n, Linear& L, bool root, int depth) {
    if (!n) return set_error(SKEL_EINVAL, "null node in skeleton tree");
    if (depth > 64) return set_error(SKEL_EINVAL, "skeleton tree deeper than 64 levels");
    switch (n->kind) {
        case NK_MAP:
            if ((int)L.st.size() >= kMaxStages)
                return set_error(SKEL_EUNSUPPORTED, "more than %d stages after unrolling loops", kMaxStages);
            L.st.push_back(Stage{n->op, n->prm, -1});
            L.seen_ops |= 1u << n->op;
            L.sct += op_name(n->op);
            return SKEL_OK;
        case NK_PIPE: {
            L.sct += "pipeline(";
            for (size_t k = 0; k < n->kids.size(); ++k) {
                if (k) L.sct += ",";
                skel_status st = lin_rec(n->kids[k], L, false, depth + 1);
                if (st) return st;
            }
            L.sct += ")";
            return SKEL_OK;
        }
        case NK_LOOP: {
            Linear body;
            skel_status st = lin_rec(n->kids[0], body, false, depth + 1);
            if (st) return st;
            const int it = n->loop.iterations;
            if ((int64_t)body.st.size() * it + (int64_t)L.st.size() > (int64_t)kMaxStages * 2)
                return set_error(SKEL_EUNSUPPORTED, "loop unrolls to more than %d stages", 2 * kMaxStages);
            for (int r = 0; r < it; ++r) L.st.insert(L.st.end(), body.st.begin(), body.st.end());
            L.seen_ops |= body.seen_ops;
            if (it == 0 && (body.seen_ops & ((1u << SKEL_OP_NBODY_FORCE) | (1u << SKEL_OP_LEAPFROG)))) {
                // keep the N-body parameters of a zero-trip loop's body
                for (const Stage& b : body.st) {
                    if (b.op == SKEL_OP_NBODY_FORCE) L.nbody_prm.eps = b.prm.eps, L.nbody_prm.G = b.prm.G;
                    if (b.op == SKEL_OP_LEAPFROG) L.nbody_prm.dt = b.prm.dt;
                }
            }
            L.loop_carried |= n->loop.carried_mask;
            L.loop_sync |= n->loop.global_sync;
            char buf[32];
            snprintf(buf, sizeof(buf), "loop[%d](", it);
            L.sct += buf;
            L.sct += body.sct;
            L.sct += ")";
            return SKEL_OK;
        }
        case NK_WHILE: {
            if (!root) return set_error(SKEL_EINVAL, "a while Loop is only valid at the root of a plan");
            if (n->kids.empty() || !n->kids[0] || n->kids[0]->kind != NK_MAPRED)
                return set_error(SKEL_EINVAL, "a while Loop's body must be a MapReduce");
            char buf[64];
            snprintf(buf, sizeof(buf), "while[%d;ch%d;cmp%d;%llu](", n->loop.iterations, n->cond.channel,
                     n->cond.cmp, (unsigned long long)n->cond.threshold);
            L.sct += buf;
            skel_status st = lin_rec(n->kids[0], L, true, depth + 1);
            if (st) return st;
            L.sct += ")";
            L.is_while = true;
            L.while_max = n->loop.iterations;
            L.wcond = n->cond;
            L.loop_carried |= n->loop.carried_mask;
            L.loop_sync |= n->loop.global_sync;
            return SKEL_OK;
        }
        case NK_MAPRED: {
            if (!root) return set_error(SKEL_EINVAL, "MapReduce is only valid at the root of a plan");
            L.sct += "mapreduce(";
            skel_status st = lin_rec(n->kids[0], L, false, depth + 1);
            if (st) return st;
            L.red = n->red;
            L.sct += n->red == SKEL_RED_HIST256_SUM ? ",hist256_sum)" : ",sum)";
            return SKEL_OK;
        }
    }
    return set_error(SKEL_EINVAL, "unknown node kind");
}

skel_status linearize(skel_node root, Linear& L) {
    L = Linear();
    skel_status st = lin_rec(root, L, true, 0);
    if (st) return st;
    auto has = [&](int op) { return (L.seen_ops >> op) & 1u; };
    const int img = has(SKEL_OP_NOISE) + has(SKEL_OP_SOLARISE) + has(SKEL_OP_BLUR5);
    const int vec = has(SKEL_OP_SAXPY);
    const int nb = has(SKEL_OP_NBODY_FORCE) + has(SKEL_OP_LEAPFROG);
    const int ff = has(SKEL_OP_FFT) + has(SKEL_OP_IFFT);
    if (has(SKEL_OP_SEGMENT)) {
        if (img || vec || nb || ff || has(SKEL_OP_MIRROR))
            return set_error(SKEL_ETYPE, "SEGMENT stages cannot share a chain with other stages");
        if (L.red >= 0) return set_error(SKEL_ETYPE, "gray-volume chains have no reduce side");
        if (L.is_while) return set_error(SKEL_ETYPE, "a while Loop's body must be an image MapReduce");
        L.dom = DOM_GRAY;
        return SKEL_OK;
    }
    if (ff) {
        if (img || vec || nb || has(SKEL_OP_MIRROR))
            return set_error(SKEL_ETYPE, "FFT / IFFT stages cannot share a chain with other stages");
        if (L.red >= 0) return set_error(SKEL_ETYPE, "FFT chains have no reduce side");
        if (L.is_while) return set_error(SKEL_ETYPE, "a while Loop's body must be an image MapReduce");
        L.dom = DOM_C32;
        return SKEL_OK;
    }
    if (nb) {
        if (img || vec || has(SKEL_OP_MIRROR) || L.red >= 0 || (L.st.size() % 2) != 0)
            return set_error(SKEL_ETYPE, "N-body stages must form Pipeline(nbody_force, leapfrog), optionally looped");
        for (size_t k = 0; k < L.st.size(); k += 2) {
            const Stage& f = L.st[k];
            const Stage& g = L.st[k + 1];
            if (f.op != SKEL_OP_NBODY_FORCE || g.op != SKEL_OP_LEAPFROG)
                return set_error(SKEL_ETYPE, "N-body stages must alternate nbody_force, leapfrog");
            if (f.prm.eps != L.st[0].prm.eps || f.prm.G != L.st[0].prm.G || g.prm.dt != L.st[1].prm.dt)
                return set_error(SKEL_EUNSUPPORTED, "N-body parameters differ between iterations");
        }
        L.dom = DOM_NBODY;
        L.nbody_iters = (int)(L.st.size() / 2);
        if (L.nbody_iters > kMaxNBodyIters)
            return set_error(SKEL_EUNSUPPORTED, "N-body loop of more than %d iterations", kMaxNBodyIters);
        if (!L.st.empty()) {
            L.nbody_prm = L.st[0].prm;
            L.nbody_prm.dt = L.st[1].prm.dt;
        }
        if (L.st.size() > 2) L.st.resize(2);   // one (force, kick-drift) step; the Loop driver repeats it
        return SKEL_OK;
    }
    if (img && vec) return set_error(SKEL_ETYPE, "image stages and fp32 vector stages cannot share a chain");
    L.dom = img ? DOM_U8 : (vec ? DOM_F32 : DOM_NONE);
    if (L.is_while && L.dom == DOM_F32)
        return set_error(SKEL_ETYPE, "a while Loop's body must be an image MapReduce (exact integer condition)");
    if (L.dom == DOM_F32 && L.red == SKEL_RED_HIST256_SUM)
        return set_error(SKEL_ETYPE, "the histogram reduce applies to RGBA uint8 images only");
    int k = 0;
    for (Stage& s : L.st)
        if (s.op == SKEL_OP_SAXPY) s.side_arg = 1 + k++;
    return SKEL_OK;
}

int expected_nargs(const Linear& L) {
    if (L.dom == DOM_NBODY) return 3;
    if (L.dom == DOM_C32 || L.dom == DOM_GRAY) return 2;
    if (L.dom == DOM_U8)
        return 2 + (L.red == SKEL_RED_HIST256_SUM ? 2 : (L.red == SKEL_RED_SUM ? 1 : 0)) + (L.is_while ? 1 : 0);
    if (L.dom == DOM_F32) {
        int ns = 0;
        for (const Stage& s : L.st) ns += s.op == SKEL_OP_SAXPY;
        return 2 + ns + (L.red >= 0 ? 1 : 0);
    }
    return 2;
}

// Dense row-major strides (the only layout the kernels address).  An empty
// buffer is dense whatever its strides.  Otherwise the dimensions of extent
// > 1 either all have stride 0 (the shorthand for "dense") or each has exactly
// its dense stride; a mix of zero and non-zero strides is rejected, since a
// zero stride would make the kernels step past the caller's allocation.
// Dimensions of extent <= 1 are never stepped, so their strides are ignored.
bool dense_strides(const skel_buffer& b, int64_t esize) {
    for (int d = 0; d < b.ndim; ++d)
        if (b.shape[d] == 0) return true;
    bool any_zero = false, any_set = false;
    for (int d = 0; d < b.ndim; ++d)
        if (b.shape[d] > 1) (b.stride_bytes[d] == 0 ? any_zero : any_set) = true;
    if (!any_set) return true;
    if (any_zero) return false;
    int64_t stride = esize;
    for (int d = b.ndim - 1; d >= 0; --d) {
        if (b.shape[d] > 1 && b.stride_bytes[d] != stride) return false;
        stride *= b.shape[d];
    }
    return true;
}

static int64_t dtype_size(int dt) {
    switch (dt) {
        case SKEL_U8: return 1;
        case SKEL_U32: return 4;
        case SKEL_U64: return 8;
        case SKEL_F32: return 4;
        case SKEL_F64: return 8;
    }
    return 0;
}

static skel_status check_buf(const skel_buffer& b, int k, int dt, int ndim, const int64_t* shape) {
    if (b.dtype != dt) return set_error(SKEL_ETYPE, "argument %d: dtype %d, expected %d", k, b.dtype, dt);
    if (b.ndim != ndim) return set_error(SKEL_ESHAPE, "argument %d: %d dims, expected %d", k, b.ndim, ndim);
    for (int d = 0; d < ndim; ++d)
        if (shape[d] >= 0 && b.shape[d] != shape[d])
            return set_error(SKEL_ESHAPE, "argument %d: dim %d is %lld, expected %lld", k, d, (long long)b.shape[d],
                             (long long)shape[d]);
    for (int d = 0; d < ndim; ++d)
        if (b.shape[d] < 0) return set_error(SKEL_ESHAPE, "argument %d: negative extent", k);
    if (!dense_strides(b, dtype_size(dt))) return set_error(SKEL_ESHAPE, "argument %d: not dense row-major", k);
    return SKEL_OK;
}

skel_status derive_shape(const Linear& L, const skel_buffer* proto, int32_t nargs, Shape& sh) {
    sh = Shape();
    if (nargs != expected_nargs(L))
        return set_error(SKEL_EINVAL, "expected %d arguments, got %d", expected_nargs(L), nargs);
    skel_status st;
    if (L.dom == DOM_U8) {
        const int64_t H = proto[0].shape[0], W = proto[0].shape[1];
        const int64_t img[3] = {H, W, 4};
        if ((st = check_buf(proto[0], 0, SKEL_U8, 3, img))) return st;
        if ((st = check_buf(proto[1], 1, SKEL_U8, 3, img))) return st;
        if (L.red == SKEL_RED_HIST256_SUM) {
            const int64_t hs[2] = {4, 256}, ss[1] = {4};
            if ((st = check_buf(proto[2], 2, SKEL_U32, 2, hs))) return st;
            if ((st = check_buf(proto[3], 3, SKEL_U64, 1, ss))) return st;
        } else if (L.red == SKEL_RED_SUM) {
            const int64_t ss[1] = {4};
            if ((st = check_buf(proto[2], 2, SKEL_U64, 1, ss))) return st;
        }
        if (L.is_while) {
            const int64_t one[1] = {1};
            if ((st = check_buf(proto[nargs - 1], nargs - 1, SKEL_U32, 1, one))) return st;
        }
        if (W > kMaxDim || H > kMaxDim)
            return set_error(SKEL_EUNSUPPORTED, "image sides are limited to %d pixels", kMaxDim);
        if (W * H * 4 >= ((int64_t)1 << 31)) return set_error(SKEL_EUNSUPPORTED, "images are limited to 2 GiB");
        sh.W = W;
        sh.H = H;
        return SKEL_OK;
    }
    if (L.dom == DOM_GRAY) {
        if (proto[0].ndim < 1 || proto[0].ndim > 4) return set_error(SKEL_ESHAPE, "argument 0: 1..4 dims");
        if ((st = check_buf(proto[0], 0, SKEL_U8, proto[0].ndim, proto[0].shape))) return st;
        if ((st = check_buf(proto[1], 1, SKEL_U8, proto[0].ndim, proto[0].shape))) return st;
        int64_t n = 1;
        for (int d = 0; d < proto[0].ndim && n > 0; ++d) {
            if (proto[0].shape[d] >= ((int64_t)1 << 31)) return set_error(SKEL_EUNSUPPORTED, "volumes are limited to 2 GiB");
            n *= proto[0].shape[d];   // < 2^62: no overflow
            if (n >= ((int64_t)1 << 31)) return set_error(SKEL_EUNSUPPORTED, "volumes are limited to 2 GiB");
        }
        if (n < 0) n = 0;
        sh.n = n;
        return SKEL_OK;
    }
    if (L.dom == DOM_C32) {
        const int64_t B = proto[0].shape[0];
        const int64_t fs[3] = {B, kFftPoints, 2};
        if ((st = check_buf(proto[0], 0, SKEL_F32, 3, fs))) return st;
        if ((st = check_buf(proto[1], 1, SKEL_F32, 3, fs))) return st;
        if (B > 65535) return set_error(SKEL_EUNSUPPORTED, "at most 65535 transforms per run");
        sh.n = B;
        return SKEL_OK;
    }
    if (L.dom == DOM_F32) {
        const int64_t n = proto[0].shape[0];
        const int64_t vs[1] = {n};
        for (int k = 0; k < nargs - (L.red >= 0 ? 1 : 0); ++k)
            if ((st = check_buf(proto[k], k, SKEL_F32, 1, vs))) return st;
        if (L.red >= 0) {
            const int64_t one[1] = {1};
            if ((st = check_buf(proto[nargs - 1], nargs - 1, SKEL_F32, 1, one))) return st;
        }
        if (n * 4 >= ((int64_t)1 << 31)) return set_error(SKEL_EUNSUPPORTED, "vectors are limited to 2 GiB");
        sh.n = n;
        return SKEL_OK;
    }
    if (L.dom == DOM_NBODY) {
        const int64_t N = proto[0].shape[0];
        const int64_t bs[2] = {N, 4};
        for (int k = 0; k < 3; ++k)
            if ((st = check_buf(proto[k], k, SKEL_F32, 2, bs))) return st;
        if (N > (1 << 24)) return set_error(SKEL_EUNSUPPORTED, "at most 2^24 bodies");
        sh.N = N;
        return SKEL_OK;
    }
    return set_error(SKEL_ETYPE, "cannot tell the domain of the chain");
}

static int pow2_floor(int64_t v) {
    int p = 1;
    while ((int64_t)p * 2 <= v) p *= 2;
    return p;
}

skel_status resolve_config(const Linear& L, const Shape& sh, const skel_plan_opts* o, Config& c) {
    c = Config();
    skel_plan_opts d;
    skel_plan_opts_default(&d);
    if (!o) o = &d;
    c.fusion = o->fusion == SKEL_FUSE_AUTO ? SKEL_FUSE_ON : o->fusion;
    if (c.fusion < SKEL_FUSE_OFF || c.fusion > SKEL_FUSE_MASK) return set_error(SKEL_EINVAL, "bad fusion mode");
    c.split_mask = o->split_mask;
    c.variant = o->variant;
    if (c.variant < 0 || c.variant > 1) return set_error(SKEL_EINVAL, "variant must be 0 or 1");
    if (L.dom == DOM_U8) {
        c.wg = o->wg ? o->wg : 256;
        if (c.wg != 64 && c.wg != 128 && c.wg != 256) return set_error(SKEL_EINVAL, "image kernels take wg 64, 128 or 256");
        if (o->tile_h) {
            c.tile_h = o->tile_h;
        } else {
            c.auto_tile = true;
            bool blur = false;
            for (const Stage& s : L.st) blur |= s.op == SKEL_OP_BLUR5;
            const int64_t nb = (sh.W + (blur ? kBandOut : kBandPx) - 1) / (blur ? kBandOut : kBandPx);
            // Enough wavefront tiles to fill 256 CUs several times over.
            int th = 256;
            while (th > (blur ? 16 : 8) && nb * ((sh.H + th - 1) / th) < 4096) th /= 2;
            c.tile_h = th;
        }
        if (c.tile_h < 1 || c.tile_h > kMaxDim) return set_error(SKEL_EINVAL, "tile_h out of range");
        c.ept = 1;
    } else if (L.dom == DOM_F32) {
        c.wg = o->wg ? o->wg : 256;
        if (c.wg < 64 || c.wg > 1024 || c.wg % 64) return set_error(SKEL_EINVAL, "wg must be a multiple of 64 up to 1024");
        const int64_t nvec = (sh.n + 3) / 4;
        c.ept = o->ept ? o->ept : (nvec >= ((int64_t)1 << 20) ? 4 : 1);
        if (c.ept < 1 || c.ept > 64) return set_error(SKEL_EINVAL, "ept out of range");
        c.tile_h = 0;
    } else if (L.dom == DOM_GRAY) {
        // one 16-byte vector per lane in 512-lane groups measured fastest on
        // volumes of 1 to 60 MiB
        c.wg = o->wg ? o->wg : 512;
        if (c.wg < 64 || c.wg > 1024 || c.wg % 64) return set_error(SKEL_EINVAL, "wg must be a multiple of 64 up to 1024");
        c.ept = o->ept ? o->ept : 1;
        if (c.ept < 1 || c.ept > 64) return set_error(SKEL_EINVAL, "ept out of range");
        c.tile_h = 0;
    } else if (L.dom == DOM_C32) {
        c.wg = 256;
        if (o->wg && o->wg != 256) return set_error(SKEL_EINVAL, "FFT passes take wg 256");
        c.tile_h = 0;
        c.ept = 1;
    } else if (L.dom == DOM_NBODY) {
        c.tile_h = o->tile_h ? o->tile_h : 4;
        if (c.tile_h < 1 || c.tile_h > 16) return set_error(SKEL_EINVAL, "N-body j-slices must be 1..16");
        c.wg = 64 * c.tile_h;
        c.ept = 1;
        (void)pow2_floor;
    }
    return SKEL_OK;
}

// Segments [first, last) of a chain of k stages under the fusion mode.
static skel_status segments(const Linear& L, const Config& c, std::vector<std::pair<int, int>>& segs, bool& red_sep) {
    const int k = (int)L.st.size();
    segs.clear();
    red_sep = false;
    if (k == 0) {
        segs.push_back({0, 0});
        return SKEL_OK;
    }
    auto is_stencil = [&](int i) { return L.st[i].op == SKEL_OP_BLUR5; };
    auto is_value = [&](int i) { return L.st[i].op == SKEL_OP_NOISE || L.st[i].op == SKEL_OP_SOLARISE || L.st[i].op == SKEL_OP_SAXPY; };
    if (c.fusion == SKEL_FUSE_OFF) {
        for (int i = 0; i < k; ++i) segs.push_back({i, i + 1});
        red_sep = L.red >= 0;
        return SKEL_OK;
    }
    if (c.fusion == SKEL_FUSE_ON) {
        int start = 0, nst = 0, nval_pre = 0, nval_post = 0;
        for (int i = 0; i < k; ++i) {
            bool cut = false;
            if (is_stencil(i) && nst == 1) cut = true;
            if (is_value(i) && ((nst == 0 ? nval_pre : nval_post) >= kMaxOps)) cut = true;
            if (cut) {
                segs.push_back({start, i});
                start = i;
                nst = nval_pre = nval_post = 0;
            }
            if (is_stencil(i)) nst++;
            if (is_value(i)) (nst == 0 ? nval_pre : nval_post)++;
        }
        segs.push_back({start, k});
        return SKEL_OK;
    }
    // SKEL_FUSE_MASK
    int start = 0;
    for (int i = 0; i < k - 1; ++i)
        if (c.split_mask & (1u << i)) {
            segs.push_back({start, i + 1});
            start = i + 1;
        }
    segs.push_back({start, k});
    red_sep = L.red >= 0 && (c.split_mask & (1u << (k - 1)));
    if (L.red < 0 && (c.split_mask >> (k - 1)) != 0 && k <= 32)
        return set_error(SKEL_EINVAL, "split_mask has bits beyond the chain");
    for (auto& s : segs) {
        int nst = 0, pre = 0, post = 0;
        for (int i = s.first; i < s.second; ++i) {
            if (is_stencil(i)) nst++;
            if (is_value(i)) (nst == 0 ? pre : post)++;
        }
        if (nst > 1) return set_error(SKEL_EINVAL, "split_mask puts two stencil stages in one kernel");
        if (pre > kMaxOps || post > kMaxOps) return set_error(SKEL_EINVAL, "more than %d value stages in one kernel", kMaxOps);
    }
    return SKEL_OK;
}

static void push_op(OpList& l, const Stage& s, int flip) {
    const int k = l.n++;
    l.op[k] = s.op == SKEL_OP_NOISE ? IOP_NOISE : IOP_SOL;
    l.flip[k] = (uint8_t)(flip & 1);
    l.seed[k] = s.prm.seed;
}

// Exclusive upper bound of the final image's values: 128 when the last stage
// that changes values is a solarise (min(v, 255 - v) <= 127, and blur and
// mirror never raise a maximum), else 256.
static int final_value_bins(const Linear& L) {
    for (int i = (int)L.st.size() - 1; i >= 0; --i) {
        if (L.st[i].op == SKEL_OP_SOLARISE) return 128;
        if (L.st[i].op == SKEL_OP_NOISE) return 256;
    }
    return 256;
}

// Compute units of the current device, read once (a function-local static is
// initialised exactly once even when plans are compiled from several threads).
int device_cu_count() {
    static const int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            return n;
        return 256;
    }();
    return cus;
}

// Default rows per tile.  With x = H * nbands / R, R the resident wavefronts
// of the launch, x rows per tile fill the device exactly once.  Shorter tiles
// leave a shorter tail: the wavefronts sharing a SIMD do not progress evenly
// (the oldest issues first), so with a single round the last wavefront of each
// SIMD runs alone at the end.  Taller tiles amortise the per-tile costs: the
// two halo rows above and below a stencil tile, and the LDS histogram clear
// and row store of a reduce work-group.  Measured on gfx950 over 512^2..8192^2
// images, the best height grows like sqrt(x): 4 sqrt(x) for stencil tiles,
// 3 sqrt(x) for reduce tiles, sqrt(x) otherwise (at least 2 rows).  When that
// gives a round or more, the height is then raised just enough to make the
// tile count a whole number of rounds: a few tiles over a round boundary form
// a tail round of their own (8192^2 stencil tiles: 32 rows = 2.06 rounds ran
// 5% slower than 34 rows = 1.94 rounds).
static int fitted_tile_h(const ImgGroupArgs& A, bool blur, bool hist, const Config& c) {
    if (A.W <= 0 || A.H <= 0) return 1;
    const double resident = (double)img_waves_per_cu(A, blur, hist, c.wg, c.variant) * device_cu_count();
    const int64_t nb = std::max<int32_t>(1, A.nbands);
    const double x = (double)A.H * nb / std::max(1.0, resident);
    const double k = blur ? 4.0 : (hist ? 3.0 : 1.0);
    int th = std::max(2, (int)std::lround(k * std::sqrt(x)));
    const double rounds = (double)nb * ((A.H + th - 1) / th) / std::max(1.0, resident);
    if (rounds >= 1.0) {
        const int64_t chunks = std::max<int64_t>(1, (int64_t)(std::lround(rounds) * resident) / nb);
        th = std::max(2, (int)((A.H + chunks - 1) / chunks));
    }
    return std::min(th, (int)A.H);
}

skel_status build_kernels(const Linear& L, const Shape& sh, const Config& c, std::vector<Kernel>& ks) {
    ks.clear();
    const int bins = final_value_bins(L);
    if (L.dom == DOM_NBODY) {
        Kernel k;
        k.first = 0;
        k.last = 2;
        k.wg = c.wg;
        k.grid = (int)((sh.N + 63) / 64);
        k.name = c.fusion == SKEL_FUSE_OFF ? "nbody_force" : "nbody_force_kick_drift";
        ks.push_back(k);
        if (c.fusion == SKEL_FUSE_OFF) {
            Kernel g = k;
            g.first = 1;
            g.name = "nbody_kick_drift";
            ks.push_back(g);
        }
        return SKEL_OK;
    }
    if (L.dom == DOM_GRAY) {
        // One kernel per fused run of stages (all of them unless unfused or
        // split by the mask).
        const int k = (int)L.st.size();
        int first = 0;
        for (int i = 0; i < k; ++i) {
            const bool split = i == k - 1 || c.fusion == SKEL_FUSE_OFF ||
                               (c.fusion == SKEL_FUSE_MASK && ((c.split_mask >> i) & 1u)) || i - first + 1 == kMaxOps;
            if (!split) continue;
            Kernel K;
            K.first = first;
            K.last = i + 1;
            K.wg = c.wg;
            memset(&K.gray, 0, sizeof(K.gray));
            K.gray.n = sh.n;
            K.gray.ept = c.ept;
            for (int j = first; j <= i; ++j) {
                uint32_t lo = L.st[j].prm.lo, hi = L.st[j].prm.hi;
                if (lo == 0 && hi == 0) lo = 85, hi = 170;
                K.gray.lo[K.gray.nops] = (uint16_t)lo;
                K.gray.hi[K.gray.nops] = (uint16_t)hi;
                K.gray.nops++;
            }
            const int64_t nvec = (sh.n + 15) / 16;
            K.grid = (int)((nvec + (int64_t)c.wg * c.ept - 1) / ((int64_t)c.wg * c.ept));
            K.name = "gray_segment";
            ks.push_back(K);
            first = i + 1;
        }
        const int nk = (int)ks.size();
        for (int g = 0; g < nk; ++g) {
            ks[g].src = g == 0 ? -1 : ((g - 1) % 2);
            ks[g].dst = g == nk - 1 ? -2 : (g % 2);
        }
        return SKEL_OK;
    }
    if (L.dom == DOM_C32) {
        // Stage i splits from stage i + 1 when unfused or split_mask bit i is
        // set: its pass B then writes natural order and the next stage starts
        // with a pass A; otherwise the two share one fused B+A kernel.
        const int k = (int)L.st.size();
        auto dir = [&](int i) { return L.st[i].op == SKEL_OP_IFFT ? 1 : -1; };
        auto split = [&](int i) {
            return c.fusion == SKEL_FUSE_OFF || (c.fusion == SKEL_FUSE_MASK && ((c.split_mask >> i) & 1u));
        };
        auto add = [&](int mode, int i, int first, int last) {
            Kernel K;
            K.first = first;
            K.last = last;
            K.wg = 512;
            K.grid = (int)(sh.n * 8);
            K.fft_mode = mode;
            memset(&K.fft, 0, sizeof(K.fft));
            K.fft.dir1 = dir(i);
            K.fft.dir2 = mode == 1 ? dir(i + 1) : 0;
            K.fft.scale1 = (mode != 0 && L.st[i].op == SKEL_OP_IFFT) ? 1.0f / (float)kFftPoints : 1.0f;
            K.name = fft_pass_name(mode);
            ks.push_back(K);
        };
        add(0, 0, 0, 1);
        for (int i = 0; i < k; ++i) {
            if (i == k - 1) {
                add(2, i, i, i + 1);
            } else if (split(i)) {
                add(2, i, i, i + 1);
                add(0, i + 1, i + 1, i + 2);
            } else {
                add(1, i, i, i + 2);
            }
        }
        const int nk = (int)ks.size();
        for (int g = 0; g < nk; ++g) {
            ks[g].src = g == 0 ? -1 : ((g - 1) % 2);
            ks[g].dst = g == nk - 1 ? -2 : (g % 2);
        }
        return SKEL_OK;
    }
    std::vector<std::pair<int, int>> segs;
    bool red_sep = false;
    skel_status st = segments(L, c, segs, red_sep);
    if (st) return st;
    const int nk = (int)segs.size();
    for (int g = 0; g < nk; ++g) {
        Kernel K;
        K.first = segs[g].first;
        K.last = segs[g].second;
        K.src = g == 0 ? -1 : ((g - 1) % 2);
        K.dst = g == nk - 1 ? -2 : (g % 2);
        K.reduce = (g == nk - 1) && L.red >= 0 && !red_sep;
        K.wg = c.wg;
        if (L.dom == DOM_U8 || L.dom == DOM_NONE) {
            int b = -1;
            for (int i = K.first; i < K.last; ++i)
                if (L.st[i].op == SKEL_OP_BLUR5) b = i;
            ImgGroupArgs& A = K.img;
            memset(&A, 0, sizeof(A));
            auto mirrors = [&](int lo, int hi) {
                int m = 0;
                for (int i = lo; i < hi; ++i) m += L.st[i].op == SKEL_OP_MIRROR;
                return m & 1;
            };
            if (b >= 0) {
                K.blur = true;
                A.in_flip = mirrors(K.first, b);
                A.out_flip = mirrors(b + 1, K.last);
                for (int i = K.first; i < b; ++i)
                    if (L.st[i].op == SKEL_OP_NOISE || L.st[i].op == SKEL_OP_SOLARISE) push_op(A.pre, L.st[i], mirrors(i + 1, b));
                for (int i = b + 1; i < K.last; ++i)
                    if (L.st[i].op == SKEL_OP_NOISE || L.st[i].op == SKEL_OP_SOLARISE) push_op(A.post, L.st[i], mirrors(b + 1, i));
            } else {
                A.in_flip = 0;
                A.out_flip = mirrors(K.first, K.last);
                for (int i = K.first; i < K.last; ++i)
                    if (L.st[i].op == SKEL_OP_NOISE || L.st[i].op == SKEL_OP_SOLARISE) push_op(A.pre, L.st[i], mirrors(K.first, i));
            }
            A.W = (int32_t)sh.W;
            A.H = (int32_t)sh.H;
            const int bw = K.blur ? kBandOut : kBandPx;
            A.nbands = (int32_t)((sh.W + bw - 1) / bw);
            A.tile_h = c.auto_tile ? fitted_tile_h(A, K.blur, K.reduce, c) : c.tile_h;
            const int64_t chunks = (sh.H + A.tile_h - 1) / A.tile_h;
            A.ntiles = (sh.W == 0 || sh.H == 0) ? 0 : (int32_t)(A.nbands * chunks);
            A.write_out = 1;
            A.hist_ks = hist_copies_log2(bins, kHistWgWords);
            A.bins = bins;
            K.bins = bins;
            K.grid = (A.ntiles + c.wg / 64 - 1) / (c.wg / 64);
            K.name = img_kernel_name(A, K.blur, K.reduce, c.variant);
        } else {
            VecGroupArgs& A = K.vec;
            memset(&A, 0, sizeof(A));
            int m = 0;
            for (int i = K.first; i < K.last; ++i) {
                if (L.st[i].op == SKEL_OP_MIRROR) {
                    m ^= 1;
                } else {
                    if (A.nops >= kMaxVecOps) return set_error(SKEL_EINVAL, "more than %d saxpy stages in one kernel", kMaxVecOps);
                    A.a[A.nops] = L.st[i].prm.a;
                    A.flip[A.nops] = (uint8_t)m;
                    K.side_args.push_back(L.st[i].side_arg);
                    A.nops++;
                }
            }
            A.out_flip = m;
            A.n = sh.n;
            A.ept = c.ept;
            A.write_out = 1;
            const int64_t nvec = (sh.n + 3) / 4;
            K.grid = (int)((nvec + (int64_t)c.wg * c.ept - 1) / ((int64_t)c.wg * c.ept));
            K.name = "vec_chain";
        }
        ks.push_back(K);
    }
    if (red_sep) {
        Kernel R;
        R.first = R.last = (int)L.st.size();
        R.src = -2;
        R.dst = -3;
        R.reduce = true;
        R.wg = c.wg;
        if (L.dom == DOM_U8) {
            ImgGroupArgs& A = R.img;
            memset(&A, 0, sizeof(A));
            A.W = (int32_t)sh.W;
            A.H = (int32_t)sh.H;
            A.nbands = (int32_t)((sh.W + kBandPx - 1) / kBandPx);
            A.tile_h = c.auto_tile ? fitted_tile_h(A, false, true, c) : c.tile_h;
            const int64_t chunks = (sh.H + A.tile_h - 1) / A.tile_h;
            A.ntiles = (sh.W == 0 || sh.H == 0) ? 0 : (int32_t)(A.nbands * chunks);
            A.write_out = 0;
            A.hist_ks = hist_copies_log2(bins, kHistWgWords);
            A.bins = bins;
            R.bins = bins;
            R.grid = (A.ntiles + c.wg / 64 - 1) / (c.wg / 64);
            R.name = img_kernel_name(A, false, true, c.variant);
        } else {
            VecGroupArgs& A = R.vec;
            memset(&A, 0, sizeof(A));
            A.n = sh.n;
            A.ept = c.ept;
            A.write_out = 0;
            const int64_t nvec = (sh.n + 3) / 4;
            R.grid = (int)((nvec + (int64_t)c.wg * c.ept - 1) / ((int64_t)c.wg * c.ept));
            R.name = "vec_chain";
        }
        ks.push_back(R);
    }
    return SKEL_OK;
}

bool config_valid(const Linear& L, const Shape& sh, const Config& c) {
    std::vector<Kernel> ks;
    std::string saved = g_err;
    const bool ok = build_kernels(L, sh, c, ks) == SKEL_OK;
    g_err = saved;
    if (!ok) return false;
    if (L.dom == DOM_U8) {
        // Partitioning constraints (Sec. 3.1): a tile's rows times the 4 pixels
        // each lane computes must divide evenly into work-groups of wg/64 tiles;
        // here every tile is one wavefront, so wg must be a multiple of 64 and
        // a work-group may not span fewer than one tile.
        if (c.wg % 64 || c.tile_h < 1) return false;
    }
    return true;
}

}  // namespace skel

extern "C" const char* skel_last_error(void) { return skel::last_error_str(); }

extern "C" void skel_plan_opts_default(skel_plan_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->fusion = SKEL_FUSE_ON;
}
