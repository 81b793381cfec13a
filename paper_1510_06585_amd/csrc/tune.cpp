// Auto Tuner (Sec. 2.2) and the feature map of the learned cost model.
//
// The paper's profile builder (Algorithm 1) walks ordered configuration
// dimensions with early stopping and keeps the best configuration per
// (SCT, workload) in a knowledge base.  Here the configuration space of one
// plan is: the fusion partition of its stage chain (where kernels split, and
// whether the reduce side runs in its own kernel) x work-group size x tile
// height (images) or vectors per thread (fp32 chains) or j-slices and fusion
// (N-body).  skel_tune measures every valid point and appends the results to
// a plain-text database that doubles as the cost model's training set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "internal.h"
#include "tune.h"

using namespace skel;

namespace skel {

std::vector<Config> enumerate_configs(const Linear& L, const Shape& sh) {
    std::vector<Config> out;
    Config base;
    skel_plan_opts d;
    skel_plan_opts_default(&d);
    resolve_config(L, sh, &d, base);
    const int k = (int)L.st.size();
    if (L.dom == DOM_NBODY) {
        for (int fused = 0; fused < 2; ++fused)
            for (int js : {1, 2, 4, 8, 16}) {
                Config c = base;
                c.fusion = fused ? SKEL_FUSE_ON : SKEL_FUSE_OFF;
                c.tile_h = js;
                c.wg = 64 * js;
                out.push_back(c);
            }
        return out;
    }
    const int nbits = std::max(0, k - 1) + (L.red >= 0 ? 1 : 0);
    std::vector<uint32_t> masks;
    if (k >= 1 && nbits <= 10)
        for (uint32_t m = 0; m < (1u << nbits); ++m) {
            uint32_t mm = m & ((1u << std::max(0, k - 1)) - 1u);
            if (L.red >= 0 && (m >> std::max(0, k - 1)) & 1u) mm |= 1u << (k - 1);
            masks.push_back(mm);
        }
    else
        masks.push_back(0);
    for (uint32_t m : masks) {
        if (L.dom == DOM_U8) {
            const int th0 = base.tile_h;
            const int variants[3][2] = {{256, th0}, {64, std::max(8, th0 / 2)}, {256, std::min(1024, th0 * 2)}};
            for (const auto& v : variants) {
                Config c = base;
                c.fusion = k >= 1 ? SKEL_FUSE_MASK : SKEL_FUSE_ON;
                c.split_mask = m;
                c.wg = v[0];
                c.tile_h = v[1];
                if (config_valid(L, sh, c)) out.push_back(c);
            }
        } else {
            for (int wg : {64, 256, 1024})
                for (int ept : {1, 4}) {
                    Config c = base;
                    c.fusion = k >= 1 ? SKEL_FUSE_MASK : SKEL_FUSE_ON;
                    c.split_mask = m;
                    c.wg = wg;
                    c.ept = ept;
                    if (config_valid(L, sh, c)) out.push_back(c);
                }
        }
    }
    return out;
}

static double lg2(double v) { return v > 0 ? std::log2(v) : 0.0; }

void features(const Linear& L, const Shape& sh, const Config& c, float* f) {
    for (int i = 0; i < kNumFeatures; ++i) f[i] = 0.0f;
    std::vector<Kernel> ks;
    build_kernels(L, sh, c, ks);
    int cnt[6] = {0, 0, 0, 0, 0, 0};
    for (const Stage& s : L.st) {
        if (s.op == SKEL_OP_NOISE) cnt[0]++;
        if (s.op == SKEL_OP_SOLARISE) cnt[1]++;
        if (s.op == SKEL_OP_MIRROR) cnt[2]++;
        if (s.op == SKEL_OP_BLUR5) cnt[3]++;
        if (s.op == SKEL_OP_SAXPY) cnt[4]++;
    }
    cnt[5] = L.red >= 0 ? 1 : 0;
    for (int i = 0; i < 6; ++i) f[i] = (float)cnt[i];
    const int k = (int)L.st.size();
    f[6] = (float)k;
    const double n = L.dom == DOM_U8 ? (double)sh.W * sh.H : (L.dom == DOM_F32 ? (double)sh.n : (double)sh.N);
    f[7] = (float)lg2(n);
    f[8] = L.dom == DOM_U8 ? 1.0f : 0.0f;
    f[9] = (float)cnt[4];   // side-vector streams of an fp32 chain
    f[10] = (float)ks.size();
    // fusion boundary bits after stages 0..4 (a new kernel starts after stage i)
    for (size_t g = 1; g < ks.size(); ++g) {
        const int b = ks[g].first - 1;
        if (b >= 0 && b < 5 && ks[g].first < k) f[11 + b] = 1.0f;
    }
    const bool any_blur = cnt[3] > 0;
    f[16] = (float)lg2(L.dom == DOM_U8 ? (any_blur ? kBandOut : kBandPx) : 4.0 * c.ept);
    const int th = (L.dom == DOM_U8 && !ks.empty()) ? ks[0].img.tile_h : c.tile_h;
    f[17] = (float)lg2(std::max(1, th));
    f[18] = (float)lg2(c.wg);
    f[19] = (float)lg2(std::max(1, c.ept));
    int worst = 0;
    bool red_fused = false;
    double bytes = 0;
    for (const Kernel& K : ks) {
        int ns = 0;
        for (int i = K.first; i < K.last; ++i) ns += L.st[i].op == SKEL_OP_BLUR5;
        worst = std::max(worst, ns);
        if (K.reduce && K.last > K.first) red_fused = true;
        if (L.dom == DOM_U8) bytes += (K.dst == -3 ? 1.0 : 2.0) * n * 4.0;
        if (L.dom == DOM_F32) bytes += ((K.dst == -3 ? 1.0 : 2.0) + K.side_args.size()) * n * 4.0;
        if (L.dom == DOM_NBODY) bytes += 48.0 * n;
    }
    f[20] = (float)worst;
    f[21] = red_fused ? 1.0f : 0.0f;
    f[22] = (float)lg2(bytes);
    f[23] = (float)lg2((double)ks.size() + (L.red >= 0 ? 1 : 0));
}

std::string composition_key(const Linear& L, const Shape& sh) {
    char buf[96];
    snprintf(buf, sizeof(buf), "|%lldx%lld|%lld|%lld", (long long)sh.H, (long long)sh.W, (long long)sh.n,
             (long long)sh.N);
    std::string s = L.sct + buf;
    for (const Stage& st : L.st) {
        if (st.op == SKEL_OP_SAXPY) {
            snprintf(buf, sizeof(buf), "|a=%.9g", (double)st.prm.a);
            s += buf;
        }
    }
    for (char& ch : s)
        if (ch == ',' || ch == ' ') ch = ';';
    return s;
}

void config_to_opts(const Config& c, skel_plan_opts* o) {
    skel_plan_opts_default(o);
    o->fusion = c.fusion;
    o->split_mask = c.split_mask;
    o->tile_h = c.tile_h;
    o->wg = c.wg;
    o->ept = c.ept;
    o->variant = c.variant;
}

}  // namespace skel

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(e_ == hipErrorOutOfMemory ? SKEL_ENOMEM : SKEL_EDEVICE, "%s: %s", \
                             #expr, hipGetErrorString(e_));                                    \
    } while (0)

extern "C" int32_t skel_feature_count(void) { return kNumFeatures; }

extern "C" skel_status skel_features(skel_node root, const skel_buffer* proto, int32_t nargs,
                                     const skel_plan_opts* opts, float* feat) {
    clear_error();
    if (!root || !feat) return set_error(SKEL_EINVAL, "null root or feature buffer");
    Linear L;
    Shape sh;
    Config c;
    skel_status st = linearize(root, L);
    if (!st && L.dom == DOM_NONE) L.dom = (nargs > 0 && proto[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
    if (!st) st = derive_shape(L, proto, nargs, sh);
    if (!st) st = resolve_config(L, sh, opts, c);
    if (st) return st;
    std::vector<Kernel> ks;
    if ((st = build_kernels(L, sh, c, ks))) return st;
    features(L, sh, c, feat);
    return SKEL_OK;
}

extern "C" skel_status skel_config_count(skel_node root, const skel_buffer* proto, int32_t nargs, int32_t* count) {
    clear_error();
    if (!root || !count) return set_error(SKEL_EINVAL, "null root or result");
    Linear L;
    Shape sh;
    skel_status st = linearize(root, L);
    if (!st && L.dom == DOM_NONE) L.dom = (nargs > 0 && proto[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
    if (!st) st = derive_shape(L, proto, nargs, sh);
    if (st) return st;
    *count = (int32_t)enumerate_configs(L, sh).size();
    return SKEL_OK;
}

extern "C" skel_status skel_tune(skel_node root, const skel_buffer* args, int32_t nargs, const char* db_path,
                                 int32_t reps, int32_t max_configs, uint64_t sample_seed, skel_plan_opts* best,
                                 double* best_us) {
    clear_error();
    if (!root || !best) return set_error(SKEL_EINVAL, "null root or result");
    Linear L;
    Shape sh;
    skel_status st = linearize(root, L);
    if (!st && L.dom == DOM_NONE) L.dom = (nargs > 0 && args[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
    if (!st) st = derive_shape(L, args, nargs, sh);
    if (st) return st;
    if (reps <= 0) reps = 10;
    std::vector<Config> cands = enumerate_configs(L, sh);
    if (cands.empty()) return set_error(SKEL_EUNSUPPORTED, "no valid configuration");
    if (max_configs > 0 && (int)cands.size() > max_configs) {
        // Sample without replacement; the default configuration stays first.
        Config def;
        skel_plan_opts d;
        skel_plan_opts_default(&d);
        resolve_config(L, sh, &d, def);
        std::mt19937_64 g(sample_seed);
        std::shuffle(cands.begin(), cands.end(), g);
        cands.resize(max_configs - 1);
        cands.insert(cands.begin(), def);
    }
    FILE* db = nullptr;
    if (db_path && *db_path) {
        db = fopen(db_path, "a");
        if (!db) return set_error(SKEL_EINVAL, "cannot open %s", db_path);
    }
    const std::string key = composition_key(L, sh);
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    double best_t = 1e300;
    Config best_c = cands[0];
    std::vector<float> times;
    skel_status result = SKEL_OK;
    for (const Config& c : cands) {
        skel_plan_opts o;
        config_to_opts(c, &o);
        skel_plan p = nullptr;
        st = skel_plan_compile(root, args, nargs, &o, &p);
        if (st) continue;
        for (int w = 0; w < 3 && !st; ++w) st = skel_plan_run(p, args, nargs, s);
        times.clear();
        for (int r = 0; r < reps && !st; ++r) {
            hipEventRecord(e0, s);
            st = skel_plan_run(p, args, nargs, s);
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            times.push_back(ms * 1000.0f);
        }
        hipStreamSynchronize(s);
        skel_plan_destroy(p);
        if (st) {
            result = st;
            break;
        }
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        if (med < best_t) {
            best_t = med;
            best_c = c;
        }
        if (db) {
            float f[kNumFeatures];
            features(L, sh, c, f);
            fprintf(db, "%s,%d,%u,%d,%d,%d,%d", key.c_str(), c.fusion, c.split_mask, c.tile_h, c.wg, c.ept,
                    c.variant);
            for (int i = 0; i < kNumFeatures; ++i) fprintf(db, ",%.6g", (double)f[i]);
            fprintf(db, ",%.4f,%.4f\n", med, (double)times.front());
        }
    }
    if (db) fclose(db);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamDestroy(s);
    if (result) return result;
    config_to_opts(best_c, best);
    if (best_us) *best_us = best_t;
    return SKEL_OK;
}
