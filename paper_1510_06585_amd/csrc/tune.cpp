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
#include <ctime>
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
    std::vector<int> u8_tile_ladder;
    if (L.dom == DOM_U8) {
        Config fc = base;
        fc.fusion = SKEL_FUSE_ON;
        fc.wg = 256;
        std::vector<Kernel> ks;
        int f = std::max(2, base.tile_h);
        if (!build_kernels(L, sh, fc, ks) && !ks.empty()) f = std::max(2, (int)ks[0].img.tile_h);
        const int hmax = std::max<int>(2, (int)std::min<int64_t>(sh.H, kMaxDim));
        for (int th : {f / 4, f / 2, f, 2 * f}) {
            th = std::min(std::max(th, 2), hmax);
            if (std::find(u8_tile_ladder.begin(), u8_tile_ladder.end(), th) == u8_tile_ladder.end())
                u8_tile_ladder.push_back(th);
        }
    }
    for (uint32_t m : masks) {
        if (L.dom == DOM_GRAY) {
            for (int ept : {1, 8}) {
                Config c = base;
                c.fusion = k >= 1 ? SKEL_FUSE_MASK : SKEL_FUSE_ON;
                c.split_mask = m;
                c.ept = ept;
                if (config_valid(L, sh, c)) out.push_back(c);
            }
        } else if (L.dom == DOM_C32) {
            Config c = base;
            c.fusion = k >= 1 ? SKEL_FUSE_MASK : SKEL_FUSE_ON;
            c.split_mask = m;
            if (config_valid(L, sh, c)) out.push_back(c);
        } else if (L.dom == DOM_U8) {
            // Work-group sizes 64, 128, 256 x four explicit tile heights around
            // the fitted default of the fully fused kernel (a quarter, a half,
            // once and twice it, within [2, H]); explicit heights, so the
            // features and the timed plan see the same tiles.
            for (int wg : {64, 128, 256})
                for (int th : u8_tile_ladder) {
                    Config c = base;
                    c.fusion = k >= 1 ? SKEL_FUSE_MASK : SKEL_FUSE_ON;
                    c.split_mask = m;
                    c.wg = wg;
                    c.tile_h = th;
                    c.auto_tile = false;
                    if (config_valid(L, sh, c)) out.push_back(c);
                }
        } else {
            for (int wg : {64, 256, 1024})
                for (int ept : {1, 2, 4, 8}) {
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
    const double n = L.dom == DOM_U8    ? (double)sh.W * sh.H
                     : L.dom == DOM_F32 ? (double)sh.n
                     : L.dom == DOM_C32 ? (double)sh.n * kFftPoints
                     : L.dom == DOM_GRAY ? (double)sh.n
                                        : (double)sh.N;
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
        if (L.dom == DOM_C32) bytes += 16.0 * n;
        if (L.dom == DOM_GRAY) bytes += 2.0 * n;
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

namespace {

// Times one configuration: compile, 3 warm-up runs, `reps` runs timed with
// HIP events on a private stream; median and minimum in microseconds.
struct Timer {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<float> times;
    skel_status init() {
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        return SKEL_OK;
    }
    ~Timer() {   // teardown: errors are not reportable here
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
    skel_status time(skel_node root, const skel_buffer* args, int32_t nargs, const Config& c, int reps,
                     double* med, double* mn) {
        skel_plan_opts o;
        config_to_opts(c, &o);
        return time_opts(root, args, nargs, o, reps, med, mn);
    }
    skel_status time_opts(skel_node root, const skel_buffer* args, int32_t nargs, const skel_plan_opts& o, int reps,
                          double* med, double* mn) {
        skel_plan p = nullptr;
        skel_status st = skel_plan_compile(root, args, nargs, &o, &p);
        if (st) return SKEL_EINVAL;
        for (int w = 0; w < 3 && !st; ++w) st = skel_plan_run(p, args, nargs, s);
        times.clear();
        hipError_t e = hipSuccess;
        for (int r = 0; r < reps && !st && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, s);
            if (e != hipSuccess) break;
            st = skel_plan_run(p, args, nargs, s);
            if (st) break;
            float ms = 0;
            e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) times.push_back(ms * 1000.0f);
        }
        const hipError_t es = hipStreamSynchronize(s);
        if (e == hipSuccess) e = es;
        skel_plan_destroy(p);
        if (st) return st == SKEL_EINVAL ? SKEL_EDEVICE : st;   // a compiled plan that fails to run is a device error
        if (e != hipSuccess) return set_error(SKEL_EDEVICE, "timing a candidate: %s", hipGetErrorString(e));
        if (times.empty()) return set_error(SKEL_EINVAL, "no timed repetitions");
        std::sort(times.begin(), times.end());
        *med = times[times.size() / 2];
        *mn = times.front();
        return SKEL_OK;
    }
};

void db_row(FILE* db, const std::string& key, const Linear& L, const Shape& sh, const Config& c, double med,
            double mn) {
    float f[kNumFeatures];
    features(L, sh, c, f);
    fprintf(db, "%s,%d,%u,%d,%d,%d,%d", key.c_str(), c.fusion, c.split_mask, c.tile_h, c.wg, c.ept, c.variant);
    for (int i = 0; i < kNumFeatures; ++i) fprintf(db, ",%.6g", (double)f[i]);
    fprintf(db, ",%.4f,%.4f\n", med, mn);
}

// Provenance of the rows that follow (the knowledge base of Sec. 3.2 keeps
// profiles across sessions and machines): one comment line per tuning session
// with the tuner, the device, the runtime version and the UTC time.  Readers
// skip lines that start with '#'.
void db_session(FILE* db, const char* tuner, const std::string& key) {
    int dev = 0, rt = 0;
    hipDeviceProp_t prop;
    memset(&prop, 0, sizeof(prop));
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) prop.gcnArchName[0] = 0;
    if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
    char when[32] = "unknown";
    const time_t now = time(nullptr);
    struct tm g;
    if (gmtime_r(&now, &g)) strftime(when, sizeof(when), "%Y-%m-%dT%H:%M:%SZ", &g);
    fprintf(db, "# skel tuning session: tuner=%s composition=%s device=%s cus=%d hip_runtime=%d utc=%s\n", tuner,
            key.c_str(), prop.gcnArchName[0] ? prop.gcnArchName : "unknown", prop.multiProcessorCount, rt, when);
}

}  // namespace

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
    if (db) db_session(db, "exhaustive", key);
    Timer T;
    if ((st = T.init())) {
        if (db) fclose(db);
        return st;
    }
    double best_t = 1e300;
    Config best_c = cands[0];
    skel_status result = SKEL_OK;
    for (const Config& c : cands) {
        double med = 0, mn = 0;
        st = T.time(root, args, nargs, c, reps, &med, &mn);
        if (st == SKEL_EINVAL) continue;   // configuration rejected by the plan compiler
        if (st) {
            result = st;
            break;
        }
        if (med < best_t) {
            best_t = med;
            best_c = c;
        }
        if (db) db_row(db, key, L, sh, c, med, mn);
    }
    if (db) fclose(db);
    if (result) return result;
    config_to_opts(best_c, best);
    if (best_us) *best_us = best_t;
    return SKEL_OK;
}

// One configuration timed with the tuner's own protocol, so that baselines
// and re-timings compare with its rows like for like.
extern "C" skel_status skel_time_config(skel_node root, const skel_buffer* args, int32_t nargs,
                                        const skel_plan_opts* opts, int32_t reps, double* median_us,
                                        double* min_us) {
    clear_error();
    if (!root || !median_us) return set_error(SKEL_EINVAL, "null root or result");
    if (reps <= 0) reps = 10;
    skel_plan_opts o;
    if (opts) o = *opts; else skel_plan_opts_default(&o);
    // Compile once up front so that an invalid request reports the plan
    // compiler's own status and message (the timer folds compile failures
    // into SKEL_EINVAL); the options are passed on as given, so defaults such
    // as fitted tile heights stay defaults.
    skel_plan p = nullptr;
    skel_status st = skel_plan_compile(root, args, nargs, &o, &p);
    if (st) return st;
    skel_plan_destroy(p);
    Timer T;
    if ((st = T.init())) return st;
    double med = 0, mn = 0;
    if ((st = T.time_opts(root, args, nargs, o, reps, &med, &mn))) return st;
    *median_us = med;
    if (min_us) *min_us = mn;
    return SKEL_OK;
}

// Algorithm 1 (the profile builder), on one GPU: the dimensions of the
// configuration space are walked in the order most likely to hold the best
// configuration, and a dimension is abandoned as soon as a candidate fails to
// improve on the best so far ("discard"):
//   1. fusion partitions, fewest kernels first (the fully fused plan leads);
//      after the first partition, a partition whose best time does not beat
//      the best so far ends the search;
//   2. per partition, work-group sizes in non-increasing order of occupancy
//      (resident wavefronts per CU), those below occ_threshold of the best
//      occupancy filtered out; a size that does not improve ends the loop;
//   3. per size, the inner parameter (tile height of images, vectors per
//      thread of fp32 chains, j-slices of N-body) in increasing order while
//      each step improves by at least `precision_us`.
// CPU fission, overlap and the CPU/GPU load distribution of the paper's
// algorithm have no counterpart on one GPU.
namespace {

struct Group {
    int wg;
    std::vector<Config> inner;   // increasing inner parameter
};

int occupancy_of(const Linear& L, const Shape& sh, const Config& c) {
    std::vector<Kernel> ks;
    if (build_kernels(L, sh, c, ks) || ks.empty()) return 0;
    if (L.dom == DOM_U8) {
        int worst = 1 << 30;
        for (const Kernel& K : ks)
            worst = std::min(worst, img_waves_per_cu(K.img, K.blur, K.reduce, K.wg, c.variant));
        return worst;
    }
    return 1;   // fp32, gray and FFT chains, N-body: occupancy does not depend on wg here
}

int inner_value(const Linear& L, const Config& c) { return (L.dom == DOM_F32 || L.dom == DOM_GRAY) ? c.ept : c.tile_h; }

}  // namespace

extern "C" skel_status skel_tune_pruned(skel_node root, const skel_buffer* args, int32_t nargs, const char* db_path,
                                        int32_t reps, double precision_us, double occ_threshold,
                                        skel_plan_opts* best, double* best_us, int32_t* timed) {
    clear_error();
    if (!root || !best) return set_error(SKEL_EINVAL, "null root or result");
    Linear L;
    Shape sh;
    skel_status st = linearize(root, L);
    if (!st && L.dom == DOM_NONE) L.dom = (nargs > 0 && args[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
    if (!st) st = derive_shape(L, args, nargs, sh);
    if (st) return st;
    if (reps <= 0) reps = 10;
    if (precision_us < 0) precision_us = 0;
    const std::vector<Config> all = enumerate_configs(L, sh);
    if (all.empty()) return set_error(SKEL_EUNSUPPORTED, "no valid configuration");

    // Group the candidate set by partition, then by work-group size.
    struct Part {
        int kernels;
        int fusion;
        uint32_t mask;
        std::vector<Group> groups;
    };
    std::vector<Part> parts;
    for (const Config& c : all) {
        Part* P = nullptr;
        for (Part& q : parts)
            if (q.fusion == c.fusion && q.mask == c.split_mask) P = &q;
        if (!P) {
            std::vector<Kernel> ks;
            build_kernels(L, sh, c, ks);
            parts.push_back(Part{(int)ks.size(), c.fusion, c.split_mask, {}});
            P = &parts.back();
        }
        Group* G = nullptr;
        for (Group& g : P->groups)
            if (g.wg == c.wg) G = &g;
        if (!G) {
            P->groups.push_back(Group{c.wg, {}});
            G = &P->groups.back();
        }
        G->inner.push_back(c);
    }
    std::stable_sort(parts.begin(), parts.end(), [](const Part& a, const Part& b) {
        if (a.kernels != b.kernels) return a.kernels < b.kernels;
        return a.mask < b.mask;
    });
    for (Part& P : parts) {
        std::vector<std::pair<int, int>> occ;   // (occupancy, index)
        for (size_t i = 0; i < P.groups.size(); ++i) {
            std::sort(P.groups[i].inner.begin(), P.groups[i].inner.end(),
                      [&](const Config& a, const Config& b) { return inner_value(L, a) < inner_value(L, b); });
            occ.push_back({occupancy_of(L, sh, P.groups[i].inner[0]), (int)i});
        }
        std::stable_sort(occ.begin(), occ.end(),
                         [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first > b.first; });
        std::vector<Group> ordered;
        for (const auto& o : occ)
            if (o.first >= occ_threshold * occ.front().first) ordered.push_back(P.groups[o.second]);
        P.groups.swap(ordered);
    }

    FILE* db = nullptr;
    if (db_path && *db_path) {
        db = fopen(db_path, "a");
        if (!db) return set_error(SKEL_EINVAL, "cannot open %s", db_path);
    }
    const std::string key = composition_key(L, sh);
    if (db) db_session(db, "pruned", key);
    Timer T;
    if ((st = T.init())) {
        if (db) fclose(db);
        return st;
    }
    double best_t = 1e300;
    Config best_c = parts.front().groups.front().inner.front();
    int ntimed = 0;
    skel_status result = SKEL_OK;
    for (size_t pi = 0; pi < parts.size() && !result; ++pi) {
        const double before_part = best_t;
        for (const Group& G : parts[pi].groups) {
            const double before_group = best_t;
            for (const Config& c : G.inner) {
                double med = 0, mn = 0;
                st = T.time(root, args, nargs, c, reps, &med, &mn);
                if (st == SKEL_EINVAL) continue;
                if (st) {
                    result = st;
                    break;
                }
                ++ntimed;
                if (db) db_row(db, key, L, sh, c, med, mn);
                if (med < best_t) {
                    const double gain = best_t - med;
                    best_t = med;
                    best_c = c;
                    if (gain < precision_us) break;   // converged along this direction
                } else {
                    break;                            // no improvement: discard larger values
                }
            }
            if (result || !(best_t < before_group)) break;   // this size did not improve: discard the rest
        }
        if (pi > 0 && !(best_t < before_part)) break;        // this partition did not improve: stop
    }
    if (db) fclose(db);
    if (result) return result;
    config_to_opts(best_c, best);
    if (best_us) *best_us = best_t;
    if (timed) *timed = ntimed;
    return SKEL_OK;
}

// Auto Tuner for batched runs (Sec. 2.2, applied to the batch execution
// model of Sec. 2).  The persistent batched kernel runs the fully fused plan
// (one kernel: the only partition a single persistent launch can hold), so the
// search is over the tile height every request is cut into and the
// work-group size (= wavefronts, hence adjacent tiles, per group), each point
// timed as a whole skel_batch_run of the caller's request set: 3 warm-up runs
// (the first lays out the work list and captures the graph), then the median
// of `reps` runs.  Exhaustive: every point.  pruned != 0: Algorithm 1's
// ordered walk -- work-group sizes in non-increasing order of resident
// wavefronts, the first size that does not improve ends the search; per size,
// tile heights increase while each improves by at least precision_us.
namespace {

constexpr int kBatchTileCands[] = {8, 12, 16, 24, 31, 40, 48, 64, 96, 128};
constexpr int kBatchWgCands[] = {64, 128, 256};

}  // namespace

extern "C" skel_status skel_tune_batch(skel_node root, const skel_buffer* args, int32_t nargs, int32_t nreq,
                                       const char* db_path, int32_t reps, int32_t pruned, double precision_us,
                                       skel_plan_opts* best, double* best_us, int32_t* timed) {
    clear_error();
    if (!root || !best || !args || nreq < 1) return set_error(SKEL_EINVAL, "null root, result or empty request set");
    Linear L;
    Shape sh;
    skel_status st = linearize(root, L);
    if (!st && L.dom == DOM_NONE) L.dom = (nargs > 0 && args[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
    if (!st) st = derive_shape(L, args, nargs, sh);
    if (st) return st;
    if (L.dom != DOM_U8 || L.is_while) return set_error(SKEL_EUNSUPPORTED, "batched runs are image chains");
    {
        // The request set is checked on the host before any device work, so a
        // bad request reports its own status rather than a failed candidate's.
        skel_plan_opts o;
        skel_plan_opts_default(&o);
        o.fusion = SKEL_FUSE_ON;
        skel_plan p0 = nullptr;
        if ((st = skel_plan_compile(root, args, nargs, &o, &p0))) return st;
        st = batch_validate(p0, args, nargs, nreq);
        const std::string why = st ? skel_last_error() : "";
        skel_plan_destroy(p0);   // clears the thread's error message
        if (st) return set_error(st, "%s", why.c_str());
    }
    if (reps <= 0) reps = 10;
    if (precision_us < 0) precision_us = 0;
    // The knowledge-base row describes the whole batch: the key names the
    // request count and total pixels, the features a square image of the
    // batch's total pixel count.
    double px = 0;
    for (int r = 0; r < nreq; ++r) px += (double)args[(size_t)r * nargs].shape[0] * args[(size_t)r * nargs].shape[1];
    Shape tot;
    tot.W = tot.H = std::max<int64_t>(1, (int64_t)std::llround(std::sqrt(px)));
    char kb[64];
    snprintf(kb, sizeof(kb), "batch%d|px%.0f|", nreq, px);
    const std::string key = kb + composition_key(L, sh);

    struct Cand {
        int wg, th, occ;
    };
    std::vector<std::vector<Cand>> by_wg;   // per work-group size, increasing tile height
    for (int wg : kBatchWgCands) {
        std::vector<Cand> v;
        for (int th : kBatchTileCands) v.push_back(Cand{wg, th, 0});
        by_wg.push_back(v);
    }
    if (pruned) {
        // resident wavefronts per CU of the fused kernel at each size (the
        // batched kernel shares its register and LDS footprint)
        skel_plan_opts d;
        skel_plan_opts_default(&d);
        for (auto& v : by_wg) {
            d.wg = v[0].wg;
            d.tile_h = v[0].th;
            Config c;
            std::vector<Kernel> ks;
            int occ = 0;
            if (!resolve_config(L, sh, &d, c) && !build_kernels(L, sh, c, ks) && ks.size() == 1)
                occ = img_waves_per_cu(ks[0].img, ks[0].blur, ks[0].reduce, ks[0].wg, c.variant);
            for (Cand& x : v) x.occ = occ;
        }
        std::stable_sort(by_wg.begin(), by_wg.end(),
                         [](const std::vector<Cand>& a, const std::vector<Cand>& b) { return a[0].occ > b[0].occ; });
    }

    FILE* db = nullptr;
    if (db_path && *db_path) {
        db = fopen(db_path, "a");
        if (!db) return set_error(SKEL_EINVAL, "cannot open %s", db_path);
    }
    if (db) db_session(db, pruned ? "batch-pruned" : "batch-exhaustive", key);
    Timer T;
    if ((st = T.init())) {
        if (db) fclose(db);
        return st;
    }
    double best_t = 1e300;
    Config best_c;
    bool have = false;
    int ntimed = 0;
    skel_status result = SKEL_OK;
    auto time_one = [&](const Cand& x, double* med, double* mn) -> skel_status {
        skel_plan_opts o;
        skel_plan_opts_default(&o);
        o.fusion = SKEL_FUSE_ON;
        o.tile_h = x.th;
        o.wg = x.wg;
        skel_plan p = nullptr;
        if (skel_plan_compile(root, args, nargs, &o, &p)) return SKEL_EINVAL;
        if (p->kernels.size() != 1) {
            skel_plan_destroy(p);
            return SKEL_EINVAL;
        }
        skel_status s2 = SKEL_OK;
        for (int w = 0; w < 3 && !s2; ++w) s2 = skel_batch_run(p, args, nargs, nreq, T.s);
        T.times.clear();
        hipError_t e = hipSuccess;
        for (int r = 0; r < reps && !s2 && e == hipSuccess; ++r) {
            e = hipEventRecord(T.e0, T.s);
            if (e != hipSuccess) break;
            s2 = skel_batch_run(p, args, nargs, nreq, T.s);
            if (s2) break;
            float ms = 0;
            e = hipEventRecord(T.e1, T.s);
            if (e == hipSuccess) e = hipEventSynchronize(T.e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, T.e0, T.e1);
            if (e == hipSuccess) T.times.push_back(ms * 1000.0f);
        }
        const hipError_t es = hipStreamSynchronize(T.s);
        if (e == hipSuccess) e = es;
        skel_plan_destroy(p);
        if (s2) return s2 == SKEL_EINVAL ? SKEL_EDEVICE : s2;
        if (e != hipSuccess) return set_error(SKEL_EDEVICE, "timing a batch candidate: %s", hipGetErrorString(e));
        if (T.times.empty()) return set_error(SKEL_EINVAL, "no timed repetitions");
        std::sort(T.times.begin(), T.times.end());
        *med = T.times[T.times.size() / 2];
        *mn = T.times.front();
        return SKEL_OK;
    };
    for (const auto& v : by_wg) {
        const double before = best_t;
        for (const Cand& x : v) {
            double med = 0, mn = 0;
            st = time_one(x, &med, &mn);
            if (st == SKEL_EINVAL) continue;
            if (st) {
                result = st;
                break;
            }
            ++ntimed;
            Config c;
            c.fusion = SKEL_FUSE_ON;
            c.tile_h = x.th;
            c.wg = x.wg;
            if (db) db_row(db, key, L, tot, c, med, mn);
            const bool better = med < best_t;
            const double gain = best_t - med;
            if (better) {
                best_t = med;
                best_c = c;
                have = true;
            }
            if (pruned && (!better || gain < precision_us)) break;
        }
        if (result) break;
        if (pruned && have && !(best_t < before)) break;
    }
    if (db) fclose(db);
    if (result) return result;
    if (!have) return set_error(SKEL_EUNSUPPORTED, "no batch configuration could be timed");
    skel_plan_opts_default(best);
    best->fusion = SKEL_FUSE_ON;
    best->tile_h = best_c.tile_h;
    best->wg = best_c.wg;
    if (best_us) *best_us = best_t;
    if (timed) *timed = ntimed;
    return SKEL_OK;
}
