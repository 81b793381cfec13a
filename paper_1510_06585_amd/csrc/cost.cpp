// Learned cost model: trains the MLP on tuning-database rows with the
// project's own HIP kernels and selects configurations for unseen
// compositions.  The paper derives configurations for new (SCT, workload)
// pairs by interpolating over the knowledge base (Sec. 3.2: radial basis
// functions up to three dimensions, Euclidean nearest neighbour above); the
// network here plays that role over the 24 features of a configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "tune.h"

using namespace skel;

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(e_ == hipErrorOutOfMemory ? SKEL_ENOMEM : SKEL_EDEVICE, "%s: %s", \
                             #expr, hipGetErrorString(e_));                                    \
    } while (0)

namespace {

constexpr int kNP = 5825;

struct Model {
    float mean[kNumFeatures];
    float stdv[kNumFeatures];
    std::vector<float> theta;
};

bool load_model(const char* path, Model& m) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char tag[64];
    int ver = 0;
    bool ok = fscanf(f, "%63s %d", tag, &ver) == 2 && strcmp(tag, "skel-cost-model") == 0 && ver == 1;
    for (int i = 0; ok && i < kNumFeatures; ++i) ok = fscanf(f, "%f", &m.mean[i]) == 1;
    for (int i = 0; ok && i < kNumFeatures; ++i) ok = fscanf(f, "%f", &m.stdv[i]) == 1;
    m.theta.assign(kNP, 0.0f);
    for (int i = 0; ok && i < kNP; ++i) ok = fscanf(f, "%f", &m.theta[i]) == 1;
    fclose(f);
    return ok;
}

bool save_model(const char* path, const Model& m) {
    FILE* f = fopen(path, "w");
    if (!f) return false;
    fprintf(f, "skel-cost-model 1\n");
    for (int i = 0; i < kNumFeatures; ++i) fprintf(f, "%.9g ", (double)m.mean[i]);
    fprintf(f, "\n");
    for (int i = 0; i < kNumFeatures; ++i) fprintf(f, "%.9g ", (double)m.stdv[i]);
    fprintf(f, "\n");
    for (int i = 0; i < kNP; ++i) fprintf(f, "%.9g\n", (double)m.theta[i]);
    fclose(f);
    return true;
}

// One database row: key, 6 config fields, 24 features, median us, min us.
bool parse_row(const std::string& line, std::vector<float>& feat, float& t_us) {
    if (line.empty() || line[0] == '#') return false;   // provenance comments
    std::vector<std::string> tok;
    std::stringstream ss(line);
    std::string x;
    while (std::getline(ss, x, ',')) tok.push_back(x);
    if ((int)tok.size() != 1 + 6 + kNumFeatures + 2) return false;
    feat.resize(kNumFeatures);
    for (int i = 0; i < kNumFeatures; ++i) feat[i] = strtof(tok[7 + i].c_str(), nullptr);
    t_us = strtof(tok[7 + kNumFeatures].c_str(), nullptr);
    return t_us > 0.0f;
}

void he_uniform(std::vector<float>& th, uint64_t seed) {
    std::mt19937_64 g(seed);
    th.assign(kNP, 0.0f);
    const int layers[3][3] = {{0, 64, 24}, {1600, 64, 64}, {5760, 1, 64}};
    for (const auto& L : layers) {
        const double lim = std::sqrt(6.0 / L[2]);
        std::uniform_real_distribution<double> u(-lim, lim);
        for (int i = 0; i < L[1] * L[2]; ++i) th[L[0] + i] = (float)u(g);
    }
}

}  // namespace

extern "C" int32_t skel_mlp_param_count(void) { return kNP; }

extern "C" skel_status skel_mlp_forward(const float* params, const float* X, int32_t n, float* y, void* stream) {
    clear_error();
    if (n < 0 || (n > 0 && (!params || !X || !y))) return set_error(SKEL_EINVAL, "bad MLP forward arguments");
    HIP_TRY(launch_mlp_forward(params, X, n, y, (hipStream_t)stream));
    return SKEL_OK;
}

extern "C" skel_status skel_mlp_grad(const float* params, const float* X, const float* t, int32_t n, float* grad,
                                     float* loss, void* stream) {
    clear_error();
    if (n <= 0 || !params || !X || !t || !grad) return set_error(SKEL_EINVAL, "bad MLP gradient arguments");
    const hipStream_t s = (hipStream_t)stream;
    float* work = nullptr;
    HIP_TRY(hipMallocAsync((void**)&work, sizeof(float) * mlp_grad_work_floats(n), s));
    hipError_t e = launch_mlp_grad(params, X, t, n, grad, loss, work, s);
    const hipError_t ef = hipFreeAsync(work, s);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return set_error(SKEL_EDEVICE, "MLP gradient: %s", hipGetErrorString(e));
    return SKEL_OK;
}

extern "C" skel_status skel_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                                     float beta1, float beta2, float eps, void* stream) {
    clear_error();
    if (!params || !grad || !m || !v || step < 1) return set_error(SKEL_EINVAL, "bad Adam arguments");
    HIP_TRY(launch_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return SKEL_OK;
}

extern "C" skel_status skel_cost_train(const char* db_path, const char* weights_out, int32_t epochs, uint64_t seed,
                                       const float* init, float* final_loss) {
    clear_error();
    if (!db_path || !weights_out || epochs < 0) return set_error(SKEL_EINVAL, "bad training arguments");
    FILE* f = fopen(db_path, "r");
    if (!f) return set_error(SKEL_EINVAL, "cannot open %s", db_path);
    std::vector<float> X, T;
    std::vector<float> feat;
    char* line = nullptr;
    size_t cap = 0;
    ssize_t len;
    while ((len = getline(&line, &cap, f)) > 0) {
        std::string sl(line, (size_t)len);
        while (!sl.empty() && (sl.back() == '\n' || sl.back() == '\r')) sl.pop_back();
        float t_us;
        if (!parse_row(sl, feat, t_us)) continue;
        X.insert(X.end(), feat.begin(), feat.end());
        T.push_back(std::log(t_us));
    }
    free(line);
    fclose(f);
    const int n = (int)T.size();
    if (n == 0) return set_error(SKEL_EINVAL, "no training rows in %s", db_path);
    Model m;
    for (int j = 0; j < kNumFeatures; ++j) {
        double s = 0, s2 = 0;
        for (int i = 0; i < n; ++i) s += X[(size_t)i * kNumFeatures + j];
        const double mu = s / n;
        for (int i = 0; i < n; ++i) {
            const double d = X[(size_t)i * kNumFeatures + j] - mu;
            s2 += d * d;
        }
        const double sd = std::sqrt(s2 / n);
        m.mean[j] = (float)mu;
        m.stdv[j] = sd > 1e-6 ? (float)sd : 1.0f;
        for (int i = 0; i < n; ++i)
            X[(size_t)i * kNumFeatures + j] = (float)((X[(size_t)i * kNumFeatures + j] - mu) / m.stdv[j]);
    }
    if (init)
        m.theta.assign(init, init + kNP);
    else
        he_uniform(m.theta, seed);
    const int B = 256;
    float *dX = nullptr, *dT = nullptr, *dP = nullptr, *dG = nullptr, *dM = nullptr, *dV = nullptr, *dW = nullptr,
          *dL = nullptr, *dY = nullptr;
    int* dI = nullptr;
    int* hI = nullptr;
    auto cleanup = [&]() {
        for (void* q : {(void*)dX, (void*)dT, (void*)dP, (void*)dG, (void*)dM, (void*)dV, (void*)dW, (void*)dL,
                        (void*)dY, (void*)dI})
            if (q) (void)hipFree(q);
        if (hI) (void)hipHostFree(hI);
    };
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) {
        if (e == hipSuccess && r != hipSuccess) e = r;
    };
    A(hipMalloc(&dX, sizeof(float) * X.size()));
    A(hipMalloc(&dT, sizeof(float) * n));
    A(hipMalloc(&dY, sizeof(float) * n));
    A(hipMalloc(&dP, sizeof(float) * kNP));
    A(hipMalloc(&dG, sizeof(float) * kNP));
    A(hipMalloc(&dM, sizeof(float) * kNP));
    A(hipMalloc(&dV, sizeof(float) * kNP));
    A(hipMalloc(&dL, sizeof(float)));
    A(hipMalloc(&dW, sizeof(float) * mlp_grad_work_floats(B)));
    A(hipMalloc(&dI, sizeof(int) * n));
    A(hipHostMalloc((void**)&hI, sizeof(int) * n, hipHostMallocDefault));
    if (e != hipSuccess) {
        cleanup();
        return set_error(SKEL_ENOMEM, "training buffers: %s", hipGetErrorString(e));
    }
    hipStream_t s;
    A(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    A(hipMemcpy(dX, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice));
    A(hipMemcpy(dT, T.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    A(hipMemcpy(dP, m.theta.data(), sizeof(float) * kNP, hipMemcpyHostToDevice));
    A(hipMemset(dM, 0, sizeof(float) * kNP));
    A(hipMemset(dV, 0, sizeof(float) * kNP));
    std::mt19937_64 g(seed ^ 0x9E3779B97F4A7C15ull);
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    int step = 0;
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        std::shuffle(perm.begin(), perm.end(), g);
        A(hipStreamSynchronize(s));   // previous epoch done with the index buffer
        memcpy(hI, perm.data(), sizeof(int) * n);
        A(hipMemcpyAsync(dI, hI, sizeof(int) * n, hipMemcpyHostToDevice, s));
        for (int off = 0; off < n && e == hipSuccess; off += B) {
            const int bs = std::min(B, n - off);
            A(launch_mlp_grad_idx(dP, dX, dT, dI + off, bs, dG, dL, dW, s));
            A(launch_mlp_adam(dP, dG, dM, dV, ++step, 1e-3f, 0.9f, 0.999f, 1e-8f, s));
        }
    }
    A(launch_mlp_forward(dP, dX, n, dY, s));
    std::vector<float> Y(n);
    A(hipStreamSynchronize(s));
    A(hipMemcpy(Y.data(), dY, sizeof(float) * n, hipMemcpyDeviceToHost));
    A(hipMemcpy(m.theta.data(), dP, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    (void)hipStreamDestroy(s);
    cleanup();
    if (e != hipSuccess) return set_error(SKEL_EDEVICE, "training: %s", hipGetErrorString(e));
    double L = 0;
    for (int i = 0; i < n; ++i) L += (double)(Y[i] - T[i]) * (Y[i] - T[i]);
    if (final_loss) *final_loss = (float)(L / n);
    if (!save_model(weights_out, m)) return set_error(SKEL_EINVAL, "cannot write %s", weights_out);
    return SKEL_OK;
}

namespace {

// Every valid configuration of the composition with its predicted run time
// (log microseconds), from one forward pass of the model over all of them.
// `weights` may name several models separated by ';' (an ensemble, e.g. the
// same data trained from different initialisations): the prediction is the
// mean of their log-time predictions.
skel_status predict_all(skel_node root, const skel_buffer* proto, int32_t nargs, const char* weights,
                        std::vector<Config>& cands, std::vector<float>& Y) {
    std::vector<std::string> paths;
    {
        std::string w(weights);
        size_t a = 0;
        while (a <= w.size()) {
            const size_t b = w.find(';', a);
            const std::string one = w.substr(a, b == std::string::npos ? std::string::npos : b - a);
            if (!one.empty()) paths.push_back(one);
            if (b == std::string::npos) break;
            a = b + 1;
        }
    }
    if (paths.empty()) return set_error(SKEL_EINVAL, "no cost model named");
    Linear L;
    Shape sh;
    skel_status st = linearize(root, L);
    if (!st && L.dom == DOM_NONE) L.dom = (nargs > 0 && proto[0].dtype == SKEL_U8) ? DOM_U8 : DOM_F32;
    if (!st) st = derive_shape(L, proto, nargs, sh);
    if (st) return st;
    cands = enumerate_configs(L, sh);
    if (cands.empty()) return set_error(SKEL_EUNSUPPORTED, "no valid configuration");
    const int n = (int)cands.size();
    std::vector<float> F((size_t)n * kNumFeatures);
    for (int i = 0; i < n; ++i) features(L, sh, cands[i], &F[(size_t)i * kNumFeatures]);
    Y.assign(n, 0.0f);
    std::vector<float> X(F.size()), Yk(n);
    for (const std::string& path : paths) {
        Model m;
        if (!load_model(path.c_str(), m)) return set_error(SKEL_EINVAL, "cannot read cost model %s", path.c_str());
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < kNumFeatures; ++j)
                X[(size_t)i * kNumFeatures + j] = (F[(size_t)i * kNumFeatures + j] - m.mean[j]) / m.stdv[j];
        float *dP = nullptr, *dX = nullptr, *dY = nullptr;
        hipError_t e = hipMalloc(&dP, sizeof(float) * kNP);
        if (!e) e = hipMalloc(&dX, sizeof(float) * X.size());
        if (!e) e = hipMalloc(&dY, sizeof(float) * n);
        if (!e) e = hipMemcpy(dP, m.theta.data(), sizeof(float) * kNP, hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(dX, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice);
        if (!e) e = launch_mlp_forward(dP, dX, n, dY, nullptr);
        if (!e) e = hipMemcpy(Yk.data(), dY, sizeof(float) * n, hipMemcpyDeviceToHost);
        for (void* q : {(void*)dP, (void*)dX, (void*)dY})
            if (q) (void)hipFree(q);
        if (e != hipSuccess) return set_error(SKEL_EDEVICE, "cost model inference: %s", hipGetErrorString(e));
        for (int i = 0; i < n; ++i) Y[i] += Yk[i] / (float)paths.size();
    }
    return SKEL_OK;
}

}  // namespace

extern "C" skel_status skel_cost_select(skel_node root, const skel_buffer* proto, int32_t nargs, const char* weights,
                                        skel_plan_opts* chosen) {
    clear_error();
    if (!root || !weights || !chosen) return set_error(SKEL_EINVAL, "null argument");
    std::vector<Config> cands;
    std::vector<float> Y;
    skel_status st = predict_all(root, proto, nargs, weights, cands, Y);
    if (st) return st;
    int best = 0;
    for (int i = 1; i < (int)Y.size(); ++i)
        if (Y[i] < Y[best]) best = i;
    config_to_opts(cands[best], chosen);
    return SKEL_OK;
}

extern "C" skel_status skel_cost_rank(skel_node root, const skel_buffer* proto, int32_t nargs, const char* weights,
                                      int32_t k, skel_plan_opts* ranked, float* pred_us, int32_t* count) {
    clear_error();
    if (!root || !weights || !ranked || !count || k < 1) return set_error(SKEL_EINVAL, "null argument or k < 1");
    *count = 0;
    std::vector<Config> cands;
    std::vector<float> Y;
    skel_status st = predict_all(root, proto, nargs, weights, cands, Y);
    if (st) return st;
    std::vector<int> idx(Y.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    // ties keep enumeration order, so the first entry is skel_cost_select's choice
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return Y[a] < Y[b]; });
    const int n = std::min<int>(k, (int)idx.size());
    for (int i = 0; i < n; ++i) {
        config_to_opts(cands[idx[i]], &ranked[i]);
        if (pred_us) pred_us[i] = std::exp(Y[idx[i]]);
    }
    *count = n;
    return SKEL_OK;
}
