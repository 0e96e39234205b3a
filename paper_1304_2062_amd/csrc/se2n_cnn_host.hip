// Host runtime of the learned corrector: the network object (FP32 master
// parameters, Adam state, bfloat16 MFMA weights), workspace layout, the
// forward / gradient / Adam / training calls and the corrected inpainting
// path, behind the C ABI of include/se2n.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/se2n.h"
#include "se2n_cnn.hpp"
#include "se2n_host.hpp"

using namespace se2n;

struct se2n_cnn_s {
    int N = 0;
    int device = 0;
    bool alive = true;
    float* params = nullptr;  // [kCnnP]
    float* m = nullptr;
    float* v = nullptr;
    float* grads = nullptr;   // gradient of the last se2n_cnn_train_step
    float* loss = nullptr;    // one float
    bf16* wf = nullptr;       // [3][9][32][32]
    bf16* wd = nullptr;
    int t = 0;                // Adam steps taken
    // measured accuracy of the network per regime (se2n_cnn_set_validation)
    struct Validation {
        int M, n_coarse, n_fine, scheme;
        double T, beta, rel_l2;
    };
    std::vector<Validation> validated;
    // kernel timing
    bool prof_on = false;
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::map<std::string, std::pair<int, double>> acc;
};

namespace {

constexpr int kTilesPerWg = 4;

int check_cnn(se2n_cnn c) {
    if (!c) return fail(SE2N_EINVAL, "network is NULL");
    if (!c->alive) return fail(SE2N_ESTATE, "network was destroyed");
    return SE2N_OK;
}

int check_shape(se2n_cnn c, int M, int B) {
    if (M < 16 || M > 8192 || M % 16) return fail(SE2N_EINVAL, "M must be a multiple of 16 in [16, 8192] (got %d)", M);
    if (B < 1 || (long)B * M * M > (1L << 31)) return fail(SE2N_EINVAL, "batch must be >= 1 with batch*M*M <= 2^31");
    (void)c;
    return SE2N_OK;
}

struct CnnWs {
    bf16 *a0, *a1, *a2, *g0, *g1;
    float *scale, *sparts;
    float *out, *parts, *slices, *lparts;
    size_t bytes;
};

CnnWs layout(const se2n_cnn c, int M, int B, bool training, char* base) {
    CnnWs w{};
    size_t off = 0;
    const size_t act = align256((size_t)B * M * M * kCnnC * sizeof(bf16));
    auto take = [&](size_t n) {
        char* p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    };
    w.scale = (float*)take((size_t)B * sizeof(float));
    w.sparts = (float*)take((size_t)B * kCnnScaleBlocks * sizeof(float));
    w.a0 = (bf16*)take(act);
    w.a1 = (bf16*)take(act);
    if (training) {
        w.a2 = (bf16*)take(act);
        w.g0 = (bf16*)take(act);
        w.g1 = (bf16*)take(act);
        w.out = (float*)take((size_t)B * c->N * M * M * sizeof(float));
        w.parts = (float*)take((size_t)cnn_wgrad_parts(M, B, kTilesPerWg) * kCnnPart * sizeof(float));
        w.slices = (float*)take((size_t)kCnnSlices * kCnnPart * sizeof(float));
        w.lparts = (float*)take((size_t)cnn_loss_blocks(c->N, M, B) * sizeof(float));
    } else {
        w.a2 = w.a0;  // the input is dead once layer 1 has run
    }
    w.bytes = off;
    return w;
}

struct Timed {
    se2n_cnn c;
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(se2n_cnn c_, const char* n, hipStream_t s) : c(c_), name(n), st(s) {
        if (c->prof_on && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, st);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess) {
            (void)hipEventRecord(b, st);
            c->pending.push_back({name, a, b});
        } else {
            (void)hipEventDestroy(a);
        }
    }
};

#define CNN_TIMED(c, name, st, call, what) \
    do {                                   \
        Timed t_(c, name, st);             \
        SE2N_HIP(call, what);              \
    } while (0)

int refresh_weights(se2n_cnn c, hipStream_t st) {
    CNN_TIMED(c, "cnn_prep", st, cnn_prep(c->params, c->wf, c->wd, st), "corrector weight preparation");
    return SE2N_OK;
}

// psi_out = psi + net(psi); `w` from layout(..., training)
int forward_impl(se2n_cnn c, const float* psi, float* out, int M, int B, const CnnWs& w, hipStream_t st) {
    const int N = c->N;
    CNN_TIMED(c, "cnn_rms", st, cnn_rms(psi, w.sparts, w.scale, N, M, B, st), "corrector input scale");
    CNN_TIMED(c, "cnn_pack", st, cnn_pack(psi, w.scale, w.a0, N, M, B, st), "corrector input packing");
    CNN_TIMED(c, "cnn_conv1", st,
              cnn_conv(CNN_HIDDEN, w.a0, c->wf, c->params + kCnnW, w.a1, nullptr, nullptr, nullptr, nullptr, N, M, B,
                       st),
              "corrector layer 1");
    CNN_TIMED(c, "cnn_conv2", st,
              cnn_conv(CNN_HIDDEN, w.a1, c->wf + kCnnW, c->params + kCnnL + kCnnW, w.a2, nullptr, nullptr, nullptr,
                       nullptr, N, M, B, st),
              "corrector layer 2");
    CNN_TIMED(c, "cnn_conv3", st,
              cnn_conv(CNN_LAST, w.a2, c->wf + 2 * kCnnW, c->params + 2 * kCnnL + kCnnW, nullptr, nullptr, psi, out,
                       w.scale, N, M, B, st),
              "corrector layer 3");
    return SE2N_OK;
}

int layer_wgrad(se2n_cnn c, const bf16* g, const bf16* a, float* grad_layer, int M, int B, const CnnWs& w,
                hipStream_t st) {
    const int nparts = cnn_wgrad_parts(M, B, kTilesPerWg);
    CNN_TIMED(c, "cnn_wgrad", st, cnn_wgrad(g, a, w.parts, M, B, kTilesPerWg, st), "corrector weight gradient");
    CNN_TIMED(c, "cnn_wgrad_reduce", st, cnn_wgrad_reduce(w.parts, nparts, w.slices, grad_layer, st),
              "corrector gradient reduction");
    return SE2N_OK;
}

int gradients_impl(se2n_cnn c, const float* coarse, const float* fine, int M, int B, float* grads, float* loss,
                   const CnnWs& w, hipStream_t st) {
    int rc = forward_impl(c, coarse, w.out, M, B, w, st);
    if (rc) return rc;
    const int N = c->N;
    const double numel = (double)B * N * M * M;
    const int nl = cnn_loss_blocks(N, M, B);
    CNN_TIMED(c, "cnn_loss", st,
              cnn_loss(w.out, fine, w.scale, w.g0, w.lparts, N, M, B, (float)(2.0 / numel), st), "corrector loss");
    if (loss) {
        CNN_TIMED(c, "cnn_loss_reduce", st, cnn_loss_reduce(w.lparts, nl, (float)(1.0 / numel), loss, st),
                  "corrector loss reduction");
    }
    // layer 3: g0 = dloss/dr
    rc = layer_wgrad(c, w.g0, w.a2, grads + 2 * kCnnL, M, B, w, st);
    if (rc) return rc;
    CNN_TIMED(c, "cnn_dgrad", st,
              cnn_conv(CNN_DGRAD, w.g0, c->wd + 2 * kCnnW, nullptr, w.g1, w.a2, nullptr, nullptr, nullptr, N, M, B,
                       st),
              "corrector input gradient (layer 3)");
    // layer 2: g1 = dloss/dz2
    rc = layer_wgrad(c, w.g1, w.a1, grads + kCnnL, M, B, w, st);
    if (rc) return rc;
    CNN_TIMED(c, "cnn_dgrad", st,
              cnn_conv(CNN_DGRAD, w.g1, c->wd + kCnnW, nullptr, w.g0, w.a1, nullptr, nullptr, nullptr, N, M, B, st),
              "corrector input gradient (layer 2)");
    // layer 1: g0 = dloss/dz1
    return layer_wgrad(c, w.g0, w.a0, grads, M, B, w, st);
}

int adam_impl(se2n_cnn c, const float* grads, float lr, float b1, float b2, float eps, hipStream_t st) {
    if (!(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
        return fail(SE2N_EINVAL, "Adam needs lr >= 0, 0 <= beta1, beta2 < 1 and eps > 0");
    c->t += 1;
    CNN_TIMED(c, "cnn_adam", st, cnn_adam(c->params, grads, c->m, c->v, c->t, lr, b1, b2, eps, st), "Adam step");
    return refresh_weights(c, st);
}

// Seeded He-normal initial weights (splitmix64 + Box-Muller): layers 1, 2;
// layer 3 and every bias zero, so the network starts as the identity map.
std::vector<float> initial_params(int N, uint64_t seed) {
    std::vector<float> p(kCnnP, 0.0f);
    uint64_t s = seed ^ 0x9E3779B97F4A7C15ull;
    auto next = [&]() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    auto normal = [&]() {
        const double u1 = unif(), u2 = unif();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    for (int l = 0; l < 2; ++l) {
        const int cin = l == 0 ? N : kCnnC;
        const double sd = std::sqrt(2.0 / (9.0 * cin));
        for (int o = 0; o < kCnnC; ++o)
            for (int ci = 0; ci < cin; ++ci)
                for (int tap = 0; tap < 9; ++tap) p[(size_t)l * kCnnL + (o * kCnnC + ci) * 9 + tap] = (float)(sd * normal());
    }
    return p;
}

// Zero the parameters of the padded channels (layer 1 inputs, layer 3 outputs >= N).
void mask_padded(std::vector<float>& p, int N) {
    for (int o = 0; o < kCnnC; ++o)
        for (int ci = N; ci < kCnnC; ++ci)
            for (int tap = 0; tap < 9; ++tap) p[(o * kCnnC + ci) * 9 + tap] = 0.0f;
    for (int o = N; o < kCnnC; ++o) {
        for (int ci = 0; ci < kCnnC; ++ci)
            for (int tap = 0; tap < 9; ++tap) p[2 * kCnnL + (o * kCnnC + ci) * 9 + tap] = 0.0f;
        p[2 * kCnnL + kCnnW + o] = 0.0f;
    }
}

int upload_params(se2n_cnn c, std::vector<float>& p) {
    mask_padded(p, c->N);
    SE2N_HIP(hipMemcpy(c->params, p.data(), kCnnP * sizeof(float), hipMemcpyHostToDevice), "parameter upload");
    SE2N_HIP(hipMemset(c->m, 0, kCnnP * sizeof(float)), "Adam state reset");
    SE2N_HIP(hipMemset(c->v, 0, kCnnP * sizeof(float)), "Adam state reset");
    c->t = 0;
    int rc = refresh_weights(c, nullptr);
    if (rc) return rc;
    SE2N_HIP(hipDeviceSynchronize(), "parameter upload");
    return SE2N_OK;
}

void free_cnn(se2n_cnn c) {
    for (void* p : {(void*)c->params, (void*)c->m, (void*)c->v, (void*)c->grads, (void*)c->loss, (void*)c->wf,
                    (void*)c->wd})
        if (p) (void)hipFree(p);
    for (auto& r : c->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
}

}  // namespace

extern "C" {

int se2n_cnn_create(se2n_cnn* out, int N, uint64_t seed) {
    clear_error();
    if (!out) return fail(SE2N_EINVAL, "out is NULL");
    if (N < 1 || N > kCnnC) return fail(SE2N_EINVAL, "the corrector takes 1 <= N <= %d orientations (got %d)", kCnnC, N);
    se2n_cnn c = new (std::nothrow) se2n_cnn_s;
    if (!c) return fail(SE2N_ENOMEM, "host allocation of the network failed");
    c->N = N;
    (void)hipGetDevice(&c->device);
    hipError_t e = hipSuccess;
    for (float** p : {&c->params, &c->m, &c->v, &c->grads})
        if (e == hipSuccess) e = dev_malloc((void**)p, kCnnP * sizeof(float));
    if (e == hipSuccess) e = dev_malloc((void**)&c->loss, 256);
    if (e == hipSuccess) e = dev_malloc((void**)&c->wf, 3 * kCnnW * sizeof(bf16));
    if (e == hipSuccess) e = dev_malloc((void**)&c->wd, 3 * kCnnW * sizeof(bf16));
    if (e != hipSuccess) {
        free_cnn(c);
        delete c;
        return fail(SE2N_ENOMEM, "hipMalloc of the network's buffers failed: %s", hipGetErrorString(e));
    }
    std::vector<float> p = initial_params(N, seed);
    const int rc = upload_params(c, p);
    if (rc) {
        free_cnn(c);
        delete c;
        return rc;
    }
    *out = c;
    return SE2N_OK;
}

int se2n_cnn_destroy(se2n_cnn c) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    (void)hipDeviceSynchronize();
    free_cnn(c);
    c->alive = false;
    delete c;
    return SE2N_OK;
}

int se2n_cnn_get_params(se2n_cnn c, float* host, int capacity, int* count) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!count) return fail(SE2N_EINVAL, "count is NULL");
    *count = kCnnP;
    if (!host) return SE2N_OK;
    if (capacity < kCnnP) return fail(SE2N_EINVAL, "capacity %d < %d parameters", capacity, kCnnP);
    SE2N_HIP(hipDeviceSynchronize(), "synchronise before reading parameters");
    SE2N_HIP(hipMemcpy(host, c->params, kCnnP * sizeof(float), hipMemcpyDeviceToHost), "parameter download");
    return SE2N_OK;
}

int se2n_cnn_set_params(se2n_cnn c, const float* host, int count) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!host) return fail(SE2N_EINVAL, "host is NULL");
    if (count != kCnnP) return fail(SE2N_EINVAL, "expected %d parameters (got %d)", kCnnP, count);
    std::vector<float> p(host, host + kCnnP);
    for (float x : p)
        if (!std::isfinite(x)) return fail(SE2N_EINVAL, "parameters must be finite");
    SE2N_HIP(hipDeviceSynchronize(), "synchronise before writing parameters");
    return upload_params(c, p);
}

int se2n_cnn_get_adam(se2n_cnn c, float* m, float* v, int capacity, int* step) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!step) return fail(SE2N_EINVAL, "step is NULL");
    *step = c->t;
    if (!m && !v) return SE2N_OK;
    if (!m || !v) return fail(SE2N_EINVAL, "m and v must both be given");
    if (capacity < kCnnP) return fail(SE2N_EINVAL, "capacity %d < %d parameters", capacity, kCnnP);
    SE2N_HIP(hipDeviceSynchronize(), "synchronise before reading the Adam state");
    SE2N_HIP(hipMemcpy(m, c->m, kCnnP * sizeof(float), hipMemcpyDeviceToHost), "Adam first moment download");
    SE2N_HIP(hipMemcpy(v, c->v, kCnnP * sizeof(float), hipMemcpyDeviceToHost), "Adam second moment download");
    return SE2N_OK;
}

int se2n_cnn_set_adam(se2n_cnn c, const float* m, const float* v, int count, int step) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!m || !v) return fail(SE2N_EINVAL, "m and v must be non-NULL");
    if (count != kCnnP) return fail(SE2N_EINVAL, "expected %d values (got %d)", kCnnP, count);
    if (step < 0) return fail(SE2N_EINVAL, "step must be >= 0 (got %d)", step);
    for (int i = 0; i < kCnnP; ++i)
        if (!std::isfinite(m[i]) || !std::isfinite(v[i]) || v[i] < 0.f)
            return fail(SE2N_EINVAL, "Adam moments must be finite, v >= 0");
    SE2N_HIP(hipDeviceSynchronize(), "synchronise before writing the Adam state");
    SE2N_HIP(hipMemcpy(c->m, m, kCnnP * sizeof(float), hipMemcpyHostToDevice), "Adam first moment upload");
    SE2N_HIP(hipMemcpy(c->v, v, kCnnP * sizeof(float), hipMemcpyHostToDevice), "Adam second moment upload");
    c->t = step;
    return SE2N_OK;
}

size_t se2n_cnn_workspace_bytes(se2n_cnn c, int M, int batch, int training) {
    clear_error();
    if (check_cnn(c) || check_shape(c, M, batch)) return 0;
    return layout(c, M, batch, training != 0, nullptr).bytes;
}

int se2n_cnn_forward(se2n_cnn c, const float* psi, float* out, int M, int batch, void* workspace, void* stream) {
    clear_error();
    int rc = check_cnn(c);
    if (!rc) rc = check_shape(c, M, batch);
    if (rc) return rc;
    if (!psi || !out || !workspace) return fail(SE2N_EINVAL, "psi, out and workspace must be non-NULL");
    const CnnWs w = layout(c, M, batch, false, (char*)workspace);
    return forward_impl(c, psi, out, M, batch, w, (hipStream_t)stream);
}

int se2n_cnn_gradients(se2n_cnn c, const float* coarse, const float* fine, int M, int batch, float* grads,
                       float* loss, void* workspace, void* stream) {
    clear_error();
    int rc = check_cnn(c);
    if (!rc) rc = check_shape(c, M, batch);
    if (rc) return rc;
    if (!coarse || !fine || !grads || !workspace)
        return fail(SE2N_EINVAL, "coarse, fine, grads and workspace must be non-NULL");
    const CnnWs w = layout(c, M, batch, true, (char*)workspace);
    return gradients_impl(c, coarse, fine, M, batch, grads, loss, w, (hipStream_t)stream);
}

int se2n_cnn_adam_step(se2n_cnn c, const float* grads, float lr, float beta1, float beta2, float eps, void* stream) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!grads) return fail(SE2N_EINVAL, "grads is NULL");
    return adam_impl(c, grads, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int se2n_cnn_train_step(se2n_cnn c, const float* coarse, const float* fine, int M, int batch, float lr, float* loss,
                        void* workspace, void* stream) {
    clear_error();
    int rc = check_cnn(c);
    if (!rc) rc = check_shape(c, M, batch);
    if (rc) return rc;
    if (!coarse || !fine || !workspace) return fail(SE2N_EINVAL, "coarse, fine and workspace must be non-NULL");
    const CnnWs w = layout(c, M, batch, true, (char*)workspace);
    rc = gradients_impl(c, coarse, fine, M, batch, c->grads, loss ? loss : c->loss, w, (hipStream_t)stream);
    if (rc) return rc;
    return adam_impl(c, c->grads, lr, 0.9f, 0.999f, 1e-8f, (hipStream_t)stream);
}

int se2n_cnn_profile(se2n_cnn c, int enable) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    for (auto& r : c->pending) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    c->pending.clear();
    c->acc.clear();
    c->prof_on = enable != 0;
    return SE2N_OK;
}

int se2n_cnn_profile_stats(se2n_cnn c, se2n_kernel_stat* out, int capacity, int* count) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!count) return fail(SE2N_EINVAL, "count is NULL");
    for (auto& r : c->pending) {
        SE2N_HIP(hipEventSynchronize(r.b), "wait for timing events");
        float ms = 0.f;
        SE2N_HIP(hipEventElapsedTime(&ms, r.a, r.b), "event elapsed time");
        auto& a = c->acc[r.name];
        a.first += 1;
        a.second += ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    c->pending.clear();
    *count = (int)c->acc.size();
    if (out) {
        int k = 0;
        for (const auto& kv : c->acc) {
            if (k >= capacity) break;
            std::memset(&out[k], 0, sizeof out[k]);
            snprintf(out[k].name, sizeof out[k].name, "%s", kv.first.c_str());
            out[k].launches = kv.second.first;
            out[k].total_ms = kv.second.second;
            ++k;
        }
    }
    return SE2N_OK;
}

size_t se2n_corrected_workspace_bytes(se2n_plan plan, se2n_cnn c) {
    clear_error();
    if (!plan || check_cnn(c)) return 0;
    const size_t pw = se2n_workspace_bytes(plan);
    if (pw == 0) return 0;
    int M = 0, N = 0;
    se2n_dtype dt = SE2N_F32;
    if (se2n_plan_info(plan, &M, &N, &dt) || dt != SE2N_F32 || N != c->N || M % 16) return 0;
    return align256(pw) + align256((size_t)N * M * M * sizeof(float)) + se2n_cnn_workspace_bytes(c, M, 1, 0);
}

int se2n_cnn_set_validation(se2n_cnn c, int M, double T, double beta, int n_coarse, int n_fine, se2n_scheme scheme,
                            double rel_l2) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (M < 16 || n_coarse < 1 || n_fine < 1 || !(T >= 0.0) || !(beta >= 0.0) || !std::isfinite(T) ||
        !std::isfinite(beta) || (scheme != SE2N_CN && scheme != SE2N_EXACT) || !(rel_l2 >= 0.0))
        return fail(SE2N_EINVAL, "bad validation record");
    for (auto& v : c->validated) {
        if (v.M == M && v.T == T && v.beta == beta && v.n_coarse == n_coarse && v.n_fine == n_fine &&
            v.scheme == (int)scheme) {
            v.rel_l2 = rel_l2;
            return SE2N_OK;
        }
    }
    c->validated.push_back({M, n_coarse, n_fine, (int)scheme, T, beta, rel_l2});
    return SE2N_OK;
}

int se2n_cnn_get_validation(se2n_cnn c, int M, double T, double beta, int n_coarse, int n_fine, se2n_scheme scheme,
                            double* rel_l2) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    if (!rel_l2) return fail(SE2N_EINVAL, "rel_l2 is NULL");
    *rel_l2 = -1.0;
    for (const auto& v : c->validated)
        if (v.M == M && v.T == T && v.beta == beta && v.n_coarse == n_coarse && v.n_fine == n_fine &&
            v.scheme == (int)scheme)
            *rel_l2 = v.rel_l2;
    return SE2N_OK;
}

int se2n_inpaint_corrected(se2n_plan plan, se2n_cnn c, const void* f, const uint8_t* mask, double sigma, double T,
                           double beta, int n_steps, int n_fine, se2n_scheme scheme, se2n_proj mode,
                           double max_rel_l2, uint8_t* rmap_out, void* out, int* used_fallback, void* workspace,
                           void* stream) {
    clear_error();
    int rc = check_cnn(c);
    if (rc) return rc;
    int M = 0, N = 0;
    se2n_dtype dt = SE2N_F32;
    rc = se2n_plan_info(plan, &M, &N, &dt);
    if (rc) return rc;
    if (dt != SE2N_F32) return fail(SE2N_EUNSUPPORTED, "the corrected path runs in FP32 plans only");
    if (N != c->N) return fail(SE2N_EINVAL, "plan N (%d) differs from the network's N (%d)", N, c->N);
    if (M % 16) return fail(SE2N_EUNSUPPORTED, "the corrector needs M divisible by 16 (got %d)", M);
    if (!f || !mask || !rmap_out || !out || !workspace)
        return fail(SE2N_EINVAL, "f, mask, rmap_out, out and workspace must be non-NULL");
    if (n_fine < 1 || n_fine < n_steps) return fail(SE2N_EINVAL, "n_fine (%d) must be >= n_steps (%d) >= 1", n_fine, n_steps);
    if (!(max_rel_l2 >= 0.0)) return fail(SE2N_EINVAL, "max_rel_l2 must be >= 0 (got %g)", max_rel_l2);
    char* base = (char*)workspace;
    // The network is applied only in a regime where its error against the
    // fine-step solve was measured to be within the bar; everywhere else the
    // fine-step plain solve runs instead.
    double measured = -1.0;
    rc = se2n_cnn_get_validation(c, M, T, beta, n_steps, n_fine, scheme, &measured);
    if (rc) return rc;
    const bool trusted = measured >= 0.0 && measured <= max_rel_l2;
    if (used_fallback) *used_fallback = trusted ? 0 : 1;
    if (!trusted)
        return se2n_inpaint(plan, f, mask, sigma, T, beta, n_fine, scheme, mode, nullptr, rmap_out, out, base, stream);
    void* pws = base;
    float* psi = (float*)(base + align256(se2n_workspace_bytes(plan)));
    char* cws = (char*)psi + align256((size_t)N * M * M * sizeof(float));
    hipStream_t st = (hipStream_t)stream;
    rc = se2n_orient(plan, f, mask, sigma, rmap_out, pws, stream);
    if (!rc) rc = se2n_lift(plan, f, mask, rmap_out, psi, stream);
    if (!rc) rc = se2n_diffuse(plan, psi, T, beta, n_steps, scheme, pws, stream);
    if (rc) return rc;
    const CnnWs w = layout(c, M, 1, false, cws);
    rc = forward_impl(c, psi, psi, M, 1, w, st);
    if (rc) return rc;
    return se2n_project(plan, psi, mode, out, stream);
}

}  // extern "C"
