// lbs_api.hip - the surrogate's C ABI (include/lbell.h): arena layout,
// parameters, training, prediction and gradients.  Host code only; every
// arithmetic step runs in the kernels of k_mlp.hip.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "lbell.h"
#include "lbs_internal.h"

using namespace lbd;

namespace lbd {
LbsLayout lbs_layout(int max_n) {
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t tiles = (size_t)(max_n + 15) / 16;
    LbsLayout L{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = up(p + bytes);
        return at;
    };
    L.P = take(sizeof(float) * MLP_NP);
    L.M = take(sizeof(float) * MLP_NP);
    L.V = take(sizeof(float) * MLP_NP);
    L.G = take(sizeof(float) * MLP_NP * tiles);
    L.Lpart = take(sizeof(float) * tiles);
    L.gsum = take(sizeof(float) * MLP_NP);
    L.X = take(sizeof(float) * MLP_IN * (size_t)max_n);
    L.Y = take(sizeof(float) * MLP_OUT * (size_t)max_n);
    L.out = take(sizeof(float) * MLP_OUT * (size_t)max_n);
    L.loss = take(sizeof(double));
    L.total = p;
    return L;
}
}  // namespace lbd

namespace {
lb_status hipc(lbs* s, hipError_t e, const char* what) {
    if (e == hipSuccess) return LB_OK;
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    return LB_EDEVICE;
}
#define HC(expr)                                          \
    do {                                                  \
        lb_status _s = hipc(s, (expr), #expr);            \
        if (_s != LB_OK) return _s;                       \
    } while (0)

// Scratch of lbs_grad_noalloc: the per-tile partial gradients and squared
// errors of up to LBS_NOALLOC_MAX_SAMPLES samples (16 samples per tile),
// 5.3 MB, one copy on every device the library runs on, held until the
// process ends.  Its address is taken once per device with that device
// current; host code uses that address only, never the array's name.
constexpr int NOALLOC_TILES = (LBS_NOALLOC_MAX_SAMPLES + 15) / 16;
static __device__ __align__(256) float scratch[(size_t)NOALLOC_TILES * MLP_NP + NOALLOC_TILES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

lb_status noalloc_scratch(float** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LB_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LB_EDEVICE;
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}

lb_status upload(lbs* s, const float* X, const float* Y, int n) {
    HC(hipMemcpyAsync(s->X, X, sizeof(float) * MLP_IN * (size_t)n, hipMemcpyHostToDevice, s->stream));
    if (Y) HC(hipMemcpyAsync(s->Y, Y, sizeof(float) * MLP_OUT * (size_t)n, hipMemcpyHostToDevice, s->stream));
    return LB_OK;
}
}  // namespace

extern "C" {

size_t lbs_arena_bytes(int max_samples) {
    if (max_samples < 1) return 0;
    return lbs_layout(max_samples).total;
}

lb_status lbs_create(int max_samples, void* dev_arena, size_t bytes, void* hip_stream, lbs** out) {
    if (!out) return LB_EINVAL;
    *out = nullptr;
    if (max_samples < 1 || !dev_arena || ((uintptr_t)dev_arena % 256) != 0) return LB_EINVAL;
    const LbsLayout L = lbs_layout(max_samples);
    if (bytes < L.total) return LB_ENOMEM;
    lbs* s = new lbs();
    s->stream = (hipStream_t)hip_stream;
    s->arena = (char*)dev_arena;
    s->max_n = max_samples;
    s->max_tiles = (max_samples + 15) / 16;
    s->P = (float*)(s->arena + L.P);
    s->M = (float*)(s->arena + L.M);
    s->V = (float*)(s->arena + L.V);
    s->G = (float*)(s->arena + L.G);
    s->Lpart = (float*)(s->arena + L.Lpart);
    s->gsum = (float*)(s->arena + L.gsum);
    s->X = (float*)(s->arena + L.X);
    s->Y = (float*)(s->arena + L.Y);
    s->out = (float*)(s->arena + L.out);
    s->loss_acc = (double*)(s->arena + L.loss);
    hipError_t e = hipMemsetAsync(s->arena, 0, L.gsum, s->stream);  // P, M, V (and the partials) start at 0
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        delete s;
        return LB_EDEVICE;
    }
    *out = s;
    return LB_OK;
}

lb_status lbs_set_params(lbs* s, const float* params) {
    if (!s || !params) return LB_EINVAL;
    HC(hipMemcpyAsync(s->P, params, sizeof(float) * MLP_NP, hipMemcpyHostToDevice, s->stream));
    HC(hipMemsetAsync(s->M, 0, sizeof(float) * MLP_NP, s->stream));
    HC(hipMemsetAsync(s->V, 0, sizeof(float) * MLP_NP, s->stream));
    HC(hipStreamSynchronize(s->stream));
    s->adam_t = 0;
    return LB_OK;
}

lb_status lbs_get_params(lbs* s, float* params) {
    if (!s || !params) return LB_EINVAL;
    HC(hipMemcpyAsync(params, s->P, sizeof(float) * MLP_NP, hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    return LB_OK;
}

lb_status lbs_train(lbs* s, const float* X, const float* Y, int n, int epochs, int batch, float lr,
                    float* loss) {
    if (!s || !X || !Y || n < 1 || n > s->max_n || epochs < 1 || batch < 1 || !(lr > 0)) return LB_EINVAL;
    lb_status st = upload(s, X, Y, n);
    if (st != LB_OK) return st;
    for (int e = 0; e < epochs; ++e) {
        HC(hipMemsetAsync(s->loss_acc, 0, sizeof(double), s->stream));
        for (int b0 = 0; b0 < n; b0 += batch) {
            const int nb = std::min(batch, n - b0);
            MlpArgs a{s->P, s->X + (size_t)b0 * MLP_IN, s->Y + (size_t)b0 * MLP_OUT, nullptr, s->G, s->Lpart, nb,
                      (float)(2.0 / (6.0 * nb)), 1};
            HC(launch_mlp(a, s->stream));
            s->adam_t++;
            MlpReduceArgs r{};
            r.G = s->G;
            r.Lpart = s->Lpart;
            r.ntiles = (nb + 15) / 16;
            r.P = s->P;
            r.M = s->M;
            r.V = s->V;
            r.lr = lr;
            r.c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)s->adam_t)));
            r.c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)s->adam_t)));
            r.loss_acc = s->loss_acc;
            r.mode = 0;
            HC(launch_mlp_reduce(r, s->stream));
        }
    }
    double acc = 0;
    HC(hipMemcpyAsync(&acc, s->loss_acc, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    if (loss) *loss = (float)(acc / (6.0 * n));
    return LB_OK;
}

lb_status lbs_predict(lbs* s, const float* X, int n, float* Y) {
    if (!s || !X || !Y || n < 1 || n > s->max_n) return LB_EINVAL;
    lb_status st = upload(s, X, nullptr, n);
    if (st != LB_OK) return st;
    MlpArgs a{s->P, s->X, nullptr, s->out, nullptr, nullptr, n, 0.f, 0};
    HC(launch_mlp(a, s->stream));
    HC(hipMemcpyAsync(Y, s->out, sizeof(float) * MLP_OUT * (size_t)n, hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    return LB_OK;
}

lb_status lbs_grad(lbs* s, const float* X, const float* Y, int n, float* grads, float* loss) {
    if (!s || !X || !Y || n < 1 || n > s->max_n) return LB_EINVAL;
    lb_status st = upload(s, X, Y, n);
    if (st != LB_OK) return st;
    HC(hipMemsetAsync(s->loss_acc, 0, sizeof(double), s->stream));
    MlpArgs a{s->P, s->X, s->Y, nullptr, s->G, s->Lpart, n, (float)(2.0 / (6.0 * n)), 1};
    HC(launch_mlp(a, s->stream));
    MlpReduceArgs r{};
    r.G = s->G;
    r.Lpart = s->Lpart;
    r.ntiles = (n + 15) / 16;
    r.gsum = s->gsum;
    r.loss_acc = s->loss_acc;
    r.mode = 1;
    HC(launch_mlp_reduce(r, s->stream));
    double acc = 0;
    if (grads) HC(hipMemcpyAsync(grads, s->gsum, sizeof(float) * MLP_NP, hipMemcpyDeviceToHost, s->stream));
    HC(hipMemcpyAsync(&acc, s->loss_acc, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    if (loss) *loss = (float)(acc / (6.0 * n));
    return LB_OK;
}

lb_status lbs_grad_noalloc(const float* params, const float* X, const float* Y, int n, float* grads, float* loss,
                           void* hip_stream) {
    if (!params || !X || !Y || !grads || n < 1 || n > LBS_NOALLOC_MAX_SAMPLES) return LB_EINVAL;
    float* sc = nullptr;
    const lb_status st = noalloc_scratch(&sc);
    if (st != LB_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;
    float* G = sc;
    float* Lpart = sc + (size_t)NOALLOC_TILES * MLP_NP;
    // the same kernels and sums as lbs_grad; every tile the sums read is
    // written first, so nothing in the scratch needs clearing
    MlpArgs a{params, X, Y, nullptr, G, Lpart, n, (float)(2.0 / (6.0 * n)), 1};
    if (launch_mlp(a, stream) != hipSuccess) return LB_EDEVICE;
    MlpReduceArgs r{};
    r.G = G;
    r.Lpart = Lpart;
    r.ntiles = (n + 15) / 16;
    r.gsum = grads;
    r.loss_out = loss;
    r.loss_div = 6.0 * n;
    r.mode = 1;
    if (launch_mlp_reduce(r, stream) != hipSuccess) return LB_EDEVICE;
    return LB_OK;
}

lb_status lbs_destroy(lbs* s) {
    if (!s) return LB_EINVAL;
    hipStreamSynchronize(s->stream);
    delete s;
    return LB_OK;
}

}  // extern "C"
