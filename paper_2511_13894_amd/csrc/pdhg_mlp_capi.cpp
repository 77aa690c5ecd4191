// C ABI of the fix predictor: create, parameters, forward, gradient, train.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pdhg.h"
#include "pdhg_internal.hpp"
#include "pdhg_mlp.hpp"

using namespace pdhg;

namespace {

constexpr int64_t kMaxBatch = 65536;

struct HipFail {
    hipError_t err;
    const char *what;
};

inline void chk(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw HipFail{e, what};
}

#define CHK(expr) chk((expr), #expr)

int hip_fail(const HipFail &f)
{
    return fail(f.err == hipErrorOutOfMemory ? PDHG_ERR_OOM : PDHG_ERR_HIP,
                std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t mix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// features (float32 host, n x 16) and labels to the device
struct DevSet {
    short *F = nullptr;
    float *Ff = nullptr, *Y = nullptr;
    int *idx = nullptr;
    ~DevSet()
    {
        for (void *q : {(void *)F, (void *)Ff, (void *)Y, (void *)idx})
            if (q) (void)hipFree(q);
    }
};

void upload(pdhg_mlp *net, DevSet &d, const float *features, const float *labels, int64_t n)
{
    CHK(hipMalloc(&d.F, sizeof(short) * 16 * (size_t)n));
    CHK(hipMalloc(&d.Ff, sizeof(float) * 16 * (size_t)n));
    CHK(hipMemcpyAsync(d.Ff, features, sizeof(float) * 16 * (size_t)n, hipMemcpyHostToDevice, net->stream));
    CHK(mlp_features_to_bf16(net->stream, d.Ff, d.F, n));
    if (labels) {
        CHK(hipMalloc(&d.Y, sizeof(float) * (size_t)n));
        CHK(hipMemcpyAsync(d.Y, labels, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, net->stream));
    }
    CHK(hipMalloc(&d.idx, sizeof(int) * (size_t)n));
}

} // namespace

extern "C" {

int pdhg_mlp_create(uint64_t seed, pdhg_mlp **out)
{
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    pdhg_mlp *net = new (std::nothrow) pdhg_mlp();
    if (!net) return fail(PDHG_ERR_OOM, "host allocation failed");
    try {
        CHK(hipStreamCreate(&net->stream));
        for (float **q : {&net->p, &net->m, &net->v, &net->grad}) CHK(hipMalloc(q, sizeof(float) * MLP_NPARAMS));
        CHK(hipMalloc(&net->w1b, sizeof(short) * 1024));
        CHK(hipMalloc(&net->w2b, sizeof(short) * 4096));
        CHK(hipMalloc(&net->w3b, sizeof(short) * 64));
        net->max_waves = (int)((((kMaxBatch + 15) / 16 + 1) / 2 + 3) / 4 * 4);
        CHK(hipMalloc(&net->part, sizeof(float) * MLP_NPARAMS * (size_t)net->max_waves));
        CHK(hipMalloc(&net->lossp, sizeof(float) * (size_t)net->max_waves));
        CHK(hipMalloc(&net->loss_acc, sizeof(double)));
        CHK(mlp_init(net, seed));
        CHK(mlp_scratch_setup()); // the no-allocation forward's staging array on this device
        CHK(hipStreamSynchronize(net->stream));
    } catch (const HipFail &f) {
        pdhg_mlp_destroy(net);
        return hip_fail(f);
    }
    *out = net;
    return PDHG_OK;
}

void pdhg_mlp_destroy(pdhg_mlp *net)
{
    if (!net) return;
    if (net->stream) (void)hipStreamSynchronize(net->stream);
    for (void *q : {(void *)net->p, (void *)net->m, (void *)net->v, (void *)net->grad, (void *)net->w1b,
                    (void *)net->w2b, (void *)net->w3b, (void *)net->part, (void *)net->lossp, (void *)net->loss_acc})
        if (q) (void)hipFree(q);
    if (net->stream) (void)hipStreamDestroy(net->stream);
    delete net;
}

int pdhg_mlp_set_params(pdhg_mlp *net, const float *params)
{
    if (!net || !params) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    try {
        CHK(hipMemcpyAsync(net->p, params, sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice, net->stream));
        CHK(hipMemsetAsync(net->m, 0, sizeof(float) * MLP_NPARAMS, net->stream));
        CHK(hipMemsetAsync(net->v, 0, sizeof(float) * MLP_NPARAMS, net->stream));
        net->adam_t = 0;
        CHK(mlp_sync(net));
        CHK(hipStreamSynchronize(net->stream));
    } catch (const HipFail &f) {
        return hip_fail(f);
    }
    return PDHG_OK;
}

int pdhg_mlp_get_params(pdhg_mlp *net, float *params)
{
    if (!net || !params) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    try {
        CHK(hipMemcpyAsync(params, net->p, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost, net->stream));
        CHK(hipStreamSynchronize(net->stream));
    } catch (const HipFail &f) {
        return hip_fail(f);
    }
    return PDHG_OK;
}

int pdhg_mlp_forward(pdhg_mlp *net, const float *features, int64_t n, float *logits)
{
    if (!net || (n > 0 && (!features || !logits)) || n < 0) return fail(PDHG_ERR_INVALID_ARG, "bad arguments");
    if (n == 0) return PDHG_OK;
    try {
        DevSet d;
        upload(net, d, features, nullptr, n);
        float *dl = nullptr;
        CHK(hipMalloc(&dl, sizeof(float) * (size_t)n));
        hipError_t e = mlp_forward(net, net->stream, d.F, n, dl);
        if (e == hipSuccess) e = hipMemcpyAsync(logits, dl, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, net->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
        (void)hipFree(dl);
        CHK(e);
    } catch (const HipFail &f) {
        return hip_fail(f);
    }
    return PDHG_OK;
}

int pdhg_mlp_gradient(pdhg_mlp *net, const float *features, const float *labels, int64_t n, double pos_weight,
                      float *grad, double *loss)
{
    if (!net || !features || !labels || !grad || n < 1 || n > kMaxBatch)
        return fail(PDHG_ERR_INVALID_ARG, "bad arguments (1 <= n <= 65536)");
    try {
        DevSet d;
        upload(net, d, features, labels, n);
        std::vector<int> idx((size_t)n);
        for (int64_t i = 0; i < n; i++) idx[i] = (int)i;
        CHK(hipMemcpyAsync(d.idx, idx.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, net->stream));
        CHK(hipMemsetAsync(net->loss_acc, 0, sizeof(double), net->stream));
        CHK(mlp_grad(net, d.F, d.Y, d.idx, 0, (int)n, (float)pos_weight));
        double l = 0.0;
        CHK(hipMemcpyAsync(grad, net->grad, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost, net->stream));
        CHK(hipMemcpyAsync(&l, net->loss_acc, sizeof(double), hipMemcpyDeviceToHost, net->stream));
        CHK(hipStreamSynchronize(net->stream));
        if (loss) *loss = l / (double)n;
    } catch (const HipFail &f) {
        return hip_fail(f);
    }
    return PDHG_OK;
}

void pdhg_default_train_params(pdhg_train_params *t)
{
    if (!t) return;
    std::memset(t, 0, sizeof(*t));
    t->epochs = 4;
    t->batch = 4096;
    t->lr = 1e-3;
    t->beta1 = 0.9;
    t->beta2 = 0.999;
    t->eps = 1e-8;
    t->pos_weight = 0.0;
    t->seed = 1;
}

int pdhg_mlp_train(pdhg_mlp *net, const float *features, const float *labels, int64_t n, const pdhg_train_params *tp,
                   pdhg_train_report *rep)
{
    if (!net || !features || !labels || n < 1 || n >= ((int64_t)1 << 31))
        return fail(PDHG_ERR_INVALID_ARG, "bad arguments");
    pdhg_train_params t;
    if (tp) t = *tp;
    else pdhg_default_train_params(&t);
    if (t.batch < 1 || t.batch > kMaxBatch || t.epochs < 0) return fail(PDHG_ERR_INVALID_ARG, "bad training parameters");
    const double t0 = now_s();
    try {
        // positive-class weight N_neg / N_pos unless given
        double pw = t.pos_weight;
        if (!(pw > 0.0)) {
            int64_t pos = 0;
            for (int64_t i = 0; i < n; i++) pos += labels[i] > 0.5f;
            pw = pos > 0 ? (double)(n - pos) / (double)pos : 1.0;
        }
        DevSet d;
        upload(net, d, features, labels, n);
        std::vector<int> idx((size_t)n);
        double first = NAN, last = NAN;
        int64_t steps = 0;
        for (int ep = 0; ep < t.epochs; ep++) {
            // seeded Fisher-Yates shuffle (splitmix64 counter stream)
            for (int64_t i = 0; i < n; i++) idx[i] = (int)i;
            for (int64_t i = n - 1; i > 0; i--) {
                const uint64_t r = mix64(t.seed ^ (((uint64_t)ep << 40) + (uint64_t)i));
                const int64_t j = (int64_t)(r % (uint64_t)(i + 1));
                std::swap(idx[i], idx[j]);
            }
            CHK(hipMemcpyAsync(d.idx, idx.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, net->stream));
            CHK(hipMemsetAsync(net->loss_acc, 0, sizeof(double), net->stream));
            for (int64_t b0 = 0; b0 < n; b0 += t.batch) {
                const int bsz = (int)std::min<int64_t>(t.batch, n - b0);
                CHK(mlp_grad(net, d.F, d.Y, d.idx, b0, bsz, (float)pw));
                net->adam_t += 1;
                CHK(mlp_adam(net, (float)t.lr, (float)t.beta1, (float)t.beta2, (float)t.eps, net->adam_t));
                steps++;
            }
            double l = 0.0;
            CHK(hipMemcpyAsync(&l, net->loss_acc, sizeof(double), hipMemcpyDeviceToHost, net->stream));
            CHK(hipStreamSynchronize(net->stream));
            l /= (double)n;
            if (ep == 0) first = l;
            last = l;
        }
        if (rep) {
            std::memset(rep, 0, sizeof(*rep));
            rep->loss_first = first;
            rep->loss_last = last;
            rep->seconds = now_s() - t0;
            rep->steps = steps;
            rep->samples_per_s = rep->seconds > 0 ? (double)n * t.epochs / rep->seconds : 0.0;
            rep->pos_weight = pw;
        }
    } catch (const HipFail &f) {
        return hip_fail(f);
    }
    return PDHG_OK;
}

} // extern "C"
