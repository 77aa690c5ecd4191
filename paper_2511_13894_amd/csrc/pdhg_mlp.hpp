// Internal declarations of the fix predictor (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pdhg.h"

#define MLP_NPARAMS 5313 // w1 (64x16), b1 (64), w2 (64x64), b2 (64), w3 (64), b3 (1)

struct pdhg_mlp {
    hipStream_t stream = nullptr;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr; // float32 master values, Adam state
    short *w1b = nullptr, *w2b = nullptr, *w3b = nullptr;           // bfloat16 weight copies
    float *part = nullptr, *lossp = nullptr;                         // per-wave partial gradients and losses
    int max_waves = 0;
    double *loss_acc = nullptr;
    int64_t adam_t = 0;
};

namespace pdhg {
hipError_t mlp_sync(pdhg_mlp *net);
hipError_t mlp_init(pdhg_mlp *net, uint64_t seed);
hipError_t mlp_features_to_bf16(hipStream_t st, const float *src, short *dst, int64_t n_rows);
hipError_t mlp_forward(const pdhg_mlp *net, hipStream_t st, const short *F, int64_t N, float *logits);
hipError_t mlp_grad(pdhg_mlp *net, const short *F, const float *Y, const int *idx, int64_t b0, int bsz, float pw);
hipError_t mlp_adam(pdhg_mlp *net, float lr, float beta1, float beta2, float eps, int64_t t);
// device address of the no-allocation forward's staging array on the current
// device (looked up once per device)
hipError_t mlp_scratch_setup();
} // namespace pdhg
