// Per-variable fix predictor on BF16 matrix cores (gfx950 MFMA):
//   h1 = relu(W1 f + b1), h2 = relu(W2 bf16(h1) + b2), logit = w3 . h2 + b3
// with 16 padded features, 64 hidden units per layer, FP32 accumulation.
//
// One wave evaluates 16 variables at a time in the transposed form
// H1^T (64 x 16) = W1 (64 x 16) F^T (16 x 16): with v_mfma_f32_16x16x16_bf16
// a lane holds A[row = lane % 16][k = 4 (lane / 16) + i], B[k = 4 (lane / 16)
// + i][col = lane % 16] and D[row = 4 (lane / 16) + i][col = lane % 16], so the
// D block of one layer is already the B operand of the next layer's K block
// and the layers chain in registers.  The 64-wide layer-2 contractions use
// gfx950's v_mfma_f32_16x16x32_bf16, two K = 32 steps instead of four K = 16
// ones: there a lane holds A[lane % 16][k = 8 (lane / 16) + i] and B[k = 8
// (lane / 16) + i][lane % 16], i < 8, and the same D layout.  A lane's 8 B
// values are its D values of two consecutive 16-row blocks, so within a K = 32
// step the hidden unit of slot (lane / 16, i) is 16 (2p + i / 4) + 4 (lane /
// 16) + i % 4; the weights are loaded in that order, and the contraction is
// the same sum over all 64 units.  The weight gradients (sums over variables)
// need the activations with the variable index as K; those tiles go through
// LDS.
#include <cmath>
#include <mutex>
#include <string>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"
#include "pdhg_mlp.hpp"

namespace pdhg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u); // round to nearest, ties to even
    return (short)(u >> 16);
}

__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                  0, 0, 0);
}

// hidden unit of K = 32 step p, slot (lane group lg, element i)
__device__ __forceinline__ int k32_unit(int p, int lg, int i) { return 16 * (2 * p + (i >> 2)) + 4 * lg + (i & 3); }

// the B operand of K = 32 step p: the D values of 16-row blocks 2p and 2p + 1
__device__ __forceinline__ bf16x8 k32_pair(const bf16x4 &lo, const bf16x4 &hi)
{
    return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// parameter offsets in the flat vector: w1 (64x16), b1, w2 (64x64), b2, w3, b3
constexpr int OFF_W1 = 0, OFF_B1 = 1024, OFF_W2 = 1088, OFF_B2 = 5184, OFF_W3 = 5248, OFF_B3 = 5312;

struct MlpW {
    const short *w1b, *w2b, *w3b; // bfloat16 copies
    const float *p;               // float32 master values (biases read from here)
};

// ----------------------------------------------------------------- forward
__global__ __launch_bounds__(kBlock) void k_mlp_forward(const short *__restrict__ F, int64_t N, MlpW w,
                                                       float *__restrict__ logits)
{
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    bf16x4 w1a[4];
    bf16x8 w2a[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; mb++) {
#pragma unroll
        for (int i = 0; i < 4; i++) w1a[mb][i] = w.w1b[(16 * mb + lr) * 16 + 4 * lg + i];
#pragma unroll
        for (int p = 0; p < 2; p++)
#pragma unroll
            for (int i = 0; i < 8; i++) w2a[mb][p][i] = w.w2b[(16 * mb + lr) * 64 + k32_unit(p, lg, i)];
    }
    const float b3 = w.p[OFF_B3];
    const int64_t ntiles = (N + 15) / 16;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t t = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; t < ntiles; t += nwaves) {
        const int64_t v = t * 16 + lr;
        bf16x4 fb = {0, 0, 0, 0};
        if (v < N) {
#pragma unroll
            for (int i = 0; i < 4; i++) fb[i] = F[v * 16 + 4 * lg + i];
        }
        bf16x4 h1b[4];
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            const f32x4 a = mfma16(w1a[mb], fb, f32x4{0, 0, 0, 0});
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float h = a[r] + w.p[OFF_B1 + 16 * mb + 4 * lg + r];
                h1b[mb][r] = f2bf(h > 0.0f ? h : 0.0f);
            }
        }
        float part = 0.0f;
        const bf16x8 h1p[2] = {k32_pair(h1b[0], h1b[1]), k32_pair(h1b[2], h1b[3])};
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            f32x4 a = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < 2; p++) a = mfma32(w2a[mb][p], h1p[p], a);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int h = 16 * mb + 4 * lg + r;
                float hv = a[r] + w.p[OFF_B2 + h];
                hv = hv > 0.0f ? hv : 0.0f;
                part += bf2f(w.w3b[h]) * hv;
            }
        }
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (lg == 0 && v < N) logits[v] = part + b3;
    }
}

// ---------------------------------------------------------------- gradient
// Each wave handles `tiles_per_wave` tiles of 16 samples of the minibatch
// (samples idx[b0 + k], k < bsz) and writes its partial gradient (5313
// values) and partial loss; k_mlp_reduce sums the partials in wave order.
__device__ __forceinline__ float softplus(float x) { return x > 0.0f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }

__global__ __launch_bounds__(kBlock) void k_mlp_grad(const short *__restrict__ F, const float *__restrict__ Y,
                                                    const int *__restrict__ idx, int64_t b0, int bsz,
                                                    int tiles_per_wave, float pw, MlpW w,
                                                    float *__restrict__ part, float *__restrict__ lossp)
{
    __shared__ short sA[kBlock / 64][64 * 16];
    __shared__ short sB[kBlock / 64][64 * 16];
    __shared__ short sF[kBlock / 64][16 * 16];
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, wid = threadIdx.x >> 6;
    const int gw = blockIdx.x * (kBlock / 64) + wid; // global wave number
    bf16x4 w1a[4];
    bf16x8 w2a[4][2], w2t[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; mb++) {
#pragma unroll
        for (int i = 0; i < 4; i++) w1a[mb][i] = w.w1b[(16 * mb + lr) * 16 + 4 * lg + i];
#pragma unroll
        for (int p = 0; p < 2; p++)
#pragma unroll
            for (int i = 0; i < 8; i++) {
                w2a[mb][p][i] = w.w2b[(16 * mb + lr) * 64 + k32_unit(p, lg, i)];
                w2t[mb][p][i] = w.w2b[k32_unit(p, lg, i) * 64 + 16 * mb + lr]; // W2^T
            }
    }
    const float b3 = w.p[OFF_B3];
    const float inv_b = 1.0f / (float)bsz;
    f32x4 gw2[4][4], gw1[4];
    float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.0f, loss = 0.0f;
#pragma unroll
    for (int mb = 0; mb < 4; mb++) {
        gw1[mb] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < 4; r++) gb1[mb][r] = gb2[mb][r] = gw3[mb][r] = 0.0f;
#pragma unroll
        for (int nb = 0; nb < 4; nb++) gw2[mb][nb] = f32x4{0, 0, 0, 0};
    }
    short *a_s = sA[wid], *b_s = sB[wid], *f_s = sF[wid];
    for (int tt = 0; tt < tiles_per_wave; tt++) {
        const int64_t k = ((int64_t)gw * tiles_per_wave + tt) * 16 + lr; // sample slot in the minibatch
        const bool valid = k < bsz;
        const int64_t row = valid ? (int64_t)idx[b0 + k] : 0;
        bf16x4 fb = {0, 0, 0, 0};
        float y = 0.0f;
        if (valid) {
#pragma unroll
            for (int i = 0; i < 4; i++) fb[i] = F[row * 16 + 4 * lg + i];
            y = Y[row];
        }
        // forward, keeping the activations
        float h1[4][4], h2[4][4];
        bf16x4 h1b[4];
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            const f32x4 a = mfma16(w1a[mb], fb, f32x4{0, 0, 0, 0});
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float h = a[r] + w.p[OFF_B1 + 16 * mb + 4 * lg + r];
                h1[mb][r] = h > 0.0f ? h : 0.0f;
                h1b[mb][r] = f2bf(h1[mb][r]);
            }
        }
        float z = 0.0f;
        const bf16x8 h1p[2] = {k32_pair(h1b[0], h1b[1]), k32_pair(h1b[2], h1b[3])};
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            f32x4 a = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < 2; p++) a = mfma32(w2a[mb][p], h1p[p], a);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int h = 16 * mb + 4 * lg + r;
                const float hv = a[r] + w.p[OFF_B2 + h];
                h2[mb][r] = hv > 0.0f ? hv : 0.0f;
                z += bf2f(w.w3b[h]) * h2[mb][r];
            }
        }
        z += __shfl_xor(z, 16, 64);
        z += __shfl_xor(z, 32, 64);
        z += b3;
        // dL/dz of the weighted binary cross-entropy, averaged over the minibatch
        float dz = 0.0f;
        if (valid) {
            const float s = 1.0f / (1.0f + expf(-z));
            dz = (s * (pw * y + 1.0f - y) - pw * y) * inv_b;
            if (lg == 0) {
                loss += pw * y * softplus(-z) + (1.0f - y) * softplus(z);
                gb3 += dz;
            }
        }
        // layer 3 and 2 gradients
        bf16x4 dh2b[4];
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int h = 16 * mb + 4 * lg + r;
                gw3[mb][r] += dz * h2[mb][r];
                const float d = h2[mb][r] > 0.0f ? dz * bf2f(w.w3b[h]) : 0.0f;
                gb2[mb][r] += d;
                dh2b[mb][r] = f2bf(d);
            }
        // dH1^T = W2^T dH2^T, masked by relu
        bf16x4 dh1b[4];
        const bf16x8 dh2p[2] = {k32_pair(dh2b[0], dh2b[1]), k32_pair(dh2b[2], dh2b[3])};
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            f32x4 a = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < 2; p++) a = mfma32(w2t[mb][p], dh2p[p], a);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float d = h1[mb][r] > 0.0f ? a[r] : 0.0f;
                gb1[mb][r] += d;
                dh1b[mb][r] = f2bf(d);
            }
        }
        // dW2 += dH2^T H1 : both tiles transposed through LDS (K = samples)
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                a_s[(16 * mb + 4 * lg + r) * 16 + lr] = dh2b[mb][r];
                b_s[(16 * mb + 4 * lg + r) * 16 + lr] = h1b[mb][r];
            }
#pragma unroll
        for (int i = 0; i < 4; i++) f_s[lr * 16 + 4 * lg + i] = fb[i];
        __syncthreads();
        bf16x4 A2[4], B2[4], Bf;
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                A2[mb][i] = a_s[(16 * mb + lr) * 16 + 4 * lg + i];
                B2[mb][i] = b_s[(16 * mb + lr) * 16 + 4 * lg + i];
            }
#pragma unroll
        for (int i = 0; i < 4; i++) Bf[i] = f_s[(4 * lg + i) * 16 + lr];
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
#pragma unroll
            for (int nb = 0; nb < 4; nb++) gw2[mb][nb] = mfma16(A2[mb], B2[nb], gw2[mb][nb]);
        // dW1 += dH1^T F
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
#pragma unroll
            for (int r = 0; r < 4; r++) a_s[(16 * mb + 4 * lg + r) * 16 + lr] = dh1b[mb][r];
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            bf16x4 A1;
#pragma unroll
            for (int i = 0; i < 4; i++) A1[i] = a_s[(16 * mb + lr) * 16 + 4 * lg + i];
            gw1[mb] = mfma16(A1, Bf, gw1[mb]);
        }
        __syncthreads();
    }
    // per-wave partial gradient, fixed lane order
    float *out = part + (size_t)gw * MLP_NPARAMS;
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * mb + 4 * lg + r;
            out[OFF_W1 + h * 16 + lr] = gw1[mb][r];
#pragma unroll
            for (int nb = 0; nb < 4; nb++) out[OFF_W2 + h * 64 + 16 * nb + lr] = gw2[mb][nb][r];
            float s1 = gb1[mb][r], s2 = gb2[mb][r], s3 = gw3[mb][r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                s1 += __shfl_xor(s1, off, 64);
                s2 += __shfl_xor(s2, off, 64);
                s3 += __shfl_xor(s3, off, 64);
            }
            if (lr == 0) {
                out[OFF_B1 + h] = s1;
                out[OFF_B2 + h] = s2;
                out[OFF_W3 + h] = s3;
            }
        }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        gb3 += __shfl_xor(gb3, off, 64);
        loss += __shfl_xor(loss, off, 64);
    }
    if (lane == 0) {
        out[OFF_B3] = gb3;
        lossp[gw] = loss;
    }
}

// grad[p] = sum over waves of part[w][p], in wave order
__global__ __launch_bounds__(kBlock) void k_mlp_reduce(const float *__restrict__ part, int nw,
                                                      const float *__restrict__ lossp, float *__restrict__ grad,
                                                      double *__restrict__ loss_acc)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < MLP_NPARAMS) {
        float acc = 0.0f;
        for (int w = 0; w < nw; w++) acc += part[(size_t)w * MLP_NPARAMS + p];
        grad[p] = acc;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double l = 0.0;
        for (int w = 0; w < nw; w++) l += (double)lossp[w];
        loss_acc[0] += l;
    }
}

// Adam (Kingma and Ba 2015) on the float32 master values, then fresh
// bfloat16 copies of the weights.  bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ __launch_bounds__(kBlock) void k_mlp_adam(float *__restrict__ p, float *__restrict__ m,
                                                    float *__restrict__ v, const float *__restrict__ g, float lr,
                                                    float beta1, float beta2, float eps, float bc1, float bc2,
                                                    short *__restrict__ w1b, short *__restrict__ w2b,
                                                    short *__restrict__ w3b)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= MLP_NPARAMS) return;
    const float gk = g[k];
    const float mk = beta1 * m[k] + (1.0f - beta1) * gk;
    const float vk = beta2 * v[k] + (1.0f - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float pk = p[k] - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
    p[k] = pk;
    if (k < OFF_B1) w1b[k - OFF_W1] = f2bf(pk);
    else if (k >= OFF_W2 && k < OFF_B2) w2b[k - OFF_W2] = f2bf(pk);
    else if (k >= OFF_W3 && k < OFF_B3) w3b[k - OFF_W3] = f2bf(pk);
}

// bfloat16 copies of the weights from the master values
__global__ __launch_bounds__(kBlock) void k_mlp_sync_bf16(const float *__restrict__ p, short *__restrict__ w1b,
                                                         short *__restrict__ w2b, short *__restrict__ w3b)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= MLP_NPARAMS) return;
    if (k < OFF_B1) w1b[k - OFF_W1] = f2bf(p[k]);
    else if (k >= OFF_W2 && k < OFF_B2) w2b[k - OFF_W2] = f2bf(p[k]);
    else if (k >= OFF_W3 && k < OFF_B3) w3b[k - OFF_W3] = f2bf(p[k]);
}

// float32 features (N x 16) to bfloat16
__global__ __launch_bounds__(kBlock) void k_to_bf16(int64_t len, const float *__restrict__ src, short *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock)
        dst[i] = f2bf(src[i]);
}

// Kaiming-uniform weights, bound sqrt(6 / fan_in), from splitmix64 of a
// counter (padding columns of W1 stay 0); zero biases; zero Adam state
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_mlp_init(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                                    uint64_t seed)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= MLP_NPARAMS) return;
    const double u = (double)(mix64(seed ^ ((uint64_t)k * 0x9E3779B97F4A7C15ULL)) >> 11) * (1.0 / 9007199254740992.0);
    float val = 0.0f;
    if (k < OFF_B1) val = ((k % 16) < 12) ? (float)((2.0 * u - 1.0) * sqrt(6.0 / 12.0)) : 0.0f;
    else if (k >= OFF_W2 && k < OFF_B2) val = (float)((2.0 * u - 1.0) * sqrt(6.0 / 64.0));
    else if (k >= OFF_W3 && k < OFF_B3) val = (float)((2.0 * u - 1.0) * sqrt(6.0 / 64.0));
    p[k] = val;
    m[k] = 0.0f;
    v[k] = 0.0f;
}

hipError_t mlp_init(pdhg_mlp *net, uint64_t seed)
{
    hipLaunchKernelGGL(k_mlp_init, dim3((MLP_NPARAMS + kBlock - 1) / kBlock), dim3(kBlock), 0, net->stream, net->p, net->m,
                       net->v, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_sync(net);
}

static MlpW weights(const pdhg_mlp *net) { return MlpW{net->w1b, net->w2b, net->w3b, net->p}; }

hipError_t mlp_sync(pdhg_mlp *net)
{
    hipLaunchKernelGGL(k_mlp_sync_bf16, dim3((MLP_NPARAMS + kBlock - 1) / kBlock), dim3(kBlock), 0, net->stream, net->p,
                       net->w1b, net->w2b, net->w3b);
    return hipGetLastError();
}

hipError_t mlp_features_to_bf16(hipStream_t st, const float *src, short *dst, int64_t n_rows)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n_rows * 16, kBlock, 65536)), dim3(kBlock), 0, st, n_rows * 16, src, dst);
    return hipGetLastError();
}

hipError_t mlp_forward(const pdhg_mlp *net, hipStream_t st, const short *F, int64_t N, float *logits)
{
    if (N <= 0) return hipSuccess;
    const int64_t tiles = (N + 15) / 16;
    const int grid = grid_for((tiles + 3) / 4, 1, 1 << 20);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kBlock), 0, st, F, N, weights(net), logits);
    return hipGetLastError();
}

// one minibatch: gradient into net->grad, loss added to net->loss_acc
hipError_t mlp_grad(pdhg_mlp *net, const short *F, const float *Y, const int *idx, int64_t b0, int bsz, float pw)
{
    const int tiles = (bsz + 15) / 16;
    const int tpw = 2;
    const int waves = (tiles + tpw - 1) / tpw;
    const int blocks = (waves + 3) / 4;
    const int nw = blocks * 4;
    if (nw > net->max_waves) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(kBlock), 0, net->stream, F, Y, idx, b0, bsz, tpw, pw,
                       weights(net), net->part, net->lossp);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAMS + kBlock - 1) / kBlock), dim3(kBlock), 0, net->stream,
                       net->part, nw, net->lossp, net->grad, net->loss_acc);
    return hipGetLastError();
}

hipError_t mlp_adam(pdhg_mlp *net, float lr, float beta1, float beta2, float eps, int64_t t)
{
    const float bc1 = 1.0f - powf(beta1, (float)t), bc2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAMS + kBlock - 1) / kBlock), dim3(kBlock), 0, net->stream, net->p,
                       net->m, net->v, net->grad, lr, beta1, beta2, eps, bc1, bc2, net->w1b, net->w2b, net->w3b);
    return hipGetLastError();
}

} // namespace pdhg

// ------------------------------------------------- forward without allocation
// For callers that cannot allocate (graph capture, serving loops): the
// bfloat16 staging copy of the features lives in this file-scope device
// array instead of a buffer allocated per call.  Every GPU the library runs
// on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and is kept per device.
namespace pdhg {
namespace {

constexpr int64_t kNoAllocMaxRows = 65536;     // variables per call
constexpr int kMaxDevices = 64;
static __device__ __align__(256) short scratch[16 * kNoAllocMaxRows]; // 2 MiB
short *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// the current device's address of `scratch` (looked up on first use)
hipError_t scratch_for_current_device(short **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (short *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

} // namespace

hipError_t mlp_scratch_setup() // at pdhg_mlp_create, on the device the network lives on
{
    short *p = nullptr;
    return scratch_for_current_device(&p);
}

} // namespace pdhg

extern "C" int pdhg_mlp_forward_noalloc(pdhg_mlp *net, const float *features, int64_t n, float *logits, void *stream)
{
    using namespace pdhg;
    if (!net || n < 0 || (n > 0 && (!features || !logits)))
        return fail(PDHG_ERR_INVALID_ARG, "bad arguments (NULL network or device pointer, or n < 0)");
    if (n > kNoAllocMaxRows)
        return fail(PDHG_ERR_INVALID_ARG, "pdhg_mlp_forward_noalloc takes at most 65536 variables per call");
    if (n == 0) return PDHG_OK;
    short *fb = nullptr;
    hipError_t e = scratch_for_current_device(&fb);
    if (e != hipSuccess) return fail(PDHG_ERR_HIP, std::string("HIP error in hipGetSymbolAddress: ") + hipGetErrorString(e));
    hipStream_t st = stream ? (hipStream_t)stream : net->stream;
    e = mlp_features_to_bf16(st, features, fb, n); // every staged row is overwritten: nothing to clear
    if (e == hipSuccess) e = mlp_forward(net, st, fb, n, logits);
    if (e != hipSuccess) return fail(PDHG_ERR_HIP, std::string("HIP error in the forward launch: ") + hipGetErrorString(e));
    return PDHG_OK;
}
