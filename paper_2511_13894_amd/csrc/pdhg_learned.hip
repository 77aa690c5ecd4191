// Learned warm start of the corner push: restart history, the 16
// per-variable features, learned fixes and their undo rule.
//
// Features of column j on the scaled model:
//   0..3   x_j, z_j, |c_j|, ||A_{:,j}||_2;
//   4..7   x_j at each of the last 4 restarts of the solve minus its current
//          value (0 where fewer than 4 restarts happened);
//   8..11  the same for z_j;
//   12     the push objective coefficient of column j (the scaled
//          Uniform[0,1) draw of the push seed);
//   13, 14 x_j - l_j and u_j - x_j (-1 where that bound is infinite);
//   15     (x_j - l_j) / (u_j - l_j) where both bounds are finite and
//          distinct, else -1.
// Each feature f is mapped to sign(v) ln(1 + |v| / s_f), s_f the root mean
// square of f over the LP (1 if that is 0).
// A learned fix puts a column that the plain rule leaves free (|z_j| <=
// eps_abs) at its nearer finite bound when the predicted probability is at
// least theta, provided the sign of z_j allows it (z_j >= -eps_abs for the
// lower bound, z_j <= eps_abs for the upper bound).  At every push check the
// push model's reduced cost chat - Ahat'y (unscaled) is tested and a learned
// fix whose reduced cost has the wrong sign (below -eps_abs at a lower fix,
// above eps_abs at an upper fix) goes back to the plain rule's bounds.
#include <cmath>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"
#include "pdhg_kernels.hpp"
#include "pdhg_mlp.hpp"

namespace pdhg {

constexpr int kNF = 16;
// the per-block feature sums reuse the check's partial-sum buffer
static_assert((Q_COUNT + 1) * 3 >= kNF, "partial-sum buffer too small for the feature sums");

__device__ __forceinline__ double zsplit(double lam, double lo, double hi)
{
    const double zp = (!is_inf_lo(lo) && lam > 0.0) ? lam : 0.0;
    const double zm = (!is_inf_up(hi) && lam < 0.0) ? -lam : 0.0;
    return zp - zm;
}

// at a restart of the solve: slot (restarts - 1) mod 4 <- candidate x, z
template <typename V>
__global__ __launch_bounds__(kBlock) void k_record_history(int n, const DevState *__restrict__ st,
                                                          const V *__restrict__ xp, const double *__restrict__ ch,
                                                          const V *__restrict__ lh, const V *__restrict__ uh,
                                                          const double *__restrict__ aty, float *__restrict__ hx,
                                                          float *__restrict__ hz)
{
    if (!st->restart_flag || st->done) return;
    const int64_t slot = (st->restarts - 1) & 3;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        hx[slot * n + j] = (float)xp[j];
        hz[slot * n + j] = (float)zsplit((double)ch[j] - aty[j], (double)lh[j], (double)uh[j]);
    }
}

hipError_t launch_record_history(pdhg_solver *s)
{
    const int g = grid_for(s->n, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL((k_record_history<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->st,
                           (const float *)s->xp, s->ch, (const float *)s->lh, (const float *)s->uh,
                           s->aty, s->hx, s->hz);
    else
        hipLaunchKernelGGL((k_record_history<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->st,
                           (const double *)s->xp, s->ch, (const double *)s->lh, (const double *)s->uh,
                           s->aty, s->hx, s->hz);
    return hipGetLastError();
}

// raw features into f (n x 16, float) and per-block sums of their squares
template <typename V>
__global__ __launch_bounds__(kBlock) void k_feat_raw(int n, const DevState *__restrict__ st, const V *__restrict__ xp,
                                                    const double *__restrict__ ch, const V *__restrict__ lh,
                                                    const V *__restrict__ uh, const double *__restrict__ aty,
                                                    const int *__restrict__ tp, const V *__restrict__ atv,
                                                    const float *__restrict__ hx, const float *__restrict__ hz,
                                                    const double *__restrict__ dc, uint64_t seed, double obj_scale,
                                                    float *__restrict__ f,
                                                    double *__restrict__ part, int nblk)
{
    const int64_t rest = st->restarts;
    const int have = rest < 4 ? (int)rest : 4;
    double sq[kNF];
#pragma unroll
    for (int q = 0; q < kNF; q++) sq[q] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        double v[kNF];
        const double xj = (double)xp[j];
        const double zj = zsplit((double)ch[j] - aty[j], (double)lh[j], (double)uh[j]);
        double cn = 0.0;
        for (int e = tp[j]; e < tp[j + 1]; e++) cn += (double)atv[e] * (double)atv[e];
        v[0] = xj;
        v[1] = zj;
        v[2] = fabs((double)ch[j]);
        v[3] = sqrt(cn);
#pragma unroll
        for (int k = 1; k <= 4; k++) {
            const int64_t slot = (rest - k) & 3;
            v[3 + k] = (k <= have && hx) ? (double)hx[slot * n + j] - xj : 0.0;
            v[7 + k] = (k <= have && hz) ? (double)hz[slot * n + j] - zj : 0.0;
        }
        const double lo = (double)lh[j], hi = (double)uh[j];
        const bool flo = !is_inf_lo(lo), fhi = !is_inf_up(hi);
        v[12] = dc[j] * (obj_scale * push_unit(seed, j));
        v[13] = flo ? xj - lo : -1.0;
        v[14] = fhi ? hi - xj : -1.0;
        v[15] = (flo && fhi && hi > lo) ? (xj - lo) / (hi - lo) : -1.0;
#pragma unroll
        for (int q = 0; q < kNF; q++) {
            if (!isfinite(v[q])) v[q] = 0.0;
            f[j * 16 + q] = (float)v[q];
            sq[q] += v[q] * v[q];
        }
    }
    block_reduce<kNF>(sq, 0u);
    if (threadIdx.x == 0)
        for (int q = 0; q < kNF; q++) part[q * nblk + blockIdx.x] = sq[q];
}

// scale of each feature: root mean square over the LP (1 if 0)
__global__ __launch_bounds__(kBlock) void k_feat_scale(int n, const double *__restrict__ part, int nblk,
                                                      double *__restrict__ scale)
{
    double v[kNF];
#pragma unroll
    for (int q = 0; q < kNF; q++) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) acc += part[q * nblk + b];
        v[q] = acc;
    }
    block_reduce<kNF>(v, 0u);
    if (threadIdx.x == 0)
        for (int q = 0; q < kNF; q++) {
            const double rms = n > 0 ? sqrt(v[q] / (double)n) : 0.0;
            scale[q] = rms > 0.0 ? rms : 1.0;
        }
}

__device__ __forceinline__ short f2bf_l(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// sign(v) ln(1 + |v| / s) in place, and the bfloat16 copy for the network
__global__ __launch_bounds__(kBlock) void k_feat_norm(int64_t n, const double *__restrict__ scale, float *__restrict__ f,
                                                     short *__restrict__ fb)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n * 16; k += (int64_t)gridDim.x * kBlock) {
        const int q = (int)(k & 15);
        float out = 0.0f;
        if (q < kNF) {
            const double v = (double)f[k];
            const double t = log1p(fabs(v) / scale[q]);
            out = (float)(v < 0.0 ? -t : t);
        }
        f[k] = out;
        fb[k] = f2bf_l(out);
    }
}

hipError_t compute_features(pdhg_solver *s, uint64_t seed)
{
    hipStream_t st = s->stream;
    // z of the candidate needs Ahat' y+ (float64 accumulation)
    if (s->fp32)
        spmv<float, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, (const float *)s->ahat_t,
                                            (const double *)s->yp, s->aty);
    else
        spmv<double, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, (const double *)s->ahat_t,
                                             (const double *)s->yp, s->aty);
    const int nb = s->red_blocks_n;
    double *scale = s->redout + 16;
    if (s->fp32)
        hipLaunchKernelGGL((k_feat_raw<float>), dim3(nb), dim3(kBlock), 0, st, s->n, s->st, (const float *)s->xp,
                           s->ch, (const float *)s->lh, (const float *)s->uh, s->aty, s->tp,
                           (const float *)s->ahat_t, s->hx, s->hz, s->dc, seed, s->p.push_obj_scale, s->feat_raw,
                           s->partials, nb);
    else
        hipLaunchKernelGGL((k_feat_raw<double>), dim3(nb), dim3(kBlock), 0, st, s->n, s->st, (const double *)s->xp,
                           s->ch, (const double *)s->lh, (const double *)s->uh, s->aty, s->tp,
                           (const double *)s->ahat_t, s->hx, s->hz, s->dc, seed, s->p.push_obj_scale, s->feat_raw,
                           s->partials, nb);
    hipLaunchKernelGGL(k_feat_scale, dim3(1), dim3(kBlock), 0, st, s->n, s->partials, nb, scale);
    hipLaunchKernelGGL(k_feat_norm, dim3(grid_for((int64_t)s->n * 16, kBlock, 65536)), dim3(kBlock), 0, st,
                       (int64_t)s->n, scale, s->feat_raw, s->feat_b);
    return hipGetLastError();
}

// learned fixes at the push start (after the plain rule)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_learned_fix(int n, const float *__restrict__ logits, float theta_logit,
                                                       const double *__restrict__ z, double eps_abs,
                                                       const double *__restrict__ l, const double *__restrict__ u,
                                                       const double *__restrict__ dc, const V *__restrict__ xs,
                                                       V *__restrict__ lh, V *__restrict__ uh, V *__restrict__ x,
                                                       int8_t *__restrict__ lfix, unsigned *__restrict__ count)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        lfix[j] = 0;
        if (fabs(z[j]) > eps_abs || logits[j] < theta_logit) continue; // plain-fixed, or not predicted
        const double lo = l[j] / dc[j], hi = u[j] / dc[j], xv = (double)xs[j];
        const double dl = is_inf_lo(lo) ? INFINITY : xv - lo;
        const double du = is_inf_up(hi) ? INFINITY : hi - xv;
        if (!(dl < INFINITY) && !(du < INFINITY)) continue; // free column
        if (dl <= du) {
            if (z[j] < -eps_abs) continue;
            lh[j] = uh[j] = x[j] = (V)lo;
            lfix[j] = 1;
        } else {
            if (z[j] > eps_abs) continue;
            lh[j] = uh[j] = x[j] = (V)hi;
            lfix[j] = 2;
        }
        atomicAdd(&count[0], 1u);
    }
}

hipError_t launch_learned_fix(pdhg_solver *s, double theta)
{
    const float tl = (float)log(theta / (1.0 - theta)); // probability >= theta <=> logit >= tl
    const int g = grid_for(s->n, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL((k_learned_fix<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->logits, tl, s->zsol,
                           s->p.eps_abs, s->l, s->u, s->dc, (const float *)s->xs, (float *)s->lh, (float *)s->uh,
                           (float *)s->x, s->lfix, s->lcount);
    else
        hipLaunchKernelGGL((k_learned_fix<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->logits, tl, s->zsol,
                           s->p.eps_abs, s->l, s->u, s->dc, (const double *)s->xs, (double *)s->lh, (double *)s->uh,
                           (double *)s->x, s->lfix, s->lcount);
    return hipGetLastError();
}

// undo rule at a push check (aty = Ahat' y+ of the check's candidate)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_learned_undo(int n, const DevState *__restrict__ st,
                                                        int8_t *__restrict__ lfix, const double *__restrict__ ch,
                                                        const double *__restrict__ aty, const double *__restrict__ dc,
                                                        const double *__restrict__ l, const double *__restrict__ u,
                                                        double eps_abs, V *__restrict__ lh, V *__restrict__ uh,
                                                        unsigned *__restrict__ count)
{
    // runs at the terminating check too (and idempotently in cycles after
    // it), so that no fix with a rejected sign survives the push
    (void)st;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int8_t f = lfix[j];
        if (!f) continue;
        const double lam = ((double)ch[j] - aty[j]) / dc[j];
        if ((f == 1 && lam < -eps_abs) || (f == 2 && lam > eps_abs)) {
            lh[j] = (V)(l[j] / dc[j]);
            uh[j] = (V)(u[j] / dc[j]);
            lfix[j] = 0;
            atomicAdd(&count[1], 1u);
        }
    }
}

hipError_t launch_learned_undo(pdhg_solver *s)
{
    const int g = grid_for(s->n, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL((k_learned_undo<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->st, s->lfix,
                           s->ch, s->aty, s->dc, s->l, s->u, s->p.eps_abs, (float *)s->lh, (float *)s->uh,
                           s->lcount);
    else
        hipLaunchKernelGGL((k_learned_undo<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->st, s->lfix,
                           s->ch, s->aty, s->dc, s->l, s->u, s->p.eps_abs, (double *)s->lh,
                           (double *)s->uh, s->lcount);
    return hipGetLastError();
}

} // namespace pdhg
