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
                                                          const double *__restrict__ xp, const double *__restrict__ ch,
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
                           (const double *)s->xp, s->ch, (const float *)s->lh, (const float *)s->uh,
                           s->aty, s->hx, s->hz);
    else
        hipLaunchKernelGGL((k_record_history<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->st,
                           (const double *)s->xp, s->ch, (const double *)s->lh, (const double *)s->uh,
                           s->aty, s->hx, s->hz);
    return hipGetLastError();
}

// raw features of column j (jl its index inside its LP, for the push draw;
// n the stride of the history arrays; rest the LP's restart count)
template <typename V>
__device__ __forceinline__ void column_features(int64_t j, int64_t jl, int64_t n, int64_t rest,
                                                const double *__restrict__ xp, const double *__restrict__ ch,
                                                const V *__restrict__ lh, const V *__restrict__ uh,
                                                const double *__restrict__ aty, const int *__restrict__ tp,
                                                const V *__restrict__ atv, const float *__restrict__ hx,
                                                const float *__restrict__ hz, const double *__restrict__ dc,
                                                uint64_t seed, double obj_scale, double (&v)[kNF])
{
    const int have = rest < 4 ? (int)rest : 4;
    const double xj = (double)xp[j];
    const double zj = zsplit(ch[j] - aty[j], (double)lh[j], (double)uh[j]);
    double cn = 0.0;
    for (int e = tp[j]; e < tp[j + 1]; e++) cn += (double)atv[e] * (double)atv[e];
    v[0] = xj;
    v[1] = zj;
    v[2] = fabs(ch[j]);
    v[3] = sqrt(cn);
#pragma unroll
    for (int k = 1; k <= 4; k++) {
        const int64_t slot = (rest - k) & 3;
        v[3 + k] = (k <= have && hx) ? (double)hx[slot * n + j] - xj : 0.0;
        v[7 + k] = (k <= have && hz) ? (double)hz[slot * n + j] - zj : 0.0;
    }
    const double lo = (double)lh[j], hi = (double)uh[j];
    const bool flo = !is_inf_lo(lo), fhi = !is_inf_up(hi);
    v[12] = dc[j] * (obj_scale * push_unit(seed, jl));
    v[13] = flo ? xj - lo : -1.0;
    v[14] = fhi ? hi - xj : -1.0;
    v[15] = (flo && fhi && hi > lo) ? (xj - lo) / (hi - lo) : -1.0;
#pragma unroll
    for (int q = 0; q < kNF; q++)
        if (!isfinite(v[q])) v[q] = 0.0;
}

// raw features into f (n x 16, float) and per-block sums of their squares
template <typename V>
__global__ __launch_bounds__(kBlock) void k_feat_raw(int n, const DevState *__restrict__ st, const double *__restrict__ xp,
                                                    const double *__restrict__ ch, const V *__restrict__ lh,
                                                    const V *__restrict__ uh, const double *__restrict__ aty,
                                                    const int *__restrict__ tp, const V *__restrict__ atv,
                                                    const float *__restrict__ hx, const float *__restrict__ hz,
                                                    const double *__restrict__ dc, uint64_t seed, double obj_scale,
                                                    float *__restrict__ f,
                                                    double *__restrict__ part, int nblk)
{
    const int64_t rest = st->restarts;
    double sq[kNF];
#pragma unroll
    for (int q = 0; q < kNF; q++) sq[q] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        double v[kNF];
        column_features<V>(j, j, n, rest, xp, ch, lh, uh, aty, tp, atv, hx, hz, dc, seed, obj_scale, v);
#pragma unroll
        for (int q = 0; q < kNF; q++) {
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
        hipLaunchKernelGGL((k_feat_raw<float>), dim3(nb), dim3(kBlock), 0, st, s->n, s->st, (const double *)s->xp,
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

// learned fix of column j at the push start (after the plain rule):
// 0 none, 1 at the lower bound, 2 at the upper bound
template <typename V>
__device__ __forceinline__ int learned_fix_one(int64_t j, const float *__restrict__ logits, float theta_logit,
                                               const double *__restrict__ z, double eps_abs,
                                               const double *__restrict__ l, const double *__restrict__ u,
                                               const double *__restrict__ dc, const double *__restrict__ xs,
                                               V *__restrict__ lh, V *__restrict__ uh, V *__restrict__ x,
                                               double *__restrict__ xa)
{
    if (fabs(z[j]) > eps_abs || logits[j] < theta_logit) return 0; // plain-fixed, or not predicted
    const double lo = l[j] / dc[j], hi = u[j] / dc[j], xv = (double)xs[j];
    const double dl = is_inf_lo(lo) ? INFINITY : xv - lo;
    const double du = is_inf_up(hi) ? INFINITY : hi - xv;
    if (!(dl < INFINITY) && !(du < INFINITY)) return 0; // free column
    if (dl <= du) {
        if (z[j] < -eps_abs) return 0;
        lh[j] = uh[j] = (V)lo;
        set_iterate<V>(j, (double)(V)lo, x, xa);
        return 1;
    }
    if (z[j] > eps_abs) return 0;
    lh[j] = uh[j] = (V)hi;
    set_iterate<V>(j, (double)(V)hi, x, xa);
    return 2;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_learned_fix(int n, const float *__restrict__ logits, float theta_logit,
                                                       const double *__restrict__ z, double eps_abs,
                                                       const double *__restrict__ l, const double *__restrict__ u,
                                                       const double *__restrict__ dc, const double *__restrict__ xs,
                                                       V *__restrict__ lh, V *__restrict__ uh, V *__restrict__ x,
                                                       double *__restrict__ xa,
                                                       int8_t *__restrict__ lfix, unsigned *__restrict__ count)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const int f = learned_fix_one<V>(j, logits, theta_logit, z, eps_abs, l, u, dc, xs, lh, uh, x, xa);
        lfix[j] = (int8_t)f;
        if (f) atomicAdd(&count[0], 1u);
    }
}

hipError_t launch_learned_fix(pdhg_solver *s, double theta)
{
    const float tl = (float)log(theta / (1.0 - theta)); // probability >= theta <=> logit >= tl
    const int g = grid_for(s->n, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL((k_learned_fix<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->logits, tl, s->zsol,
                           s->p.eps_abs, s->l, s->u, s->dc, (const double *)s->xs, (float *)s->lh, (float *)s->uh,
                           (float *)s->x, (double *)s->xa, s->lfix, s->lcount);
    else
        hipLaunchKernelGGL((k_learned_fix<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->logits, tl, s->zsol,
                           s->p.eps_abs, s->l, s->u, s->dc, (const double *)s->xs, (double *)s->lh, (double *)s->uh,
                           (double *)s->x, (double *)s->xa, s->lfix, s->lcount);
    return hipGetLastError();
}

// undo rule for column j at a push check (aty = Ahat' y+ of the check's
// candidate): true if its learned fix went back to the plain rule's bounds
template <typename V>
__device__ __forceinline__ bool learned_undo_one(int64_t j, int8_t *__restrict__ lfix, const double *__restrict__ ch,
                                                 const double *__restrict__ aty, const double *__restrict__ dc,
                                                 const double *__restrict__ l, const double *__restrict__ u,
                                                 double eps_abs, V *__restrict__ lh, V *__restrict__ uh)
{
    const int8_t f = lfix[j];
    if (!f) return false;
    const double lam = (ch[j] - aty[j]) / dc[j];
    if (!((f == 1 && lam < -eps_abs) || (f == 2 && lam > eps_abs))) return false;
    lh[j] = (V)(l[j] / dc[j]);
    uh[j] = (V)(u[j] / dc[j]);
    lfix[j] = 0;
    return true;
}

// runs at the terminating check too (and idempotently in cycles after it),
// so that no fix with a rejected sign survives the push
template <typename V>
__global__ __launch_bounds__(kBlock) void k_learned_undo(int n, int8_t *__restrict__ lfix, const double *__restrict__ ch,
                                                        const double *__restrict__ aty, const double *__restrict__ dc,
                                                        const double *__restrict__ l, const double *__restrict__ u,
                                                        double eps_abs, V *__restrict__ lh, V *__restrict__ uh,
                                                        unsigned *__restrict__ count)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
        if (learned_undo_one<V>(j, lfix, ch, aty, dc, l, u, eps_abs, lh, uh)) atomicAdd(&count[1], 1u);
}

hipError_t launch_learned_undo(pdhg_solver *s)
{
    const int g = grid_for(s->n, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL((k_learned_undo<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->lfix, s->ch, s->aty,
                           s->dc, s->l, s->u, s->p.eps_abs, (float *)s->lh, (float *)s->uh, s->lcount);
    else
        hipLaunchKernelGGL((k_learned_undo<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->lfix, s->ch, s->aty,
                           s->dc, s->l, s->u, s->p.eps_abs, (double *)s->lh, (double *)s->uh, s->lcount);
    return hipGetLastError();
}

// ----------------------------------------------------------- the batch ---
// The same rules per LP of a batch, over its 256-column reduction tiles
// {lp, first column, columns, 0}: each LP's own restart count, push seed,
// feature scales and counters (lcount[2 lp], lcount[2 lp + 1]).

template <typename V>
__global__ __launch_bounds__(kBlock) void kb_record_history(const int4 *__restrict__ rn, int n,
                                                           const DevState *__restrict__ sts, const double *__restrict__ xp,
                                                           const double *__restrict__ ch, const V *__restrict__ lh,
                                                           const V *__restrict__ uh, const double *__restrict__ aty,
                                                           float *__restrict__ hx, float *__restrict__ hz)
{
    const int4 tl = rn[blockIdx.x];
    const DevState &d = sts[tl.x];
    if (!d.restart_flag || d.done || (int)threadIdx.x >= tl.z) return;
    const int64_t slot = (d.restarts - 1) & 3, j = tl.y + threadIdx.x;
    hx[slot * n + j] = (float)xp[j];
    hz[slot * n + j] = (float)zsplit(ch[j] - aty[j], (double)lh[j], (double)uh[j]);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void kb_feat_raw(const int4 *__restrict__ rn, int n, const int *__restrict__ coff,
                                                     const DevState *__restrict__ sts, const double *__restrict__ xp,
                                                     const double *__restrict__ ch, const V *__restrict__ lh,
                                                     const V *__restrict__ uh, const double *__restrict__ aty,
                                                     const int *__restrict__ tp, const V *__restrict__ atv,
                                                     const float *__restrict__ hx, const float *__restrict__ hz,
                                                     const double *__restrict__ dc, const uint64_t *__restrict__ seeds,
                                                     double obj_scale, float *__restrict__ f, double *__restrict__ part,
                                                     int ntile)
{
    const int4 tl = rn[blockIdx.x];
    double v[kNF];
#pragma unroll
    for (int q = 0; q < kNF; q++) v[q] = 0.0;
    if ((int)threadIdx.x < tl.z) {
        const int64_t j = tl.y + threadIdx.x;
        column_features<V>(j, j - coff[tl.x], n, sts[tl.x].restarts, xp, ch, lh, uh, aty, tp, atv, hx, hz, dc,
                           seeds[tl.x], obj_scale, v);
#pragma unroll
        for (int q = 0; q < kNF; q++) {
            f[j * 16 + q] = (float)v[q];
            v[q] *= v[q];
        }
    }
    block_reduce<kNF>(v, 0u);
    if (threadIdx.x == 0)
        for (int q = 0; q < kNF; q++) part[(size_t)q * ntile + blockIdx.x] = v[q];
}

// one workgroup per LP: feature scales from its tiles' sums, in tile order
__global__ __launch_bounds__(kBlock) void kb_feat_scale(const int *__restrict__ rn_start, const int *__restrict__ coff,
                                                       const double *__restrict__ part, int ntile,
                                                       double *__restrict__ scale)
{
    const int lp = blockIdx.x;
    double v[kNF];
#pragma unroll
    for (int q = 0; q < kNF; q++) {
        double acc = 0.0;
        for (int t = rn_start[lp] + threadIdx.x; t < rn_start[lp + 1]; t += kBlock) acc += part[(size_t)q * ntile + t];
        v[q] = acc;
    }
    block_reduce<kNF>(v, 0u);
    if (threadIdx.x == 0) {
        const double nl = (double)(coff[lp + 1] - coff[lp]);
        for (int q = 0; q < kNF; q++) {
            const double rms = nl > 0 ? sqrt(v[q] / nl) : 0.0;
            scale[(size_t)lp * kNF + q] = rms > 0.0 ? rms : 1.0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void kb_feat_norm(const int4 *__restrict__ rn, const double *__restrict__ scale,
                                                      float *__restrict__ f, short *__restrict__ fb)
{
    const int4 tl = rn[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    const int64_t j = tl.y + threadIdx.x;
    const double *sc = scale + (size_t)tl.x * kNF;
#pragma unroll
    for (int q = 0; q < kNF; q++) {
        const double v = (double)f[j * 16 + q];
        const double t = log1p(fabs(v) / sc[q]);
        const float out = (float)(v < 0.0 ? -t : t);
        f[j * 16 + q] = out;
        fb[j * 16 + q] = f2bf_l(out);
    }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void kb_learned_fix(const int4 *__restrict__ rn, const int *__restrict__ active,
                                                        const float *__restrict__ logits, float theta_logit,
                                                        const double *__restrict__ z, double eps_abs,
                                                        const double *__restrict__ l, const double *__restrict__ u,
                                                        const double *__restrict__ dc, const double *__restrict__ xs,
                                                        V *__restrict__ lh, V *__restrict__ uh, V *__restrict__ x,
                                                        double *__restrict__ xa,
                                                        int8_t *__restrict__ lfix, unsigned *__restrict__ count)
{
    const int4 tl = rn[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    const int64_t j = tl.y + threadIdx.x;
    const int f = active[tl.x] ? learned_fix_one<V>(j, logits, theta_logit, z, eps_abs, l, u, dc, xs, lh, uh, x, xa) : 0;
    lfix[j] = (int8_t)f;
    if (f) atomicAdd(&count[2 * tl.x], 1u);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void kb_learned_undo(const int4 *__restrict__ rn, int8_t *__restrict__ lfix,
                                                         const double *__restrict__ ch, const double *__restrict__ aty,
                                                         const double *__restrict__ dc, const double *__restrict__ l,
                                                         const double *__restrict__ u, double eps_abs,
                                                         V *__restrict__ lh, V *__restrict__ uh,
                                                         unsigned *__restrict__ count)
{
    const int4 tl = rn[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    if (learned_undo_one<V>(tl.y + threadIdx.x, lfix, ch, aty, dc, l, u, eps_abs, lh, uh))
        atomicAdd(&count[2 * tl.x + 1], 1u);
}

hipError_t batch_record_history(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    if (s->fp32)
        hipLaunchKernelGGL((kb_record_history<float>), dim3(b->n_rn), dim3(kBlock), 0, s->stream, b->rn, s->n, b->sts,
                           (const double *)s->xp, s->ch, (const float *)s->lh, (const float *)s->uh, s->aty, s->hx,
                           s->hz);
    else
        hipLaunchKernelGGL((kb_record_history<double>), dim3(b->n_rn), dim3(kBlock), 0, s->stream, b->rn, s->n,
                           b->sts, (const double *)s->xp, s->ch, (const double *)s->lh, (const double *)s->uh, s->aty,
                           s->hx, s->hz);
    return hipGetLastError();
}

hipError_t batch_compute_features(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    // z of every LP's candidate needs Ahat' y+ on all columns (float64 accumulation)
    if (s->fp32)
        spmv<float, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, (const float *)s->ahat_t,
                                            (const double *)s->yp, s->aty);
    else
        spmv<double, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, (const double *)s->ahat_t,
                                             (const double *)s->yp, s->aty);
    if (s->fp32)
        hipLaunchKernelGGL((kb_feat_raw<float>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, s->n, b->d_coff, b->sts,
                           (const double *)s->xp, s->ch, (const float *)s->lh, (const float *)s->uh, s->aty, s->tp,
                           (const float *)s->ahat_t, s->hx, s->hz, s->dc, b->seeds, s->p.push_obj_scale, s->feat_raw,
                           b->fpart, b->n_rn);
    else
        hipLaunchKernelGGL((kb_feat_raw<double>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, s->n, b->d_coff, b->sts,
                           (const double *)s->xp, s->ch, (const double *)s->lh, (const double *)s->uh, s->aty, s->tp,
                           (const double *)s->ahat_t, s->hx, s->hz, s->dc, b->seeds, s->p.push_obj_scale,
                           s->feat_raw, b->fpart, b->n_rn);
    hipLaunchKernelGGL(kb_feat_scale, dim3(b->count), dim3(kBlock), 0, st, b->rn_start, b->d_coff, b->fpart, b->n_rn,
                       b->fscale);
    hipLaunchKernelGGL(kb_feat_norm, dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, b->fscale, s->feat_raw, s->feat_b);
    return hipGetLastError();
}

hipError_t batch_learned_fix(pdhg_batch *b, double theta)
{
    pdhg_solver *s = b->s;
    const float tl = (float)log(theta / (1.0 - theta)); // probability >= theta <=> logit >= tl
    if (s->fp32)
        hipLaunchKernelGGL((kb_learned_fix<float>), dim3(b->n_rn), dim3(kBlock), 0, s->stream, b->rn, b->active,
                           s->logits, tl, s->zsol, s->p.eps_abs, s->l, s->u, s->dc, (const double *)s->xs,
                           (float *)s->lh, (float *)s->uh, (float *)s->x, (double *)s->xa, s->lfix, s->lcount);
    else
        hipLaunchKernelGGL((kb_learned_fix<double>), dim3(b->n_rn), dim3(kBlock), 0, s->stream, b->rn, b->active,
                           s->logits, tl, s->zsol, s->p.eps_abs, s->l, s->u, s->dc, (const double *)s->xs,
                           (double *)s->lh, (double *)s->uh, (double *)s->x, (double *)s->xa, s->lfix, s->lcount);
    return hipGetLastError();
}

hipError_t batch_learned_undo(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    if (s->fp32)
        hipLaunchKernelGGL((kb_learned_undo<float>), dim3(b->n_rn), dim3(kBlock), 0, s->stream, b->rn, s->lfix, s->ch,
                           s->aty, s->dc, s->l, s->u, s->p.eps_abs, (float *)s->lh, (float *)s->uh, s->lcount);
    else
        hipLaunchKernelGGL((kb_learned_undo<double>), dim3(b->n_rn), dim3(kBlock), 0, s->stream, b->rn, s->lfix,
                           s->ch, s->aty, s->dc, s->l, s->u, s->p.eps_abs, (double *)s->lh, (double *)s->uh,
                           s->lcount);
    return hipGetLastError();
}

} // namespace pdhg
