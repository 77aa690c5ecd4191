// Batch engine: many independent LPs of uneven sizes solved and corner-pushed
// together.  The LPs form one block-diagonal model with global indices; each
// half-iteration is a single launch over instance-aligned row tiles of every
// LP, so the whole chip works on all LPs at once and large and small ones
// balance without any barrier between workgroups.  Every LP keeps its own
// DevState (step sizes, Halpern counter, restart state, done flag), its own
// scaling, step size and checks; checks reduce per-tile partial sums of each
// LP in a fixed order, so an LP's trajectory does not depend on the others.
#include <cmath>

#include <algorithm>
#include <vector>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"
#include "pdhg_kernels.hpp"

namespace pdhg {

constexpr int kRedRows = kBlock; // rows per reduction tile (one per thread)

// ------------------------------------------------------------ iteration ---
template <typename V, int T, int NT>
__global__ __launch_bounds__(NT) void kb_primal(const int4 *__restrict__ tiles, const int *__restrict__ tp,
                                               const int *__restrict__ ti, const V *__restrict__ atv,
                                               const double *__restrict__ y, const double *__restrict__ ch,
                                               const V *__restrict__ lh, const V *__restrict__ uh,
                                               V *__restrict__ x, const double *__restrict__ xa, V *__restrict__ xbar,
                                               double *__restrict__ xp, const DevState *__restrict__ sts, int i,
                                               int store_cand)
{
    __shared__ int s_ptr[T + 1];
    __shared__ double s_prod[kTileU * NT];
    __shared__ double s_sum[T];
    const int4 tl = tiles[xcd_range_block(blockIdx.x, gridDim.x)];
    const DevState *st = sts + tl.x;
    if (st->done) return;
    const int r0 = tl.y, rows = tl.z;
    const int tid = threadIdx.x;
    const bool mine = tid < rows;
    const int j = r0 + tid;
    double xj = 0, cj = 0, lo = 0, hi = 0, aj = 0;
    if (mine) {
        aj = xa[j];
        xj = iterate_value<V>(x[j], aj);
        cj = ch[j];
        lo = (double)lh[j];
        hi = (double)uh[j];
    }
    tile_row_sums<V, double, T, NT>(r0, rows, tp, ti, atv, y, s_ptr, s_prod, s_sum);
    if (!mine) return;
    primal_update<V>(j, s_sum[tid], xj, cj, lo, hi, aj, x, xbar, xp, st, i, store_cand);
}

template <typename V, int T, int NT>
__global__ __launch_bounds__(NT) void kb_dual(const int4 *__restrict__ tiles, const int *__restrict__ rp,
                                             const int *__restrict__ ci, const V *__restrict__ av,
                                             const V *__restrict__ xbar, const double *__restrict__ bh,
                                             const int8_t *__restrict__ sense, double *__restrict__ y,
                                             const double *__restrict__ ya, double *__restrict__ yp,
                                             const DevState *__restrict__ sts, int i, int store_cand)
{
    __shared__ int s_ptr[T + 1];
    __shared__ double s_prod[kTileU * NT];
    __shared__ double s_sum[T];
    const int4 tl = tiles[xcd_range_block(blockIdx.x, gridDim.x)];
    const DevState *st = sts + tl.x;
    if (st->done) return;
    const int r0 = tl.y, rows = tl.z;
    const int tid = threadIdx.x;
    const bool mine = tid < rows;
    const int r = r0 + tid;
    double yr = 0, br = 0, ar = 0;
    int8_t sn = '=';
    if (mine) {
        yr = y[r];
        br = bh[r];
        ar = ya[r];
        sn = sense[r];
    }
    tile_row_sums<V, V, T, NT>(r0, rows, rp, ci, av, xbar, s_ptr, s_prod, s_sum);
    if (!mine) return;
    dual_update(r, s_sum[tid], yr, br, ar, sn, y, yp, st, i, store_cand);
}

template <typename V>
static void launch_primal_b(pdhg_batch *b, int i, int store, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    pdhg_solver *s = b->s;
#define PDHG_BP_CASE(TT, RR, NT)                                                                               \
    case TT:                                                                                                   \
        PDHG_LAUNCH(e0, e1, (kb_primal<V, RR, NT>), dim3(b->n_ptiles), dim3(NT), s->stream, b->ptiles, s->tp, \
                           s->ti, (const V *)s->ahat_t, (const double *)s->y, s->chc,                         \
                           (const V *)s->lh, (const V *)s->uh, (V *)s->x, (const double *)s->xa, (V *)s->xbar,\
                           (double *)s->xp, b->sts, i, store);                                                \
        break;
    switch (-b->kern_at) {
        PDHG_BP_CASE(32, 32, 256)
        PDHG_BP_CASE(128, 128, 256)
        PDHG_BP_CASE(256, 256, 256)
        PDHG_BP_CASE(1032, 32, 64)
        PDHG_BP_CASE(1064, 64, 64)
    default:
        PDHG_BP_CASE(64, 64, 256)
    }
#undef PDHG_BP_CASE
}

template <typename V>
static void launch_dual_b(pdhg_batch *b, int i, int store, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    pdhg_solver *s = b->s;
#define PDHG_BD_CASE(TT, RR, NT)                                                                               \
    case TT:                                                                                                   \
        PDHG_LAUNCH(e0, e1, (kb_dual<V, RR, NT>), dim3(b->n_dtiles), dim3(NT), s->stream, b->dtiles, s->rp,   \
                           s->ci, (const V *)s->ahat, (const V *)s->xbar, (const double *)s->bhc, s->sense,    \
                           (double *)s->y, (const double *)s->ya, (double *)s->yp, b->sts, i, store);         \
        break;
    switch (-b->kern_a) {
        PDHG_BD_CASE(32, 32, 256)
        PDHG_BD_CASE(128, 128, 256)
        PDHG_BD_CASE(256, 256, 256)
        PDHG_BD_CASE(1032, 32, 64)
        PDHG_BD_CASE(1064, 64, 64)
    default:
        PDHG_BD_CASE(64, 64, 256)
    }
#undef PDHG_BD_CASE
}

// ---------------------------------------------------------------- checks ---
// ex / ety (mixed mode, else NULL): the rounding error's products, added to
// ax / aty to give the float64 products, which are written back
__global__ __launch_bounds__(kBlock) void kb_check_rows(const int4 *__restrict__ rm, double *__restrict__ ax,
                                                       const double *__restrict__ ex,
                                                       const double *__restrict__ bh, const int8_t *__restrict__ sense,
                                                       const double *__restrict__ dr, const double *__restrict__ yc,
                                                       const double *__restrict__ ya, double *__restrict__ part,
                                                       int ntile, const DevState *__restrict__ sts)
{
    const int4 tl = rm[blockIdx.x];
    if (sts[tl.x].done) return;
    double v[6] = {0, 0, 0, 0, 0, 0}; // PH2, P2, PINF, BTY, DY2, NAN
    if ((int)threadIdx.x < tl.z) {
        const int i = tl.y + threadIdx.x;
        double axi = ax[i];
        if (ex) {
            axi += ex[i];
            ax[i] = axi;
        }
        double r = bh[i] - axi;
        const int8_t s = sense[i];
        if (s == '<') r = r < 0.0 ? r : 0.0;
        else if (s == '>') r = r > 0.0 ? r : 0.0;
        else if (s == 'N') r = 0.0; // dropped by the dual push
        const double ru = r / dr[i];
        const double yi = yc[i];
        const double dy = yi - ya[i];
        v[0] = r * r;
        v[1] = ru * ru;
        v[2] = fabs(ru);
        v[3] = bh[i] * yi;
        v[4] = dy * dy;
        v[5] = isfinite(yi) ? 0.0 : 1.0;
    }
    block_reduce<6>(v, 1u << 2);
    if (threadIdx.x == 0) {
        part[Q_PH2 * ntile + blockIdx.x] = v[0];
        part[Q_P2 * ntile + blockIdx.x] = v[1];
        part[Q_PINF * ntile + blockIdx.x] = v[2];
        part[Q_BTY * ntile + blockIdx.x] = v[3];
        part[Q_DY2 * ntile + blockIdx.x] = v[4];
        part[Q_NAN * ntile + blockIdx.x] = v[5];
    }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void kb_check_cols(const int4 *__restrict__ rn, double *__restrict__ aty,
                                                       const double *__restrict__ ety,
                                                       const double *__restrict__ ch, const V *__restrict__ lh,
                                                       const V *__restrict__ uh, const double *__restrict__ dc,
                                                       const double *__restrict__ xc, const double *__restrict__ xa,
                                                       const double *__restrict__ c0, const double *__restrict__ l0,
                                                       const double *__restrict__ u0, int orig,
                                                       double *__restrict__ part, int ntile,
                                                       const DevState *__restrict__ sts)
{
    const int4 tl = rn[blockIdx.x];
    if (sts[tl.x].done) return;
    double v[7] = {0, 0, 0, 0, 0, 0, 0}; // DH2, D2, DINF, CTX, BND, DX2, NAN
    if ((int)threadIdx.x < tl.z) {
        const int j = tl.y + threadIdx.x;
        double cj, lo, hi;
        check_model<V>(orig != 0, j, ch, lh, uh, c0, l0, u0, dc, cj, lo, hi);
        double atyj = aty[j];
        if (ety) {
            atyj += ety[j];
            aty[j] = atyj;
        }
        const double lam = cj - atyj;
        const double zp = (!is_inf_lo(lo) && lam > 0.0) ? lam : 0.0;
        const double zm = (!is_inf_up(hi) && lam < 0.0) ? -lam : 0.0;
        const double rd = lam - (zp - zm);
        const double rdu = rd / dc[j];
        const double xj = xc[j];
        const double dx = xj - xa[j];
        v[0] = rd * rd;
        v[1] = rdu * rdu;
        v[2] = fabs(rdu);
        v[3] = cj * xj;
        if (zp > 0.0) v[4] += lo * zp;
        if (zm > 0.0) v[4] -= hi * zm;
        v[5] = dx * dx;
        v[6] = isfinite(xj) ? 0.0 : 1.0;
    }
    block_reduce<7>(v, 1u << 2);
    if (threadIdx.x == 0) {
        part[Q_DH2 * ntile + blockIdx.x] = v[0];
        part[Q_D2 * ntile + blockIdx.x] = v[1];
        part[Q_DINF * ntile + blockIdx.x] = v[2];
        part[Q_CTX * ntile + blockIdx.x] = v[3];
        part[Q_BND * ntile + blockIdx.x] = v[4];
        part[Q_DX2 * ntile + blockIdx.x] = v[5];
        part[Q_COUNT * ntile + blockIdx.x] = v[6];
    }
}

// one workgroup per LP: its tiles' partials in a fixed order, then decide
__global__ __launch_bounds__(kBlock) void kb_check_final(DevState *__restrict__ sts, const double *__restrict__ pm,
                                                        int ntm, const double *__restrict__ pn, int ntn,
                                                        const int *__restrict__ rm_start,
                                                        const int *__restrict__ rn_start, int mode, int len)
{
    DevState *st = sts + blockIdx.x;
    if (st->done) return;
    const int m0 = rm_start[blockIdx.x], m1 = rm_start[blockIdx.x + 1];
    const int n0 = rn_start[blockIdx.x], n1 = rn_start[blockIdx.x + 1];
    double v[Q_COUNT + 1];
    fold_check_partials(v, pm, (size_t)ntm, m0, m1, pn, (size_t)ntn, n0, n1);
    block_reduce<Q_COUNT + 1>(v, (1u << Q_PINF) | (1u << Q_DINF));
    if (threadIdx.x == 0) check_decide(st, v, mode, len);
}

// restart copies per tile: column tiles first, then row tiles (mixed mode:
// the stored difference x - x_a becomes 0)
template <typename V>
__global__ __launch_bounds__(kBlock) void kb_restart_apply(const int4 *__restrict__ rn, int ntn,
                                                          const int4 *__restrict__ rm,
                                                          const DevState *__restrict__ sts, V *__restrict__ x,
                                                          double *__restrict__ xa, const double *__restrict__ xp,
                                                          double *__restrict__ y, double *__restrict__ ya,
                                                          const double *__restrict__ yp)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    const bool col = (int)blockIdx.x < ntn;
    const int4 tl = col ? rn[blockIdx.x] : rm[blockIdx.x - ntn];
    const DevState *st = sts + tl.x;
    if (!st->restart_flag || st->done) return;
    if ((int)threadIdx.x >= tl.z) return;
    const int k = tl.y + threadIdx.x;
    if (col) {
        const double v = xp[k];
        x[k] = delta ? (V)0 : (V)v;
        xa[k] = v;
    } else {
        const double v = yp[k];
        y[k] = v;
        ya[k] = v;
    }
}

// Anchored objective and right-hand side per LP (mixed mode): chc = ch -
// (pa + pb), bhc = bh - (qa + qb) with pa + pb = E' y_a and qa + qb = Ahat
// x_a in float64 (pb, qb may be NULL; qa may be the output), for every LP
// that restarted at this check (the check left E' y+ in ety and the float64
// Ahat x+ in ax), or for every LP with `always` (a phase start); column
// tiles, then row tiles.
__global__ __launch_bounds__(kBlock) void kb_defect_set(const int4 *__restrict__ rn, int ntn,
                                                       const int4 *__restrict__ rm,
                                                       const DevState *__restrict__ sts, int always,
                                                       const double *ch, const double *pa, const double *pb,
                                                       double *chc, const double *bh, const double *qa,
                                                       const double *qb, double *bhc)
{
    const bool col = (int)blockIdx.x < ntn;
    const int4 tl = col ? rn[blockIdx.x] : rm[blockIdx.x - ntn];
    const DevState *st = sts + tl.x;
    if (!always && (!st->restart_flag || st->done)) return;
    if ((int)threadIdx.x >= tl.z) return;
    const int k = tl.y + threadIdx.x;
    if (col) chc[k] = ch[k] - (pb ? pa[k] + pb[k] : pa[k]);
    else bhc[k] = bh[k] - (qb ? qa[k] + qb[k] : qa[k]);
}

__global__ void kb_advance(DevState *sts, int count, int len)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || sts[i].done) return;
    sts[i].t += len;
    sts[i].k0 += len;
}

// products over the iteration tiles, skipping the LPs that have stopped:
// by their DevState (checks) or by a per-LP flag (power iteration, skip[lp])
template <typename VM, typename VV, int T, int NT>
__global__ __launch_bounds__(NT) void kb_spmv(const int4 *__restrict__ tiles, const int *__restrict__ ptr,
                                             const int *__restrict__ idx, const VM *__restrict__ val,
                                             const VV *__restrict__ vec, double *__restrict__ out,
                                             const DevState *__restrict__ sts, const double *__restrict__ skip)
{
    __shared__ int s_ptr[T + 1];
    __shared__ double s_prod[kTileU * NT];
    __shared__ double s_sum[T];
    const int4 tl = tiles[xcd_range_block(blockIdx.x, gridDim.x)];
    if (sts ? sts[tl.x].done != 0 : skip[tl.x] != 0.0) return; // uniform over the workgroup
    tile_row_sums<VM, VV, T, NT>(tl.y, tl.z, ptr, idx, val, vec, s_ptr, s_prod, s_sum);
    if ((int)threadIdx.x < tl.z) out[tl.y + threadIdx.x] = s_sum[threadIdx.x];
}

template <typename VM, typename VV>
static void launch_spmv_b(pdhg_batch *b, int kern, const int4 *tiles, int ntiles, const int *ptr, const int *idx,
                          const VM *val, const VV *vec, double *out, const double *skip = nullptr)
{
    if (ntiles <= 0) return;
    hipStream_t st = b->s->stream;
#define PDHG_BS_CASE(TT, RR, NT)                                                                               \
    case TT:                                                                                                   \
        hipLaunchKernelGGL((kb_spmv<VM, VV, RR, NT>), dim3(ntiles), dim3(NT), 0, st, tiles, ptr, idx, val, vec, \
                           out, skip ? nullptr : b->sts, skip);                                               \
        break;
    switch (-kern) {
        PDHG_BS_CASE(32, 32, 256)
        PDHG_BS_CASE(128, 128, 256)
        PDHG_BS_CASE(256, 256, 256)
        PDHG_BS_CASE(1032, 32, 64)
        PDHG_BS_CASE(1064, 64, 64)
    default:
        PDHG_BS_CASE(64, 64, 256)
    }
#undef PDHG_BS_CASE
}

template <typename V>
static void check_b(pdhg_batch *b, int mode, int len)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    // mode 0 checks the iterate at a phase start, where it is the anchor
    // (in the mixed mode x holds its difference from x_a, which is 0 there)
    const double *xc = (const double *)(mode ? s->xp : (s->fp32 ? s->xa : s->x));
    const double *yc = (const double *)(mode ? s->yp : s->y);
    launch_spmv_b<V, double>(b, b->kern_a, b->dtiles, b->n_dtiles, s->rp, s->ci, (const V *)s->ahat, xc, s->ax);
    launch_spmv_b<V, double>(b, b->kern_at, b->ptiles, b->n_ptiles, s->tp, s->ti, (const V *)s->ahat_t, yc, s->aty);
    if (s->aerr) { // mixed mode: the rounding error's products complete the float64 ones
        launch_spmv_b<float, double>(b, b->kern_a, b->dtiles, b->n_dtiles, s->rp, s->ci, (const float *)s->aerr, xc,
                                     s->ex);
        launch_spmv_b<float, double>(b, b->kern_at, b->ptiles, b->n_ptiles, s->tp, s->ti, (const float *)s->aerr_t,
                                     yc, s->ety);
    }
    double *pm = b->part, *pn = b->part + (size_t)(Q_COUNT + 1) * b->n_rm;
    hipLaunchKernelGGL(kb_check_rows, dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, s->ax,
                       (const double *)(s->aerr ? s->ex : nullptr), (const double *)s->bh, s->sense,
                       s->dr, yc, (const double *)s->ya, pm, b->n_rm, b->sts);
    hipLaunchKernelGGL((kb_check_cols<V>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, s->aty,
                       (const double *)(s->aerr ? s->ety : nullptr), s->ch,
                       (const V *)s->lh, (const V *)s->uh, s->dc, xc, (const double *)s->xa, s->c, s->l, s->u,
                       s->model_original ? 1 : 0, pn, b->n_rn, b->sts);
    hipLaunchKernelGGL(kb_check_final, dim3(b->count), dim3(kBlock), 0, st, b->sts, pm, b->n_rm, pn, b->n_rn,
                       b->rm_start, b->rn_start, mode, len);
    if (mode == 1 && s->hx) (void)batch_record_history(b); // before the restart copies
    if (mode == 2 && s->learned_active) (void)batch_learned_undo(b);
    if (mode != 0 && s->aerr) // the check left E' y+ in ety and Ahat x+ (float64) in ax
        hipLaunchKernelGGL(kb_defect_set, dim3(b->n_rn + b->n_rm), dim3(kBlock), 0, st, b->rn, b->n_rn, b->rm, b->sts, 0,
                           s->ch, (const double *)s->ety, (const double *)nullptr, s->chc, (const double *)s->bh,
                           (const double *)s->ax, (const double *)nullptr, s->bhc);
    if (mode != 0)
        hipLaunchKernelGGL((kb_restart_apply<V>), dim3(b->n_rn + b->n_rm), dim3(kBlock), 0, st, b->rn, b->n_rn, b->rm,
                           b->sts, (V *)s->x, (double *)s->xa, (const double *)s->xp, (double *)s->y, (double *)s->ya,
                           (const double *)s->yp);
}

hipError_t batch_iterations(pdhg_batch *b, int count, bool check_at_end, int mode, bool timed_launch)
{
    pdhg_solver *s = b->s;
    const int timed = (timed_launch && count >= 2) ? count / 2 : -1;
    for (int i = 0; i < count; i++) {
        const int store = (check_at_end && i == count - 1) ? 1 : 0;
        hipEvent_t *ev = i == timed ? s->ev : nullptr;
        if (s->fp32) launch_primal_b<float>(b, i, store, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
        else launch_primal_b<double>(b, i, store, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
        if (s->fp32) launch_dual_b<float>(b, i, store, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
        else launch_dual_b<double>(b, i, store, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (check_at_end) {
        if (s->fp32) check_b<float>(b, mode, count);
        else check_b<double>(b, mode, count);
    } else {
        hipLaunchKernelGGL(kb_advance, dim3((b->count + 255) / 256), dim3(256), 0, s->stream, b->sts, b->count, count);
    }
    return hipGetLastError();
}

hipError_t batch_capture_cycle(pdhg_batch *b, int len, int mode)
{
    if (b->graph && b->graph_len == len && b->graph_mode == mode) return hipSuccess;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t el = batch_iterations(b, len, true, mode, false);
    e = hipStreamEndCapture(b->s->stream, &g);
    if (el != hipSuccess) return el;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    b->graph_len = len;
    b->graph_mode = mode;
    return hipSuccess;
}

// ---------------------------------------------------- per-LP reductions ---
// partial sum of squares of a vector over one reduction tile
template <typename T>
__global__ __launch_bounds__(kBlock) void kb_sumsq(const int4 *__restrict__ tiles, const T *__restrict__ v,
                                                  double *__restrict__ part)
{
    const int4 tl = tiles[blockIdx.x];
    double q[1] = {0.0};
    if ((int)threadIdx.x < tl.z) {
        const double a = (double)v[tl.y + threadIdx.x];
        q[0] = a * a;
    }
    block_reduce<1>(q, 0u);
    if (threadIdx.x == 0) part[blockIdx.x] = q[0];
}

// per-LP power step (the single-LP rule): ps = {lambda[count], done[count],
// steps[count]}; rho = u'u from the LP's row tiles, w'w from its column tiles
__global__ __launch_bounds__(kBlock) void kb_power_finish(const int *__restrict__ rm_start,
                                                         const double *__restrict__ pm,
                                                         const int *__restrict__ rn_start,
                                                         const double *__restrict__ pn, int count, double tol,
                                                         double *__restrict__ ps)
{
    const int lp = blockIdx.x;
    if (ps[count + lp] != 0.0) return;
    double q[2] = {0.0, 0.0};
    for (int t = rm_start[lp] + threadIdx.x; t < rm_start[lp + 1]; t += kBlock) q[0] += pm[t];
    for (int t = rn_start[lp] + threadIdx.x; t < rn_start[lp + 1]; t += kBlock) q[1] += pn[t];
    block_reduce<2>(q, 0u);
    if (threadIdx.x == 0) {
        const double rho = q[0], ww = q[1], lam = sqrt(ww);
        ps[lp] = lam;
        ps[2 * count + lp] += 1.0;
        if (!(lam > 0.0) || sqrt(fmax(ww - rho * rho, 0.0)) <= tol * rho) ps[count + lp] = 1.0;
    }
}

// the power iteration's start on every column of an LP, numbered from the
// LP's first column (so an LP gets the start it gets when solved alone)
__global__ __launch_bounds__(kBlock) void kb_fill_start(const int4 *__restrict__ rn, const int *__restrict__ coff,
                                                       double *__restrict__ v)
{
    const int4 tl = rn[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    const int j = tl.y + threadIdx.x;
    v[j] = power_start(j - coff[tl.x]);
}

// ps[3 count + lp] = the LP's ||v|| from its column tiles' partials
__global__ __launch_bounds__(kBlock) void kb_start_norm(const int *__restrict__ rn_start, const double *__restrict__ pn,
                                                       int count, double *__restrict__ ps)
{
    const int lp = blockIdx.x;
    double q[1] = {0.0};
    for (int t = rn_start[lp] + threadIdx.x; t < rn_start[lp + 1]; t += kBlock) q[0] += pn[t];
    block_reduce<1>(q, 0u);
    if (threadIdx.x == 0) ps[3 * count + lp] = sqrt(q[0]);
}

__global__ __launch_bounds__(kBlock) void kb_div_start(const int4 *__restrict__ rn, const double *__restrict__ ps,
                                                      int count, double *__restrict__ v)
{
    const int4 tl = rn[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    const int j = tl.y + threadIdx.x;
    v[j] = v[j] / ps[3 * count + tl.x];
}

__global__ __launch_bounds__(kBlock) void kb_normalize(const int4 *__restrict__ rn, const double *__restrict__ w,
                                                      const double *__restrict__ ps, int count, double *__restrict__ v)
{
    const int4 tl = rn[blockIdx.x];
    const double l = ps[tl.x];
    if (ps[count + tl.x] != 0.0 || !(l > 0.0) || (int)threadIdx.x >= tl.z) return;
    const int j = tl.y + threadIdx.x;
    v[j] = w[j] / l;
}

__global__ void kb_set_step(DevState *sts, int count, const double *ps, double safety)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double l = ps[i];
    const double sig = (ps[2 * count + i] > 0.0 && l > 0.0) ? sqrt(l) : 0.0;
    sts[i].sigma_est = sig;
    sts[i].eta = sig > 1e-12 ? safety / sig : safety;
}

// per LP: 1 + ||b||, 1 + ||c|| from row-tile and column-tile partials
__global__ __launch_bounds__(kBlock) void kb_set_norms(DevState *__restrict__ sts, const double *__restrict__ pm,
                                                      const double *__restrict__ pn, const int *__restrict__ rm_start,
                                                      const int *__restrict__ rn_start)
{
    double q[2] = {0.0, 0.0};
    for (int t = rn_start[blockIdx.x] + threadIdx.x; t < rn_start[blockIdx.x + 1]; t += kBlock) q[0] += pn[t];
    for (int t = rm_start[blockIdx.x] + threadIdx.x; t < rm_start[blockIdx.x + 1]; t += kBlock) q[1] += pm[t];
    block_reduce<2>(q, 0u);
    if (threadIdx.x != 0) return;
    sts[blockIdx.x].nc1 = 1.0 + sqrt(q[0]);
    sts[blockIdx.x].nb1 = 1.0 + sqrt(q[1]);
}

// per LP: omega = ||chat|| / ||bhat|| and a fresh restart state; LPs that do
// not take part in the phase are parked as done
__global__ __launch_bounds__(kBlock) void kb_phase_start(DevState *__restrict__ sts, const double *__restrict__ pm,
                                                        const double *__restrict__ pn, const int *__restrict__ rm_start,
                                                        const int *__restrict__ rn_start, const int *__restrict__ active)
{
    double q[2] = {0.0, 0.0};
    for (int t = rn_start[blockIdx.x] + threadIdx.x; t < rn_start[blockIdx.x + 1]; t += kBlock) q[0] += pn[t];
    for (int t = rm_start[blockIdx.x] + threadIdx.x; t < rm_start[blockIdx.x + 1]; t += kBlock) q[1] += pm[t];
    block_reduce<2>(q, 0u);
    if (threadIdx.x != 0) return;
    DevState *st = sts + blockIdx.x;
    st->restart_flag = 0;
    if (!active[blockIdx.x]) {
        st->done = 1;
        return;
    }
    const double nc = sqrt(q[0]), nb = sqrt(q[1]);
    const double om = (nc > 1e-10 && nb > 1e-10) ? nc / nb : 1.0;
    st->omega = om;
    st->tau = st->eta / om;
    st->sigma = st->eta * om;
    st->k0 = 0;
    st->t = 0;
    st->restarts = 0;
    st->done = 0;
    st->status = PDHG_ITER_LIMIT;
    st->checks = 0;
}

hipError_t batch_setup(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    double *pm = b->part, *pn = b->part + (size_t)(Q_COUNT + 1) * b->n_rm;
    // 1 + ||b||, 1 + ||c|| per LP
    hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, s->b, pm);
    hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, s->c, pn);
    hipLaunchKernelGGL(kb_set_norms, dim3(b->count), dim3(kBlock), 0, st, b->sts, pm, pn, b->rm_start, b->rn_start);
    // power iteration per LP on its block of Ahat'Ahat
    double *v = s->xu, *w = s->zsol, *u = s->ax; // float64 work vectors of the right lengths
    hipMemsetAsync(b->lp_scalar, 0, sizeof(double) * 4 * (size_t)b->count, st);
    if (b->n_rn > 0) { // start: v = (1 + U) / ||1 + U|| per LP, the norm in lp_scalar[3 count + lp]
        hipLaunchKernelGGL(kb_fill_start, dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, b->d_coff, v);
        hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, v, pn);
        hipLaunchKernelGGL(kb_start_norm, dim3(b->count), dim3(kBlock), 0, st, b->rn_start, pn, b->count, b->lp_scalar);
        hipLaunchKernelGGL(kb_div_start, dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, b->lp_scalar, b->count, v);
    }
    std::vector<double> done((size_t)b->count, 0.0);
    constexpr int kPowerBatch = 32; // steps launched between reads of the done flags
    for (int it = 0; it < s->p.power_iters && s->m > 0 && s->n > 0; it += kPowerBatch) {
        const int len = std::min(kPowerBatch, s->p.power_iters - it);
        for (int k = 0; k < len; k++) {
            const double *pdone = b->lp_scalar + b->count; // LPs whose power iteration has stopped
            if (s->fp32) {
                launch_spmv_b<float, double>(b, b->kern_a, b->dtiles, b->n_dtiles, s->rp, s->ci,
                                             (const float *)s->ahat, v, u, pdone);
                launch_spmv_b<float, double>(b, b->kern_at, b->ptiles, b->n_ptiles, s->tp, s->ti,
                                             (const float *)s->ahat_t, u, w, pdone);
            } else {
                launch_spmv_b<double, double>(b, b->kern_a, b->dtiles, b->n_dtiles, s->rp, s->ci,
                                              (const double *)s->ahat, v, u, pdone);
                launch_spmv_b<double, double>(b, b->kern_at, b->ptiles, b->n_ptiles, s->tp, s->ti,
                                              (const double *)s->ahat_t, u, w, pdone);
            }
            hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, u, pm);
            hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, w, pn);
            hipLaunchKernelGGL(kb_power_finish, dim3(b->count), dim3(kBlock), 0, st, b->rm_start, pm, b->rn_start, pn,
                               b->count, s->p.power_tol, b->lp_scalar);
            hipLaunchKernelGGL(kb_normalize, dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, w, b->lp_scalar, b->count, v);
        }
        hipError_t e = hipMemcpyAsync(done.data(), b->lp_scalar + b->count, sizeof(double) * done.size(),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (std::all_of(done.begin(), done.end(), [](double d) { return d != 0.0; })) break;
    }
    hipLaunchKernelGGL(kb_set_step, dim3((b->count + 255) / 256), dim3(256), 0, st, b->sts, b->count, b->lp_scalar,
                       s->p.eta_safety);
    return hipGetLastError();
}

template <typename V>
static hipError_t phase_begin_b(pdhg_batch *b, bool fresh)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    hipError_t e = launch_start_vectors(s, fresh);
    if (e != hipSuccess) return e;
    double *pm = b->part, *pn = b->part + (size_t)(Q_COUNT + 1) * b->n_rm;
    hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, s->ch, pn);
    hipLaunchKernelGGL((kb_sumsq<double>), dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, (const double *)s->bh, pm);
    hipLaunchKernelGGL(kb_phase_start, dim3(b->count), dim3(kBlock), 0, st, b->sts, pm, pn, b->rm_start, b->rn_start,
                       b->active);
    check_b<V>(b, 0, 0); // anchor KKT parts of every LP's start point
    return hipGetLastError();
}

// mixed mode: every LP's anchored data at its current anchor
hipError_t batch_defect_refresh(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    s->defect_stale = false;
    if (!s->aerr) {
        defect_alias(s);
        return hipSuccess;
    }
    // the LPs taking part in the phase (the tiles skip the others): fl32(Ahat)
    // x_a into bhc, E x_a into ex, E' y_a into ety
    const double *xa = (const double *)s->xa, *ya = (const double *)s->ya;
    launch_spmv_b<float, double>(b, b->kern_a, b->dtiles, b->n_dtiles, s->rp, s->ci, (const float *)s->ahat, xa,
                                 s->bhc);
    launch_spmv_b<float, double>(b, b->kern_a, b->dtiles, b->n_dtiles, s->rp, s->ci, (const float *)s->aerr, xa, s->ex);
    launch_spmv_b<float, double>(b, b->kern_at, b->ptiles, b->n_ptiles, s->tp, s->ti, (const float *)s->aerr_t, ya,
                                 s->ety);
    hipLaunchKernelGGL(kb_defect_set, dim3(b->n_rn + b->n_rm), dim3(kBlock), 0, s->stream, b->rn, b->n_rn, b->rm,
                       b->sts, 1, s->ch, (const double *)s->ety, (const double *)nullptr, s->chc,
                       (const double *)s->bh, (const double *)s->bhc, (const double *)s->ex, s->bhc);
    return hipGetLastError();
}

hipError_t batch_phase_begin(pdhg_batch *b, bool fresh)
{
    b->s->defect_stale = true;
    return b->s->fp32 ? phase_begin_b<float>(b, fresh) : phase_begin_b<double>(b, fresh);
}

// --------------------------------------------------------- KKT reports ---
__global__ __launch_bounds__(kBlock) void kb_report_rows(const int4 *__restrict__ rm, const double *__restrict__ bv,
                                                        const int8_t *__restrict__ s0, const double *__restrict__ ax,
                                                        const double *__restrict__ y, double *__restrict__ part,
                                                        int ntile)
{
    const int4 tl = rm[blockIdx.x];
    const double tol = 1e-6;
    double v[6] = {0, 0, 0, 0, 0, 0}; // P2, PINF, BTY, POFF, DZERO, CAND
    if ((int)threadIdx.x < tl.z) {
        const int i = tl.y + threadIdx.x;
        double r = bv[i] - ax[i];
        const int8_t sn = s0[i];
        if (sn == '<') r = r < 0.0 ? r : 0.0;
        else if (sn == '>') r = r > 0.0 ? r : 0.0;
        v[0] = r * r;
        v[1] = fabs(r);
        v[2] = bv[i] * y[i];
        if (sn != '=') {
            const double slack = (sn == '<') ? (bv[i] - ax[i]) : (ax[i] - bv[i]);
            const double zs = (sn == '<') ? -y[i] : y[i];
            const bool off = slack > tol;
            v[3] = off ? 1.0 : 0.0;
            v[4] = fabs(zs) <= tol ? 1.0 : 0.0;
            v[5] = (off && fabs(zs) < tol) ? 1.0 : 0.0;
        }
    }
    block_reduce<6>(v, 1u << 1);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; q++) part[q * ntile + blockIdx.x] = v[q];
}

__global__ __launch_bounds__(kBlock) void kb_report_cols(const int4 *__restrict__ rn, const double *__restrict__ c,
                                                        const double *__restrict__ l, const double *__restrict__ u,
                                                        const double *__restrict__ aty, const double *__restrict__ x,
                                                        double *__restrict__ zout, double *__restrict__ part,
                                                        int ntile)
{
    const int4 tl = rn[blockIdx.x];
    const double tol = 1e-6;
    double v[7] = {0, 0, 0, 0, 0, 0, 0}; // D2, DINF, CTX, BND, POFF, DZERO, CAND
    if ((int)threadIdx.x < tl.z) {
        const int j = tl.y + threadIdx.x;
        const double lam = c[j] - aty[j];
        const double zp = (!is_inf_lo(l[j]) && lam > 0.0) ? lam : 0.0;
        const double zm = (!is_inf_up(u[j]) && lam < 0.0) ? -lam : 0.0;
        const double z = zp - zm;
        const double rd = lam - z;
        v[0] = rd * rd;
        v[1] = fabs(rd);
        v[2] = c[j] * x[j];
        if (zp > 0.0) v[3] += l[j] * zp;
        if (zm > 0.0) v[3] -= u[j] * zm;
        const bool off = (x[j] - l[j] > tol) && (u[j] - x[j] > tol);
        v[4] = off ? 1.0 : 0.0;
        v[5] = fabs(z) <= tol ? 1.0 : 0.0;
        v[6] = (off && fabs(z) < tol) ? 1.0 : 0.0;
        if (zout) zout[j] = z;
    }
    block_reduce<7>(v, 1u << 1);
    if (threadIdx.x == 0)
        for (int q = 0; q < 7; q++) part[q * ntile + blockIdx.x] = v[q];
}

// per LP: out[lp * R_COUNT + r]
__global__ __launch_bounds__(kBlock) void kb_report_final(const double *__restrict__ pr, int ntm,
                                                         const double *__restrict__ pc, int ntn,
                                                         const int *__restrict__ rm_start,
                                                         const int *__restrict__ rn_start, double *__restrict__ out)
{
    const int m0 = rm_start[blockIdx.x], m1 = rm_start[blockIdx.x + 1];
    const int n0 = rn_start[blockIdx.x], n1 = rn_start[blockIdx.x + 1];
    double v[13];
#pragma unroll
    for (int q = 0; q < 6; q++) {
        double acc = 0.0;
        for (int t = m0 + threadIdx.x; t < m1; t += kBlock)
            acc = (q == 1) ? fmax(acc, pr[q * ntm + t]) : acc + pr[q * ntm + t];
        v[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < 7; q++) {
        double acc = 0.0;
        for (int t = n0 + threadIdx.x; t < n1; t += kBlock)
            acc = (q == 1) ? fmax(acc, pc[q * ntn + t]) : acc + pc[q * ntn + t];
        v[6 + q] = acc;
    }
    block_reduce<13>(v, (1u << 1) | (1u << 7));
    if (threadIdx.x != 0) return;
    double *o = out + (size_t)blockIdx.x * R_COUNT;
    o[R_P2] = v[0];
    o[R_PINF] = v[1];
    o[R_BTY] = v[2];
    o[R_D2] = v[6];
    o[R_DINF] = v[7];
    o[R_CTX] = v[8];
    o[R_BND] = v[9];
    o[R_POFF] = v[3] + v[10];
    o[R_DZERO] = v[4] + v[11];
    o[R_CAND] = v[5] + v[12];
}

hipError_t batch_report(pdhg_batch *b, const double *x, const double *y, double *z, pdhg_kkt_report *out)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    spmv<double, double, double, double>(st, s->lanes_a, s->m, s->rp, s->ci, s->av, x, s->ax);
    spmv<double, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, s->atv, y, s->aty);
    double *pr = b->part, *pc = b->part + (size_t)(Q_COUNT + 1) * b->n_rm;
    hipLaunchKernelGGL(kb_report_rows, dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, s->b, s->sense0, s->ax, y, pr, b->n_rm);
    hipLaunchKernelGGL(kb_report_cols, dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, s->c, s->l, s->u, s->aty, x, z, pc,
                       b->n_rn);
    hipLaunchKernelGGL(kb_report_final, dim3(b->count), dim3(kBlock), 0, st, pr, b->n_rm, pc, b->n_rn, b->rm_start,
                       b->rn_start, b->rep);
    hipMemcpyAsync(b->rep_host, b->rep, sizeof(double) * R_COUNT * (size_t)b->count, hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(b->sts_host, b->sts, sizeof(DevState) * (size_t)b->count, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < b->count; i++) {
        const double *v = b->rep_host + (size_t)i * R_COUNT;
        pdhg_kkt_report *k = out + i;
        const int64_t mi = b->roff[i + 1] - b->roff[i];
        k->rp2 = sqrt(v[R_P2]);
        k->rd2 = sqrt(v[R_D2]);
        k->rpinf = v[R_PINF];
        k->rdinf = v[R_DINF];
        k->pobj = v[R_CTX];
        k->dobj = v[R_BTY] + v[R_BND];
        k->gap = k->pobj - k->dobj;
        k->rel_p = k->rp2 / b->sts_host[i].nb1;
        k->rel_d = k->rd2 / b->sts_host[i].nc1;
        k->rel_gap = fabs(k->gap) / (1.0 + fabs(k->pobj) + fabs(k->dobj));
        k->p_off = (int64_t)v[R_POFF];
        k->d_zero = (int64_t)v[R_DZERO];
        k->candidates = (int64_t)v[R_CAND];
        k->est_primal = k->p_off > mi ? k->p_off - mi : 0;
        k->est_dual = mi > k->d_zero ? mi - k->d_zero : 0;
    }
    return hipGetLastError();
}

// --------------------------------------------------------------- push ---
template <typename V>
__global__ __launch_bounds__(kBlock) void kb_push_cols(const int4 *__restrict__ rn, const int *__restrict__ coff,
                                                      const int *__restrict__ active, const double *__restrict__ z,
                                                      const double *__restrict__ xs, const double *__restrict__ dc,
                                                      double eps_abs, const uint64_t *__restrict__ seeds, double scale,
                                                      V *__restrict__ lh, V *__restrict__ uh, double *__restrict__ ch,
                                                      V *__restrict__ x, double *__restrict__ xa,
                                                      double *__restrict__ part, int ntile)
{
    const int4 tl = rn[blockIdx.x];
    double v[2] = {0.0, 0.0};
    if (active[tl.x] && (int)threadIdx.x < tl.z) {
        const int j = tl.y + threadIdx.x;
        const int64_t jl = j - coff[tl.x]; // column number inside its LP
        const double xv = xs[j];
        if (z[j] > eps_abs) {
            uh[j] = (V)xv;
            v[1] = 1.0;
        } else if (z[j] < -eps_abs) {
            lh[j] = (V)xv;
            v[0] = 1.0;
        }
        ch[j] = dc[j] * (scale * push_unit(seeds[tl.x], jl));
        set_iterate<V>(j, xv, x, xa); // the solve's x
    }
    block_reduce<2>(v, 0u);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[ntile + blockIdx.x] = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void kb_push_rows(const int4 *__restrict__ rm, const int *__restrict__ active,
                                                      const double *__restrict__ yu, double eps_abs,
                                                      int8_t *__restrict__ sense, double *__restrict__ y,
                                                      double *__restrict__ part)
{
    const int4 tl = rm[blockIdx.x];
    double v[1] = {0.0};
    if (active[tl.x] && (int)threadIdx.x < tl.z) {
        const int i = tl.y + threadIdx.x;
        const int8_t sn = sense[i];
        if ((sn == '<' && yu[i] < -eps_abs) || (sn == '>' && yu[i] > eps_abs)) {
            sense[i] = '=';
            v[0] = 1.0;
        }
        y[i] = 0.0;
    }
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void kb_push_final(const double *__restrict__ pn, int ntn,
                                                       const double *__restrict__ pm, const int *__restrict__ rm_start,
                                                       const int *__restrict__ rn_start, double *__restrict__ out)
{
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = rn_start[blockIdx.x] + threadIdx.x; t < rn_start[blockIdx.x + 1]; t += kBlock) {
        v[0] += pn[t];
        v[1] += pn[ntn + t];
    }
    for (int t = rm_start[blockIdx.x] + threadIdx.x; t < rm_start[blockIdx.x + 1]; t += kBlock) v[2] += pm[t];
    block_reduce<3>(v, 0u);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; q++) out[(size_t)blockIdx.x * R_COUNT + q] = v[q];
}

template <typename V>
static hipError_t push_setup_b(pdhg_batch *b, pdhg_push_result *out, double theta)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    double *pm = b->part, *pn = b->part + (size_t)(Q_COUNT + 1) * b->n_rm;
    hipLaunchKernelGGL((kb_push_cols<V>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, b->d_coff, b->active, s->zsol,
                       (const double *)s->xs, s->dc, s->p.eps_abs, b->seeds, s->p.push_obj_scale, (V *)s->lh,
                       (V *)s->uh, s->ch, (V *)s->x, (double *)s->xa, pn, b->n_rn);
    hipLaunchKernelGGL(kb_push_rows, dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, b->active, s->yu, s->p.eps_abs,
                       s->sense, (double *)s->y, pm);
    if (theta > 0.0) { // learned warm start on the columns the plain rule leaves free
        hipError_t el = batch_learned_fix(b, theta);
        if (el != hipSuccess) return el;
    }
    hipLaunchKernelGGL(kb_push_final, dim3(b->count), dim3(kBlock), 0, st, pn, b->n_rn, pm, b->rm_start, b->rn_start,
                       b->rep);
    hipMemcpyAsync(b->rep_host, b->rep, sizeof(double) * R_COUNT * (size_t)b->count, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < b->count; i++) {
        out[i].n_fix_lower = (int64_t)b->rep_host[(size_t)i * R_COUNT + 0];
        out[i].n_fix_upper = (int64_t)b->rep_host[(size_t)i * R_COUNT + 1];
        out[i].n_rows_to_eq = (int64_t)b->rep_host[(size_t)i * R_COUNT + 2];
    }
    return phase_begin_b<V>(b, false);
}

hipError_t batch_push_setup(pdhg_batch *b, const uint64_t *seeds, pdhg_push_result *out, double theta)
{
    b->s->model_original = false;
    // every pushed LP iterates again: its tiles must be in the lists before the
    // phase-start check below uses them
    hipError_t ec = batch_compact_tiles(b, true);
    if (ec != hipSuccess) return ec;
    hipError_t e = hipMemcpyAsync(b->seeds, seeds, sizeof(uint64_t) * (size_t)b->count, hipMemcpyHostToDevice,
                                  b->s->stream);
    if (e != hipSuccess) return e;
    return b->s->fp32 ? push_setup_b<float>(b, out, theta) : push_setup_b<double>(b, out, theta);
}

// LPs whose push made no check (or did not run) keep the solve's x
__global__ __launch_bounds__(kBlock) void kb_keep_unpushed(const int4 *__restrict__ rn, const DevState *__restrict__ sts,
                                                          const int *__restrict__ active, const double *__restrict__ xu,
                                                          double *__restrict__ xpush)
{
    const int4 tl = rn[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    if (active[tl.x] && sts[tl.x].checks > 0) return;
    const int j = tl.y + threadIdx.x;
    xpush[j] = xu[j];
}

hipError_t batch_keep_unpushed(pdhg_batch *b)
{
    hipLaunchKernelGGL(kb_keep_unpushed, dim3(b->n_rn), dim3(kBlock), 0, b->s->stream, b->rn, b->sts, b->active,
                       b->s->xu, b->s->xpush);
    return hipGetLastError();
}

// ---------------------------------------------------------- dual push ---
// The single-LP dual push of pdhg_iter.hip over every LP taking part, each
// with its own seed and its own column and row numbering for the draws.  LPs
// not taking part keep their model; their entries of the work vectors are 0.
__global__ __launch_bounds__(kBlock) void kb_dpush_rows(const int4 *__restrict__ rm, const int *__restrict__ active,
                                                       const int8_t *__restrict__ sense0, const double *__restrict__ bv,
                                                       const double *__restrict__ ax, const double *__restrict__ yu,
                                                       double eps_abs, int8_t *__restrict__ sense,
                                                       double *__restrict__ yn, double *__restrict__ part)
{
    const int4 tl = rm[blockIdx.x];
    double v[1] = {0.0}; // rows dropped, dual held at the solve's
    if ((int)threadIdx.x < tl.z) {
        const int i = tl.y + threadIdx.x;
        if (active[tl.x]) {
            const int8_t sn = sense0[i];
            const double slack = sn == '<' ? bv[i] - ax[i] : (sn == '>' ? ax[i] - bv[i] : 0.0);
            const bool drop = sn != '=' && slack > eps_abs;
            sense[i] = drop ? (int8_t)'N' : sn;
            yn[i] = drop ? yu[i] : 0.0;
            v[0] = drop ? 1.0 : 0.0;
        } else {
            yn[i] = 0.0;
        }
    }
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename V>
__global__ __launch_bounds__(kBlock) void kb_dpush_cols(const int4 *__restrict__ rn, const int *__restrict__ coff,
                                                       const int *__restrict__ active, const double *__restrict__ xk,
                                                       const double *__restrict__ l, const double *__restrict__ u,
                                                       const double *__restrict__ c, const double *__restrict__ aty,
                                                       const double *__restrict__ atyn, const double *__restrict__ dc,
                                                       double eps_abs, const uint64_t *__restrict__ seeds,
                                                       V *__restrict__ lh, V *__restrict__ uh, double *__restrict__ ch,
                                                       V *__restrict__ x, double *__restrict__ xa,
                                                       double *__restrict__ w0, double *__restrict__ part, int ntile)
{
    const int4 tl = rn[blockIdx.x];
    double v[1] = {0.0}; // columns off both bounds
    if ((int)threadIdx.x < tl.z) {
        const int j = tl.y + threadIdx.x;
        if (active[tl.x]) {
            const double xj = xk[j];
            const bool at_lo = !is_inf_lo(l[j]) && xj - l[j] <= eps_abs;
            const bool at_up = !is_inf_up(u[j]) && u[j] - xj <= eps_abs;
            lh[j] = at_lo ? (V)0 : (V)-INFINITY;
            uh[j] = at_up ? (V)0 : (V)INFINITY;
            const double lam = c[j] - aty[j];
            const double rj = (at_lo && at_up) ? 0.0 : at_lo ? fmin(lam, 0.0) : at_up ? fmax(lam, 0.0) : lam;
            ch[j] = dc[j] * (c[j] - atyn[j] - rj);
            const double uj = push_unit(seeds[tl.x], (int64_t)(j - coff[tl.x]));
            w0[j] = (at_lo && at_up) ? 0.0 : (at_up ? -uj : uj);
            x[j] = (V)0;
            xa[j] = 0.0;
            v[0] = (!at_lo && !at_up) ? 1.0 : 0.0;
        } else {
            w0[j] = 0.0;
        }
    }
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[ntile + blockIdx.x] = 0.0;
    }
}

// aw = A w0 (unscaled); an LP's first row is the first row of its first
// reduction tile, its column count the difference of its column offsets.
__global__ __launch_bounds__(kBlock) void kb_dpush_rhs(const int4 *__restrict__ rm, const int *__restrict__ rm_start,
                                                      const int *__restrict__ coff, const int *__restrict__ active,
                                                      const int8_t *__restrict__ sense, const double *__restrict__ dr,
                                                      const double *__restrict__ ys, const double *__restrict__ aw,
                                                      const uint64_t *__restrict__ seeds, double scale,
                                                      double *__restrict__ bh, double *__restrict__ y)
{
    const int4 tl = rm[blockIdx.x];
    if (!active[tl.x] || (int)threadIdx.x >= tl.z) return;
    const int i = tl.y + threadIdx.x;
    if (sense[i] == 'N') {
        bh[i] = 0.0;
        y[i] = 0.0;
        return;
    }
    const int row0 = rm[rm_start[tl.x]].y;
    const int64_t n_lp = coff[tl.x + 1] - coff[tl.x];
    const double vi = push_unit(seeds[tl.x], n_lp + (i - row0));
    const int8_t sn = sense[i];
    const double g = sn == '>' ? aw[i] - vi : (sn == '<' ? aw[i] + vi : aw[i]);
    bh[i] = dr[i] * (scale * g);
    y[i] = ys[i];
}

// The pushed y: the push's candidate on the rows kept; the solve's y on the
// dropped rows and on every row of an LP whose push made no check or did not run.
__global__ __launch_bounds__(kBlock) void kb_dpush_final(const int4 *__restrict__ rm, const DevState *__restrict__ sts,
                                                        const int *__restrict__ active, const int8_t *__restrict__ sense,
                                                        const double *__restrict__ yu, double *__restrict__ ypush)
{
    const int4 tl = rm[blockIdx.x];
    if ((int)threadIdx.x >= tl.z) return;
    const int i = tl.y + threadIdx.x;
    if (!active[tl.x] || sts[tl.x].checks == 0 || sense[i] == 'N') ypush[i] = yu[i];
}

// Needs batch_report() of (xk, yu) just before: s->ax holds A xk, s->aty A'yu.
template <typename V>
static hipError_t dual_push_setup_b(pdhg_batch *b, const double *xk, int64_t *cols_free, int64_t *rows_fixed)
{
    pdhg_solver *s = b->s;
    hipStream_t st = s->stream;
    double *pm = b->part, *pn = b->part + (size_t)(Q_COUNT + 1) * b->n_rm;
    hipLaunchKernelGGL(kb_dpush_rows, dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, b->active, s->sense0, s->b, s->ax,
                       s->yu, s->p.eps_abs, s->sense, s->ypush, pm);
    spmv<double, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, s->atv, s->ypush, s->zpush);
    hipLaunchKernelGGL((kb_dpush_cols<V>), dim3(b->n_rn), dim3(kBlock), 0, st, b->rn, b->d_coff, b->active, xk, s->l,
                       s->u, s->c, s->aty, s->zpush, s->dc, s->p.eps_abs, b->seeds, (V *)s->lh, (V *)s->uh, s->ch,
                       (V *)s->x, (double *)s->xa, s->w0, pn, b->n_rn);
    // A w0 into ax (read above, free now): the rows of LPs not taking part keep their bhat
    spmv<double, double, double, double>(st, s->lanes_a, s->m, s->rp, s->ci, s->av, s->w0, s->ax);
    hipLaunchKernelGGL(kb_dpush_rhs, dim3(b->n_rm), dim3(kBlock), 0, st, b->rm, b->rm_start, b->d_coff, b->active,
                       s->sense, s->dr, (const double *)s->ys, s->ax, b->seeds, s->p.push_obj_scale, (double *)s->bh,
                       (double *)s->y);
    hipLaunchKernelGGL(kb_push_final, dim3(b->count), dim3(kBlock), 0, st, pn, b->n_rn, pm, b->rm_start, b->rn_start,
                       b->rep);
    hipMemcpyAsync(b->rep_host, b->rep, sizeof(double) * R_COUNT * (size_t)b->count, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < b->count; i++) {
        cols_free[i] = (int64_t)b->rep_host[(size_t)i * R_COUNT + 0];
        rows_fixed[i] = (int64_t)b->rep_host[(size_t)i * R_COUNT + 2];
    }
    return phase_begin_b<V>(b, false);
}

hipError_t batch_dual_push_setup(pdhg_batch *b, const uint64_t *seeds, const double *xk, int64_t *cols_free,
                                 int64_t *rows_fixed)
{
    b->s->model_original = false;
    hipError_t ec = batch_compact_tiles(b, true); // every LP taking part iterates again
    if (ec != hipSuccess) return ec;
    hipError_t e = hipMemcpyAsync(b->seeds, seeds, sizeof(uint64_t) * (size_t)b->count, hipMemcpyHostToDevice,
                                  b->s->stream);
    if (e != hipSuccess) return e;
    return b->s->fp32 ? dual_push_setup_b<float>(b, xk, cols_free, rows_fixed)
                      : dual_push_setup_b<double>(b, xk, cols_free, rows_fixed);
}

hipError_t batch_dual_push_finish(pdhg_batch *b)
{
    hipLaunchKernelGGL(kb_dpush_final, dim3(b->n_rm), dim3(kBlock), 0, b->s->stream, b->rm, b->sts, b->active,
                       b->s->sense, b->s->yu, b->s->ypush);
    return hipGetLastError();
}

// ------------------------------------------------------------- kernels ---
static void build_tiles(const std::vector<int> &off, int count, int rows_per, std::vector<int4> &tiles,
                        std::vector<int> *start)
{
    tiles.clear();
    if (start) start->assign((size_t)count + 1, 0);
    for (int i = 0; i < count; i++) {
        if (start) (*start)[i] = (int)tiles.size();
        for (int r = off[i]; r < off[i + 1]; r += rows_per) {
            int4 t;
            t.x = i;
            t.y = r;
            t.z = off[i + 1] - r < rows_per ? off[i + 1] - r : rows_per;
            t.w = 0;
            tiles.push_back(t);
        }
    }
    if (start) (*start)[count] = (int)tiles.size();
}

static int tile_rows(int kern) { return -kern > 1000 ? -kern - 1000 : -kern; }

// ---------------------------------------------- push on the free columns ---
// The compaction of the block-diagonal model keeps each LP's free columns
// contiguous and in order, so the batch only needs the column-side
// structures of the compact numbering: LP offsets, primal iteration tiles,
// column reduction tiles.  out[i] = first compact column of LP i (i <= count),
// out[count + 1 + i] = first compact transpose entry of LP i.
__global__ void kb_compact_offsets(int count, const int *__restrict__ coff, const int *__restrict__ newid,
                                   const int *__restrict__ tpc, int *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > count) return;
    const int k = newid[coff[i]];
    out[i] = k;
    out[count + 1 + i] = tpc[k];
}

hipError_t batch_push_compact_begin(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    hipError_t e = push_compact_begin(s);
    if (e != hipSuccess || !s->pc.active) return e;
    hipStream_t st = s->stream;
    const int cnt = b->count;
    std::vector<int> h(2 * ((size_t)cnt + 1));
    int *dv = nullptr;
    int4 *rn = nullptr;
    int *rn_start = nullptr, *d_coff = nullptr;
    e = hipMalloc(&dv, sizeof(int) * h.size());
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kb_compact_offsets, dim3((cnt + 1 + 255) / 256), dim3(256), 0, st, cnt, b->d_coff,
                           s->pc.newid, s->pc.tp, dv);
        e = hipMemcpyAsync(h.data(), dv, sizeof(int) * h.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(dv);
    }
    std::vector<int> coff(h.begin(), h.begin() + cnt + 1);
    std::vector<int64_t> nnz((size_t)cnt);
    for (int i = 0; i < cnt; i++) nnz[i] = (int64_t)h[cnt + 2 + i] - h[cnt + 1 + i];
    std::vector<int4> pt, rt;
    std::vector<int> rs;
    build_tiles(coff, cnt, tile_rows(b->kern_at), pt, nullptr);
    build_tiles(coff, cnt, kBlock, rt, &rs);
    if (e == hipSuccess) e = hipMalloc(&rn, sizeof(int4) * (rt.size() > 0 ? rt.size() : 1));
    if (e == hipSuccess) e = hipMalloc(&rn_start, sizeof(int) * rs.size());
    if (e == hipSuccess) e = hipMalloc(&d_coff, sizeof(int) * coff.size());
    if (e == hipSuccess && !rt.empty()) e = hipMemcpy(rn, rt.data(), sizeof(int4) * rt.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(rn_start, rs.data(), sizeof(int) * rs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_coff, coff.data(), sizeof(int) * coff.size(), hipMemcpyHostToDevice);
    // at most as many primal tiles as the full model's: the buffer holds them
    if (e == hipSuccess && !pt.empty()) e = hipMemcpy(b->ptiles, pt.data(), sizeof(int4) * pt.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        for (void *q : {(void *)rn, (void *)rn_start, (void *)d_coff})
            if (q) (void)hipFree(q);
        (void)push_compact_end(s, false);
        // the device tile list may hold compact tiles by now: put the full ones back
        if (!b->ptiles_all.empty())
            (void)hipMemcpy(b->ptiles, b->ptiles_all.data(), sizeof(int4) * b->ptiles_all.size(), hipMemcpyHostToDevice);
        b->n_ptiles = (int)b->ptiles_all.size();
        return e;
    }
    b->full.coff = b->coff;
    b->full.nnz_of = b->nnz_of;
    b->full.ptiles_all = b->ptiles_all;
    b->full.rn = b->rn;
    b->full.n_rn = b->n_rn;
    b->full.rn_start = b->rn_start;
    b->full.d_coff = b->d_coff;
    b->coff = coff;
    b->nnz_of = nnz;
    b->ptiles_all = pt;
    b->n_ptiles = (int)pt.size();
    b->rn = rn;
    b->n_rn = (int)rt.size();
    b->rn_start = rn_start;
    b->d_coff = d_coff;
    b->full.active = true;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return hipSuccess;
}

hipError_t batch_push_compact_end(pdhg_batch *b, bool scatter)
{
    pdhg_solver *s = b->s;
    hipError_t e = push_compact_end(s, scatter);
    if (!b->full.active) return e;
    for (void *q : {(void *)b->rn, (void *)b->rn_start, (void *)b->d_coff})
        if (q) (void)hipFree(q);
    b->coff = b->full.coff;
    b->nnz_of = b->full.nnz_of;
    b->ptiles_all = b->full.ptiles_all;
    b->rn = b->full.rn;
    b->n_rn = b->full.n_rn;
    b->rn_start = b->full.rn_start;
    b->d_coff = b->full.d_coff;
    b->full = {};
    const hipError_t e2 = b->ptiles_all.empty() ? hipSuccess
                                                : hipMemcpy(b->ptiles, b->ptiles_all.data(),
                                                            sizeof(int4) * b->ptiles_all.size(), hipMemcpyHostToDevice);
    b->n_ptiles = (int)b->ptiles_all.size();
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return e != hipSuccess ? e : e2;
}

// (Re)build the iteration tiles for a kernel choice and upload them.
hipError_t batch_set_kernels(pdhg_batch *b, int kern_at, int kern_a)
{
    std::vector<int4> pt, dt;
    build_tiles(b->coff, b->count, tile_rows(kern_at), pt, nullptr);
    build_tiles(b->roff, b->count, tile_rows(kern_a), dt, nullptr);
    if (b->ptiles) (void)hipFree(b->ptiles);
    if (b->dtiles) (void)hipFree(b->dtiles);
    b->ptiles = b->dtiles = nullptr;
    hipError_t e = hipMalloc(&b->ptiles, sizeof(int4) * (pt.size() > 0 ? pt.size() : 1));
    if (e == hipSuccess) e = hipMalloc(&b->dtiles, sizeof(int4) * (dt.size() > 0 ? dt.size() : 1));
    if (e == hipSuccess && !pt.empty())
        e = hipMemcpy(b->ptiles, pt.data(), sizeof(int4) * pt.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !dt.empty())
        e = hipMemcpy(b->dtiles, dt.data(), sizeof(int4) * dt.size(), hipMemcpyHostToDevice);
    b->n_ptiles = (int)pt.size();
    b->n_dtiles = (int)dt.size();
    b->ptiles_all = std::move(pt);
    b->dtiles_all = std::move(dt);
    b->kern_at = kern_at;
    b->kern_a = kern_a;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return e;
}

// Iteration tiles of the LPs still iterating (all = false) or of every LP
// (all = true, at the start of a phase).  Tiles of a stopped LP exit at once,
// but a launch over them still dispatches their workgroups: once a quarter
// of the tiles in use belong to stopped LPs, the lists are rebuilt without
// them (in place: the device buffers hold every tile) and the captured cycle
// graph, whose launches carry the tile counts, is dropped.  Tile order does
// not enter any LP's arithmetic.
hipError_t batch_compact_tiles(pdhg_batch *b, bool all)
{
    std::vector<int4> pt, dt;
    if (all) {
        if (b->n_ptiles == (int)b->ptiles_all.size() && b->n_dtiles == (int)b->dtiles_all.size()) return hipSuccess;
        pt = b->ptiles_all;
        dt = b->dtiles_all;
    } else {
        for (const int4 &t : b->ptiles_all)
            if (!b->sts_host[t.x].done) pt.push_back(t);
        for (const int4 &t : b->dtiles_all)
            if (!b->sts_host[t.x].done) dt.push_back(t);
        if (pt.empty() || dt.empty()) return hipSuccess; // nothing left to run: the phase ends
        if (4 * pt.size() > 3 * (size_t)b->n_ptiles && 4 * dt.size() > 3 * (size_t)b->n_dtiles) return hipSuccess;
    }
    hipStream_t st = b->s->stream;
    hipError_t e = hipMemcpyAsync(b->ptiles, pt.data(), sizeof(int4) * pt.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->dtiles, dt.data(), sizeof(int4) * dt.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st); // the host vectors die on return
    if (e != hipSuccess) return e;
    b->n_ptiles = (int)pt.size();
    b->n_dtiles = (int)dt.size();
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return hipSuccess;
}

// Time every tiled kernel on scratch output vectors and keep the fastest.
hipError_t batch_autotune(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    const size_t vb = s->fp32 ? sizeof(float) : sizeof(double);
    void *sx = nullptr, *sxbar = nullptr, *sxp = nullptr, *sy = nullptr, *syp = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&sx, vb * (size_t)(s->n > 0 ? s->n : 1));
    if (e == hipSuccess) e = hipMalloc(&sxbar, vb * (size_t)(s->n > 0 ? s->n : 1));
    if (e == hipSuccess) e = hipMalloc(&sxp, sizeof(double) * (size_t)(s->n > 0 ? s->n : 1));
    if (e == hipSuccess) e = hipMalloc(&sy, sizeof(double) * (size_t)(s->m > 0 ? s->m : 1));
    if (e == hipSuccess) e = hipMalloc(&syp, sizeof(double) * (size_t)(s->m > 0 ? s->m : 1));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipMemcpyAsync(sx, s->x, vb * (size_t)s->n, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sxbar, s->x, vb * (size_t)s->n, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sy, s->y, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, s->stream);
    const int cands[] = {-32, -64, -128, -256, -1032, -1064};
    void *keep[5] = {s->x, s->xbar, s->xp, s->y, s->yp};
    s->x = sx;
    s->xbar = sxbar;
    s->xp = sxp;
    s->y = sy;
    s->yp = syp;
    int best_at = b->kern_at, best_a = b->kern_a;
    for (int half = 0; half < 2 && e == hipSuccess; half++) {
        float best = 1e30f;
        for (int c : cands) {
            e = half == 0 ? batch_set_kernels(b, c, best_a) : batch_set_kernels(b, best_at, c);
            if (e != hipSuccess) break;
            for (int rep = 0; rep < 4; rep++) {
                if (rep == 1) hipEventRecord(e0, s->stream);
                if (half == 0) {
                    if (s->fp32) launch_primal_b<float>(b, 0, 0);
                    else launch_primal_b<double>(b, 0, 0);
                } else {
                    if (s->fp32) launch_dual_b<float>(b, 0, 0);
                    else launch_dual_b<double>(b, 0, 0);
                }
            }
            hipEventRecord(e1, s->stream);
            e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            if (ms < best) {
                best = ms;
                if (half == 0) best_at = c;
                else best_a = c;
            }
        }
    }
    s->x = keep[0];
    s->xbar = keep[1];
    s->xp = keep[2];
    s->y = keep[3];
    s->yp = keep[4];
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void *q : {sx, sxbar, sxp, sy, syp})
        if (q) (void)hipFree(q);
    if (e != hipSuccess) return e;
    return batch_set_kernels(b, best_at, best_a);
}

} // namespace pdhg
