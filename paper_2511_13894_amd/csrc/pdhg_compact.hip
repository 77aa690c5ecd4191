// The corner push on its free columns only.
//
// Algorithm 1 fixes a column by giving it equal lower and upper bounds (the
// solve's value).  Under the push iteration such a column's x+ is that bound
// at every step, so its only effect is the constant term Ahat_j x_j in the
// dual product.  The push can therefore iterate on the LP of the free columns
// with bhat replaced by btilde = bhat - Ahat_fixed x_fixed:
//   * the row residuals are the same (btilde - Ahat_free x_free = bhat - Ahat x);
//   * a fixed column's reduced cost is absorbed by its two finite bounds, so
//     it adds nothing to the dual residual;
//   * its objective terms appear in both objectives and cancel in the gap;
// hence the same weighted KKT, restarts and stopping test, with the fixed
// columns' share of the matrix and n-vectors gone from every push iteration.
// The solver's fields point at the compact model while the push iterates and
// at the full model again once it ends.  In the learned push a learned fix may
// be undone at a check, so only the plain rule's fixes are dropped: learned
// fixes stay in the compact model with their flags and original bounds.
#include <hipcub/hipcub.hpp>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"

namespace pdhg {

// flag[j] = 1 for a column the compact model keeps (lhat_j != uhat_j, or a
// learned fix, which an undo may free again), 0 for a fixed one; flag[n] = 0
template <typename V>
__global__ __launch_bounds__(kBlock) void k_free_flags(int n, const V *__restrict__ lh, const V *__restrict__ uh,
                                                      const int8_t *__restrict__ lfix, int *__restrict__ flag)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n) flag[j] = (lh[j] != uh[j] || (lfix && lfix[j])) ? 1 : 0;
    else if (j == n) flag[j] = 0;
}

// the learned push's per-column state on the kept columns
__global__ __launch_bounds__(kBlock) void k_gather_learned(int nf, const int *__restrict__ keep,
                                                          const int8_t *__restrict__ lfix, const double *__restrict__ l,
                                                          const double *__restrict__ u, int8_t *__restrict__ lfixc,
                                                          double *__restrict__ lc, double *__restrict__ uc)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nf) return;
    const int j = keep[k];
    lfixc[k] = lfix[j];
    lc[k] = l[j];
    uc[k] = u[j];
}

// keep[newid[j]] = j for every free column j
__global__ __launch_bounds__(kBlock) void k_keep_list(int n, const int *__restrict__ flag, const int *__restrict__ newid,
                                                     int *__restrict__ keep)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n && flag[j]) keep[newid[j]] = (int)j;
}

// len[k] = entries of free column keep[k]; len[nf] = 0
__global__ __launch_bounds__(kBlock) void k_col_len(int nf, const int *__restrict__ keep, const int *__restrict__ tp,
                                                   int *__restrict__ len)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nf) len[k] = tp[keep[k] + 1] - tp[keep[k]];
    else if (k == nf) len[k] = 0;
}

// the transpose's rows of the free columns, in the compact order
template <typename V>
__global__ __launch_bounds__(kBlock) void k_copy_cols(int nf, const int *__restrict__ keep, const int *__restrict__ tp,
                                                     const int *__restrict__ ti, const V *__restrict__ atv,
                                                     const int *__restrict__ tpc, int *__restrict__ tic,
                                                     V *__restrict__ atvc)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nf) return;
    const int j = keep[k], b = tp[j], e = tp[j + 1], o = tpc[k];
    for (int q = 0; q < e - b; q++) {
        tic[o + q] = ti[b + q];
        atvc[o + q] = atv[b + q];
    }
}

// cnt[i] = entries of row i in free columns (one wave per row); cnt[m] = 0
__global__ __launch_bounds__(kBlock) void k_row_free_count(int m, const int *__restrict__ rp, const int *__restrict__ ci,
                                                          const int *__restrict__ flag, int *__restrict__ cnt)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
    const int lane = (int)(threadIdx.x & 63);
    if (i > m) return;
    if (i == m) {
        if (lane == 0) cnt[m] = 0;
        return;
    }
    int c = 0;
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) c += flag[ci[e]];
    c = group_sum<64>(c);
    if (lane == 0) cnt[i] = c;
}

// row i's entries in free columns, in their order, with compact column
// numbers (one wave per row; a ballot gives each kept entry its slot)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_copy_rows(int m, const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const V *__restrict__ av, const int *__restrict__ flag,
                                                     const int *__restrict__ newid, const int *__restrict__ rpc,
                                                     int *__restrict__ cic, V *__restrict__ avc)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
    const int lane = (int)(threadIdx.x & 63);
    if (i >= m) return;
    const uint64_t below = (1ull << lane) - 1ull;
    int o = rpc[i];
    for (int e0 = rp[i]; e0 < rp[i + 1]; e0 += 64) {
        const int e = e0 + lane;
        const bool in = e < rp[i + 1];
        const int col = in ? ci[e] : 0;
        const bool keep = in && flag[col] != 0;
        const uint64_t mask = __ballot(keep);
        if (keep) {
            const int slot = o + __popcll(mask & below);
            cic[slot] = newid[col];
            avc[slot] = av[e];
        }
        o += __popcll(mask);
    }
}

// xf = the fixed columns' value (their common bound), 0 on free columns
template <typename V>
__global__ __launch_bounds__(kBlock) void k_fixed_values(int n, const int *__restrict__ flag, const V *__restrict__ lh,
                                                        double *__restrict__ xf)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n) xf[j] = flag[j] ? 0.0 : (double)lh[j];
}

__global__ __launch_bounds__(kBlock) void k_btilde(int m, const double *__restrict__ bh, const double *__restrict__ ax,
                                                  double *__restrict__ bt)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) bt[i] = bh[i] - ax[i];
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_gather_free(int nf, const int *__restrict__ keep, const double *__restrict__ ch,
                                                       const double *__restrict__ dc, const V *__restrict__ lh,
                                                       const V *__restrict__ uh, const V *__restrict__ x,
                                                       const double *__restrict__ xa, const double *__restrict__ xp,
                                                       double *__restrict__ chc, double *__restrict__ dcc,
                                                       V *__restrict__ lhc, V *__restrict__ uhc, V *__restrict__ xc,
                                                       double *__restrict__ xac, double *__restrict__ xpc)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nf) return;
    const int j = keep[k];
    chc[k] = ch[j];
    dcc[k] = dc[j];
    lhc[k] = lh[j];
    uhc[k] = uh[j];
    xc[k] = x[j];
    xac[k] = xa[j];
    xpc[k] = xp[j];
}

// back to the full vectors: free columns from the compact ones, fixed
// columns at their bound (their x+ at every push iteration; in the mixed
// mode as the anchor, stored difference 0)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_expand(int n, const int *__restrict__ flag, const int *__restrict__ newid,
                                                  const V *__restrict__ lh, const V *__restrict__ xc,
                                                  const double *__restrict__ xac, const double *__restrict__ xpc,
                                                  V *__restrict__ x, double *__restrict__ xa, double *__restrict__ xp)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    if (flag[j]) {
        const int k = newid[j];
        x[j] = xc[k];
        xa[j] = xac[k];
        xp[j] = xpc[k];
    } else {
        const double v = (double)lh[j];
        x[j] = delta ? (V)0 : lh[j];
        xa[j] = v;
        xp[j] = v;
    }
}

namespace {

// out[0..len] = exclusive prefix sums of in[0..len] (in[len] = 0 gives out[len] = the total)
hipError_t exclusive_scan(hipStream_t st, const int *in, int *out, int len)
{
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, len + 1, st);
    if (e != hipSuccess) return e;
    void *tmp = nullptr;
    if ((e = hipMalloc(&tmp, bytes > 0 ? bytes : 1)) != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, len + 1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    return e;
}

int read_int(hipStream_t st, const int *p, hipError_t &e)
{
    int v = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&v, p, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return v;
}

template <typename T>
hipError_t alloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count > 0 ? count : 1));
}

void free_compact(pdhg_solver::PushCompact &c)
{
    void *ptrs[] = {c.flag, c.newid, c.keep, c.tp, c.ti, c.rp, c.ci, c.ahat, c.ahat_t, c.lh, c.uh,
                    c.x, c.xa, c.xbar, c.xp, c.ch, c.dc, c.bt, c.lfix, c.l, c.u, c.aerr, c.aerr_t};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    c = pdhg_solver::PushCompact{};
}

template <typename V>
hipError_t begin_impl(pdhg_solver *s)
{
    auto &c = s->pc;
    hipStream_t st = s->stream;
    const int n = s->n, m = s->m;
    const int gn1 = grid_for((int64_t)n + 1, kBlock, 1 << 30);
    hipError_t e = alloc(&c.flag, (size_t)n + 1);
    if (e == hipSuccess) e = alloc(&c.newid, (size_t)n + 1);
    if (e != hipSuccess) return e;
    const int8_t *lfix = s->learned_active ? s->lfix : nullptr;
    hipLaunchKernelGGL((k_free_flags<V>), dim3(gn1), dim3(kBlock), 0, st, n, (const V *)s->lh, (const V *)s->uh, lfix,
                       c.flag);
    if ((e = exclusive_scan(st, c.flag, c.newid, n)) != hipSuccess) return e;
    const int nf = read_int(st, c.newid + n, e);
    if (e != hipSuccess) return e;
    if (nf == n) { // nothing fixed: iterate on the full model
        free_compact(c);
        return hipSuccess;
    }
    c.nf = nf;
    if ((e = alloc(&c.keep, (size_t)nf)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_keep_list, dim3(gn1), dim3(kBlock), 0, st, n, c.flag, c.newid, c.keep);
    // transpose rows (the primal half) of the free columns
    int *len = nullptr;
    if ((e = alloc(&len, (size_t)nf + 1)) != hipSuccess) return e;
    if ((e = alloc(&c.tp, (size_t)nf + 1)) != hipSuccess) {
        (void)hipFree(len);
        return e;
    }
    hipLaunchKernelGGL(k_col_len, dim3(grid_for((int64_t)nf + 1, kBlock, 1 << 30)), dim3(kBlock), 0, st, nf, c.keep,
                       s->tp, len);
    e = exclusive_scan(st, len, c.tp, nf);
    (void)hipFree(len);
    if (e != hipSuccess) return e;
    const int nnz_f = read_int(st, c.tp + nf, e);
    if (e != hipSuccess) return e;
    c.nnz = nnz_f;
    if ((e = alloc(&c.ti, (size_t)nnz_f)) != hipSuccess) return e;
    if ((e = alloc(reinterpret_cast<V **>(&c.ahat_t), (size_t)nnz_f)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_copy_cols<V>), dim3(grid_for(nf, kBlock, 1 << 30)), dim3(kBlock), 0, st, nf, c.keep, s->tp,
                       s->ti, (const V *)s->ahat_t, c.tp, c.ti, (V *)c.ahat_t);
    if (s->aerr) { // mixed mode: the free columns' rounding errors as well (same indices rewritten)
        if ((e = alloc(reinterpret_cast<float **>(&c.aerr_t), (size_t)nnz_f)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_copy_cols<float>), dim3(grid_for(nf, kBlock, 1 << 30)), dim3(kBlock), 0, st, nf, c.keep,
                           s->tp, s->ti, (const float *)s->aerr_t, c.tp, c.ti, (float *)c.aerr_t);
    }
    // rows of A (the dual half) restricted to the free columns
    int *cnt = nullptr;
    if ((e = alloc(&cnt, (size_t)m + 1)) != hipSuccess) return e;
    if ((e = alloc(&c.rp, (size_t)m + 1)) != hipSuccess) {
        (void)hipFree(cnt);
        return e;
    }
    const int gw = grid_for(((int64_t)m + 1) * 64, kBlock, 1 << 30); // one wave per row
    hipLaunchKernelGGL(k_row_free_count, dim3(gw), dim3(kBlock), 0, st, m, s->rp, s->ci, c.flag, cnt);
    e = exclusive_scan(st, cnt, c.rp, m);
    (void)hipFree(cnt);
    if (e != hipSuccess) return e;
    const int nnz_rows = read_int(st, c.rp + m, e);
    if (e != hipSuccess) return e;
    if (nnz_rows != nnz_f) return hipErrorInvalidValue; // A and its transpose disagree
    if ((e = alloc(&c.ci, (size_t)nnz_f)) != hipSuccess) return e;
    if ((e = alloc(reinterpret_cast<V **>(&c.ahat), (size_t)nnz_f)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_copy_rows<V>), dim3(gw), dim3(kBlock), 0, st, m, s->rp, s->ci, (const V *)s->ahat, c.flag,
                       c.newid, c.rp, c.ci, (V *)c.ahat);
    if (s->aerr) {
        if ((e = alloc(reinterpret_cast<float **>(&c.aerr), (size_t)nnz_f)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_copy_rows<float>), dim3(gw), dim3(kBlock), 0, st, m, s->rp, s->ci,
                           (const float *)s->aerr, c.flag, c.newid, c.rp, c.ci, (float *)c.aerr);
    }
    // btilde = bhat - Ahat xf, the float64 product on the full model (aty is free here)
    double *xf = s->aty;
    hipLaunchKernelGGL((k_fixed_values<V>), dim3(gn1), dim3(kBlock), 0, st, n, c.flag, (const V *)s->lh, xf);
    if ((e = exact_product(s, false, xf, s->ax)) != hipSuccess) return e;
    if ((e = alloc(&c.bt, (size_t)m)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_btilde, dim3(grid_for(m, kBlock, 1 << 30)), dim3(kBlock), 0, st, m, (const double *)s->bh,
                       s->ax, c.bt);
    // the free columns' vectors
    if ((e = alloc(&c.ch, (size_t)nf)) != hipSuccess) return e;
    if ((e = alloc(&c.dc, (size_t)nf)) != hipSuccess) return e;
    V **vecs[] = {reinterpret_cast<V **>(&c.lh), reinterpret_cast<V **>(&c.uh), reinterpret_cast<V **>(&c.x),
                  reinterpret_cast<V **>(&c.xbar)};
    for (V **q : vecs)
        if ((e = alloc(q, (size_t)nf)) != hipSuccess) return e;
    for (double **q : {reinterpret_cast<double **>(&c.xa), reinterpret_cast<double **>(&c.xp)}) // float64 anchor, candidate
        if ((e = alloc(q, (size_t)nf)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_gather_free<V>), dim3(grid_for(nf, kBlock, 1 << 30)), dim3(kBlock), 0, st, nf, c.keep,
                       s->ch, s->dc, (const V *)s->lh, (const V *)s->uh, (const V *)s->x, (const double *)s->xa,
                       (const double *)s->xp, c.ch, c.dc, (V *)c.lh, (V *)c.uh, (V *)c.x, (double *)c.xa,
                       (double *)c.xp);
    if (lfix) {
        if ((e = alloc(&c.lfix, (size_t)nf)) != hipSuccess) return e;
        if ((e = alloc(&c.l, (size_t)nf)) != hipSuccess) return e;
        if ((e = alloc(&c.u, (size_t)nf)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_gather_learned, dim3(grid_for(nf, kBlock, 1 << 30)), dim3(kBlock), 0, st, nf, c.keep, lfix,
                           s->l, s->u, c.lfix, c.l, c.u);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    // put the compact model in place
    c.n0 = s->n;
    c.nnz0 = s->nnz;
    c.udeg_at0 = s->udeg_at;
    c.red_blocks_n0 = s->red_blocks_n;
    c.tp0 = s->tp;
    c.ti0 = s->ti;
    c.rp0 = s->rp;
    c.ci0 = s->ci;
    c.ahat0 = s->ahat;
    c.ahat_t0 = s->ahat_t;
    c.lh0 = s->lh;
    c.uh0 = s->uh;
    c.bh0 = s->bh;
    c.x0 = s->x;
    c.xa0 = s->xa;
    c.xbar0 = s->xbar;
    c.xp0 = s->xp;
    c.ch0 = s->ch;
    c.dc0 = s->dc;
    c.aerr0 = s->aerr;
    c.aerr_t0 = s->aerr_t;
    c.chc0 = s->chc;
    c.bhc0 = s->bhc;
    c.segs0 = s->segs;
    s->n = nf;
    s->nnz = nnz_f;
    s->red_blocks_n = grid_for(nf, kBlock, kMaxRedBlocks);
    s->tp = c.tp;
    s->ti = c.ti;
    s->rp = c.rp;
    s->ci = c.ci;
    s->ahat = c.ahat;
    s->ahat_t = c.ahat_t;
    s->lh = c.lh;
    s->uh = c.uh;
    s->bh = c.bt;
    s->x = c.x;
    s->xa = c.xa;
    s->xbar = c.xbar;
    s->xp = c.xp;
    s->ch = c.ch;
    s->dc = c.dc;
    if (s->aerr) { // the full model's chc and bhc (n >= nf entries) serve the compact model
        s->aerr = c.aerr;
        s->aerr_t = c.aerr_t;
    }
    defect_alias(s);
    s->defect_stale = true;
    if (lfix) {
        c.lfix0 = s->lfix;
        c.l0 = s->l;
        c.u0 = s->u;
        s->lfix = c.lfix;
        s->l = c.l;
        s->u = c.u;
    }
    c.active = true;
    if (s->graph_exec) { // captured on the full model's arrays
        (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
        s->graph_mode = -1;
    }
    if (s->kern_a == kRowSegs && (e = plan_row_segments(s)) != hipSuccess) return e; // of the compact rows
    return detect_uniform_columns(s); // of the compact model (on failure the caller restores the full one)
}

template <typename V>
hipError_t end_impl(pdhg_solver *s, bool scatter)
{
    auto &c = s->pc;
    hipError_t e = hipSuccess;
    if (scatter)
        hipLaunchKernelGGL((k_expand<V>), dim3(grid_for(c.n0, kBlock, 1 << 30)), dim3(kBlock), 0, s->stream, c.n0,
                           c.flag, c.newid, (const V *)c.lh0, (const V *)c.x, (const double *)c.xa,
                           (const double *)c.xp, (V *)c.x0, (double *)c.xa0, (double *)c.xp0);
    e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s->stream); // the compact arrays are freed below
    if (e == hipSuccess) e = e2;
    s->n = c.n0;
    s->nnz = c.nnz0;
    s->udeg_at = c.udeg_at0;
    s->red_blocks_n = c.red_blocks_n0;
    s->tp = c.tp0;
    s->ti = c.ti0;
    s->rp = c.rp0;
    s->ci = c.ci0;
    s->ahat = c.ahat0;
    s->ahat_t = c.ahat_t0;
    s->lh = c.lh0;
    s->uh = c.uh0;
    s->bh = c.bh0;
    s->x = c.x0;
    s->xa = c.xa0;
    s->xbar = c.xbar0;
    s->xp = c.xp0;
    s->ch = c.ch0;
    s->dc = c.dc0;
    s->aerr = c.aerr0;
    s->aerr_t = c.aerr_t0;
    s->chc = c.chc0;
    s->bhc = c.bhc0;
    s->segs = c.segs0;
    s->defect_stale = true;
    if (c.lfix0) {
        s->lfix = c.lfix0;
        s->l = c.l0;
        s->u = c.u0;
    }
    if (s->graph_exec) {
        (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
        s->graph_mode = -1;
    }
    free_compact(c);
    return e;
}

} // namespace

hipError_t push_compact_begin(pdhg_solver *s)
{
    if (s->pc.active) return hipSuccess;
    const hipError_t e = s->fp32 ? begin_impl<float>(s) : begin_impl<double>(s);
    if (e != hipSuccess && !s->pc.active) free_compact(s->pc); // a failed build leaves the full model in place
    return e;
}

hipError_t push_compact_end(pdhg_solver *s, bool scatter)
{
    if (!s->pc.active) return hipSuccess;
    return s->fp32 ? end_impl<float>(s, scatter) : end_impl<double>(s, scatter);
}

} // namespace pdhg
