// The PDHG iteration (primal and dual halves with fused projections,
// extrapolation and Halpern averaging), the periodic check (residuals, gap,
// weighted KKT, restart and primal-weight update, termination), the corner
// push setup of Algorithm 1, and float64 KKT reports on the original model.
#include <cmath>
#include <cstdio>
#include <vector>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"
#include "pdhg_kernels.hpp"

namespace pdhg {

// ------------------------------------------------------------ iteration ---
template <typename V, int L>
__global__ __launch_bounds__(kBlock) void k_primal(int n, const int *__restrict__ tp, const int *__restrict__ ti,
                                                  const V *__restrict__ atv, const double *__restrict__ y,
                                                  const double *__restrict__ ch, const V *__restrict__ lh,
                                                  const V *__restrict__ uh, V *__restrict__ x,
                                                  const double *__restrict__ xa, V *__restrict__ xbar,
                                                  double *__restrict__ xp, const DevState *__restrict__ st, int i,
                                                  int store_cand)
{
    const int64_t gi = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int64_t j = gi / L;
    const int lane = (int)(gi % L);
    if (j >= n) return;
    // the epilogue's operands are loaded by every lane of the group (one
    // request per group), none behind a divergent branch; the stop flag is
    // uniform (issuing the product's loads before the test, or testing only
    // after the product, measured no faster)
    const double aj = xa[j], xj = iterate_value<V>(x[j], aj), cj = ch[j], lo = (double)lh[j], hi = (double)uh[j];
    if (st->done) return;
    double acc = lane_dot<L, double>(tp[j], tp[j + 1], lane, ti, atv, y);
    acc = group_sum<L>(acc);
    if (lane != 0) return;
    primal_update<V>(j, acc, xj, cj, lo, hi, aj, x, xbar, xp, st, i, store_cand);
}

// Dual half on rows [row0, row1), one row of A per group of L lanes, for the
// workgroup that takes logical block lb:  h = Ahat xbar, then the update.
template <typename V, int L>
__device__ __forceinline__ void dual_rows(int row0, int row1, int lb, const int *__restrict__ rp,
                                          const int *__restrict__ ci, const V *__restrict__ av,
                                          const V *__restrict__ xbar, const double *__restrict__ bh,
                                          const int8_t *__restrict__ sense, double *__restrict__ y,
                                          const double *__restrict__ ya, double *__restrict__ yp,
                                          const DevState *__restrict__ st, int i, int store_cand)
{
    const int64_t gi = (int64_t)lb * kBlock + threadIdx.x;
    const int64_t r = row0 + gi / L;
    const int lane = (int)(gi % L);
    if (r >= row1) return;
    const double yr = y[r], br = bh[r], ar = ya[r]; // epilogue operands (see k_primal)
    const int8_t sn = sense[r];
    if (st->done) return;
    double acc = lane_dot<L, double>(rp[r], rp[r + 1], lane, ci, av, xbar);
    acc = group_sum<L>(acc);
    if (lane != 0) return;
    dual_update(r, acc, yr, br, ar, sn, y, yp, st, i, store_cand);
}

// Dual half, one row of A per group of L lanes:  h = Ahat xbar.
template <typename V, int L>
__global__ __launch_bounds__(kBlock) void k_dual(int m, const int *__restrict__ rp, const int *__restrict__ ci,
                                                const V *__restrict__ av, const V *__restrict__ xbar,
                                                const double *__restrict__ bh, const int8_t *__restrict__ sense,
                                                double *__restrict__ y, const double *__restrict__ ya,
                                                double *__restrict__ yp, const DevState *__restrict__ st, int i,
                                                int store_cand)
{
    dual_rows<V, L>(0, m, xcd_block(blockIdx.x, gridDim.x), rp, ci, av, xbar, bh, sense, y, ya, yp, st, i,
                    store_cand);
}

// ------------------------------------------------------- row segments ---
// Rows of one kind share a lane-group width.  A row whose entries sit in
// consecutive columns (a source row of a transportation model) streams its
// share of xbar: many lanes finish it in few rounds of loads.  A row whose
// columns are spread out (a sink row, one column per source) gathers one
// cache line per entry, and the next rows gather the same lines: narrower
// groups put more such rows in a workgroup, whose shared L1 then serves them.
// Each segment has its own workgroups in one launch; a workgroup finds its
// segment from its index (a uniform branch) and maps itself onto the XCDs
// as a launch of the segment alone would.
__device__ __forceinline__ int seg_of(const RowSegs &sg, int b)
{
    int k = 0;
    while (k + 1 < sg.count && b >= sg.blk0[k + 1]) k++;
    return k;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_dual_segs(RowSegs sg, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const V *__restrict__ av,
                                                     const V *__restrict__ xbar, const double *__restrict__ bh,
                                                     const int8_t *__restrict__ sense, double *__restrict__ y,
                                                     const double *__restrict__ ya, double *__restrict__ yp,
                                                     const DevState *__restrict__ st, int i, int store_cand)
{
    const int k = seg_of(sg, blockIdx.x);
    const int lb = xcd_block(blockIdx.x - sg.blk0[k], sg.blk0[k + 1] - sg.blk0[k]);
    const int r0 = sg.row0[k], r1 = sg.row0[k + 1];
#define PDHG_SEG_CASE(LL)                                                                                       \
    case LL:                                                                                                    \
        dual_rows<V, LL>(r0, r1, lb, rp, ci, av, xbar, bh, sense, y, ya, yp, st, i, store_cand);               \
        break;
    switch (sg.lanes[k]) {
        PDHG_SEG_CASE(1)
        PDHG_SEG_CASE(2)
        PDHG_SEG_CASE(4)
        PDHG_SEG_CASE(8)
        PDHG_SEG_CASE(16)
        PDHG_SEG_CASE(32)
    default:
        PDHG_SEG_CASE(64)
    }
#undef PDHG_SEG_CASE
}

// out = M vec on the same segments (the check products of this dual half)
template <typename VM, typename VV, int L>
__device__ __forceinline__ void spmv_rows(int row0, int row1, int lb, const int *__restrict__ ptr,
                                          const int *__restrict__ idx, const VM *__restrict__ val,
                                          const VV *__restrict__ vec, double *__restrict__ out)
{
    const int64_t gi = (int64_t)lb * kBlock + threadIdx.x;
    const int64_t r = row0 + gi / L;
    const int lane = (int)(gi % L);
    if (r >= row1) return;
    double acc = lane_dot<L, double>(ptr[r], ptr[r + 1], lane, idx, val, vec);
    acc = group_sum<L>(acc);
    if (lane == 0) out[r] = acc;
}

template <typename VM, typename VV>
__global__ __launch_bounds__(kBlock) void k_spmv_segs(RowSegs sg, const int *__restrict__ ptr,
                                                     const int *__restrict__ idx, const VM *__restrict__ val,
                                                     const VV *__restrict__ vec, double *__restrict__ out)
{
    const int k = seg_of(sg, blockIdx.x);
    const int lb = xcd_block(blockIdx.x - sg.blk0[k], sg.blk0[k + 1] - sg.blk0[k]);
    const int r0 = sg.row0[k], r1 = sg.row0[k + 1];
#define PDHG_SEG_CASE(LL)                                                                                       \
    case LL:                                                                                                    \
        spmv_rows<VM, VV, LL>(r0, r1, lb, ptr, idx, val, vec, out);                                            \
        break;
    switch (sg.lanes[k]) {
        PDHG_SEG_CASE(1)
        PDHG_SEG_CASE(2)
        PDHG_SEG_CASE(4)
        PDHG_SEG_CASE(8)
        PDHG_SEG_CASE(16)
        PDHG_SEG_CASE(32)
    default:
        PDHG_SEG_CASE(64)
    }
#undef PDHG_SEG_CASE
}

// adj[r] = entries of row r whose next entry lies in the next column
// (columns are sorted within a row); one wave per row
__global__ __launch_bounds__(kBlock) void k_row_adjacent(int m, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, int *__restrict__ adj)
{
    const int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= m) return;
    const int beg = rp[w], end = rp[w + 1];
    int c = 0;
    for (int e = beg + lane; e + 1 < end; e += 64) c += ci[e + 1] == ci[e] + 1 ? 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) adj[w] = c;
}

// ------------------------------------------------------- long rows ---
// One row per workgroup of kBlock threads, for rows of hundreds of entries
// or more: the threads stride over the row four entries at a time, with all
// index and value loads issued before the gathers, and a block reduction in
// a fixed order gives the row sum to thread 0, which runs the update.
template <typename VM, typename VV>
__device__ __forceinline__ double row_block_sum(int beg, int end, const int *__restrict__ idx,
                                                const VM *__restrict__ val, const VV *__restrict__ vec)
{
    double acc = 0.0;
    for (int e0 = beg + (int)threadIdx.x; e0 < end; e0 += 4 * kBlock) {
        int id[4];
        double v[4], g[4];
        // every lane loads: positions past the row's end reload its last
        // entry (e0 < end here), so no load is merged with a fallback value
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = e0 + u * kBlock;
            const int ec = e < end ? e : end - 1;
            id[u] = idx[ec];
            v[u] = (double)val[ec];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) g[u] = (double)vec[id[u]];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (e0 + u * kBlock < end) acc += v[u] * g[u];
    }
    double q[1] = {acc};
    block_reduce<1>(q, 0u);
    return q[0];
}

// ---------------------------------------------------- check products ---
// A check's products use the structure of the iteration kernel of the same
// half (LDS tiles, one row per workgroup, or lane groups): they cost what an
// iteration half costs, and an LP inside a batch (same tiles) gets the same
// row sums as when it is solved alone.
template <typename VM, typename VV, int T, int NT>
__global__ __launch_bounds__(NT) void k_spmv_tiled(int rows_total, const int *__restrict__ ptr,
                                                  const int *__restrict__ idx, const VM *__restrict__ val,
                                                  const VV *__restrict__ vec, double *__restrict__ out)
{
    __shared__ int s_ptr[T + 1];
    __shared__ double s_prod[kTileU * NT];
    __shared__ double s_sum[T];
    const int r0 = xcd_block(blockIdx.x, gridDim.x) * T;
    const int rows = rows_total - r0 < T ? rows_total - r0 : T;
    tile_row_sums<VM, VV, T, NT>(r0, rows, ptr, idx, val, vec, s_ptr, s_prod, s_sum);
    if ((int)threadIdx.x < rows) out[r0 + threadIdx.x] = s_sum[threadIdx.x];
}

template <typename VM, typename VV>
__global__ __launch_bounds__(kBlock) void k_spmv_rowblock(const int *__restrict__ ptr, const int *__restrict__ idx,
                                                         const VM *__restrict__ val, const VV *__restrict__ vec,
                                                         double *__restrict__ out)
{
    const int r = xcd_block(blockIdx.x, gridDim.x);
    const double h = row_block_sum<VM, VV>(ptr[r], ptr[r + 1], idx, val, vec);
    if (threadIdx.x == 0) out[r] = h;
}

// out = M vec (float64) with the kernel structure `kern` (lanes_* encoding)
template <typename VM, typename VV>
static void check_spmv(hipStream_t st, int kern, int rows, const int *ptr, const int *idx, const VM *val,
                       const VV *vec, double *out)
{
    if (rows <= 0) return;
    if (kern > 0) {
        spmv<VM, VV, double, double>(st, kern, rows, ptr, idx, val, vec, out);
        return;
    }
    if (kern == kRowBlock) {
        hipLaunchKernelGGL((k_spmv_rowblock<VM, VV>), dim3(rows), dim3(kBlock), 0, st, ptr, idx, val, vec, out);
        return;
    }
    const int T = -kern;
    const int rows_per = T > 1000 ? T - 1000 : T;
    const int grid = (rows + rows_per - 1) / rows_per;
#define PDHG_CS_CASE(TT, RR, NT)                                                                                 \
    case TT:                                                                                                     \
        hipLaunchKernelGGL((k_spmv_tiled<VM, VV, RR, NT>), dim3(grid), dim3(NT), 0, st, rows, ptr, idx, val, vec, \
                           out);                                                                                 \
        break;
    switch (T) {
        PDHG_CS_CASE(32, 32, 256)
        PDHG_CS_CASE(64, 64, 256)
        PDHG_CS_CASE(128, 128, 256)
        PDHG_CS_CASE(1032, 32, 64)
        PDHG_CS_CASE(1064, 64, 64)
    default:
        PDHG_CS_CASE(256, 256, 256)
    }
#undef PDHG_CS_CASE
}

__global__ __launch_bounds__(kBlock) void k_add_to(int64_t len, double *__restrict__ out, const double *__restrict__ add)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock)
        out[i] += add[i];
}

// out = M vec for a matrix with A's rows (Ahat, or its float rounding error
// in mixed mode) in the dual half's kernel structure; the sliced layout
// holds only the float matrix, so with it the products use lane groups
template <typename VM, typename VV>
static void row_product(const pdhg_solver *s, const VM *val, const VV *vec, double *out)
{
    if (s->m <= 0) return;
    if (s->kern_a == kRowSegs) {
        const RowSegs &sg = s->segs;
        hipLaunchKernelGGL((k_spmv_segs<VM, VV>), dim3(sg.blk0[sg.count]), dim3(kBlock), 0, s->stream, sg, s->rp,
                           s->ci, val, vec, out);
        return;
    }
    check_spmv<VM, VV>(s->stream, s->kern_a == kSell ? s->lanes_a : s->kern_a, s->m, s->rp, s->ci, val, vec, out);
}

hipError_t solver_product(pdhg_solver *s, bool transpose, const double *vec, double *out);

hipError_t exact_product(pdhg_solver *s, bool transpose, const double *vec, double *out)
{
    hipError_t e = solver_product(s, transpose, vec, out);
    if (e != hipSuccess || !s->aerr) return e;
    hipStream_t st = s->stream;
    if (transpose) { // ety is free outside a check cycle
        check_spmv<float, double>(st, s->kern_at, s->n, s->tp, s->ti, (const float *)s->aerr_t, vec, s->ety);
        hipLaunchKernelGGL(k_add_to, dim3(grid_for(s->n, kBlock, 8192)), dim3(kBlock), 0, st, (int64_t)s->n, out,
                           (const double *)s->ety);
    } else {
        row_product<float, double>(s, (const float *)s->aerr, vec, s->ex);
        hipLaunchKernelGGL(k_add_to, dim3(grid_for(s->m, kBlock, 8192)), dim3(kBlock), 0, st, (int64_t)s->m, out,
                           (const double *)s->ex);
    }
    return hipGetLastError();
}

hipError_t solver_product(pdhg_solver *s, bool transpose, const double *vec, double *out)
{
    if (transpose) {
        if (s->fp32) check_spmv<float, double>(s->stream, s->kern_at, s->n, s->tp, s->ti, (const float *)s->ahat_t, vec, out);
        else check_spmv<double, double>(s->stream, s->kern_at, s->n, s->tp, s->ti, (const double *)s->ahat_t, vec, out);
    } else if (s->kern_a == kSell) {
        sell_product(s, vec, out);
    } else {
        if (s->fp32) row_product<float, double>(s, (const float *)s->ahat, vec, out);
        else row_product<double, double>(s, (const double *)s->ahat, vec, out);
    }
    return hipGetLastError();
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_primal_rowblock(int n, const int *__restrict__ tp,
                                                           const int *__restrict__ ti, const V *__restrict__ atv,
                                                           const double *__restrict__ y, const double *__restrict__ ch,
                                                           const V *__restrict__ lh, const V *__restrict__ uh,
                                                           V *__restrict__ x, const double *__restrict__ xa,
                                                           V *__restrict__ xbar, double *__restrict__ xp,
                                                           const DevState *__restrict__ st, int i, int store_cand)
{
    if (st->done) return;
    const int j = xcd_block(blockIdx.x, gridDim.x);
    double xj = 0, cj = 0, lo = 0, hi = 0, aj = 0;
    if (threadIdx.x == 0) {
        aj = xa[j];
        xj = iterate_value<V>(x[j], aj);
        cj = ch[j];
        lo = (double)lh[j];
        hi = (double)uh[j];
    }
    const double g = row_block_sum<V, double>(tp[j], tp[j + 1], ti, atv, y);
    if (threadIdx.x == 0) primal_update<V>(j, g, xj, cj, lo, hi, aj, x, xbar, xp, st, i, store_cand);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_dual_rowblock(int m, const int *__restrict__ rp, const int *__restrict__ ci,
                                                         const V *__restrict__ av, const V *__restrict__ xbar,
                                                         const double *__restrict__ bh,
                                                         const int8_t *__restrict__ sense, double *__restrict__ y,
                                                         const double *__restrict__ ya, double *__restrict__ yp,
                                                         const DevState *__restrict__ st, int i, int store_cand)
{
    if (st->done) return;
    const int r = xcd_block(blockIdx.x, gridDim.x);
    double yr = 0, br = 0, ar = 0;
    int8_t sn = 0;
    if (threadIdx.x == 0) {
        yr = y[r];
        br = bh[r];
        ar = ya[r];
        sn = sense[r];
    }
    const double h = row_block_sum<V, V>(rp[r], rp[r + 1], ci, av, xbar);
    if (threadIdx.x == 0) dual_update(r, h, yr, br, ar, sn, y, yp, st, i, store_cand);
}

template <typename V, int T, int NT>
__global__ __launch_bounds__(NT) void k_primal_tiled(int n, const int *__restrict__ tp, const int *__restrict__ ti,
                                                    const V *__restrict__ atv, const double *__restrict__ y,
                                                    const double *__restrict__ ch, const V *__restrict__ lh,
                                                    const V *__restrict__ uh, V *__restrict__ x,
                                                    const double *__restrict__ xa, V *__restrict__ xbar,
                                                    double *__restrict__ xp, const DevState *__restrict__ st, int i,
                                                    int store_cand)
{
    __shared__ int s_ptr[T + 1];
    __shared__ double s_prod[kTileU * NT];
    __shared__ double s_sum[T];
    const int r0 = xcd_block(blockIdx.x, gridDim.x) * T;
    const int rows = n - r0 < T ? n - r0 : T; // >= 1: the grid covers n
    const int tid = threadIdx.x;
    const bool mine = tid < rows;
    const int j = r0 + tid;
    // Epilogue operands, independent of the product: every thread loads
    // (threads past the tile reload its first row), so no load waits on a
    // divergent branch.  The stop flag is uniform: the whole workgroup
    // leaves together.
    const int jc = mine ? j : r0;
    const double aj = xa[jc], xj = iterate_value<V>(x[jc], aj), cj = ch[jc], lo = (double)lh[jc],
                 hi = (double)uh[jc];
    if (st->done) return;
    tile_row_sums<V, double, T, NT>(r0, rows, tp, ti, atv, y, s_ptr, s_prod, s_sum);
    if (!mine) return;
    primal_update<V>(j, s_sum[tid], xj, cj, lo, hi, aj, x, xbar, xp, st, i, store_cand);
}

template <typename V, int T, int NT>
__global__ __launch_bounds__(NT) void k_dual_tiled(int m, const int *__restrict__ rp, const int *__restrict__ ci,
                                                  const V *__restrict__ av, const V *__restrict__ xbar,
                                                  const double *__restrict__ bh, const int8_t *__restrict__ sense,
                                                  double *__restrict__ y, const double *__restrict__ ya,
                                                  double *__restrict__ yp, const DevState *__restrict__ st, int i,
                                                  int store_cand)
{
    __shared__ int s_ptr[T + 1];
    __shared__ double s_prod[kTileU * NT];
    __shared__ double s_sum[T];
    const int r0 = xcd_block(blockIdx.x, gridDim.x) * T;
    const int rows = m - r0 < T ? m - r0 : T; // >= 1: the grid covers m
    const int tid = threadIdx.x;
    const bool mine = tid < rows;
    const int r = r0 + tid;
    const int rc = mine ? r : r0; // as in k_primal_tiled: unconditional epilogue loads
    const double yr = y[rc], br = bh[rc], ar = ya[rc];
    const int8_t sn = sense[rc];
    if (st->done) return;
    tile_row_sums<V, V, T, NT>(r0, rows, rp, ci, av, xbar, s_ptr, s_prod, s_sum);
    if (!mine) return;
    dual_update(r, s_sum[tid], yr, br, ar, sn, y, yp, st, i, store_cand);
}

// Primal half when every column of A has the same D <= 3 entries (every
// transpose row starts at j*D: network and transportation LPs, and their
// push models on the free columns): one thread per column, with no
// row-pointer loads, so the column's index and value loads go out with the
// epilogue's in the first round and the gathers in the second.  The products
// are rounded before they are summed in entry order, as the 256-row LDS
// tiles (one thread per row) sum them: the two give the same bits.
template <typename V, int D>
__global__ __launch_bounds__(kBlock) void k_primal_udeg(int n, const int *__restrict__ ti, const V *__restrict__ atv,
                                                       const double *__restrict__ y, const double *__restrict__ ch,
                                                       const V *__restrict__ lh, const V *__restrict__ uh,
                                                       V *__restrict__ x, const double *__restrict__ xa,
                                                       V *__restrict__ xbar, double *__restrict__ xp,
                                                       const DevState *__restrict__ st, int i, int store_cand)
{
    const int64_t j = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (j >= n) return;
    int id[D];
    double v[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        id[d] = ti[j * D + d];
        v[d] = (double)atv[j * D + d];
    }
    const double aj = xa[j], xj = iterate_value<V>(x[j], aj), cj = ch[j], lo = (double)lh[j], hi = (double)uh[j];
    if (st->done) return;
    double g[D];
#pragma unroll
    for (int d = 0; d < D; d++) g[d] = y[id[d]];
    double acc = 0.0;
    {
#pragma clang fp contract(off)
        // separate roundings of each product and each sum, as the tiles' LDS products
#pragma unroll
        for (int d = 0; d < D; d++) acc = acc + v[d] * g[d];
    }
    primal_update<V>(j, acc, xj, cj, lo, hi, aj, x, xbar, xp, st, i, store_cand);
}

template <typename V>
static void launch_primal(pdhg_solver *s, int i, int store, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    const int L = s->kern_at;
    if (s->n <= 0) return;
    // uniform columns, kernel chosen by the library: the 256-row tiles' sums with fewer loads
    // (an explicit lanes_at = -256 keeps the tiles)
    if (uses_uniform_kernel(s)) {
        const int grid = (s->n + kBlock - 1) / kBlock;
#define PDHG_UD_CASE(DD)                                                                                       \
    case DD:                                                                                                   \
        PDHG_LAUNCH(e0, e1, (k_primal_udeg<V, DD>), dim3(grid), dim3(kBlock), s->stream, s->n, s->ti,        \
                    (const V *)s->ahat_t, (const double *)s->y, s->chc, (const V *)s->lh, (const V *)s->uh,    \
                    (V *)s->x, (const double *)s->xa, (V *)s->xbar, (double *)s->xp, s->st, i, store);                   \
        break;
        switch (s->udeg_at) {
            PDHG_UD_CASE(1)
            PDHG_UD_CASE(2)
        default:
            PDHG_UD_CASE(3)
        }
#undef PDHG_UD_CASE
        return;
    }
    if (L == kRowBlock) {
        PDHG_LAUNCH(e0, e1, (k_primal_rowblock<V>), dim3(s->n), dim3(kBlock), s->stream, s->n, s->tp, s->ti,
                    (const V *)s->ahat_t, (const double *)s->y, s->chc, (const V *)s->lh, (const V *)s->uh,
                    (V *)s->x, (const double *)s->xa, (V *)s->xbar, (double *)s->xp, s->st, i, store);
        return;
    }
    if (L < 0) { // LDS-tiled kernel: -T (256 threads) or -(1000 + T) (64 threads)
        const int T = -L;
        const int rows_per = T > 1000 ? T - 1000 : T;
        const int grid = (s->n + rows_per - 1) / rows_per;
#define PDHG_PT_CASE(TT, RR, NT)                                                                                \
    case TT:                                                                                                    \
        PDHG_LAUNCH(e0, e1, (k_primal_tiled<V, RR, NT>), dim3(grid), dim3(NT), s->stream, s->n, s->tp, s->ti, \
                           (const V *)s->ahat_t, (const double *)s->y, s->chc, (const V *)s->lh,          \
                           (const V *)s->uh, (V *)s->x, (const double *)s->xa, (V *)s->xbar, (double *)s->xp, s->st, i,  \
                           store);                                                                              \
        break;
        switch (T) {
            PDHG_PT_CASE(32, 32, 256)
            PDHG_PT_CASE(64, 64, 256)
            PDHG_PT_CASE(128, 128, 256)
            PDHG_PT_CASE(1032, 32, 64)
            PDHG_PT_CASE(1064, 64, 64)
        default:
            PDHG_PT_CASE(256, 256, 256)
        }
#undef PDHG_PT_CASE
        return;
    }
    const int grid = (int)(((int64_t)s->n * L + kBlock - 1) / kBlock);
#define PDHG_PRIMAL_CASE(LL)                                                                                    \
    case LL:                                                                                                    \
        PDHG_LAUNCH(e0, e1, (k_primal<V, LL>), dim3(grid), dim3(kBlock), s->stream, s->n, s->tp, s->ti,      \
                           (const V *)s->ahat_t, (const double *)s->y, s->chc, (const V *)s->lh,          \
                           (const V *)s->uh, (V *)s->x, (const double *)s->xa, (V *)s->xbar, (double *)s->xp, s->st, i,  \
                           store);                                                                              \
        break;
    switch (L) {
        PDHG_PRIMAL_CASE(1)
        PDHG_PRIMAL_CASE(2)
        PDHG_PRIMAL_CASE(4)
        PDHG_PRIMAL_CASE(8)
        PDHG_PRIMAL_CASE(16)
        PDHG_PRIMAL_CASE(32)
    default:
        PDHG_PRIMAL_CASE(64)
    }
#undef PDHG_PRIMAL_CASE
}

template <typename V>
static void launch_dual(pdhg_solver *s, int i, int store, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    const int L = s->kern_a;
    if (s->m <= 0) return;
    if (L == kSell) {
        sell_dual(s, i, store, e0, e1);
        return;
    }
    if (L == kRowSegs) {
        const RowSegs &sg = s->segs;
        PDHG_LAUNCH(e0, e1, (k_dual_segs<V>), dim3(sg.blk0[sg.count]), dim3(kBlock), s->stream, sg, s->rp, s->ci,
                    (const V *)s->ahat, (const V *)s->xbar, (const double *)s->bhc, s->sense, (double *)s->y,
                    (const double *)s->ya, (double *)s->yp, s->st, i, store);
        return;
    }
    if (L == kRowBlock) {
        PDHG_LAUNCH(e0, e1, (k_dual_rowblock<V>), dim3(s->m), dim3(kBlock), s->stream, s->m, s->rp, s->ci,
                    (const V *)s->ahat, (const V *)s->xbar, (const double *)s->bhc, s->sense, (double *)s->y,
                    (const double *)s->ya, (double *)s->yp, s->st, i, store);
        return;
    }
    if (L < 0) {
        const int T = -L;
        const int rows_per = T > 1000 ? T - 1000 : T;
        const int grid = (s->m + rows_per - 1) / rows_per;
#define PDHG_DT_CASE(TT, RR, NT)                                                                                \
    case TT:                                                                                                    \
        PDHG_LAUNCH(e0, e1, (k_dual_tiled<V, RR, NT>), dim3(grid), dim3(NT), s->stream, s->m, s->rp, s->ci,   \
                           (const V *)s->ahat, (const V *)s->xbar, (const double *)s->bhc, s->sense, (double *)s->y,\
                           (const double *)s->ya, (double *)s->yp, s->st, i, store);                                      \
        break;
        switch (T) {
            PDHG_DT_CASE(32, 32, 256)
            PDHG_DT_CASE(64, 64, 256)
            PDHG_DT_CASE(128, 128, 256)
            PDHG_DT_CASE(1032, 32, 64)
            PDHG_DT_CASE(1064, 64, 64)
        default:
            PDHG_DT_CASE(256, 256, 256)
        }
#undef PDHG_DT_CASE
        return;
    }
    const int grid = (int)(((int64_t)s->m * L + kBlock - 1) / kBlock);
#define PDHG_DUAL_CASE(LL)                                                                                      \
    case LL:                                                                                                    \
        PDHG_LAUNCH(e0, e1, (k_dual<V, LL>), dim3(grid), dim3(kBlock), s->stream, s->m, s->rp, s->ci,        \
                           (const V *)s->ahat, (const V *)s->xbar, (const double *)s->bhc, s->sense, (double *)s->y,\
                           (const double *)s->ya, (double *)s->yp, s->st, i, store);                                      \
        break;
    switch (L) {
        PDHG_DUAL_CASE(1)
        PDHG_DUAL_CASE(2)
        PDHG_DUAL_CASE(4)
        PDHG_DUAL_CASE(8)
        PDHG_DUAL_CASE(16)
        PDHG_DUAL_CASE(32)
    default:
        PDHG_DUAL_CASE(64)
    }
#undef PDHG_DUAL_CASE
}

// ---------------------------------------------------------------- checks ---
// Row part of a check on the candidate (xc, yc) of the scaled current model:
// rP_hat (current senses), unscaled rP = rP_hat / Dr, b'y, ||yc - ya||^2.
// In the mixed mode ex (else NULL) holds E xc, the float matrix's rounding
// error times the candidate: ax + ex is the float64 product, written back.
__global__ __launch_bounds__(kBlock) void k_check_rows(int m, double *__restrict__ ax, const double *__restrict__ ex,
                                                      const double *__restrict__ bh,
                                                      const int8_t *__restrict__ sense, const double *__restrict__ dr,
                                                      const double *__restrict__ yc, const double *__restrict__ ya,
                                                      double *__restrict__ part, int nblk, const DevState *st)
{
    if (st->done) return;
    double v[6] = {0, 0, 0, 0, 0, 0}; // PH2, P2, PINF, BTY, DY2, NAN
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        double axi = ax[i];
        if (ex) {
            axi += ex[i];
            ax[i] = axi;
        }
        double r = (double)bh[i] - axi;
        const int8_t s = sense[i];
        if (s == '<') r = r < 0.0 ? r : 0.0;
        else if (s == '>') r = r > 0.0 ? r : 0.0;
        else if (s == 'N') r = 0.0; // dropped by the dual push
        const double ru = r / dr[i];
        const double yi = (double)yc[i];
        const double dy = yi - (double)ya[i];
        v[0] += r * r;
        v[1] += ru * ru;
        v[2] = fmax(v[2], fabs(ru));
        v[3] += (double)bh[i] * yi;
        v[4] += dy * dy;
        v[5] += isfinite(yi) ? 0.0 : 1.0;
    }
    block_reduce<6>(v, 1u << 2);
    if (threadIdx.x == 0) {
        part[Q_PH2 * nblk + blockIdx.x] = v[0];
        part[Q_P2 * nblk + blockIdx.x] = v[1];
        part[Q_PINF * nblk + blockIdx.x] = v[2];
        part[Q_BTY * nblk + blockIdx.x] = v[3];
        part[Q_DY2 * nblk + blockIdx.x] = v[4];
        part[Q_NAN * nblk + blockIdx.x] = v[5];
    }
}

// Column part: lambda_hat = chat - Ahat'yc, zhat split by the finite bounds,
// rD_hat = lambda_hat - zhat, unscaled rD = rD_hat / Dc, chat'xc, bound terms
// of the dual objective, ||xc - xa||^2.
// ety (mixed mode, else NULL) = E' yc: aty + ety is the float64 product, written back.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_check_cols(int n, double *__restrict__ aty, const double *__restrict__ ety,
                                                      const double *__restrict__ ch,
                                                      const V *__restrict__ lh, const V *__restrict__ uh,
                                                      const double *__restrict__ dc, const double *__restrict__ xc,
                                                      const double *__restrict__ xa, const double *__restrict__ c0,
                                                      const double *__restrict__ l0, const double *__restrict__ u0,
                                                      int orig, double *__restrict__ part, int nblk,
                                                      const DevState *st)
{
    if (st->done) return;
    double v[7] = {0, 0, 0, 0, 0, 0, 0}; // DH2, D2, DINF, CTX, BND, DX2, NAN
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
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
        v[0] += rd * rd;
        v[1] += rdu * rdu;
        v[2] = fmax(v[2], fabs(rdu));
        v[3] += cj * xj;
        if (zp > 0.0) v[4] += lo * zp;
        if (zm > 0.0) v[4] -= hi * zm;
        v[5] += dx * dx;
        v[6] += isfinite(xj) ? 0.0 : 1.0;
    }
    block_reduce<7>(v, 1u << 2);
    if (threadIdx.x == 0) {
        part[Q_DH2 * nblk + blockIdx.x] = v[0];
        part[Q_D2 * nblk + blockIdx.x] = v[1];
        part[Q_DINF * nblk + blockIdx.x] = v[2];
        part[Q_CTX * nblk + blockIdx.x] = v[3];
        part[Q_BND * nblk + blockIdx.x] = v[4];
        part[Q_DX2 * nblk + blockIdx.x] = v[5];
        part[(Q_COUNT)*nblk + blockIdx.x] = v[6];
    }
}

// Reduce the check partials of one LP in a fixed order, then decide.
__global__ __launch_bounds__(kBlock) void k_check_final(DevState *st, const double *__restrict__ pm, int gm,
                                                       const double *__restrict__ pn, int gn, int mode, int len)
{
    if (st->done) return;
    // slot q of the row partials lives at pm[q * gm + b], of the column
    // partials at pn[q * gn + b]; slot Q_COUNT holds the column NaN count
    double v[Q_COUNT + 1];
    fold_check_partials(v, pm, (size_t)gm, 0, gm, pn, (size_t)gn, 0, gn);
    block_reduce<Q_COUNT + 1>(v, (1u << Q_PINF) | (1u << Q_DINF));
    if (threadIdx.x == 0) check_decide(st, v, mode, len);
}

// On restart: x = x_anchor = x+, y = y_anchor = y+ (candidate of the check);
// in the mixed mode the stored difference x - x_a becomes 0.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_restart_apply(int n, int m, const DevState *st, V *__restrict__ x,
                                                         double *__restrict__ xa, const double *__restrict__ xp,
                                                         double *__restrict__ y, double *__restrict__ ya,
                                                         const double *__restrict__ yp)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    if (!st->restart_flag || st->done) return;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) {
            const double v = xp[i];
            x[i] = delta ? (V)0 : (V)v;
            xa[i] = v;
        } else {
            const int64_t r = i - n;
            const double v = yp[r];
            y[r] = v;
            ya[r] = v;
        }
    }
}

// Anchored objective and right-hand side (mixed mode): chc = ch - (pa + pb)
// and bhc = bh - (qa + qb), where pa + pb = E' y_a and qa + qb = Ahat x_a in
// float64 (pb, qb may be NULL; qa may be the output itself).  At a restart the
// candidate becomes the anchor and the check has just left E' y+ in ety and
// the float64 product Ahat x+ in ax; with `always` (a phase start)
// regardless of the restart flag.
__global__ __launch_bounds__(kBlock) void k_defect_set(int n, int m, const DevState *st, int always,
                                                      const double *ch, const double *pa, const double *pb,
                                                      double *chc, const double *bh, const double *qa,
                                                      const double *qb, double *bhc)
{
    if (!always && (!st->restart_flag || st->done)) return;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) {
            chc[i] = ch[i] - (pb ? pa[i] + pb[i] : pa[i]);
        } else {
            const int64_t r = i - n;
            bhc[r] = bh[r] - (qb ? qa[r] + qb[r] : qa[r]);
        }
    }
}

__global__ void k_advance(DevState *st, int len)
{
    if (st->done) return;
    st->t += len;
    st->k0 += len;
}

template <typename V>
static void check_impl(pdhg_solver *s, const double *xc, const double *yc, double *pm, double *pn)
{
    hipStream_t st = s->stream;
    if (s->kern_a == kSell) sell_product(s, xc, s->ax);
    else row_product<V, double>(s, (const V *)s->ahat, xc, s->ax);
    check_spmv<V, double>(st, s->kern_at, s->n, s->tp, s->ti, (const V *)s->ahat_t, yc, s->aty);
    if (s->aerr) { // mixed mode: the float64 products are these plus E xc and E' yc
        row_product<float, double>(s, (const float *)s->aerr, xc, s->ex);
        check_spmv<float, double>(st, s->kern_at, s->n, s->tp, s->ti, (const float *)s->aerr_t, yc, s->ety);
    }
    const int gm = s->red_blocks_m, gn = s->red_blocks_n;
    hipLaunchKernelGGL(k_check_rows, dim3(gm), dim3(kBlock), 0, st, s->m, s->ax, (const double *)(s->aerr ? s->ex : nullptr),
                       (const double *)s->bh, s->sense, s->dr, yc, (const double *)s->ya, pm, gm, s->st);
    hipLaunchKernelGGL((k_check_cols<V>), dim3(gn), dim3(kBlock), 0, st, s->n, s->aty,
                       (const double *)(s->aerr ? s->ety : nullptr), s->ch,
                       (const V *)s->lh, (const V *)s->uh, s->dc, xc, (const double *)s->xa, s->c, s->l, s->u,
                       s->model_original ? 1 : 0, pn, gn, s->st);
}

hipError_t launch_check(pdhg_solver *s, int mode, int len)
{
    const bool use_cand = mode != 0;
    const int gm = s->red_blocks_m, gn = s->red_blocks_n;
    double *pm = s->partials;
    double *pn = s->partials + (size_t)(Q_COUNT + 1) * gm;
    // mode 0 checks the iterate at a phase start, where it is the anchor
    // (in the mixed mode x holds its difference from x_a, which is 0 there)
    const double *xc = (const double *)(use_cand ? s->xp : (s->fp32 ? s->xa : s->x));
    if (s->fp32) check_impl<float>(s, xc, (const double *)(use_cand ? s->yp : s->y), pm, pn);
    else check_impl<double>(s, xc, (const double *)(use_cand ? s->yp : s->y), pm, pn);
    hipLaunchKernelGGL(k_check_final, dim3(1), dim3(kBlock), 0, s->stream, s->st, pm, gm, pn, gn, mode, len);
    if (mode == 1 && s->hx) { // restart history for the learned push (before the restart copies)
        hipError_t e = launch_record_history(s);
        if (e != hipSuccess) return e;
    }
    if (mode == 2 && s->learned_active) { // undo learned fixes the push model's duals reject
        hipError_t e = launch_learned_undo(s);
        if (e != hipSuccess) return e;
    }
    if (mode != 0) {
        const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
        if (s->aerr) // the check left E' y+ in ety and Ahat x+ (float64) in ax
            hipLaunchKernelGGL(k_defect_set, dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->st, 0, s->ch,
                               (const double *)s->ety, (const double *)nullptr, s->chc, (const double *)s->bh,
                               (const double *)s->ax, (const double *)nullptr, s->bhc);
        if (s->fp32)
            hipLaunchKernelGGL((k_restart_apply<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->st,
                               (float *)s->x, (double *)s->xa, (const double *)s->xp, (double *)s->y, (double *)s->ya,
                               (const double *)s->yp);
        else
            hipLaunchKernelGGL((k_restart_apply<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->st,
                               (double *)s->x, (double *)s->xa, (const double *)s->xp, (double *)s->y, (double *)s->ya,
                               (const double *)s->yp);
    }
    return hipGetLastError();
}

// bad |= 1 if some row of `ptr` (rows + 1 entries) does not hold exactly D entries
__global__ __launch_bounds__(kBlock) void k_uniform_rows(int rows, const int *__restrict__ ptr, int D,
                                                        unsigned *__restrict__ bad)
{
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r <= rows; r += (int64_t)gridDim.x * kBlock)
        if (ptr[r] != (int)(r * D)) {
            atomicOr(bad, 1u);
            return;
        }
}

__global__ void k_zero_u32(unsigned *p) { *p = 0u; }

hipError_t detect_uniform_columns(pdhg_solver *s)
{
    s->udeg_at = 0;
    if (s->n <= 0 || s->nnz % s->n != 0) return hipSuccess;
    const int D = s->nnz / s->n;
    if (D < 1 || D > 3) return hipSuccess;
    unsigned *d_bad = (unsigned *)s->redout; // small scratch of the handle, free outside a check
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s->stream, d_bad);
    hipLaunchKernelGGL(k_uniform_rows, dim3(grid_for((int64_t)s->n + 1, kBlock, 4096)), dim3(kBlock), 0, s->stream,
                       s->n, s->tp, D, d_bad);
    unsigned bad = 1;
    hipError_t e = hipMemcpyAsync(&bad, d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess && bad == 0) s->udeg_at = D;
    return e;
}

hipError_t defect_refresh(pdhg_solver *s)
{
    s->defect_stale = false;
    if (!s->aerr) {
        defect_alias(s);
        return hipSuccess;
    }
    hipStream_t st = s->stream;
    const double *xa = (const double *)s->xa, *ya = (const double *)s->ya;
    // fl32(Ahat) x_a into bhc, E x_a into ex, E' y_a into ety
    if (s->kern_a == kSell) sell_product(s, xa, s->bhc);
    else row_product<float, double>(s, (const float *)s->ahat, xa, s->bhc);
    row_product<float, double>(s, (const float *)s->aerr, xa, s->ex);
    check_spmv<float, double>(st, s->kern_at, s->n, s->tp, s->ti, (const float *)s->aerr_t, ya, s->ety);
    const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
    hipLaunchKernelGGL(k_defect_set, dim3(g), dim3(kBlock), 0, st, s->n, s->m, s->st, 1, s->ch,
                       (const double *)s->ety, (const double *)nullptr, s->chc, (const double *)s->bh,
                       (const double *)s->bhc, (const double *)s->ex, s->bhc);
    return hipGetLastError();
}

hipError_t launch_advance(pdhg_solver *s, int len)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s->stream, s->st, len);
    return hipGetLastError();
}

hipError_t launch_iterations(pdhg_solver *s, int count, bool check_at_end, int mode, bool timed_launch)
{
    const int timed = (timed_launch && count >= 2) ? count / 2 : -1; // one sampled iteration
    for (int i = 0; i < count; i++) {
        const int store = (check_at_end && i == count - 1) ? 1 : 0;
        hipEvent_t *ev = i == timed ? s->ev : nullptr;
        if (s->fp32) launch_primal<float>(s, i, store, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
        else launch_primal<double>(s, i, store, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
        if (s->fp32) launch_dual<float>(s, i, store, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
        else launch_dual<double>(s, i, store, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (check_at_end) return launch_check(s, mode, count);
    return launch_advance(s, count);
}

// capture `len` iterations + the check into a graph (replayed per cycle)
hipError_t capture_cycle(pdhg_solver *s, int len, int mode)
{
    if (s->graph_exec && s->graph_len == len && s->graph_mode == mode) return hipSuccess;
    if (s->graph_exec) {
        hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t el = launch_iterations(s, len, true, mode, false);
    e = hipStreamEndCapture(s->stream, &g);
    if (el != hipSuccess) return el;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    s->graph_len = len;
    s->graph_mode = mode;
    return hipSuccess;
}

// ----------------------------------------------------------- phase start ---
// partial sums of chat^2 (cols) and bhat^2 (rows) for the initial weight
template <typename V>
__global__ __launch_bounds__(kBlock) void k_sumsq2(int n, const V *__restrict__ a, int m, const double *__restrict__ bvec,
                                                  double *__restrict__ part, int nblk)
{
    double v[2] = {0.0, 0.0};
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const double q = (double)a[j];
        v[0] += q * q;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const double q = (double)bvec[i];
        v[1] += q * q;
    }
    block_reduce<2>(v, 0u);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[nblk + blockIdx.x] = v[1];
    }
}

// omega = ||chat|| / ||bhat|| (both > 1e-10, else 1); tau, sigma; counters reset
__global__ __launch_bounds__(kBlock) void k_phase_start(DevState *st, const double *__restrict__ part, int nblk)
{
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        v[0] += part[b];
        v[1] += part[nblk + b];
    }
    block_reduce<2>(v, 0u);
    if (threadIdx.x != 0) return;
    const double nc = sqrt(v[0]), nb = sqrt(v[1]);
    const double om = (nc > 1e-10 && nb > 1e-10) ? nc / nb : 1.0;
    st->omega = om;
    st->tau = st->eta / om;
    st->sigma = st->eta * om;
    st->k0 = 0;
    st->t = 0;
    st->restarts = 0;
    st->done = 0;
    st->status = PDHG_ITER_LIMIT;
    st->restart_flag = 0;
    st->checks = 0;
}

// x = clamp(0, lhat, uhat), y = 0, anchors = (x, y) (mixed mode: x_a = that
// point, stored difference x - x_a = 0)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_start_point(int n, int m, const V *__restrict__ lh, const V *__restrict__ uh,
                                                       V *__restrict__ x, double *__restrict__ xa,
                                                       double *__restrict__ y, double *__restrict__ ya)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) {
            V v = (V)0;
            v = v < lh[i] ? lh[i] : v;
            v = v > uh[i] ? uh[i] : v;
            x[i] = delta ? (V)0 : v;
            xa[i] = (double)v;
        } else {
            y[i - n] = 0.0;
            ya[i - n] = 0.0;
        }
    }
}

// anchors = the current iterate (mixed mode: x_a += x - x_a, then the
// differences are 0)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_copy_anchor(int n, int m, V *__restrict__ x, double *__restrict__ xa,
                                                       const double *__restrict__ y, double *__restrict__ ya)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) {
            if (delta) {
                xa[i] += (double)x[i];
                x[i] = (V)0;
            } else {
                xa[i] = (double)x[i];
            }
        } else {
            ya[i - n] = y[i - n];
        }
    }
}

template <typename V>
static void start_vectors(pdhg_solver *s, bool fresh_start)
{
    hipStream_t st = s->stream;
    const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
    if (fresh_start)
        hipLaunchKernelGGL((k_start_point<V>), dim3(g), dim3(kBlock), 0, st, s->n, s->m, (const V *)s->lh,
                           (const V *)s->uh, (V *)s->x, (double *)s->xa, (double *)s->y, (double *)s->ya);
    else
        hipLaunchKernelGGL((k_copy_anchor<V>), dim3(g), dim3(kBlock), 0, st, s->n, s->m, (V *)s->x, (double *)s->xa,
                           (const double *)s->y, (double *)s->ya);
}

// x = clamp(0, lhat, uhat), y = 0 (fresh) or anchors = current (x, y)
hipError_t launch_start_vectors(pdhg_solver *s, bool fresh_start)
{
    if (s->fp32) start_vectors<float>(s, fresh_start);
    else start_vectors<double>(s, fresh_start);
    return hipGetLastError();
}

template <typename V>
static hipError_t phase_start(pdhg_solver *s, bool fresh_start)
{
    hipStream_t st = s->stream;
    s->defect_stale = true; // a new anchor (and possibly a new model)
    start_vectors<V>(s, fresh_start);
    const int nb = grid_for(s->n > s->m ? s->n : s->m, kBlock, kMaxRedBlocks);
    hipLaunchKernelGGL((k_sumsq2<double>), dim3(nb), dim3(kBlock), 0, st, s->n, s->ch, s->m, (const double *)s->bh,
                       s->partials, nb);
    hipLaunchKernelGGL(k_phase_start, dim3(1), dim3(kBlock), 0, st, s->st, s->partials, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_check(s, 0, 0); // anchor KKT parts of the start point
}

// 1 + ||b||_2 and 1 + ||c||_2 of the original model (relative tests)
__global__ __launch_bounds__(kBlock) void k_set_norms(DevState *st, const double *__restrict__ part, int nblk)
{
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        v[0] += part[b];
        v[1] += part[nblk + b];
    }
    block_reduce<2>(v, 0u);
    if (threadIdx.x != 0) return;
    st->nc1 = 1.0 + sqrt(v[0]);
    st->nb1 = 1.0 + sqrt(v[1]);
}

hipError_t init_norms(pdhg_solver *s)
{
    const int nb = grid_for(s->n > s->m ? s->n : s->m, kBlock, kMaxRedBlocks);
    hipLaunchKernelGGL((k_sumsq2<double>), dim3(nb), dim3(kBlock), 0, s->stream, s->n, s->c, s->m, s->b, s->partials, nb);
    hipLaunchKernelGGL(k_set_norms, dim3(1), dim3(kBlock), 0, s->stream, s->st, s->partials, nb);
    return hipGetLastError();
}

hipError_t init_iteration(pdhg_solver *s)
{
    return s->fp32 ? phase_start<float>(s, true) : phase_start<double>(s, true);
}

// caller's start point (xu, yu unscaled) -> x = clamp(x / Dc, lhat, uhat),
// y = y / Dr projected on the sign of its row (the projections of the method);
// mixed mode: x_a = that x in float64 and the stored difference 0
template <typename V>
__global__ __launch_bounds__(kBlock) void k_set_start(int n, int m, const double *__restrict__ xu,
                                                     const double *__restrict__ yu, const double *__restrict__ dc,
                                                     const double *__restrict__ dr, const V *__restrict__ lh,
                                                     const V *__restrict__ uh, const int8_t *__restrict__ sense,
                                                     V *__restrict__ x, double *__restrict__ xa, double *__restrict__ y)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) {
            const double v = fmin(fmax(xu[i] / dc[i], (double)lh[i]), (double)uh[i]);
            if (delta) {
                xa[i] = v;
                x[i] = (V)0;
            } else {
                x[i] = (V)v;
            }
        } else {
            const int64_t r = i - n;
            double v = yu[r] / dr[r];
            if (sense[r] == '<') v = fmin(v, 0.0);
            else if (sense[r] == '>') v = fmax(v, 0.0);
            y[r] = v;
        }
    }
}

hipError_t set_start(pdhg_solver *s)
{
    const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
    if (s->fp32) {
        hipLaunchKernelGGL((k_set_start<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->xu, s->yu, s->dc,
                           s->dr, (const float *)s->lh, (const float *)s->uh, s->sense, (float *)s->x, (double *)s->xa,
                           (double *)s->y);
        return phase_start<float>(s, false);
    }
    hipLaunchKernelGGL((k_set_start<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->xu, s->yu, s->dc,
                       s->dr, (const double *)s->lh, (const double *)s->uh, s->sense, (double *)s->x, (double *)s->xa,
                       (double *)s->y);
    return phase_start<double>(s, false);
}

// (xp, yp) <- (x, y): the candidate of a phase that has not reached a check
template <typename V>
__global__ __launch_bounds__(kBlock) void k_candidate_from_iterate(int n, int m, const V *__restrict__ x,
                                                                  const double *__restrict__ xa,
                                                                  double *__restrict__ xp, const double *__restrict__ y,
                                                                  double *__restrict__ yp)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) xp[i] = iterate_value<V>(x[i], xa[i]);
        else yp[i - n] = y[i - n];
    }
}

hipError_t candidate_from_iterate(pdhg_solver *s)
{
    const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL((k_candidate_from_iterate<float>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m,
                           (const float *)s->x, (const double *)s->xa, (double *)s->xp, (const double *)s->y,
                           (double *)s->yp);
    else
        hipLaunchKernelGGL((k_candidate_from_iterate<double>), dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m,
                           (const double *)s->x, (const double *)s->xa, (double *)s->xp, (const double *)s->y,
                           (double *)s->yp);
    return hipGetLastError();
}

// xo = Dc (xh + xd) (xd: an optional float difference), yo = Dr yh
__global__ __launch_bounds__(kBlock) void k_unscale(int n, int m, const double *__restrict__ dc,
                                                   const double *__restrict__ dr, const double *__restrict__ xh,
                                                   const float *__restrict__ xd, const double *__restrict__ yh,
                                                   double *__restrict__ xo, double *__restrict__ yo)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += (int64_t)gridDim.x * kBlock) {
        if (i < n) {
            if (xo) xo[i] = dc[i] * (xd ? xh[i] + (double)xd[i] : xh[i]);
        } else {
            if (yo) yo[i - n] = dr[i - n] * yh[i - n];
        }
    }
}

hipError_t unscale(pdhg_solver *s, const double *xh, const double *yh, double *xo, double *yo)
{
    const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
    hipLaunchKernelGGL(k_unscale, dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->dc, s->dr, xh,
                       (const float *)nullptr, yh, xo, yo);
    return hipGetLastError();
}

hipError_t unscale_iterate(pdhg_solver *s, double *xo, double *yo)
{
    const int g = grid_for((int64_t)s->n + s->m, kBlock, 8192);
    if (s->fp32)
        hipLaunchKernelGGL(k_unscale, dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->dc, s->dr,
                           (const double *)s->xa, (const float *)s->x, (const double *)s->y, xo, yo);
    else
        hipLaunchKernelGGL(k_unscale, dim3(g), dim3(kBlock), 0, s->stream, s->n, s->m, s->dc, s->dr,
                           (const double *)s->x, (const float *)nullptr, (const double *)s->y, xo, yo);
    return hipGetLastError();
}

// ------------------------------------------------------------- KKT report ---
// rows: rP (original senses), its inf-norm, b'y, slack counts
__global__ __launch_bounds__(kBlock) void k_report_rows(int m, const double *__restrict__ b, const int8_t *__restrict__ s0,
                                                       const double *__restrict__ ax, const double *__restrict__ y,
                                                       double *__restrict__ part, int nblk)
{
    const double tol = 1e-6;
    double v[6] = {0, 0, 0, 0, 0, 0}; // P2, PINF, BTY, POFF, DZERO, CAND
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        double r = b[i] - ax[i];
        const int8_t sn = s0[i];
        if (sn == '<') r = r < 0.0 ? r : 0.0;
        else if (sn == '>') r = r > 0.0 ? r : 0.0;
        v[0] += r * r;
        v[1] = fmax(v[1], fabs(r));
        v[2] += b[i] * y[i];
        if (sn != '=') {
            const double slack = (sn == '<') ? (b[i] - ax[i]) : (ax[i] - b[i]);
            const double zs = (sn == '<') ? -y[i] : y[i];
            const bool off = slack > tol;
            v[3] += off ? 1.0 : 0.0;
            v[4] += fabs(zs) <= tol ? 1.0 : 0.0;
            v[5] += (off && fabs(zs) < tol) ? 1.0 : 0.0;
        }
    }
    block_reduce<6>(v, 1u << 1);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; q++) part[q * nblk + blockIdx.x] = v[q];
}

// columns: z split, rD, c'x, bound terms of the dual objective, counts
__global__ __launch_bounds__(kBlock) void k_report_cols(int n, const double *__restrict__ c, const double *__restrict__ l,
                                                       const double *__restrict__ u, const double *__restrict__ aty,
                                                       const double *__restrict__ x, double *__restrict__ zout,
                                                       double *__restrict__ part, int nblk)
{
    const double tol = 1e-6;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // D2, DINF, CTX, BND, POFF, DZERO, CAND, unused
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const double lam = c[j] - aty[j];
        const double zp = (!is_inf_lo(l[j]) && lam > 0.0) ? lam : 0.0;
        const double zm = (!is_inf_up(u[j]) && lam < 0.0) ? -lam : 0.0;
        const double z = zp - zm;
        const double rd = lam - z;
        v[0] += rd * rd;
        v[1] = fmax(v[1], fabs(rd));
        v[2] += c[j] * x[j];
        if (zp > 0.0) v[3] += l[j] * zp;
        if (zm > 0.0) v[3] -= u[j] * zm;
        const double zc = z;
        const bool off = (x[j] - l[j] > tol) && (u[j] - x[j] > tol);
        v[4] += off ? 1.0 : 0.0;
        v[5] += fabs(zc) <= tol ? 1.0 : 0.0;
        v[6] += (off && fabs(zc) < tol) ? 1.0 : 0.0;
        if (zout) zout[j] = z;
    }
    block_reduce<8>(v, 1u << 1);
    if (threadIdx.x == 0)
        for (int q = 0; q < 8; q++) part[q * nblk + blockIdx.x] = v[q];
}

__global__ __launch_bounds__(kBlock) void k_report_final(const double *__restrict__ pr, int gm, const double *__restrict__ pc,
                                                        int gn, double *__restrict__ out)
{
    double v[13];
#pragma unroll
    for (int q = 0; q < 6; q++) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < gm; b += kBlock) acc = (q == 1) ? fmax(acc, pr[q * gm + b]) : acc + pr[q * gm + b];
        v[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < 7; q++) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < gn; b += kBlock) acc = (q == 1) ? fmax(acc, pc[q * gn + b]) : acc + pc[q * gn + b];
        v[6 + q] = acc;
    }
    block_reduce<13>(v, (1u << 1) | (1u << 7));
    if (threadIdx.x != 0) return;
    // rows: P2 PINF BTY POFF DZERO CAND | cols: D2 DINF CTX BND POFF DZERO CAND
    out[R_P2] = v[0];
    out[R_PINF] = v[1];
    out[R_BTY] = v[2];
    out[R_D2] = v[6];
    out[R_DINF] = v[7];
    out[R_CTX] = v[8];
    out[R_BND] = v[9];
    out[R_POFF] = v[3] + v[10];
    out[R_DZERO] = v[4] + v[11];
    out[R_CAND] = v[5] + v[12];
}

hipError_t report(pdhg_solver *s, const double *x, const double *y, double *z, pdhg_kkt_report *k)
{
    hipStream_t st = s->stream;
    spmv<double, double, double, double>(st, s->lanes_a, s->m, s->rp, s->ci, s->av, x, s->ax);
    spmv<double, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, s->atv, y, s->aty);
    const int gm = s->red_blocks_m, gn = s->red_blocks_n;
    double *pr = s->partials;
    double *pc = s->partials + (size_t)6 * gm;
    hipLaunchKernelGGL(k_report_rows, dim3(gm), dim3(kBlock), 0, st, s->m, s->b, s->sense0, s->ax, y, pr, gm);
    hipLaunchKernelGGL(k_report_cols, dim3(gn), dim3(kBlock), 0, st, s->n, s->c, s->l, s->u, s->aty, x, z, pc, gn);
    hipLaunchKernelGGL(k_report_final, dim3(1), dim3(kBlock), 0, st, pr, gm, pc, gn, s->redout);
    hipMemcpyAsync(s->rep_host, s->redout, sizeof(double) * R_COUNT, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    const double *v = s->rep_host;
    const double nb1 = s->st_host->nb1, nc1 = s->st_host->nc1;
    k->rp2 = sqrt(v[R_P2]);
    k->rd2 = sqrt(v[R_D2]);
    k->rpinf = v[R_PINF];
    k->rdinf = v[R_DINF];
    k->pobj = v[R_CTX];
    k->dobj = v[R_BTY] + v[R_BND];
    k->gap = k->pobj - k->dobj;
    k->rel_p = k->rp2 / nb1;
    k->rel_d = k->rd2 / nc1;
    k->rel_gap = fabs(k->gap) / (1.0 + fabs(k->pobj) + fabs(k->dobj));
    k->p_off = (int64_t)v[R_POFF];
    k->d_zero = (int64_t)v[R_DZERO];
    k->candidates = (int64_t)v[R_CAND];
    k->est_primal = k->p_off > s->m ? k->p_off - s->m : 0;
    k->est_dual = s->m > k->d_zero ? s->m - k->d_zero : 0;
    return hipGetLastError();
}

// ------------------------------------------------------------- corner push ---
// Algorithm 1 on the columns: ub_j <- x_j if z_j > eps_abs, lb_j <- x_j if
// z_j < -eps_abs (bounds stored scaled: the scaled solve candidate itself),
// objective Uniform[0,1) scaled like c, start x at the solve's x.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_push_cols(int n, const double *__restrict__ z, const double *__restrict__ xs,
                                                     const double *__restrict__ dc, double eps_abs, uint64_t seed,
                                                     double scale, V *__restrict__ lh, V *__restrict__ uh,
                                                     double *__restrict__ ch, V *__restrict__ x, double *__restrict__ xa,
                                                     double *__restrict__ part, int nblk)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    double v[2] = {0.0, 0.0}; // fixes at the lower, upper side
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const double xv = xs[j];
        if (z[j] > eps_abs) {
            uh[j] = (V)xv;
            v[1] += 1.0;
        } else if (z[j] < -eps_abs) {
            lh[j] = (V)xv;
            v[0] += 1.0;
        }
        ch[j] = dc[j] * (scale * push_unit(seed, j));
        x[j] = delta ? (V)0 : (V)xv; // the iterate starts at the solve's x (mixed mode: as the anchor)
        xa[j] = xv;
    }
    block_reduce<2>(v, 0u);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[nblk + blockIdx.x] = v[1];
    }
}

// inequality rows whose slack reduced cost is non-trivial become equalities; y = 0
__global__ __launch_bounds__(kBlock) void k_push_rows(int m, const double *__restrict__ yu, double eps_abs,
                                                     int8_t *__restrict__ sense, double *__restrict__ y,
                                                     double *__restrict__ part)
{
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const int8_t sn = sense[i];
        if ((sn == '<' && yu[i] < -eps_abs) || (sn == '>' && yu[i] > eps_abs)) {
            sense[i] = '=';
            v[0] += 1.0;
        }
        y[i] = 0.0;
    }
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_sum3(const double *__restrict__ p, int n0, int n1, double *__restrict__ out)
{
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n0; b += kBlock) {
        v[0] += p[b];
        v[1] += p[n0 + b];
    }
    for (int b = threadIdx.x; b < n1; b += kBlock) v[2] += p[2 * n0 + b];
    block_reduce<3>(v, 0u);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
        out[2] = v[2];
    }
}

template <typename V>
static hipError_t push_setup_impl(pdhg_solver *s, uint64_t seed, pdhg_push_result *r, double theta)
{
    hipStream_t st = s->stream;
    const int gn = s->red_blocks_n, gm = s->red_blocks_m;
    double *pcnt = s->partials + (size_t)(Q_COUNT + 1) * (gm + gn); // past the check slots
    hipLaunchKernelGGL((k_push_cols<V>), dim3(gn), dim3(kBlock), 0, st, s->n, s->zsol, (const double *)s->xs, s->dc,
                       s->p.eps_abs, seed, s->p.push_obj_scale, (V *)s->lh, (V *)s->uh, s->ch, (V *)s->x,
                       (double *)s->xa, pcnt, gn);
    hipLaunchKernelGGL(k_push_rows, dim3(gm), dim3(kBlock), 0, st, s->m, s->yu, s->p.eps_abs, s->sense, (double *)s->y,
                       pcnt + 2 * gn);
    hipLaunchKernelGGL(k_sum3, dim3(1), dim3(kBlock), 0, st, pcnt, gn, gm, s->redout);
    if (theta > 0.0) { // learned warm start on the columns the plain rule leaves free
        hipError_t e = launch_learned_fix(s, theta);
        if (e != hipSuccess) return e;
    }
    hipMemcpyAsync(s->rep_host, s->redout, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    r->n_fix_lower = (int64_t)s->rep_host[0];
    r->n_fix_upper = (int64_t)s->rep_host[1];
    r->n_rows_to_eq = (int64_t)s->rep_host[2];
    return phase_start<V>(s, false);
}

hipError_t push_setup(pdhg_solver *s, uint64_t seed, pdhg_push_result *r, double theta)
{
    s->model_original = false;
    return s->fp32 ? push_setup_impl<float>(s, seed, r, theta) : push_setup_impl<double>(s, seed, r, theta);
}

// -------------------------------------------------------- dual push ---
// The mirror image of Algorithm 1 on the dual side, anchored at the solve's
// ybar as Algorithm 1 is at its x.  Rows: an inequality row with slack beyond
// eps_abs leaves the push model (sense 'N'), its dual held at ybar_i; yn
// carries ybar on those rows and 0 elsewhere.  ax = A x (unscaled).
__global__ __launch_bounds__(kBlock) void k_dpush_rows(int m, const int8_t *__restrict__ sense0,
                                                      const double *__restrict__ b, const double *__restrict__ ax,
                                                      const double *__restrict__ yu, double eps_abs,
                                                      int8_t *__restrict__ sense, double *__restrict__ yn,
                                                      double *__restrict__ part)
{
    double v[1] = {0.0}; // rows dropped, dual held at the solve's
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const int8_t sn = sense0[i];
        const double slack = sn == '<' ? b[i] - ax[i] : (sn == '>' ? ax[i] - b[i] : 0.0);
        const bool drop = sn != '=' && slack > eps_abs;
        sense[i] = drop ? (int8_t)'N' : sn;
        yn[i] = drop ? yu[i] : 0.0;
        v[0] += drop ? 1.0 : 0.0;
    }
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Columns: the cone of push variable w_j from where the solve's x sits: R off
// both bounds (z_j = 0 on the face), R+ within eps_abs of the lower bound only
// (z_j >= 0), R- of the upper bound only (z_j <= 0), {0} of both (z_j free);
// bounds 0 or infinite, the same scaled and unscaled.  Objective
// c~ = c - A_N'ybar_N - r, r_j the part of lambda_j = c_j - a_j'ybar that the
// cone rejects, so ybar lies on the face; stored scaled.  w0 (unscaled, for
// the anchored right-hand side A w0) is U_j in the cone; the iterate starts at 0.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_dpush_cols(int n, const double *__restrict__ xu, const double *__restrict__ l,
                                                      const double *__restrict__ u, const double *__restrict__ c,
                                                      const double *__restrict__ aty, const double *__restrict__ atyn,
                                                      const double *__restrict__ dc, double eps_abs, uint64_t seed,
                                                      V *__restrict__ lh, V *__restrict__ uh, double *__restrict__ ch,
                                                      V *__restrict__ x, double *__restrict__ xa,
                                                      double *__restrict__ w0, double *__restrict__ part, int nblk)
{
    double v[1] = {0.0}; // columns off both bounds
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const double xj = xu[j];
        const bool at_lo = !is_inf_lo(l[j]) && xj - l[j] <= eps_abs;
        const bool at_up = !is_inf_up(u[j]) && u[j] - xj <= eps_abs;
        lh[j] = at_lo ? (V)0 : (V)-INFINITY;
        uh[j] = at_up ? (V)0 : (V)INFINITY;
        const double lam = c[j] - aty[j];
        const double rj = (at_lo && at_up) ? 0.0 : at_lo ? fmin(lam, 0.0) : at_up ? fmax(lam, 0.0) : lam;
        ch[j] = dc[j] * (c[j] - atyn[j] - rj);
        const double uj = push_unit(seed, j);
        w0[j] = (at_lo && at_up) ? 0.0 : (at_up ? -uj : uj);
        x[j] = (V)0;
        xa[j] = 0.0;
        v[0] += (!at_lo && !at_up) ? 1.0 : 0.0;
    }
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[nblk + blockIdx.x] = 0.0;
    }
}

// Rows kept: y starts at the solve's and the right-hand side is the anchored
// g_i = scale (a_i'w0 - s_i v_i), scaled like b, v_i = U_(n+i), s_i = +1 on
// '>' rows, -1 on '<', 0 on '='; bh holds a_i'w0 (unscaled) on entry.
// Dropped rows: bh = 0, y = 0 (their dual lives in the objective).
__global__ __launch_bounds__(kBlock) void k_dpush_rhs(int m, int n, const int8_t *__restrict__ sense,
                                                     const double *__restrict__ dr, const double *__restrict__ ys,
                                                     uint64_t seed, double scale, double *__restrict__ bh,
                                                     double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const int8_t sn = sense[i];
        if (sn == 'N') {
            bh[i] = 0.0;
            y[i] = 0.0;
        } else {
            const double aw = bh[i];
            const double vi = push_unit(seed, (int64_t)n + i);
            const double g = sn == '>' ? aw - vi : (sn == '<' ? aw + vi : aw);
            bh[i] = dr[i] * (scale * g);
            y[i] = ys[i];
        }
    }
}

// The pushed y: the push's on the rows kept, the solve's on the dropped ones.
__global__ __launch_bounds__(kBlock) void k_dpush_final(int m, const int8_t *__restrict__ sense,
                                                       const double *__restrict__ yu, double *__restrict__ ypush)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
        if (sense[i] == 'N') ypush[i] = yu[i];
}

// Needs report() of (xk, yu) just before: s->ax holds A xk and s->aty A'yu.
// xk is the solve's x or the corner push's xhat (unscaled).  w0 (n) and yn
// (m) are float64 work buffers of the caller; atyn (n) another.
template <typename V>
static hipError_t dual_push_setup_impl(pdhg_solver *s, uint64_t seed, const double *xk, double *w0, double *yn,
                                       double *atyn, int64_t *n_cols_free, int64_t *n_rows_fixed)
{
    hipStream_t st = s->stream;
    const int gn = s->red_blocks_n, gm = s->red_blocks_m;
    double *pcnt = s->partials + (size_t)(Q_COUNT + 1) * (gm + gn); // past the check slots
    hipLaunchKernelGGL(k_dpush_rows, dim3(gm), dim3(kBlock), 0, st, s->m, s->sense0, s->b, s->ax, s->yu, s->p.eps_abs,
                       s->sense, yn, pcnt + 2 * gn);
    spmv<double, double, double, double>(st, s->lanes_at, s->n, s->tp, s->ti, s->atv, yn, atyn);
    hipLaunchKernelGGL((k_dpush_cols<V>), dim3(gn), dim3(kBlock), 0, st, s->n, xk, s->l, s->u, s->c, s->aty, atyn,
                       s->dc, s->p.eps_abs, seed, (V *)s->lh, (V *)s->uh, s->ch, (V *)s->x, (double *)s->xa, w0,
                       pcnt, gn);
    spmv<double, double, double, double>(st, s->lanes_a, s->m, s->rp, s->ci, s->av, w0, (double *)s->bh);
    hipLaunchKernelGGL(k_dpush_rhs, dim3(gm), dim3(kBlock), 0, st, s->m, s->n, s->sense, s->dr, (const double *)s->ys,
                       seed, s->p.push_obj_scale, (double *)s->bh, (double *)s->y);
    hipLaunchKernelGGL(k_sum3, dim3(1), dim3(kBlock), 0, st, pcnt, gn, gm, s->redout);
    hipMemcpyAsync(s->rep_host, s->redout, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *n_cols_free = (int64_t)s->rep_host[0];
    *n_rows_fixed = (int64_t)s->rep_host[2];
    return phase_start<V>(s, false);
}

hipError_t dual_push_setup(pdhg_solver *s, uint64_t seed, const double *xk, double *w0, double *yn, double *atyn,
                           int64_t *n_cols_free, int64_t *n_rows_fixed)
{
    s->model_original = false;
    return s->fp32 ? dual_push_setup_impl<float>(s, seed, xk, w0, yn, atyn, n_cols_free, n_rows_fixed)
                   : dual_push_setup_impl<double>(s, seed, xk, w0, yn, atyn, n_cols_free, n_rows_fixed);
}

hipError_t dual_push_finish(pdhg_solver *s)
{
    const int g = grid_for(s->m, kBlock, 8192);
    hipLaunchKernelGGL(k_dpush_final, dim3(g), dim3(kBlock), 0, s->stream, s->m, s->sense, s->yu, s->ypush);
    return hipGetLastError();
}

// ------------------------------------------------------- kernel choice ---
// From measured sweeps on the 100k x 400k, 7k x 10M and 800k x 3.2M LPs:
// LDS tiles up to 48 entries per row (256-row tiles for 2-3 entries: 56 against
// 63 us for one lane per row on the multicommodity primal); beyond, lane
// groups: for the primal half sized to the mean, at most 32; for the dual
// half per row segment (on the 7k x 10M dual, row segments of 32 and 16
// lanes beat one 32-lane group per row, 64 lanes, one workgroup per row and
// the sliced ELLPACK layout, which stay available as explicit or autotuned
// choices).
int choose_kernel(double mean_row, bool dual_half)
{
    if (mean_row <= 3.0) return -256; // 2-3 entries per row: 256-row tiles match or beat one lane per row
    if (mean_row <= 16.0) return -64; // measured best for 6 and 15 entries per row
    if (mean_row <= 48.0) return -32; // 24 entries per row
    // long rows: a lane group per row; the dual half picks the width per
    // segment of rows of one kind (plan_row_segments)
    if (dual_half) return kRowSegs;
    const int l = lanes_for_mean(mean_row);
    return l > 32 ? 32 : l;
}

// Segments from the rows' column pattern: a row is contiguous when at least
// half of its entries continue in the next column; runs of rows of one kind
// (rows of fewer than two entries join the current run) become segments.
// Each segment spreads over all 8 XCDs, so every XCD gets its share of each
// kind of row.  Lane-group width per segment from its mean row length l: the
// smallest power of two w >= l/4 (about one round of four loads per lane), at
// most 32; spread-out rows take 16 once l >= 512, where sharing each gathered
// line among more rows of a workgroup outweighs the extra rounds (sink rows of
// 2,000 entries at stride 5,000: 16 lanes beat 8 and 32; sink rows of 90
// entries: 32 beat 16).  More runs than kMaxSegs give one segment of 32.
static RowSegs row_segments(const std::vector<int> &rp, const std::vector<int> &adj)
{
    const int m = (int)adj.size();
    std::vector<int> start, cls;
    for (int r = 0; r < m; r++) {
        const int len = rp[r + 1] - rp[r];
        int c = cls.empty() ? 0 : cls.back();
        if (len >= 2) c = 2 * adj[r] >= len - 1 ? 1 : 0;
        if (cls.empty() || c != cls.back()) {
            start.push_back(r);
            cls.push_back(c);
        }
    }
    RowSegs sg;
    if (m <= 0) return sg;
    const bool one = (int)start.size() > kMaxSegs;
    sg.count = one ? 1 : (int)start.size();
    for (int k = 0; k < sg.count; k++) {
        const int r0 = one ? 0 : start[k], r1 = one || k + 1 == sg.count ? m : start[k + 1];
        const double mean = (double)(rp[r1] - rp[r0]) / (r1 - r0);
        int w = 1;
        while (w < 32 && 4 * w < mean) w <<= 1;
        if (one) w = 32;
        else if (cls[k] == 0 && mean >= 512.0) w = 16;
        sg.row0[k] = r0;
        sg.lanes[k] = w;
        const int64_t blocks = ((int64_t)(r1 - r0) * w + kBlock - 1) / kBlock;
        sg.blk0[k + 1] = sg.blk0[k] + (int)((blocks + 7) / 8 * 8);
    }
    sg.row0[sg.count] = m;
    return sg;
}

hipError_t plan_row_segments(pdhg_solver *s)
{
    const int m = s->m;
    s->segs = RowSegs{};
    if (m <= 0) return hipSuccess;
    std::vector<int> rp((size_t)m + 1), adj((size_t)m);
    int *d_adj = nullptr;
    hipError_t e = hipMalloc(&d_adj, sizeof(int) * (size_t)m);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_row_adjacent, dim3(grid_for((int64_t)m * 64, kBlock, 1 << 30)), dim3(kBlock), 0,
                           s->stream, m, s->rp, s->ci, d_adj);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(adj.data(), d_adj, sizeof(int) * (size_t)m, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(rp.data(), s->rp, sizeof(int) * ((size_t)m + 1), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream); // the host vectors die on return
    if (d_adj) (void)hipFree(d_adj);
    if (e != hipSuccess) return e;
    s->segs = row_segments(rp, adj);
    if (s->p.verbosity > 0)
        for (int k = 0; k < s->segs.count; k++)
            fprintf(stderr, "[pdhg] dual row segment %d: rows %d..%d, %d lanes, %d workgroups\n", k, s->segs.row0[k],
                    s->segs.row0[k + 1] - 1, s->segs.lanes[k], s->segs.blk0[k + 1] - s->segs.blk0[k]);
    return hipSuccess;
}

// Time every candidate of each half on scratch output vectors (3 launches
// each after one warm-up) and keep the fastest.  The iterate is untouched.
hipError_t autotune(pdhg_solver *s)
{
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
    const int cands[] = {-32, -64, -128, -256, -1032, -1064, 1, 2, 4, 8, 16, 32, 64, kRowBlock, kSell, kRowSegs};
    void *keep[5] = {s->x, s->xbar, s->xp, s->y, s->yp};
    s->x = sx;
    s->xbar = sxbar;
    s->xp = sxp;
    s->y = sy;
    s->yp = syp;
    for (int half = 0; half < 2 && e == hipSuccess; half++) {
        float best = 1e30f;
        int best_k = half == 0 ? s->kern_at : s->kern_a;
        for (int c : cands) {
            if (c == kSell && (half == 0 || !s->sell_idx)) continue; // dual half, layout built
            if (c == kRowSegs && (half == 0 || s->segs.count == 0)) continue; // dual half, segments planned
            if (half == 0) s->kern_at = c;
            else s->kern_a = c;
            for (int rep = 0; rep < 4; rep++) {
                if (rep == 1) hipEventRecord(e0, s->stream);
                if (half == 0) {
                    if (s->fp32) launch_primal<float>(s, 0, 0);
                    else launch_primal<double>(s, 0, 0);
                } else {
                    if (s->fp32) launch_dual<float>(s, 0, 0);
                    else launch_dual<double>(s, 0, 0);
                }
            }
            hipEventRecord(e1, s->stream);
            e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            if (ms < best) {
                best = ms;
                best_k = c;
            }
        }
        if (half == 0) s->kern_at = best_k;
        else s->kern_a = best_k;
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
    return e;
}

// ------------------------------------------------------------ copy probe ---
// one 16-byte element per thread, non-temporal loads and stores: the
// fastest plain copy measured on the MI355X (about 6.4 TB/s for 2 GiB)
__global__ __launch_bounds__(kBlock) void k_copy16(int64_t n16, const uint4 *__restrict__ src, uint4 *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n16) return;
    uint4 v;
    v.x = __builtin_nontemporal_load(&src[i].x);
    v.y = __builtin_nontemporal_load(&src[i].y);
    v.z = __builtin_nontemporal_load(&src[i].z);
    v.w = __builtin_nontemporal_load(&src[i].w);
    __builtin_nontemporal_store(v.x, &dst[i].x);
    __builtin_nontemporal_store(v.y, &dst[i].y);
    __builtin_nontemporal_store(v.z, &dst[i].z);
    __builtin_nontemporal_store(v.w, &dst[i].w);
}

hipError_t copy_probe(int64_t bytes, int reps, double *gbps)
{
    const int64_t n16 = bytes / 16;
    uint4 *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, (size_t)n16 * 16);
    if (e == hipSuccess) e = hipMalloc(&b, (size_t)n16 * 16);
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipMemsetAsync(a, 1, (size_t)n16 * 16, st);
    const int grid = grid_for(n16, kBlock, 1 << 30);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, st, n16, a, b); // warm-up
        hipEventRecord(e0, st);
        for (int r = 0; r < reps; r++) hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, st, n16, a, b);
        hipEventRecord(e1, st);
        e = hipStreamSynchronize(st);
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) *gbps = (double)(2 * n16 * 16) * reps / (ms * 1e-3) / 1e9;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return e;
}

} // namespace pdhg
