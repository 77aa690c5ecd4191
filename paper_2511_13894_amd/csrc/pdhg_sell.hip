// Sliced ELLPACK layout of Ahat for the dual half when rows are long
// (hundreds to thousands of entries).  Slices of 32 consecutive rows store
// their entries interleaved: entry k of the slice's row `lane` sits at
// soff[s] + 32 k + lane, padded with zero values to the slice's longest row.
// A workgroup of 256 threads (8 groups of 32 lanes, a lane per row) handles
// one work item (slice, chunk of kSellChunk positions): the 32 lanes of a
// group read 32 consecutive index and value words, and rows whose columns
// advance together (the sink rows of a transportation model: entry k of
// row j is column 5000 k + j) gather consecutive x-bar words; a row whose
// columns are contiguous (a source row) walks its own cache lines, which
// stay in L1 across the group's next steps.  The 8 groups' partial sums
// are reduced in LDS in a fixed order, each work item writes 32 partials,
// and a second kernel sums each row's partials in chunk order before the
// dual update (or the check product).  Deterministic.
#include <algorithm>
#include <vector>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"
#include "pdhg_kernels.hpp"

namespace pdhg {

constexpr int kSellC = 32;      // rows per slice
constexpr int kSellChunk = 256; // entry positions per work item
constexpr int kSellG = kBlock / kSellC; // lane groups per workgroup

template <typename VM, typename VV>
__global__ __launch_bounds__(kBlock) void k_sell_partial(const int2 *__restrict__ wi,
                                                        const int64_t *__restrict__ soff,
                                                        const int *__restrict__ slen, const int *__restrict__ idx,
                                                        const VM *__restrict__ val, const VV *__restrict__ vec,
                                                        double *__restrict__ part, const DevState *__restrict__ st)
{
    __shared__ double red[kSellG][kSellC];
    if (st && st->done) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int2 w = wi[b];
    const int lane = threadIdx.x % kSellC, g = threadIdx.x / kSellC;
    const int k0 = w.y * kSellChunk, k1 = min(k0 + kSellChunk, slen[w.x]);
    const int64_t base = soff[w.x] + lane;
    double acc = 0.0;
    for (int kk = k0 + g; kk < k1; kk += 4 * kSellG) {
        int id[4];
        double v[4], x[4];
        // positions past the slice's end reload its last position (kk < k1
        // here), so every lane loads and no load is merged with a fallback
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = kk + u * kSellG;
            const int64_t e = base + (int64_t)(k < k1 ? k : k1 - 1) * kSellC;
            id[u] = idx[e];
            v[u] = (double)val[e];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = (double)vec[id[u]];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (kk + u * kSellG < k1) acc += v[u] * x[u];
    }
    red[g][lane] = acc;
    __syncthreads();
    if (g == 0) {
        double t = red[0][lane];
#pragma unroll
        for (int q = 1; q < kSellG; q++) t += red[q][lane];
        part[(size_t)b * kSellC + lane] = t;
    }
}

// h = the row's partials summed in chunk order; then the dual update
__global__ __launch_bounds__(kBlock) void k_sell_dual_finish(int m, const int *__restrict__ wi_start,
                                                            const double *__restrict__ part,
                                                            const double *__restrict__ bh,
                                                            const int8_t *__restrict__ sense, double *__restrict__ y,
                                                            const double *__restrict__ ya, double *__restrict__ yp,
                                                            const DevState *__restrict__ st, int i, int store_cand)
{
    if (st->done) return;
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= m) return;
    const int s = r / kSellC, lane = r % kSellC;
    double h = 0.0;
    for (int w = wi_start[s]; w < wi_start[s + 1]; w++) h += part[(size_t)w * kSellC + lane];
    dual_update(r, h, y[r], bh[r], ya[r], sense[r], y, yp, st, i, store_cand);
}

__global__ __launch_bounds__(kBlock) void k_sell_product_finish(int m, const int *__restrict__ wi_start,
                                                               const double *__restrict__ part,
                                                               double *__restrict__ out)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= m) return;
    const int s = r / kSellC, lane = r % kSellC;
    double h = 0.0;
    for (int w = wi_start[s]; w < wi_start[s + 1]; w++) h += part[(size_t)w * kSellC + lane];
    out[r] = h;
}

// fill the layout from the scaled CSR copy, one thread per slot of every
// slice (slots past the last row are rows of length 0: all padding)
template <typename V>
__global__ __launch_bounds__(kBlock) void k_sell_fill(int m, int slots, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const V *__restrict__ ahat,
                                                     const int64_t *__restrict__ soff, const int *__restrict__ slen,
                                                     int *__restrict__ idx, V *__restrict__ val)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= slots) return;
    const int s = r / kSellC, lane = r % kSellC;
    const int beg = r < m ? rp[r] : 0, len = r < m ? rp[r + 1] - rp[r] : 0;
    const int pad_col = len > 0 ? ci[beg + len - 1] : 0;
    for (int k = 0; k < slen[s]; k++) {
        const int64_t e = soff[s] + (int64_t)k * kSellC + lane;
        idx[e] = k < len ? ci[beg + k] : pad_col;
        val[e] = k < len ? ahat[beg + k] : (V)0;
    }
}

hipError_t sell_build(pdhg_solver *s, const std::vector<int> &rp_host)
{
    const int m = s->m;
    const int ns = (m + kSellC - 1) / kSellC;
    std::vector<int> slen((size_t)ns + 1, 0), wi_start((size_t)ns + 1, 0);
    std::vector<int64_t> soff((size_t)ns + 1, 0);
    std::vector<int2> wi;
    for (int sl = 0; sl < ns; sl++) {
        int L = 0;
        for (int r = sl * kSellC; r < std::min(m, (sl + 1) * kSellC); r++) L = std::max(L, rp_host[r + 1] - rp_host[r]);
        slen[sl] = L;
        soff[sl + 1] = soff[sl] + (int64_t)L * kSellC;
        wi_start[sl] = (int)wi.size();
        for (int c = 0; c * kSellChunk < L; c++) wi.push_back(make_int2(sl, c));
    }
    wi_start[ns] = (int)wi.size();
    const size_t vb = s->fp32 ? sizeof(float) : sizeof(double);
    const size_t total = (size_t)(soff[ns] > 0 ? soff[ns] : 1);
    hipStream_t st = s->stream;
    hipError_t e = hipMalloc(&s->sell_idx, sizeof(int) * total);
    if (e == hipSuccess) e = hipMalloc(&s->sell_val, vb * total);
    if (e == hipSuccess) e = hipMalloc(&s->sell_soff, sizeof(int64_t) * soff.size());
    if (e == hipSuccess) e = hipMalloc(&s->sell_len, sizeof(int) * slen.size());
    if (e == hipSuccess) e = hipMalloc(&s->sell_wi_start, sizeof(int) * wi_start.size());
    if (e == hipSuccess) e = hipMalloc(&s->sell_wi, sizeof(int2) * (wi.empty() ? 1 : wi.size()));
    if (e == hipSuccess) e = hipMalloc(&s->sell_part, sizeof(double) * kSellC * (wi.empty() ? 1 : wi.size()));
    if (e == hipSuccess) e = hipMemcpyAsync(s->sell_soff, soff.data(), sizeof(int64_t) * soff.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->sell_len, slen.data(), sizeof(int) * slen.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->sell_wi_start, wi_start.data(), sizeof(int) * wi_start.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !wi.empty())
        e = hipMemcpyAsync(s->sell_wi, wi.data(), sizeof(int2) * wi.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    s->n_sell_wi = (int)wi.size();
    const int slots = ns * kSellC;
    if (slots > 0) {
        const int g = (slots + kBlock - 1) / kBlock;
        if (s->fp32)
            hipLaunchKernelGGL((k_sell_fill<float>), dim3(g), dim3(kBlock), 0, st, m, slots, s->rp, s->ci,
                               (const float *)s->ahat, s->sell_soff, s->sell_len, s->sell_idx, (float *)s->sell_val);
        else
            hipLaunchKernelGGL((k_sell_fill<double>), dim3(g), dim3(kBlock), 0, st, m, slots, s->rp, s->ci,
                               (const double *)s->ahat, s->sell_soff, s->sell_len, s->sell_idx, (double *)s->sell_val);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st); // the host vectors die on return
    return e;
}

template <typename V>
static void sell_dual_impl(pdhg_solver *s, int i, int store, hipEvent_t e0, hipEvent_t e1)
{
    if (s->m <= 0) return;
    // timed: the start event on the first kernel's begin, the stop event on the second's end
    const dim3 gp(s->n_sell_wi > 0 ? s->n_sell_wi : 1), gf((s->m + kBlock - 1) / kBlock), bk(kBlock);
    const DevState *st = s->st;
    if (s->n_sell_wi > 0) {
        if (e0)
            hipExtLaunchKernelGGL((k_sell_partial<V, V>), gp, bk, 0, s->stream, e0, nullptr, 0, s->sell_wi,
                                  s->sell_soff, s->sell_len, s->sell_idx, (const V *)s->sell_val, (const V *)s->xbar,
                                  s->sell_part, st);
        else
            hipLaunchKernelGGL((k_sell_partial<V, V>), gp, bk, 0, s->stream, s->sell_wi, s->sell_soff, s->sell_len,
                               s->sell_idx, (const V *)s->sell_val, (const V *)s->xbar, s->sell_part, st);
    }
    hipEvent_t f0 = s->n_sell_wi > 0 ? nullptr : e0;
    if (f0 || e1)
        hipExtLaunchKernelGGL(k_sell_dual_finish, gf, bk, 0, s->stream, f0, e1, 0, s->m, s->sell_wi_start, s->sell_part,
                              (const double *)s->bhc, s->sense, (double *)s->y, (const double *)s->ya, (double *)s->yp,
                              st, i, store);
    else
        hipLaunchKernelGGL(k_sell_dual_finish, gf, bk, 0, s->stream, s->m, s->sell_wi_start, s->sell_part,
                           (const double *)s->bhc, s->sense, (double *)s->y, (const double *)s->ya, (double *)s->yp,
                           st, i, store);
}

void sell_dual(pdhg_solver *s, int i, int store, hipEvent_t e0, hipEvent_t e1)
{
    if (s->fp32) sell_dual_impl<float>(s, i, store, e0, e1);
    else sell_dual_impl<double>(s, i, store, e0, e1);
}

template <typename VV>
static void sell_product_impl(pdhg_solver *s, const VV *vec, double *out)
{
    if (s->m <= 0) return;
    if (s->n_sell_wi > 0) {
        if (s->fp32)
            hipLaunchKernelGGL((k_sell_partial<float, VV>), dim3(s->n_sell_wi), dim3(kBlock), 0, s->stream, s->sell_wi,
                               s->sell_soff, s->sell_len, s->sell_idx, (const float *)s->sell_val, vec, s->sell_part,
                               (const DevState *)nullptr);
        else
            hipLaunchKernelGGL((k_sell_partial<double, VV>), dim3(s->n_sell_wi), dim3(kBlock), 0, s->stream,
                               s->sell_wi, s->sell_soff, s->sell_len, s->sell_idx, (const double *)s->sell_val, vec,
                               s->sell_part, (const DevState *)nullptr);
    }
    hipLaunchKernelGGL(k_sell_product_finish, dim3((s->m + kBlock - 1) / kBlock), dim3(kBlock), 0, s->stream, s->m,
                       s->sell_wi_start, s->sell_part, out);
}

void sell_product(pdhg_solver *s, const double *vec, double *out) { sell_product_impl<double>(s, vec, out); }
void sell_product(pdhg_solver *s, const float *vec, double *out) { sell_product_impl<float>(s, vec, out); }

} // namespace pdhg
