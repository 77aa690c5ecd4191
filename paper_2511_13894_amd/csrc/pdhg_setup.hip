// Setup on the device: explicit transpose of A, Ruiz + Pock-Chambolle
// scaling, and the power iteration that sets the step size.
#include <algorithm>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"
#include "pdhg_kernels.hpp"

namespace pdhg {

// ---------------------------------------------------------------- transpose
// row id of every entry (one wave per row, lanes stride the row)
__global__ __launch_bounds__(kBlock) void k_rowid(int m, const int *__restrict__ rp, int *__restrict__ rowid)
{
    const int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= m) return;
    for (int e = rp[w] + lane; e < rp[w + 1]; e += 64) rowid[e] = (int)w;
}

__global__ __launch_bounds__(kBlock) void k_count_cols(int nnz, const int *__restrict__ ci, int *__restrict__ cnt)
{
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock)
        atomicAdd(&cnt[ci[e]], 1);
}

// exclusive scan of cnt[0..len) into out[0..len] in three passes:
// per-block scans with block totals, a scan of the totals, and the offsets.
constexpr int kScanItems = 4; // items per thread
constexpr int kScanTile = kBlock * kScanItems;

__device__ int block_exclusive_scan(int v, int *total)
{
    __shared__ int wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; w++) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(int len, const int *__restrict__ in, int *__restrict__ out,
                                                      int *__restrict__ tile_sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int vals[kScanItems];
    int local = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        vals[q] = (base + q < len) ? in[base + q] : 0;
        local += vals[q];
    }
    int total;
    int excl = block_exclusive_scan(local, &total);
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        if (base + q < len) out[base + q] = excl;
        excl += vals[q];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// one workgroup scans the tile totals sequentially in chunks of kBlock
__global__ __launch_bounds__(kBlock) void k_scan_totals(int tiles, int *__restrict__ tile_sums, int *__restrict__ grand)
{
    int carry = 0;
    for (int base = 0; base < tiles; base += kBlock) {
        int i = base + threadIdx.x;
        int v = i < tiles ? tile_sums[i] : 0;
        int total;
        int excl = block_exclusive_scan(v, &total);
        if (i < tiles) tile_sums[i] = carry + excl;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int len, int *__restrict__ out, const int *__restrict__ tile_sums)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) out[i] += tile_sums[i / kScanTile];
}

__global__ void k_set_last(int *out, int len, const int *grand) { out[len] = *grand; }

// place every entry of A into its transpose row (order inside a row is
// arbitrary here; k_rank_sort makes it ascending by row index)
__global__ __launch_bounds__(kBlock) void k_scatter(int nnz, const int *__restrict__ ci, const int *__restrict__ rowid,
                                                   int *__restrict__ cursor, int *__restrict__ ti_u,
                                                   int *__restrict__ perm_u)
{
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        int pos = atomicAdd(&cursor[ci[e]], 1);
        ti_u[pos] = rowid[e];
        perm_u[pos] = (int)e;
    }
}

// rows inside a transpose row are distinct, so an entry's sorted position is
// the number of smaller row indices in its segment: a deterministic order
__global__ __launch_bounds__(kBlock) void k_rank_sort(int nnz, const int *__restrict__ ci, const int *__restrict__ tp,
                                                     const int *__restrict__ ti_u, const int *__restrict__ perm_u,
                                                     int *__restrict__ ti, int *__restrict__ tperm)
{
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock) {
        const int e = perm_u[p];
        const int j = ci[e];
        const int beg = tp[j], end = tp[j + 1];
        const int key = ti_u[p];
        int rank = 0;
        for (int q = beg; q < end; q++) rank += ti_u[q] < key;
        ti[beg + rank] = key;
        tperm[beg + rank] = e;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(int nnz, const int *__restrict__ perm, const double *__restrict__ src,
                                                  T *__restrict__ dst)
{
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock)
        dst[p] = (T)src[perm[p]];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_convert(int64_t len, const double *__restrict__ src, T *__restrict__ dst)
{
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < len; p += (int64_t)gridDim.x * kBlock)
        dst[p] = (T)src[p];
}

__global__ void k_fill_u32(unsigned *p, unsigned v) { *p = v; }

// rounding error of the float copy, v - fl32(v) (exact in float64), stored as
// float (its own rounding is 2^-24 of an error already 2^-24 of v); with a
// permutation, gathered into the transpose's order
__global__ __launch_bounds__(kBlock) void k_round_err(int64_t len, const int *__restrict__ perm,
                                                     const double *__restrict__ src, float *__restrict__ dst)
{
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < len; p += (int64_t)gridDim.x * kBlock) {
        const double v = src[perm ? perm[p] : p];
        dst[p] = (float)(v - (double)(float)v);
    }
}

static hipError_t exclusive_scan(hipStream_t st, int len, const int *in, int *out, int *work)
{
    // out has len+1 entries; work holds ceil(len/kScanTile) + 1 ints
    const int tiles = (len + kScanTile - 1) / kScanTile;
    if (len > 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, st, len, in, out, work);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, st, tiles, work, work + tiles);
        hipLaunchKernelGGL(k_scan_add, dim3((len + kBlock - 1) / kBlock), dim3(kBlock), 0, st, len, out, work);
        hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, out, len, work + tiles);
    } else {
        hipMemsetAsync(out, 0, sizeof(int), st);
    }
    return hipGetLastError();
}

// ------------------------------------------------------ device ingest ---
// Rows: row_ptr[0] = 0, row_ptr[m] = nnz, non-decreasing; within a row the
// columns in range and strictly ascending (the canonical form: a device
// model is not re-sorted), values finite.  One wave per row (the lanes
// stride its entries; each compares its column with the previous entry's).
__global__ __launch_bounds__(kBlock) void k_ingest_rows(int m, int n, int64_t nnz, const int64_t *__restrict__ rp64,
                                                       const int32_t *__restrict__ ci_in,
                                                       const double *__restrict__ av_in, const double *__restrict__ b_in,
                                                       const char *__restrict__ sense_in, int *__restrict__ rp,
                                                       int *__restrict__ ci, double *__restrict__ av,
                                                       double *__restrict__ b, int8_t *__restrict__ sense0,
                                                       unsigned *__restrict__ bad)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
    const int lane = (int)(threadIdx.x & 63);
    if (i > m) return;
    unsigned flags = 0;
    const int64_t p0 = rp64[i];
    const bool p0_ok = p0 >= 0 && p0 <= nnz;
    if (lane == 0) rp[i] = (int)(p0_ok ? p0 : 0);
    if ((i == 0 && p0 != 0) || !p0_ok) flags |= BAD_ROWPTR;
    if (i == m) {
        if (p0 != nnz) flags |= BAD_ROWPTR;
    } else {
        const int64_t p1 = rp64[i + 1];
        if (p1 < p0 || p1 > nnz || !p0_ok) {
            flags |= BAD_ROWPTR;
        } else {
            for (int64_t e = p0 + lane; e < p1; e += 64) {
                const int col = ci_in[e];
                const double v = av_in[e];
                if (col < 0 || col >= n) flags |= BAD_COL;
                else if (e > p0 && col <= ci_in[e - 1]) flags |= BAD_ORDER;
                if (!isfinite(v)) flags |= BAD_VAL;
                ci[e] = col;
                av[e] = v;
            }
        }
        if (lane == 0) {
            const double bi = b_in[i];
            if (!isfinite(bi)) flags |= BAD_B;
            b[i] = bi;
            const char sn = sense_in ? sense_in[i] : '=';
            if (sn != '=' && sn != '<' && sn != '>') flags |= BAD_SENSE;
            sense0[i] = (int8_t)sn;
        }
    }
    if (flags) atomicOr(bad, flags);
}

__global__ __launch_bounds__(kBlock) void k_ingest_cols(int n, const double *__restrict__ c_in,
                                                       const double *__restrict__ l_in,
                                                       const double *__restrict__ u_in, double *__restrict__ c,
                                                       double *__restrict__ l, double *__restrict__ u,
                                                       unsigned *__restrict__ bad)
{
    unsigned flags = 0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        const double cj = c_in[j];
        const double lo = l_in ? l_in[j] : 0.0, hi = u_in ? u_in[j] : INFINITY;
        if (!isfinite(cj)) flags |= BAD_C;
        if (isnan(lo) || isnan(hi) || lo > hi) flags |= BAD_BOUND;
        c[j] = cj;
        l[j] = lo <= -1e20 ? -INFINITY : lo;
        u[j] = hi >= 1e20 ? INFINITY : hi;
    }
    if (flags) atomicOr(bad, flags);
}

hipError_t ingest_device(pdhg_solver *s, const DeviceModel &dm, unsigned *bad)
{
    hipStream_t st = s->stream;
    unsigned *d_bad = nullptr;
    hipError_t e = hipMalloc(&d_bad, sizeof(unsigned));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, d_bad, 0u);
    hipLaunchKernelGGL(k_ingest_rows, dim3(grid_for(((int64_t)dm.m + 1) * 64, kBlock, 1 << 30)), dim3(kBlock), 0, st, dm.m,
                       dm.n, dm.nnz, dm.row_ptr, dm.col_idx, dm.val, dm.b, dm.sense, s->rp, s->ci, s->av, s->b,
                       s->sense0, d_bad);
    if (dm.n > 0)
        hipLaunchKernelGGL(k_ingest_cols, dim3(grid_for(dm.n, kBlock, 1 << 20)), dim3(kBlock), 0, st, dm.n, dm.c, dm.l,
                           dm.u, s->c, s->l, s->u, d_bad);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(bad, d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_bad);
    return e;
}

// ------------------------------------------------ batch from device arrays
// blockIdx.y is the LP; x-blocks stride over its rows (r = m checks the end
// pointer, and the last LP writes the block's final one)
__global__ __launch_bounds__(kBlock) void k_batch_rows(const BatchPart *__restrict__ parts, int count,
                                                      int64_t *__restrict__ rp, double *__restrict__ b,
                                                      char *__restrict__ sense, unsigned *__restrict__ bad)
{
    const BatchPart q = parts[blockIdx.y];
    unsigned flags = 0;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r <= q.m; r += (int64_t)gridDim.x * kBlock) {
        const int64_t v = q.row_ptr[r];
        const bool ok = v >= 0 && v <= q.nnz;
        if (!ok || (r == 0 && v != 0) || (r == q.m && v != q.nnz)) flags |= BAD_ROWPTR;
        if (r < q.m) {
            rp[q.roff + r] = q.nzoff + (ok ? v : 0);
            b[q.roff + r] = q.b[r];
            sense[q.roff + r] = q.sense ? q.sense[r] : '=';
        } else if ((int)blockIdx.y == count - 1) {
            rp[q.roff + r] = q.nzoff + (ok ? v : 0);
        }
    }
    if (flags) atomicOr(bad, flags);
}

__global__ __launch_bounds__(kBlock) void k_batch_entries(const BatchPart *__restrict__ parts,
                                                         int32_t *__restrict__ ci, double *__restrict__ val,
                                                         unsigned *__restrict__ bad)
{
    const BatchPart q = parts[blockIdx.y];
    unsigned flags = 0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < q.nnz; e += (int64_t)gridDim.x * kBlock) {
        const int32_t col = q.col_idx[e];
        if (col < 0 || col >= q.n) flags |= BAD_COL;
        ci[q.nzoff + e] = (col < 0 || col >= q.n) ? q.coff : q.coff + col;
        val[q.nzoff + e] = q.val[e];
    }
    if (flags) atomicOr(bad, flags);
}

__global__ __launch_bounds__(kBlock) void k_batch_cols(const BatchPart *__restrict__ parts, double *__restrict__ c,
                                                      double *__restrict__ l, double *__restrict__ u)
{
    const BatchPart q = parts[blockIdx.y];
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < q.n; j += (int64_t)gridDim.x * kBlock) {
        c[q.coff + j] = q.c[j];
        l[q.coff + j] = q.l ? q.l[j] : 0.0;
        u[q.coff + j] = q.u ? q.u[j] : INFINITY;
    }
}

hipError_t batch_assemble_device(hipStream_t st, const std::vector<BatchPart> &parts, int M, int N, int64_t NZ,
                                 DeviceModel *dm, std::vector<void *> &temps, unsigned *bad)
{
    const int count = (int)parts.size();
    int64_t max_m = 0, max_n = 0, max_nz = 0;
    for (const BatchPart &q : parts) {
        max_m = q.m > max_m ? q.m : max_m;
        max_n = q.n > max_n ? q.n : max_n;
        max_nz = q.nnz > max_nz ? q.nnz : max_nz;
    }
    auto get = [&](void **ptr, size_t bytes) {
        hipError_t e = hipMalloc(ptr, bytes > 0 ? bytes : 1);
        if (e == hipSuccess) temps.push_back(*ptr);
        return e;
    };
    void *rp = nullptr, *ci = nullptr, *val = nullptr, *b = nullptr, *c = nullptr, *l = nullptr, *u = nullptr,
         *sense = nullptr, *d_parts = nullptr, *d_bad = nullptr;
    hipError_t e = get(&rp, sizeof(int64_t) * ((size_t)M + 1));
    if (e == hipSuccess) e = get(&ci, sizeof(int32_t) * (size_t)NZ);
    if (e == hipSuccess) e = get(&val, sizeof(double) * (size_t)NZ);
    if (e == hipSuccess) e = get(&b, sizeof(double) * (size_t)M);
    if (e == hipSuccess) e = get(&sense, (size_t)M);
    if (e == hipSuccess) e = get(&c, sizeof(double) * (size_t)N);
    if (e == hipSuccess) e = get(&l, sizeof(double) * (size_t)N);
    if (e == hipSuccess) e = get(&u, sizeof(double) * (size_t)N);
    if (e == hipSuccess) e = get(&d_parts, sizeof(BatchPart) * (size_t)count);
    if (e == hipSuccess) e = get(&d_bad, sizeof(unsigned));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(d_parts, parts.data(), sizeof(BatchPart) * (size_t)count, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, (unsigned *)d_bad, 0u);
    const BatchPart *pp = (const BatchPart *)d_parts;
    hipLaunchKernelGGL(k_batch_rows, dim3(grid_for(max_m + 1, kBlock, 256), count), dim3(kBlock), 0, st, pp, count,
                       (int64_t *)rp, (double *)b, (char *)sense, (unsigned *)d_bad);
    if (max_nz > 0)
        hipLaunchKernelGGL(k_batch_entries, dim3(grid_for(max_nz, kBlock, 1024), count), dim3(kBlock), 0, st, pp,
                           (int32_t *)ci, (double *)val, (unsigned *)d_bad);
    hipLaunchKernelGGL(k_batch_cols, dim3(grid_for(max_n, kBlock, 256), count), dim3(kBlock), 0, st, pp, (double *)c,
                       (double *)l, (double *)u);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(bad, d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *dm = DeviceModel{M, N, NZ, (const int64_t *)rp, (const int32_t *)ci, (const double *)val, (const double *)b,
                      (const double *)c, (const double *)l, (const double *)u, (const char *)sense};
    return hipSuccess;
}

const char *ingest_error(unsigned bad)
{
    if (bad & BAD_ROWPTR) return "row_ptr[0] != 0, row_ptr[m] != nnz or row_ptr not non-decreasing";
    if (bad & BAD_COL) return "column index out of range";
    if (bad & BAD_ORDER) return "a device model's rows need ascending, unique column indices";
    if (bad & BAD_VAL) return "non-finite matrix value";
    if (bad & BAD_B) return "non-finite b";
    if (bad & BAD_C) return "non-finite c";
    if (bad & BAD_BOUND) return "bad bounds (NaN or l > u)";
    if (bad & BAD_SENSE) return "sense must be '=', '<' or '>'";
    return "invalid model";
}

hipError_t build_transpose(pdhg_solver *s)
{
    hipStream_t st = s->stream;
    const int m = s->m, n = s->n, nnz = s->nnz;
    const int tiles = (n + kScanTile - 1) / kScanTile;
    int *rowid = nullptr, *cnt = nullptr, *ti_u = nullptr, *perm_u = nullptr, *work = nullptr;
    hipError_t e = hipSuccess;
    size_t nz = (size_t)(nnz > 0 ? nnz : 1);
    if ((e = hipMalloc(&rowid, nz * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMalloc(&cnt, (size_t)(n + 1) * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMalloc(&ti_u, nz * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMalloc(&perm_u, nz * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMalloc(&work, (size_t)(tiles + 2) * sizeof(int))) != hipSuccess) return e;
    hipMemsetAsync(cnt, 0, (size_t)(n + 1) * sizeof(int), st);
    const int big = grid_for(nnz, kBlock, 65536);
    if (m > 0) hipLaunchKernelGGL(k_rowid, dim3(grid_for((int64_t)m * 64, kBlock, 1 << 30)), dim3(kBlock), 0, st, m, s->rp, rowid);
    if (nnz > 0) hipLaunchKernelGGL(k_count_cols, dim3(big), dim3(kBlock), 0, st, nnz, s->ci, cnt);
    exclusive_scan(st, n, cnt, s->tp, work);
    // cursor = copy of the row starts
    hipMemcpyAsync(cnt, s->tp, (size_t)(n + 1) * sizeof(int), hipMemcpyDeviceToDevice, st);
    if (nnz > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(big), dim3(kBlock), 0, st, nnz, s->ci, rowid, cnt, ti_u, perm_u);
        hipLaunchKernelGGL(k_rank_sort, dim3(big), dim3(kBlock), 0, st, nnz, s->ci, s->tp, ti_u, perm_u, s->ti, s->tperm);
        hipLaunchKernelGGL((k_gather<double>), dim3(big), dim3(kBlock), 0, st, nnz, s->tperm, s->av, s->atv);
    }
    e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(st);
    hipFree(rowid);
    hipFree(cnt);
    hipFree(ti_u);
    hipFree(perm_u);
    hipFree(work);
    return e != hipSuccess ? e : e2;
}

// ----------------------------------------------------------------- scaling
// per-row reduction over L lanes: MODE 0 max|a|, MODE 1 sum |a|^p
template <int L, int MODE>
__global__ __launch_bounds__(kBlock) void k_row_norm(int rows, const int *__restrict__ ptr,
                                                    const double *__restrict__ val, double p,
                                                    double *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t row = g / L;
    const int lane = (int)(g % L);
    if (row >= rows) return;
    double acc = 0.0;
    for (int e = ptr[row] + lane; e < ptr[row + 1]; e += L) {
        double a = fabs(val[e]);
        if (MODE == 0) acc = fmax(acc, a);
        else acc += (p == 1.0) ? a : pow(a, p);
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
        double o = __shfl_xor(acc, off, L);
        acc = (MODE == 0) ? fmax(acc, o) : acc + o;
    }
    if (lane == 0) out[row] = acc > 0.0 ? sqrt(acc) : 1.0;
}

template <int MODE>
static void row_norm(hipStream_t st, int lanes, int rows, const int *ptr, const double *val, double p, double *out)
{
    if (rows <= 0) return;
    const int grid = (int)(((int64_t)rows * lanes + kBlock - 1) / kBlock);
#define PDHG_RN_CASE(LL)                                                                                    \
    case LL:                                                                                                \
        hipLaunchKernelGGL((k_row_norm<LL, MODE>), dim3(grid), dim3(kBlock), 0, st, rows, ptr, val, p, out); \
        break;
    switch (lanes) {
        PDHG_RN_CASE(1)
        PDHG_RN_CASE(2)
        PDHG_RN_CASE(4)
        PDHG_RN_CASE(8)
        PDHG_RN_CASE(16)
        PDHG_RN_CASE(32)
    default:
        PDHG_RN_CASE(64)
    }
#undef PDHG_RN_CASE
}

// Ahat_e <- Ahat_e / (r_i q_j) for entry e = (i, j)
__global__ __launch_bounds__(kBlock) void k_apply_scale(int nnz, const int *__restrict__ rowid,
                                                       const int *__restrict__ ci, double *__restrict__ val,
                                                       const double *__restrict__ r, const double *__restrict__ q)
{
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock)
        val[e] = val[e] / (r[rowid[e]] * q[ci[e]]);
}

__global__ __launch_bounds__(kBlock) void k_div_vec(int len, double *__restrict__ d, const double *__restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) d[i] = d[i] / r[i];
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t len, double *__restrict__ d, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock) d[i] = v;
}

// scaled data: chat = Dc c, bhat = Dr b, lhat = l / Dc, uhat = u / Dc
template <typename V>
__global__ __launch_bounds__(kBlock) void k_scaled_cols(int n, const double *__restrict__ dc, const double *__restrict__ c,
                                                       const double *__restrict__ l, const double *__restrict__ u,
                                                       double *__restrict__ ch, V *__restrict__ lh, V *__restrict__ uh)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    ch[j] = dc[j] * c[j];
    lh[j] = (V)(l[j] / dc[j]);
    uh[j] = (V)(u[j] / dc[j]);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_scaled_rows(int m, const double *__restrict__ dr, const double *__restrict__ b,
                                                       const int8_t *__restrict__ s0, V *__restrict__ bh,
                                                       int8_t *__restrict__ sense)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    bh[i] = (V)(dr[i] * b[i]);
    sense[i] = s0[i];
}

template <typename V>
static void make_scaled(pdhg_solver *s, const double *ahat64)
{
    hipStream_t st = s->stream;
    const int big = grid_for(s->nnz, kBlock, 65536);
    if (s->nnz > 0) {
        hipLaunchKernelGGL((k_convert<V>), dim3(big), dim3(kBlock), 0, st, (int64_t)s->nnz, ahat64, (V *)s->ahat);
        hipLaunchKernelGGL((k_gather<V>), dim3(big), dim3(kBlock), 0, st, s->nnz, s->tperm, ahat64, (V *)s->ahat_t);
        if (s->aerr) {
            hipLaunchKernelGGL(k_round_err, dim3(big), dim3(kBlock), 0, st, (int64_t)s->nnz, (const int *)nullptr,
                               ahat64, (float *)s->aerr);
            hipLaunchKernelGGL(k_round_err, dim3(big), dim3(kBlock), 0, st, (int64_t)s->nnz, (const int *)s->tperm,
                               ahat64, (float *)s->aerr_t);
        }
    }
    if (s->n > 0)
        hipLaunchKernelGGL((k_scaled_cols<V>), dim3(grid_for(s->n, kBlock, 1 << 30)), dim3(kBlock), 0, st, s->n, s->dc,
                           s->c, s->l, s->u, s->ch, (V *)s->lh, (V *)s->uh);
    if (s->m > 0)
        hipLaunchKernelGGL((k_scaled_rows<double>), dim3(grid_for(s->m, kBlock, 1 << 30)), dim3(kBlock), 0, st, s->m,
                           s->dr, s->b, s->sense0, (double *)s->bh, s->sense);
}

hipError_t scale_problem(pdhg_solver *s)
{
    hipStream_t st = s->stream;
    const int m = s->m, n = s->n, nnz = s->nnz;
    double *ah = nullptr, *aht = nullptr, *r = nullptr, *q = nullptr;
    int *rowid = nullptr;
    hipError_t e;
    size_t nz = (size_t)(nnz > 0 ? nnz : 1);
    if ((e = hipMalloc(&ah, nz * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&aht, nz * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&r, (size_t)(m > 0 ? m : 1) * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&q, (size_t)(n > 0 ? n : 1) * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&rowid, nz * sizeof(int))) != hipSuccess) return e;
    hipMemcpyAsync(ah, s->av, (size_t)nnz * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (m > 0) hipLaunchKernelGGL(k_rowid, dim3(grid_for((int64_t)m * 64, kBlock, 1 << 30)), dim3(kBlock), 0, st, m, s->rp, rowid);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(m, kBlock, 4096)), dim3(kBlock), 0, st, (int64_t)m, s->dr, 1.0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, (int64_t)n, s->dc, 1.0);
    const int big = grid_for(nnz, kBlock, 65536);
    const int gm = grid_for(m, kBlock, 1 << 30), gn = grid_for(n, kBlock, 1 << 30);
    auto pass = [&](int mode, double alpha) {
        // row statistics over A's rows, column statistics over the transpose's rows
        if (nnz > 0) hipLaunchKernelGGL((k_gather<double>), dim3(big), dim3(kBlock), 0, st, nnz, s->tperm, ah, aht);
        if (mode == 0) {
            row_norm<0>(st, s->lanes_a, m, s->rp, ah, 1.0, r);
            row_norm<0>(st, s->lanes_at, n, s->tp, aht, 1.0, q);
        } else {
            row_norm<1>(st, s->lanes_a, m, s->rp, ah, 2.0 - alpha, r);
            row_norm<1>(st, s->lanes_at, n, s->tp, aht, alpha, q);
        }
        if (nnz > 0) hipLaunchKernelGGL(k_apply_scale, dim3(big), dim3(kBlock), 0, st, nnz, rowid, s->ci, ah, r, q);
        if (m > 0) hipLaunchKernelGGL(k_div_vec, dim3(gm), dim3(kBlock), 0, st, m, s->dr, r);
        if (n > 0) hipLaunchKernelGGL(k_div_vec, dim3(gn), dim3(kBlock), 0, st, n, s->dc, q);
    };
    for (int it = 0; it < s->p.ruiz_iters; it++) pass(0, 0.0);
    if (s->p.pc_alpha >= 0.0) pass(1, s->p.pc_alpha);
    if (s->fp32) make_scaled<float>(s, ah);
    else make_scaled<double>(s, ah);
    e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(st);
    hipFree(ah);
    hipFree(aht);
    hipFree(r);
    hipFree(q);
    hipFree(rowid);
    return e != hipSuccess ? e : e2;
}

// --------------------------------------------------------- power iteration
// Power iteration on M = Ahat'Ahat from v = 1/sqrt(n).  A step forms
// u = Ahat v and w = Ahat'u; with v of unit length, rho = u'u is its Rayleigh
// quotient and ||w - rho v||^2 = w'w - rho^2.  The iteration stops at the
// first step with sqrt(w'w - rho^2) <= tol * rho (or when w = 0), keeping
// lambda = ||w||, which lies in [rho, lambda_max(M)].  pw = {lambda, done,
// steps}: the decision stays on the device and later steps of a launched
// batch leave v and pw alone.

// partial sums of squares per block
__global__ __launch_bounds__(kBlock) void k_sumsq_partials(int len, const double *__restrict__ w, double *__restrict__ part)
{
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock)
        v[0] += w[i] * w[i];
    block_reduce<1>(v, 0u);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_power_start(int64_t len, double *__restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) v[i] = power_start(i);
}

// out[0] = sqrt of the sum of part[0, g), fixed order
__global__ __launch_bounds__(kBlock) void k_norm_finish(int g, const double *__restrict__ part, double *__restrict__ out)
{
    double q[1] = {0.0};
    for (int i = threadIdx.x; i < g; i += kBlock) q[0] += part[i];
    block_reduce<1>(q, 0u);
    if (threadIdx.x == 0) out[0] = sqrt(q[0]);
}

__global__ __launch_bounds__(kBlock) void k_div_scalar(int64_t len, double *__restrict__ v, const double *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) v[i] = v[i] / d[0];
}

// rho = sum of part[0, gm), w'w = sum of part[gm, gm + gn), fixed order
__global__ __launch_bounds__(kBlock) void k_power_finish(int gm, int gn, const double *__restrict__ part, double tol,
                                                        double *__restrict__ pw)
{
    if (pw[1] != 0.0) return;
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < gm; i += kBlock) v[0] += part[i];
    for (int i = threadIdx.x; i < gn; i += kBlock) v[1] += part[gm + i];
    block_reduce<2>(v, 0u);
    if (threadIdx.x == 0) {
        const double rho = v[0], ww = v[1], lam = sqrt(ww);
        pw[0] = lam;
        pw[2] += 1.0;
        if (!(lam > 0.0) || sqrt(fmax(ww - rho * rho, 0.0)) <= tol * rho) pw[1] = 1.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_normalize(int len, const double *__restrict__ w, const double *__restrict__ pw,
                                                     double *__restrict__ v)
{
    const double l = pw[0];
    if (pw[1] != 0.0 || !(l > 0.0)) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) v[i] = w[i] / l;
}

__global__ void k_set_step(pdhg::DevState *st, const double *pw, double safety)
{
    const double l = pw[0];
    const double sig = (pw[2] > 0.0 && l > 0.0) ? sqrt(l) : 0.0;
    st->sigma_est = sig;
    st->eta = sig > 1e-12 ? safety / sig : safety;
}

hipError_t power_iteration(pdhg_solver *s)
{
    hipStream_t st = s->stream;
    const int m = s->m, n = s->n;
    double *v = nullptr, *w = nullptr, *u = nullptr, *pw = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&v, (size_t)(n > 0 ? n : 1) * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&w, (size_t)(n > 0 ? n : 1) * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&u, (size_t)(m > 0 ? m : 1) * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&pw, 4 * sizeof(double))) != hipSuccess) return e;
    hipMemsetAsync(pw, 0, 4 * sizeof(double), st);
    const int gm = grid_for(m, kBlock, kMaxRedBlocks), gn = grid_for(n, kBlock, kMaxRedBlocks);
    if (n > 0) { // start: v = (1 + U) / ||1 + U||, the norm kept in pw[3]
        const int gv = grid_for(n, kBlock, 1 << 30);
        hipLaunchKernelGGL(k_power_start, dim3(gv), dim3(kBlock), 0, st, (int64_t)n, v);
        hipLaunchKernelGGL(k_sumsq_partials, dim3(gn), dim3(kBlock), 0, st, n, v, s->partials);
        hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(kBlock), 0, st, gn, s->partials, pw + 3);
        hipLaunchKernelGGL(k_div_scalar, dim3(gv), dim3(kBlock), 0, st, (int64_t)n, v, pw + 3);
    }
    double pw_host[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int kPowerBatch = 32; // steps launched between reads of the done flag
    for (int it = 0; it < s->p.power_iters && n > 0 && m > 0; it += kPowerBatch) {
        const int len = std::min(kPowerBatch, s->p.power_iters - it);
        for (int k = 0; k < len; k++) {
            (void)solver_product(s, false, v, u);
            (void)solver_product(s, true, u, w);
            hipLaunchKernelGGL(k_sumsq_partials, dim3(gm), dim3(kBlock), 0, st, m, u, s->partials);
            hipLaunchKernelGGL(k_sumsq_partials, dim3(gn), dim3(kBlock), 0, st, n, w, s->partials + gm);
            hipLaunchKernelGGL(k_power_finish, dim3(1), dim3(kBlock), 0, st, gm, gn, s->partials, s->p.power_tol, pw);
            hipLaunchKernelGGL(k_normalize, dim3(grid_for(n, kBlock, 1 << 30)), dim3(kBlock), 0, st, n, w, pw, v);
        }
        if ((e = hipMemcpyAsync(pw_host, pw, 4 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) break;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
        if (pw_host[1] != 0.0) break;
    }
    s->power_steps = (int64_t)pw_host[2];
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, st, s->st, pw, s->p.eta_safety);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(st);
    hipFree(v);
    hipFree(w);
    hipFree(u);
    hipFree(pw);
    return e != hipSuccess ? e : e2;
}

} // namespace pdhg
