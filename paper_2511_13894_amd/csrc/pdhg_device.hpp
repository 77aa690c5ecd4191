// Device-side building blocks: wave64 / workgroup reductions and the
// row-compressed sparse product with L lanes per row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pdhg_internal.hpp"

namespace pdhg {

// Sum over a group of L consecutive lanes (L a power of two <= 64); every lane
// of the group ends with the group's sum.  Butterfly order is fixed, so the
// result is deterministic.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Workgroup reduction of NQ values (sum, or max where is_max bit q is set);
// thread 0 receives the results.  Uses kBlock/64 LDS slots per quantity.
template <int NQ>
__device__ __forceinline__ void block_reduce(double (&v)[NQ], unsigned is_max_mask)
{
    __shared__ double lds[NQ][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        v[q] = ((is_max_mask >> q) & 1u) ? wave_max(v[q]) : wave_sum(v[q]);
        if (lane == 0) lds[q][wid] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            double acc = lds[q][0];
            for (int w = 1; w < kBlock / 64; w++)
                acc = ((is_max_mask >> q) & 1u) ? fmax(acc, lds[q][w]) : acc + lds[q][w];
            v[q] = acc;
        }
    }
    __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs (bid % 8).  Map them
// so that every XCD works on one contiguous range of logical blocks: rows
// that gather the same cache lines then meet in the same L2.
__device__ __forceinline__ int xcd_range_block(int bid, int nblk)
{
    const int x = bid & 7, q = nblk >> 3, r = nblk & 7;
    const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + (bid >> 3);
}

// The mapping of a single LP's launches.  Up to kXcdChunkMin workgroups
// (a launch whose workgroups are resident together) take the contiguous
// ranges above.  A larger launch runs in many rounds, and with ranges each
// XCD would own one region of the matrix: where the rows change kind along
// the matrix (the node-balance, then the capacity rows of a multicommodity
// LP) the XCDs get unequal work.  There chunks of kXcdChunk logical blocks
// are dealt round-robin to the XCDs instead: neighbouring rows still share an
// L2 within a chunk, and every region spreads over all 8 XCDs.  A tail of
// fewer than 8 chunks keeps the dispatch order.  (The batch engine keeps the
// ranges: one LP's tiles then stay in one L2.)
constexpr int kXcdChunk = 16;
constexpr int kXcdChunkMin = 8192;

__device__ __forceinline__ int xcd_block(int bid, int nblk)
{
    if (nblk < kXcdChunkMin) return xcd_range_block(bid, nblk);
    const int full = nblk / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (bid >= full) return bid;
    const int x = bid & 7, k = bid >> 3;
    return ((k / kXcdChunk) * 8 + x) * kXcdChunk + k % kXcdChunk;
}

// One lane's share of a row's product: the terms e = beg+lane, beg+lane+L, ...
// below end, accumulated in that order.  Four terms' index, value and
// gathered loads are issued before the first of them is accumulated, so a
// lane waits for one round of loads per four terms instead of per term.
template <int L, typename ACC, typename VM, typename VX>
__device__ __forceinline__ ACC lane_dot(int beg, int end, int lane, const int *__restrict__ idx,
                                        const VM *__restrict__ val, const VX *__restrict__ x)
{
    ACC acc = 0;
    int e = beg + lane;
    for (; e + 3 * L < end; e += 4 * L) {
        const int i0 = idx[e], i1 = idx[e + L], i2 = idx[e + 2 * L], i3 = idx[e + 3 * L];
        const ACC v0 = (ACC)val[e], v1 = (ACC)val[e + L], v2 = (ACC)val[e + 2 * L], v3 = (ACC)val[e + 3 * L];
        const ACC g0 = (ACC)x[i0], g1 = (ACC)x[i1], g2 = (ACC)x[i2], g3 = (ACC)x[i3];
        acc += v0 * g0;
        acc += v1 * g1;
        acc += v2 * g2;
        acc += v3 * g3;
    }
    // the last up to three terms of the lane: their loads go out together too
    // (positions past the end reload the lane's first one, whose term is not
    // added), summed in the same order as a sequential tail
    if (e < end) {
        const int e1 = e + L, e2 = e + 2 * L;
        const int c1 = e1 < end ? e1 : e, c2 = e2 < end ? e2 : e;
        const int i0 = idx[e], i1 = idx[c1], i2 = idx[c2];
        const ACC v0 = (ACC)val[e], v1 = (ACC)val[c1], v2 = (ACC)val[c2];
        const ACC g0 = (ACC)x[i0], g1 = (ACC)x[i1], g2 = (ACC)x[i2];
        acc += v0 * g0;
        if (e1 < end) acc += v1 * g1;
        if (e2 < end) acc += v2 * g2;
    }
    return acc;
}

// Row-compressed product out[r] = sum_e val[e] * x[idx[e]] over rows r < rows,
// L lanes per row, accumulation in ACC.  One group of L lanes walks a row with
// stride L (coalesced for L >= 2 on long rows, one lane per row when L = 1).
template <int L, typename VM, typename VX, typename ACC, typename VO>
__global__ __launch_bounds__(kBlock) void k_spmv(int rows, const int *__restrict__ ptr,
                                                 const int *__restrict__ idx, const VM *__restrict__ val,
                                                 const VX *__restrict__ x, VO *__restrict__ out)
{
    const int64_t g = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int64_t row = g / L;
    const int lane = (int)(g % L);
    if (row >= rows) return;
    const int beg = ptr[row], end = ptr[row + 1];
    ACC acc = lane_dot<L, ACC>(beg, end, lane, idx, val, x);
    acc = group_sum<L>(acc);
    if (lane == 0) out[row] = (VO)acc;
}

// Launch k_spmv with the lane count chosen at run time.
template <typename VM, typename VX, typename ACC, typename VO>
inline void spmv(hipStream_t st, int lanes, int rows, const int *ptr, const int *idx, const VM *val,
                 const VX *x, VO *out)
{
    if (rows <= 0) return;
    const int64_t threads = (int64_t)rows * lanes;
    const int grid = (int)((threads + kBlock - 1) / kBlock);
#define PDHG_SPMV_CASE(LL)                                                                       \
    case LL:                                                                                     \
        hipLaunchKernelGGL((k_spmv<LL, VM, VX, ACC, VO>), dim3(grid), dim3(kBlock), 0, st, rows, \
                           ptr, idx, val, x, out);                                               \
        break;
    switch (lanes) {
        PDHG_SPMV_CASE(1)
        PDHG_SPMV_CASE(2)
        PDHG_SPMV_CASE(4)
        PDHG_SPMV_CASE(8)
        PDHG_SPMV_CASE(16)
        PDHG_SPMV_CASE(32)
    default:
        PDHG_SPMV_CASE(64)
    }
#undef PDHG_SPMV_CASE
}

__device__ __forceinline__ bool is_inf_lo(double v) { return v <= -1e20; }
__device__ __forceinline__ bool is_inf_up(double v) { return v >= 1e20; }

} // namespace pdhg
