// Device functions shared by the single-LP and the batched kernels: the
// fused update epilogues, the LDS-tiled row sums, the check decisions and
// the push objective's counter-based generator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pdhg_device.hpp"
#include "pdhg_internal.hpp"

namespace pdhg {

// Halpern weights for iteration number k (0-based since the last restart).
__device__ __forceinline__ void halpern_weights(const DevState *st, int i, double &w, double &wa, double &g)
{
    const double k = (double)(st->k0 + i);
    w = (k + 1.0) / (k + 2.0);
    wa = 1.0 / (k + 2.0);
    g = st->gamma;
}

// Storage.  Float64 mode: every vector is double.  Mixed mode (V = float):
// the matrix values, the bounds lhat, uhat and two n-vectors are float, and
// the iterate x and the extrapolation xbar are stored as float DIFFERENCES
// from the float64 anchor x_a (x - x_a, xbar - x_a); the anchor, the
// candidate x+ and every m-vector (y, y_anchor, y+) are double.  The float
// rounding of a difference shrinks as the restart cycle converges, so the
// iteration keeps float64 accuracy near the optimum (rounding x itself to
// float stalls primal-degenerate LPs, where the rows cancel).  With the float
// matrix fl32(Ahat) = Ahat - E, the kernels read a float64 objective and
// right-hand side fixed at every anchor:
//   bhat - Ahat xbar = (bhat - Ahat x_a) - fl32(Ahat)(xbar - x_a) - E (xbar - x_a),
//   chat - Ahat'y    = (chat - E'y_a) - fl32(Ahat)'y - E'(y - y_a),
// so the only errors are E times a difference (and the differences' own
// rounding).  All arithmetic — products, sums, projections, Halpern averages —
// is double in registers; only the stores round to V.

// Primal half, one row of the transpose (= one column j of A) per group of L
// lanes:  g = Ahat' y;  x+ = clamp(x - tau (chat - g),
// lhat, uhat);  xbar = 2 x+ - x;  x <- w ((1+gamma) x+ - gamma x) + wa x_a.
// xj is the iterate itself (mixed: x_a + stored difference), aj the anchor.
// At the last iteration before a check the candidate x+ is stored as well.
template <typename V>
__device__ __forceinline__ void primal_update(int64_t j, double g, double xj, double cj, double lo, double hi,
                                              double aj, V *__restrict__ x, V *__restrict__ xbar,
                                              double *__restrict__ xp, const DevState *__restrict__ st, int i,
                                              int store_cand)
{
    constexpr bool delta = sizeof(V) == sizeof(float);
    double xn = xj - st->tau * (cj - g);
    xn = xn < lo ? lo : xn;
    xn = xn > hi ? hi : xn;
    const double xb = 2.0 * xn - xj;
    // x and xbar go out as non-temporal stores: only the next launch reads
    // them (the dual half xbar, the next primal half x), from beyond this
    // XCD's L2 in any case, and lines left dirty in the L2 are written back
    // before the launch can end (c2 push: 5.8 -> 5.4 us per launch)
    __builtin_nontemporal_store((V)(delta ? xb - aj : xb), &xbar[j]);
    if (store_cand) xp[j] = xn;
    double xnew = xn;
    if (st->halpern) {
        double w, wa, gm;
        halpern_weights(st, i, w, wa, gm);
        xnew = w * ((1.0 + gm) * xn - gm * xj) + wa * aj;
    }
    __builtin_nontemporal_store((V)(delta ? xnew - aj : xnew), &x[j]);
}

// set the iterate of column j to v (mixed mode: as the anchor, difference 0;
// a phase start that follows makes the anchor the iterate in either mode)
template <typename V>
__device__ __forceinline__ void set_iterate(int64_t j, double v, V *__restrict__ x, double *__restrict__ xa)
{
    if (sizeof(V) == sizeof(float)) {
        xa[j] = v;
        x[j] = (V)0;
    } else {
        x[j] = (V)v;
        xa[j] = v;
    }
}

// the iterate from its stored form
template <typename V>
__device__ __forceinline__ double iterate_value(V stored, double anchor)
{
    return sizeof(V) == sizeof(float) ? anchor + (double)stored : (double)stored;
}

// Dual half:  y+ = proj_Y(y + sigma (bhat - h));  y <- w ((1+gamma) y+ - gamma y) + wa y_anchor.
__device__ __forceinline__ void dual_update(int64_t r, double h, double yr, double br, double ar, int8_t sn,
                                            double *__restrict__ y, double *__restrict__ yp,
                                            const DevState *__restrict__ st, int i, int store_cand)
{
    double yn = yr + st->sigma * (br - h);
    if (sn == '<') yn = yn < 0.0 ? yn : 0.0;
    else if (sn == '>') yn = yn > 0.0 ? yn : 0.0;
    else if (sn == 'N') yn = 0.0; // a row the dual push drops: y_i = 0
    if (store_cand) yp[r] = yn;
    double ynew = yn;
    if (st->halpern) {
        double w, wa, gm;
        halpern_weights(st, i, w, wa, gm);
        ynew = w * ((1.0 + gm) * yn - gm * yr) + wa * ar;
    }
    y[r] = ynew;
}

// ------------------------------------------------- LDS-tiled short rows ---
// A workgroup of NT threads owns a tile of T consecutive rows.  The tile's
// entries stream through LDS in chunks of kTileU * NT: every thread loads
// entries k, k+NT, ..., k+(kTileU-1)NT (coalesced index and value loads), all
// of them before their gathers and all gathers before the first product, so
// the latencies of one thread's entries overlap instead of adding up.  The
// tile's entry range comes from two uniform loads of the row pointers, so the
// entry loads need not wait for the per-row pointers to reach LDS.  Products
// go to LDS and G = NT/T threads per row sum their row's products in a fixed
// order.  Row sums go to LDS and threads 0..T-1 run the update epilogue on
// contiguous rows, with the epilogue's vector loads issued before the product
// phase.
constexpr int kTileU = 8; // entries per thread per chunk

template <typename VM, typename VV, int T, int NT>
__device__ __forceinline__ void tile_row_sums(int r0, int rows, const int *__restrict__ ptr,
                                              const int *__restrict__ idx, const VM *__restrict__ val,
                                              const VV *__restrict__ vec, int *s_ptr, double *s_prod,
                                              double *s_sum)
{
    constexpr int G = NT / T;
    constexpr int C = kTileU * NT;
    const int tid = threadIdx.x;
    const int beg = ptr[r0], end = ptr[r0 + rows]; // uniform across the workgroup
    // The tile's row pointers (rows + 1 <= NT + 1 of them) stay in registers
    // until the products go to LDS: storing them at once would wait for
    // their loads, and with them for every load issued earlier.
    const int pa = ptr[r0 + (tid < rows ? tid : rows)];
    const int pb = T >= NT ? ptr[r0 + (tid + NT < rows ? tid + NT : rows)] : 0;
    const int my_row = tid / G, sub = tid % G;
    const bool have = my_row < rows;
    double acc = 0.0;
    for (int cs = beg; cs < end; cs += C) {
        const int ce = cs + C < end ? cs + C : end;
        int id[kTileU];
        double v[kTileU], g[kTileU];
        // Slice u of the chunk is tested once for the whole workgroup; inside
        // a live slice every lane loads, lanes past the chunk's end reloading
        // its last entry.  A per-lane conditional load would be merged with
        // the fallback value right after it and so wait for each load in turn.
#pragma unroll
        for (int u = 0; u < kTileU; u++) {
            id[u] = 0;
            v[u] = 0.0;
            if (cs + u * NT < ce) {
                const int k = cs + tid + u * NT;
                const int kc = k < ce ? k : ce - 1;
                id[u] = idx[kc];
                v[u] = (double)val[kc];
            }
        }
#pragma unroll
        for (int u = 0; u < kTileU; u++) g[u] = cs + u * NT < ce ? (double)vec[id[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < kTileU; u++) {
            const int k = cs + tid + u * NT;
            if (k < ce) s_prod[k - cs] = v[u] * g[u];
        }
        if (cs == beg) {
            if (tid <= rows) s_ptr[tid] = pa;
            if (T >= NT && tid + NT <= rows) s_ptr[tid + NT] = pb;
        }
        __syncthreads(); // products, and on the first chunk the row pointers
        const int rb = have ? s_ptr[my_row] : 0, re = have ? s_ptr[my_row + 1] : 0;
        const int lo = rb > cs ? rb : cs, hi = re < ce ? re : ce;
        // the row's products in the same sequential order, read four at a time
        int q = lo + sub;
        for (; q + 3 * G < hi; q += 4 * G) {
            const double p0 = s_prod[q - cs], p1 = s_prod[q + G - cs];
            const double p2 = s_prod[q + 2 * G - cs], p3 = s_prod[q + 3 * G - cs];
            acc += p0;
            acc += p1;
            acc += p2;
            acc += p3;
        }
        for (; q < hi; q += G) acc += s_prod[q - cs];
        __syncthreads();
    }
    acc = group_sum<G>(acc);
    if (have && sub == 0) s_sum[my_row] = acc;
    __syncthreads();
}

// The check's quantities from per-block (or per-tile) partials: slot q folds
// its partials lo..hi-1 (row slots from pm + q*sm over [m0, m1), column slots
// from pn + q*sn over [n0, n1)), thread t taking lo+t, lo+t+kBlock, ... in
// that order, by sum or, for the infinity norms, by max.  Each round issues
// every slot's load (indices clamped into the range) before combining any,
// so a round costs one memory latency instead of one per slot.
__device__ __forceinline__ void fold_check_partials(double (&v)[Q_COUNT + 1], const double *pm, size_t sm, int m0,
                                                    int m1, const double *pn, size_t sn, int n0, int n1)
{
    constexpr unsigned row_slots =
        (1u << Q_PH2) | (1u << Q_P2) | (1u << Q_PINF) | (1u << Q_BTY) | (1u << Q_DY2) | (1u << Q_NAN);
    constexpr unsigned max_slots = (1u << Q_PINF) | (1u << Q_DINF);
    const int len = m1 - m0 > n1 - n0 ? m1 - m0 : n1 - n0;
    const int rounds = (len + kBlock - 1) / kBlock;
#pragma unroll
    for (int q = 0; q < Q_COUNT + 1; q++) v[q] = 0.0;
    for (int r = 0; r < rounds; r++) {
        const int off = (int)threadIdx.x + r * kBlock;
        double a[Q_COUNT + 1];
#pragma unroll
        for (int q = 0; q < Q_COUNT + 1; q++) {
            const bool row = (row_slots >> q) & 1u;
            const int lo = row ? m0 : n0, hi = row ? m1 : n1;
            const double *src = row ? pm + (size_t)q * sm : pn + (size_t)q * sn;
            const int k = lo + off;
            a[q] = hi > lo ? src[k < hi ? k : hi - 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < Q_COUNT + 1; q++) {
            const bool row = (row_slots >> q) & 1u;
            if ((row ? m0 : n0) + off < (row ? m1 : n1))
                v[q] = ((max_slots >> q) & 1u) ? fmax(v[q], a[q]) : v[q] + a[q];
        }
    }
}

__device__ __forceinline__ double kkt_weighted(double om, double p2, double d2, double g2)
{
    return sqrt(om * om * p2 + d2 / (om * om) + g2);
}

// The check's decisions for one LP, from its reduced quantities v[Q_*] (and
// v[Q_COUNT], the column NaN count):
//   mode 0: record the anchor's weighted-KKT parts (start of a phase);
//   mode 1: solve check (termination on all three relative tests, restart);
//   mode 2: push check (termination on the primal test only, restart);
//   mode 3: dual push check (termination on the dual test only, restart).
// `len` is the number of iterations since the last state update.
__device__ inline void check_decide(DevState *st, const double *v, int mode, int len)
{
    const double ph2 = v[Q_PH2], p2 = v[Q_P2], bty = v[Q_BTY], dy2 = v[Q_DY2];
    const double dh2 = v[Q_DH2], d2 = v[Q_D2], ctx = v[Q_CTX], bnd = v[Q_BND], dx2 = v[Q_DX2];
    const double nans = v[Q_NAN] + v[Q_COUNT];
    const double pobj = ctx, dobj = bty + bnd, gap = pobj - dobj;
    if (mode == 0) {
        st->anc_p2 = ph2;
        st->anc_d2 = dh2;
        st->anc_g2 = gap * gap;
        st->kkt_prev = kkt_weighted(st->omega, ph2, dh2, gap * gap);
        return;
    }
    const int64_t t_now = st->t + len, k_now = st->k0 + len;
    st->t = t_now;
    st->checks += 1;
    st->rel_p = sqrt(p2) / st->nb1;
    st->rel_d = sqrt(d2) / st->nc1;
    st->rel_gap = fabs(gap) / (1.0 + fabs(pobj) + fabs(dobj));
    st->pobj = pobj;
    st->dobj = dobj;
    st->restart_flag = 0;
    if (nans > 0.0) {
        st->done = 1;
        st->status = PDHG_NUMERICAL;
        st->k0 = k_now;
        return;
    }
    const double eps = st->eps_rel;
    if (mode == 1 && st->rel_p <= eps && st->rel_d <= eps && st->rel_gap <= eps) {
        st->done = 1;
        st->status = PDHG_OPTIMAL;
        st->k0 = k_now;
        return;
    }
    if ((mode == 2 && st->rel_p <= eps) || (mode == 3 && st->rel_d <= eps)) {
        st->done = 1;
        st->status = PDHG_PUSH_DONE;
        st->k0 = k_now;
        return;
    }
    const double om = st->omega;
    const double kc = kkt_weighted(om, ph2, dh2, gap * gap);
    const double ka = kkt_weighted(om, st->anc_p2, st->anc_d2, st->anc_g2);
    st->kkt_c = kc;
    const bool restart = (kc <= st->r_suff * ka) || (kc <= st->r_nec * ka && kc > st->kkt_prev) ||
                         ((double)k_now >= st->r_art * (double)t_now);
    st->kkt_prev = kc;
    if (!restart) {
        st->k0 = k_now;
        return;
    }
    const double dx = sqrt(dx2), dy = sqrt(dy2);
    double om2 = om;
    if (dx > 1e-10 && dy > 1e-10) {
        const double th = st->pw_smooth;
        om2 = exp(th * log(dy / dx) + (1.0 - th) * log(om));
    }
    st->omega = om2;
    st->tau = st->eta / om2;
    st->sigma = st->eta * om2;
    st->anc_p2 = ph2;
    st->anc_d2 = dh2;
    st->anc_g2 = gap * gap;
    st->kkt_prev = kkt_weighted(om2, ph2, dh2, gap * gap);
    st->k0 = 0;
    st->restarts += 1;
    st->restart_flag = 1;
}

// Objective coefficient and bounds of column j as a check evaluates them.
// During the solve the scaled original model is rebuilt in float64 from c,
// l, u and Dc (the values the setup stored before rounding them to the
// working precision), so that a float32 copy of chat, lhat, uhat cannot move
// the tested objectives; after a push rewrote the model, its stored values.
template <typename V>
__device__ __forceinline__ void check_model(bool orig, int64_t j, const double *ch, const V *lh, const V *uh,
                                            const double *c0, const double *l0, const double *u0, const double *dc,
                                            double &cj, double &lo, double &hi)
{
    if (orig) {
        cj = dc[j] * c0[j];
        lo = l0[j] / dc[j];
        hi = u0[j] / dc[j];
    } else {
        cj = ch[j];
        lo = (double)lh[j];
        hi = (double)uh[j];
    }
}

// splitmix64 (Steele, Lea and Flood 2014)
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// the push objective's Uniform[0,1) draw of column j: top 53 bits of
// splitmix64(seed xor j * golden-ratio constant), times 2^-53
__device__ __forceinline__ double push_unit(uint64_t seed, int64_t j)
{
    const uint64_t h = splitmix64(seed ^ ((uint64_t)j * 0x9E3779B97F4A7C15ULL));
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

// The power iteration's start vector, before scaling to unit length:
// v_j = 1 + U_j, U_j the same counter-based draw with a fixed seed.  Positive
// like a constant start (a large weight on the top singular vector of a
// nonnegative matrix), but not in the null space of matrices whose scaled
// rows sum to zero, such as [1, -1], where a constant start gives u = 0.
constexpr uint64_t kPowerSeed = 0x5DEECE66DULL;
__device__ __forceinline__ double power_start(int64_t j) { return 1.0 + push_unit(kPowerSeed, j); }

} // namespace pdhg
