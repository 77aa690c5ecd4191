// C ABI of the library: argument checks, ingest, the host loop that replays
// iteration cycles, and the corner-push orchestration.  All arithmetic of the
// method runs in the kernels of pdhg_setup.hip and pdhg_iter.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "pdhg.h"
#include "pdhg_internal.hpp"
#include "pdhg_mlp.hpp"

namespace pdhg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

hipError_t init_norms(pdhg_solver *s);

// candidates a push needs with the gate on (section 4.2): max(rows * m, min)
double gate_threshold(const pdhg_params &p, int64_t m)
{
    const double a = p.push_gate_rows * (double)m, b = (double)p.push_gate_min;
    return a > b ? a : b;
}

// byte model of the two kernels: v = bytes per matrix value and per entry of
// lhat, uhat, x, xbar (4 in the mixed mode, 8 otherwise); chat, the anchors
// and the m-vectors are float64; 4 bytes per index
void model_bytes(const pdhg_solver *s, int64_t *bytes_primal, int64_t *bytes_dual)
{
    const int64_t v = s->fp32 ? 4 : 8, m = s->m, n = s->n, nz = s->nnz;
    // primal: row pointers (none for uniform columns), indices + values, y
    // gathered once, reads x, chat, x_anchor, lhat, uhat, writes x, xbar
    *bytes_primal = (uses_uniform_kernel(s) ? 0 : 4 * (n + 1)) + (4 + v) * nz + 8 * m + (5 * v + 16) * n;
    // dual: row pointers, indices + values, xbar gathered once, reads y, bhat,
    // y_anchor, sense byte, writes y
    *bytes_dual = 4 * (m + 1) + (4 + v) * nz + v * n + 4 * 8 * m + m;
}
} // namespace pdhg

using namespace pdhg;

namespace {

struct HipFailure {
    hipError_t err;
    const char *what;
};

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw HipFailure{e, what};
}

#define HIPCHK(expr) hip_check((expr), #expr)

template <typename T>
void dalloc(T **p, size_t count)
{
    hip_check(hipMalloc((void **)p, sizeof(T) * (count > 0 ? count : 1)), "hipMalloc");
}

// The handle's current answer (unscaled, device): the solve's, the primal
// push's (xhat, y, z) or the dual push's (x, yhat, zhat).
const double *cur_x(const pdhg_solver *s) { return s->primal_pushed ? s->xpush : s->xu; }
const double *cur_y(const pdhg_solver *s) { return s->dual_pushed ? s->ypush : s->yu; }
const double *cur_z(const pdhg_solver *s) { return s->dual_pushed ? s->zpush : s->zsol; }

void free_all(pdhg_solver *s)
{
    (void)push_compact_end(s, false);
    void *ptrs[] = {s->rp,   s->ci, s->av,  s->tp,   s->ti,     s->tperm, s->atv,  s->b,   s->c,       s->l,
                    s->u,    s->sense0, s->dr, s->dc, s->ahat, s->ahat_t, s->x,   s->y,     s->xa,   s->ya,
                    s->xbar, s->xp, s->yp,  s->ch,   s->bh,     s->lh,    s->uh,   s->xs,  s->ys,      s->sense,
                    s->ax,   s->aty, s->xu, s->yu,   s->zsol,   s->xpush, s->partials, s->redout, s->st,
                    s->hx,   s->hz,  s->feat_raw, s->feat_b, s->logits, s->lfix, s->lcount, s->sell_idx,
                    s->sell_val, s->sell_soff, s->sell_len, s->sell_wi_start, s->sell_wi, s->sell_part,
                    s->ypush, s->zpush, s->w0, s->aerr, s->aerr_t, s->ex, s->ety,
                    s->aerr ? (void *)s->chc : nullptr, s->aerr ? (void *)s->bhc : nullptr};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->st_host) (void)hipHostFree(s->st_host);
    if (s->rep_host) (void)hipHostFree(s->rep_host);
    if (s->cnt_host) (void)hipHostFree(s->cnt_host);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    for (hipEvent_t &e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// iteration loop of one phase (mode 1 solve, mode 2 push) for at most
// `iters` iterations; returns the status
int run_phase(pdhg_solver *s, int64_t iters, int mode, double t0)
{
    const int K = s->p.check_every;
    const int64_t target = s->t_host + std::max<int64_t>(iters, 0);
    const int depth = 4; // cycles enqueued before the host looks at the state
    bool time_out = false;
    if (s->st_host->done) return s->st_host->status;
    if (s->defect_stale) HIPCHK(defect_refresh(s)); // anchored data at the phase's anchor (mixed mode)
    while (s->t_host < target) {
        int enq = 0;
        bool any_check = false;
        bool events = false;
        while (s->t_host < target && enq < depth) {
            const int64_t to_check = s->next_check - s->t_host;
            const int64_t left = target - s->t_host;
            const bool check = to_check <= left;
            const int len = (int)(check ? to_check : left);
            // with timing on, the first segment of every batch runs eagerly with
            // events around one primal and one dual launch; the rest replay
            const bool timed = s->p.timing && enq == 0 && len >= 2;
            if (check && len == K && s->p.use_graph && !timed) {
                HIPCHK(capture_cycle(s, K, mode));
                HIPCHK(hipGraphLaunch(s->graph_exec, s->stream));
            } else {
                HIPCHK(launch_iterations(s, len, check, mode, timed));
            }
            events = events || timed;
            s->t_host += len;
            if (check) {
                s->next_check += K;
                any_check = true;
            }
            enq++;
        }
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (events && !s->st_host->done) {
            float a = 0.0f, b2 = 0.0f;
            if (hipEventElapsedTime(&a, s->ev[0], s->ev[1]) == hipSuccess &&
                hipEventElapsedTime(&b2, s->ev[2], s->ev[3]) == hipSuccess) {
                s->t_primal_ms += a;
                s->t_dual_ms += b2;
                s->t_samples += 1;
                int64_t bp = 0, bd = 0;
                model_bytes(s, &bp, &bd); // of the model iterated now (the push may run on fewer columns)
                s->t_bytes_primal += (double)bp;
                s->t_bytes_dual += (double)bd;
            }
            (void)hipGetLastError(); // a failed timing query must not leak into later checks
        }
        s->has_candidate = s->st_host->checks > 0;
        (void)any_check;
        if (s->st_host->done) {
            s->t_host = s->st_host->t; // cycles enqueued after the stop did nothing
            break;
        }
        if (s->p.time_limit > 0.0 && now_s() - t0 > s->p.time_limit) {
            time_out = true;
            break;
        }
    }
    if (s->st_host->done) return s->st_host->status;
    return time_out ? PDHG_TIME_LIMIT : PDHG_ITER_LIMIT;
}

// unscaled solution (xu, yu) and its z / KKT report, for the current phase
void solution_report(pdhg_solver *s, pdhg_kkt_report *k)
{
    if (!s->has_candidate) HIPCHK(candidate_from_iterate(s));
    HIPCHK(unscale(s, (const double *)s->xp, (const double *)s->yp, s->xu, s->yu));
    HIPCHK(report(s, s->xu, s->yu, s->zsol, k));
}

int solve_iters(pdhg_solver *s, int64_t iters, pdhg_result *r)
{
    const double t0 = now_s();
    int st = run_phase(s, iters, 1, t0);
    pdhg_kkt_report k{};
    solution_report(s, &k);
    s->solved = s->has_candidate;
    if (r) {
        std::memset(r, 0, sizeof(*r));
        r->status = st;
        r->iters = s->t_host;
        r->restarts = s->st_host->restarts;
        r->rel_p = k.rel_p;
        r->rel_d = k.rel_d;
        r->rel_gap = k.rel_gap;
        r->pobj = k.pobj;
        r->dobj = k.dobj;
        r->seconds = now_s() - t0;
    }
    return PDHG_OK;
}

bool row_sorted_unique(const int64_t *rp, const int32_t *ci, int m)
{
    for (int i = 0; i < m; i++)
        for (int64_t e = rp[i] + 1; e < rp[i + 1]; e++)
            if (ci[e] <= ci[e - 1]) return false;
    return true;
}

// one batch phase (mode 1 solve, mode 2 push), lockstep cycles over all LPs;
// returns when every LP taking part is done or `iters` iterations have run
bool run_batch_phase(pdhg_batch *b, int64_t iters, int mode, double t0)
{
    pdhg_solver *s = b->s;
    const int K = s->p.check_every;
    const int depth = 4;
    const int64_t target = b->t_host + std::max<int64_t>(iters, 0);
    bool time_out = false;
    // algorithmic bytes of one primal / dual launch over the LPs that have not
    // stopped (tiles of stopped LPs exit at once), from the last host view
    // (the single-LP byte model, per LP)
    const double vbytes = s->fp32 ? 4.0 : 8.0;
    auto active_bytes = [&](double &bp, double &bd) {
        bp = bd = 0.0;
        for (int i = 0; i < b->count; i++) {
            if (b->sts_host[i].done) continue;
            const double mi = (double)(b->roff[i + 1] - b->roff[i]), ni = (double)(b->coff[i + 1] - b->coff[i]);
            const double nz = (double)b->nnz_of[i];
            bp += 4.0 * (ni + 1) + (4.0 + vbytes) * nz + 8.0 * mi + (5.0 * vbytes + 16.0) * ni;
            bd += 4.0 * (mi + 1) + (4.0 + vbytes) * nz + vbytes * ni + 33.0 * mi;
        }
    };
    HIPCHK(batch_compact_tiles(b, true));
    if (s->defect_stale) HIPCHK(batch_defect_refresh(b)); // anchored data at every LP's anchor (mixed mode)
    while (b->t_host < target) {
        int enq = 0;
        bool events = false;
        double bp_now = 0.0, bd_now = 0.0;
        if (s->p.timing) active_bytes(bp_now, bd_now);
        while (b->t_host < target && enq < depth) {
            const int64_t to_check = b->next_check - b->t_host;
            const int64_t left = target - b->t_host;
            const bool check = to_check <= left;
            const int len = (int)(check ? to_check : left);
            const bool timed = s->p.timing && enq == 0 && len >= 2;
            if (check && len == K && s->p.use_graph && !timed) {
                HIPCHK(batch_capture_cycle(b, K, mode));
                HIPCHK(hipGraphLaunch(b->graph, s->stream));
            } else {
                HIPCHK(batch_iterations(b, len, check, mode, timed));
            }
            events = events || timed;
            b->t_host += len;
            if (check) b->next_check += K;
            enq++;
        }
        HIPCHK(hipMemcpyAsync(b->sts_host, b->sts, sizeof(DevState) * (size_t)b->count, hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (events) {
            float a = 0.0f, b2 = 0.0f;
            if (hipEventElapsedTime(&a, s->ev[0], s->ev[1]) == hipSuccess &&
                hipEventElapsedTime(&b2, s->ev[2], s->ev[3]) == hipSuccess) {
                s->t_primal_ms += a;
                s->t_dual_ms += b2;
                s->t_samples += 1;
                b->timed_bytes_primal += bp_now;
                b->timed_bytes_dual += bd_now;
            }
            (void)hipGetLastError();
        }
        bool all_done = true;
        for (int i = 0; i < b->count; i++) all_done = all_done && b->sts_host[i].done;
        if (all_done) break;
        HIPCHK(batch_compact_tiles(b, false));
        if (s->p.time_limit > 0.0 && now_s() - t0 > s->p.time_limit) {
            time_out = true;
            break;
        }
    }
    return time_out;
}

void free_batch(pdhg_batch *b)
{
    (void)batch_push_compact_end(b, false);
    void *ptrs[] = {b->d_coff, b->ptiles, b->dtiles, b->rn, b->rm, b->rn_start, b->rm_start, b->sts,
                    b->part, b->lp_scalar, b->rep, b->active, b->seeds, b->fpart, b->fscale};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (b->sts_host) (void)hipHostFree(b->sts_host);
    if (b->rep_host) (void)hipHostFree(b->rep_host);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->s) {
        free_all(b->s);
        delete b->s;
    }
}

} // namespace

extern "C" {

void pdhg_default_params(pdhg_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eps_rel = 1e-6;
    p->eps_abs = 1e-6;
    p->max_iter = 1000000;
    p->check_every = 64;
    p->ruiz_iters = 10;
    p->restart_suff = 0.2;
    p->restart_nec = 0.8;
    p->restart_art = 0.36;
    p->pw_smooth = 0.5;
    p->pc_alpha = 1.0;
    p->power_iters = 4000;
    p->halpern = 1;
    p->eta_safety = 0.99;
    p->reflect_gamma = 1.0;
    p->power_tol = 1e-3;
    p->push_min_iters = 100;
    p->precision = PDHG_FP64;
    p->push_obj_scale = 1.0;
    p->push_max_iter = 1000000;
    p->time_limit = 0.0;
    p->stream = nullptr;
    p->verbosity = 0;
    p->lanes_at = 0;
    p->lanes_a = 0;
    p->use_graph = 1;
    p->timing = 0;
    p->autotune = 0;
    p->record_history = 0;
    p->push_compact = 1;
    p->push_gate = 0;
    p->push_gate_rows = 2.0;
    p->push_gate_min = 100000;
}

const char *pdhg_last_error(void) { return g_last_error.c_str(); }

int32_t pdhg_struct_size(int32_t which)
{
    switch (which) {
    case 0: return (int32_t)sizeof(pdhg_params);
    case 1: return (int32_t)sizeof(pdhg_result);
    case 2: return (int32_t)sizeof(pdhg_kkt_report);
    case 3: return (int32_t)sizeof(pdhg_push_result);
    case 4: return (int32_t)sizeof(pdhg_timing);
    case 5: return (int32_t)sizeof(pdhg_lp_desc);
    case 6: return (int32_t)sizeof(pdhg_batch_report);
    case 7: return (int32_t)sizeof(pdhg_dual_push_result);
    default: return -1;
    }
}

// Validate the parameters (NULL: the defaults) into p; returns PDHG_OK or the error.
static int check_params(const pdhg_params *params, pdhg_params &p)
{
    if (params) p = *params;
    else pdhg_default_params(&p);
    if (p.check_every < 1 || p.ruiz_iters < 0 || p.power_iters < 0 || p.push_min_iters < 1 ||
        (p.precision != PDHG_FP64 && p.precision != PDHG_FP32_MIXED) || !(p.eps_rel > 0.0) || !(p.eta_safety > 0.0) ||
        !(p.power_tol >= 0.0) || !(p.push_gate_rows >= 0.0) || p.push_gate_min < 0)
        return fail(PDHG_ERR_INVALID_ARG, "invalid parameter");
    // every remaining tolerance, factor and cap: a NaN would turn each test
    // that reads it into "false" (no fix, no restart, no stop)
    if (!(p.eps_abs >= 0.0 && std::isfinite(p.eps_abs)) || !(std::isfinite(p.eps_rel)))
        return fail(PDHG_ERR_INVALID_ARG, "eps_abs must be finite and >= 0, eps_rel finite");
    if (!(p.push_obj_scale > 0.0 && std::isfinite(p.push_obj_scale)))
        return fail(PDHG_ERR_INVALID_ARG, "push_obj_scale must be finite and > 0");
    if (p.max_iter < 0 || p.push_max_iter < 0) return fail(PDHG_ERR_INVALID_ARG, "negative iteration cap");
    if (!(p.reflect_gamma >= 0.0 && p.reflect_gamma <= 1.0))
        return fail(PDHG_ERR_INVALID_ARG, "reflect_gamma must lie in [0, 1]");
    if (!(p.pw_smooth >= 0.0 && p.pw_smooth <= 1.0)) return fail(PDHG_ERR_INVALID_ARG, "pw_smooth must lie in [0, 1]");
    if (!(p.restart_suff >= 0.0 && p.restart_suff <= 1.0) || !(p.restart_nec >= 0.0 && p.restart_nec <= 1.0) ||
        !(p.restart_art >= 0.0 && std::isfinite(p.restart_art)))
        return fail(PDHG_ERR_INVALID_ARG, "restart factors: suff and nec in [0, 1], art finite and >= 0");
    if (std::isnan(p.pc_alpha) || std::isnan(p.time_limit) || !std::isfinite(p.eta_safety))
        return fail(PDHG_ERR_INVALID_ARG, "NaN pc_alpha or time_limit, or infinite eta_safety");
    if (p.halpern != 0 && p.halpern != 1) return fail(PDHG_ERR_INVALID_ARG, "halpern must be 0 or 1");
    for (int half = 0; half < 2; half++) { // 0: primal half (lanes_at), 1: dual half (lanes_a)
        const int32_t k = half ? p.lanes_a : p.lanes_at;
        const bool lane_ok = k >= 1 && k <= 64 && !(k & (k - 1));
        const bool tile_ok = k == -32 || k == -64 || k == -128 || k == -256 || k == -1032 || k == -1064 ||
                             k == kRowBlock || (half == 1 && (k == kSell || k == kRowSegs));
        if (k != 0 && !lane_ok && !tile_ok)
            return fail(PDHG_ERR_INVALID_ARG, "lanes must be 0, a power of two in 1..64, one of "
                                              "-32/-64/-128/-256/-1032/-1064/-2256, or -3032/-4000 (lanes_a only)");
    }

    return PDHG_OK;
}

// Where a model's arrays come from: canonical host arrays (rows sorted and
// unique, bounds with infinities, senses filled in), or the caller's device
// arrays, which the device checks and converts (pdhg_create_device).
struct ModelSource {
    const int *rp = nullptr, *ci = nullptr;
    const double *av = nullptr, *b = nullptr, *c = nullptr, *l = nullptr, *u = nullptr;
    const int8_t *sense = nullptr;
    const DeviceModel *dev = nullptr;
};

// Upload (or take over on the device) one model, build its transpose and
// scale it.  With `single` the step size, norms and start point of a lone LP
// are set up as well; a batch does those per LP (pdhg_batch.hip).
static int build_solver(int m, int n, int nz, const pdhg_params &p, const ModelSource &src, bool single,
                        pdhg_solver **out)
{
    pdhg_solver *s = new (std::nothrow) pdhg_solver();
    if (!s) return fail(PDHG_ERR_OOM, "host allocation failed");
    try {
        s->m = m;
        s->n = n;
        s->nnz = nz;
        s->p = p;
        s->fp32 = p.precision == PDHG_FP32_MIXED;
        if (p.timing)
            for (hipEvent_t &e : s->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        if (p.stream) s->stream = (hipStream_t)p.stream;
        else {
            HIPCHK(hipStreamCreate(&s->stream));
            s->own_stream = true;
        }
        const double mean_a = m > 0 ? (double)nz / m : 1.0, mean_at = n > 0 ? (double)nz / n : 1.0;
        s->lanes_a = lanes_for_mean(mean_a);
        s->lanes_at = lanes_for_mean(mean_at);
        s->kern_a = p.lanes_a ? p.lanes_a : choose_kernel(mean_a, true);
        s->kern_at = p.lanes_at ? p.lanes_at : choose_kernel(mean_at, false);
        s->red_blocks_m = grid_for(m, kBlock, kMaxRedBlocks);
        s->red_blocks_n = grid_for(n, kBlock, kMaxRedBlocks);
        const size_t vb = s->fp32 ? sizeof(float) : sizeof(double);
        const size_t M = (size_t)m, N = (size_t)n, NZ = (size_t)nz;
        dalloc(&s->rp, M + 1);
        dalloc(&s->ci, NZ);
        dalloc(&s->av, NZ);
        dalloc(&s->tp, N + 1);
        dalloc(&s->ti, NZ);
        dalloc(&s->tperm, NZ);
        dalloc(&s->atv, NZ);
        dalloc(&s->b, M);
        dalloc(&s->c, N);
        dalloc(&s->l, N);
        dalloc(&s->u, N);
        dalloc(&s->sense0, M);
        dalloc(&s->sense, M);
        dalloc(&s->dr, M);
        dalloc(&s->dc, N);
        auto vall = [&](void **ptr, size_t cnt) { hip_check(hipMalloc(ptr, vb * (cnt > 0 ? cnt : 1)), "hipMalloc"); };
        vall(&s->ahat, NZ);
        vall(&s->ahat_t, NZ);
        for (void **q : {&s->x, &s->xbar, &s->lh, &s->uh}) vall(q, N);
        for (void **q : {&s->xa, &s->xp, &s->xs}) // anchor, candidate, solution: float64
            hip_check(hipMalloc(q, sizeof(double) * (N > 0 ? N : 1)), "hipMalloc");
        dalloc(&s->ch, N);
        for (void **q : {&s->y, &s->ya, &s->yp, &s->bh, &s->ys}) // m-vectors stay float64
            hip_check(hipMalloc(q, sizeof(double) * (M > 0 ? M : 1)), "hipMalloc");
        if (s->fp32) { // the float matrix's rounding error, its products and the anchored data
            hip_check(hipMalloc(&s->aerr, sizeof(float) * (NZ > 0 ? NZ : 1)), "hipMalloc");
            hip_check(hipMalloc(&s->aerr_t, sizeof(float) * (NZ > 0 ? NZ : 1)), "hipMalloc");
            dalloc(&s->ex, M);
            dalloc(&s->ety, N);
            dalloc(&s->chc, N);
            dalloc(&s->bhc, M);
        } else {
            defect_alias(s);
        }
        dalloc(&s->ax, M);
        dalloc(&s->aty, N);
        dalloc(&s->xu, N);
        dalloc(&s->yu, M);
        dalloc(&s->zsol, N);
        dalloc(&s->xpush, N);
        const size_t nparts = (size_t)(Q_COUNT + 1) * (s->red_blocks_m + s->red_blocks_n) * 3 + 4 * kMaxRedBlocks;
        dalloc(&s->partials, nparts);
        if (p.record_history) {
            dalloc(&s->hx, 4 * N);
            dalloc(&s->hz, 4 * N);
        }
        dalloc(&s->redout, 64);
        dalloc(&s->st, 1);
        HIPCHK(hipHostMalloc((void **)&s->st_host, sizeof(DevState), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&s->rep_host, sizeof(double) * 64, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&s->cnt_host, sizeof(int64_t) * 16, hipHostMallocDefault));

        hipStream_t st = s->stream;
        std::vector<int> rp_host;
        if (src.dev) { // the caller's device arrays: checked and converted on the device
            unsigned bad = 0;
            HIPCHK(ingest_device(s, *src.dev, &bad));
            if (bad) {
                free_all(s);
                delete s;
                return fail(PDHG_ERR_INVALID_ARG, ingest_error(bad));
            }
            if (s->kern_a == kSell) { // the sliced layout is planned on the host
                rp_host.resize(M + 1);
                HIPCHK(hipMemcpy(rp_host.data(), s->rp, sizeof(int) * (M + 1), hipMemcpyDeviceToHost));
            }
        } else {
            HIPCHK(hipMemcpyAsync(s->rp, src.rp, sizeof(int) * (M + 1), hipMemcpyHostToDevice, st));
            if (nz > 0) {
                HIPCHK(hipMemcpyAsync(s->ci, src.ci, sizeof(int) * NZ, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(s->av, src.av, sizeof(double) * NZ, hipMemcpyHostToDevice, st));
            }
            if (m > 0) {
                HIPCHK(hipMemcpyAsync(s->b, src.b, sizeof(double) * M, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(s->sense0, src.sense, M, hipMemcpyHostToDevice, st));
            }
            if (n > 0) {
                HIPCHK(hipMemcpyAsync(s->c, src.c, sizeof(double) * N, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(s->l, src.l, sizeof(double) * N, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(s->u, src.u, sizeof(double) * N, hipMemcpyHostToDevice, st));
            }
            rp_host.assign(src.rp, src.rp + M + 1);
        }
        DevState hs{};
        hs.gamma = p.reflect_gamma;
        hs.eps_rel = p.eps_rel;
        hs.r_suff = p.restart_suff;
        hs.r_nec = p.restart_nec;
        hs.r_art = p.restart_art;
        hs.pw_smooth = p.pw_smooth;
        hs.halpern = p.halpern;
        hs.status = PDHG_ITER_LIMIT;
        *s->st_host = hs;
        HIPCHK(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(build_transpose(s));
        HIPCHK(detect_uniform_columns(s));
        HIPCHK(scale_problem(s));
        if (s->aerr) { // until the first anchor: the data themselves (anchor 0)
            if (n > 0) HIPCHK(hipMemcpyAsync(s->chc, s->ch, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
            if (m > 0) HIPCHK(hipMemcpyAsync(s->bhc, s->bh, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
        }
        if (s->kern_a == kRowSegs || (single && p.autotune)) HIPCHK(plan_row_segments(s));
        if (s->kern_a == kSell) HIPCHK(sell_build(s, rp_host));
        if (single) {
            HIPCHK(power_iteration(s));
            HIPCHK(init_norms(s));
            HIPCHK(init_iteration(s));
            if (p.autotune) HIPCHK(autotune(s));
        }
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        s->t_host = 0;
        s->next_check = p.check_every;
    } catch (const HipFailure &f) {
        std::string msg = std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err);
        int code = (f.err == hipErrorOutOfMemory) ? PDHG_ERR_OOM : PDHG_ERR_HIP;
        free_all(s);
        delete s;
        return fail(code, msg);
    }
    *out = s;
    set_error("");
    return PDHG_OK;
}

// Validate and canonicalise a host model (rows sorted, duplicates summed),
// then build the solver on it (build_solver).
static int create_model(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                        const double *val, const double *b, const double *c, const double *l, const double *u,
                        const char *sense, const pdhg_params *params, bool single, pdhg_solver **out)
{
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (m < 0 || n < 0 || nnz < 0) return fail(PDHG_ERR_INVALID_ARG, "negative dimension");
    if (!row_ptr || (nnz > 0 && (!col_idx || !val)) || (m > 0 && !b) || (n > 0 && !c))
        return fail(PDHG_ERR_INVALID_ARG, "NULL array");
    if (nnz >= (int64_t)1 << 31) return fail(PDHG_ERR_INVALID_ARG, "nnz must stay below 2^31");
    if (row_ptr[0] != 0 || row_ptr[m] != nnz) return fail(PDHG_ERR_INVALID_ARG, "row_ptr[0] != 0 or row_ptr[m] != nnz");
    for (int i = 0; i < m; i++)
        if (row_ptr[i + 1] < row_ptr[i]) return fail(PDHG_ERR_INVALID_ARG, "row_ptr not non-decreasing");
    for (int64_t e = 0; e < nnz; e++) {
        if (col_idx[e] < 0 || col_idx[e] >= n) return fail(PDHG_ERR_INVALID_ARG, "column index out of range");
        if (!std::isfinite(val[e])) return fail(PDHG_ERR_INVALID_ARG, "non-finite matrix value");
    }
    for (int i = 0; i < m; i++) {
        if (!std::isfinite(b[i])) return fail(PDHG_ERR_INVALID_ARG, "non-finite b");
        if (sense && sense[i] != '=' && sense[i] != '<' && sense[i] != '>')
            return fail(PDHG_ERR_INVALID_ARG, "sense must be '=', '<' or '>'");
    }
    for (int j = 0; j < n; j++) {
        const double lo = l ? l[j] : 0.0, hi = u ? u[j] : INFINITY;
        if (!std::isfinite(c[j])) return fail(PDHG_ERR_INVALID_ARG, "non-finite c");
        if (std::isnan(lo) || std::isnan(hi) || lo > hi) return fail(PDHG_ERR_INVALID_ARG, "bad bounds (NaN or l > u)");
    }
    pdhg_params p;
    if (int rc = check_params(params, p)) return rc;

    // canonical rows (ascending columns, duplicates summed), host side ingest
    std::vector<int> rp((size_t)m + 1);
    std::vector<int> ci;
    std::vector<double> av;
    if (row_sorted_unique(row_ptr, col_idx, m)) {
        for (int i = 0; i <= m; i++) rp[i] = (int)row_ptr[i];
        ci.assign(col_idx, col_idx + nnz);
        av.assign(val, val + nnz);
    } else {
        ci.reserve((size_t)nnz);
        av.reserve((size_t)nnz);
        std::vector<std::pair<int, double>> row;
        rp[0] = 0;
        for (int i = 0; i < m; i++) {
            row.clear();
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) row.emplace_back(col_idx[e], val[e]);
            std::stable_sort(row.begin(), row.end(), [](auto &a, auto &b2) { return a.first < b2.first; });
            for (size_t q = 0; q < row.size(); q++) {
                if (!ci.empty() && (int)ci.size() > rp[i] && ci.back() == row[q].first) av.back() += row[q].second;
                else {
                    ci.push_back(row[q].first);
                    av.push_back(row[q].second);
                }
            }
            rp[i + 1] = (int)ci.size();
        }
    }
    const int nz = rp[m];
    std::vector<double> lv((size_t)n), uv((size_t)n);
    std::vector<int8_t> sv((size_t)m);
    for (int j = 0; j < n; j++) {
        const double lo = l ? l[j] : 0.0, hi = u ? u[j] : INFINITY;
        lv[j] = lo <= -1e20 ? -INFINITY : lo;
        uv[j] = hi >= 1e20 ? INFINITY : hi;
    }
    for (int i = 0; i < m; i++) sv[i] = (int8_t)(sense ? sense[i] : '=');

    ModelSource src;
    src.rp = rp.data();
    src.ci = ci.data();
    src.av = av.data();
    src.b = b;
    src.c = c;
    src.l = lv.data();
    src.u = uv.data();
    src.sense = sv.data();
    return build_solver(m, n, nz, p, src, single, out);
}

int pdhg_create_device(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                       const double *val, const double *b, const double *c, const double *l, const double *u,
                       const char *sense, const pdhg_params *params, pdhg_solver **out)
{
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (m < 0 || n < 0 || nnz < 0) return fail(PDHG_ERR_INVALID_ARG, "negative dimension");
    if (!row_ptr || (nnz > 0 && (!col_idx || !val)) || (m > 0 && !b) || (n > 0 && !c))
        return fail(PDHG_ERR_INVALID_ARG, "NULL array");
    if (nnz >= (int64_t)1 << 31) return fail(PDHG_ERR_INVALID_ARG, "nnz must stay below 2^31");
    pdhg_params p;
    if (int rc = check_params(params, p)) return rc;
    DeviceModel dm{m, n, nnz, row_ptr, col_idx, val, b, c, l, u, sense};
    ModelSource src;
    src.dev = &dm;
    return build_solver(m, n, (int)nnz, p, src, true, out);
}

int pdhg_create(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                const double *b, const double *c, const double *l, const double *u, const char *sense,
                const pdhg_params *params, pdhg_solver **out)
{
    return create_model(m, n, nnz, row_ptr, col_idx, val, b, c, l, u, sense, params, true, out);
}

int pdhg_iterate(pdhg_solver *s, int64_t iters, pdhg_result *r)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (iters < 0) return fail(PDHG_ERR_INVALID_ARG, "negative iteration count");
    if (s->in_push) return fail(PDHG_ERR_STATE, "the handle is in its push phase");
    try {
        return solve_iters(s, iters, r);
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
}

int pdhg_solve(pdhg_solver *s, pdhg_result *r)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (s->in_push) return fail(PDHG_ERR_STATE, "the handle is in its push phase");
    const int64_t left = s->p.max_iter - s->t_host;
    return pdhg_iterate(s, left > 0 ? left : 0, r);
}

// The corner push; with a network or caller logits (host, n float32), the
// learned warm start on top of the plain rule.
static int corner_push_common(pdhg_solver *s, uint64_t seed, pdhg_push_result *r, pdhg_mlp *net,
                              const float *logits_host, double theta)
{
    const bool learned = net != nullptr || logits_host != nullptr;
    if (!s || !r) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (!s->solved || s->in_push) return fail(PDHG_ERR_STATE, "corner push needs a solve first (and runs once)");
    std::memset(r, 0, sizeof(*r));
    const double t0 = now_s();
    try {
        hipStream_t st = s->stream;
        // CP1: the solve's candidate (x, y) and z on the original model
        HIPCHK(hipMemcpyAsync(s->xs, s->xp, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(s->ys, s->yp, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, st));
        HIPCHK(unscale(s, (const double *)s->xs, (const double *)s->ys, s->xu, s->yu));
        HIPCHK(report(s, s->xu, s->yu, s->zsol, &r->before));
        if (s->p.push_gate && (double)r->before.candidates < gate_threshold(s->p, s->m)) {
            // section 4.2's selection rule: too few candidates to be worth a push
            HIPCHK(hipMemcpyAsync(s->xpush, s->xu, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            r->after = r->before;
            r->status = PDHG_PUSH_SKIPPED;
            r->rel_p_push = NAN;
            r->seconds = now_s() - t0;
            s->in_push = true; // the handle's one push (skipped); pdhg_get_solution gives the solve's x
            s->primal_pushed = true;
            return PDHG_OK;
        }
        if (learned) { // predictor on the solve's state, before the model changes
            const size_t n = (size_t)(s->n > 0 ? s->n : 1);
            if (!s->logits) dalloc(&s->logits, n);
            if (!s->lfix) dalloc(&s->lfix, n);
            if (!s->lcount) dalloc(&s->lcount, 2);
            HIPCHK(hipMemsetAsync(s->lcount, 0, 2 * sizeof(unsigned), st));
            if (net) {
                if (!s->feat_raw) dalloc(&s->feat_raw, 16 * n);
                if (!s->feat_b) dalloc(&s->feat_b, 16 * n);
                HIPCHK(compute_features(s, seed));
                HIPCHK(mlp_forward(net, st, s->feat_b, s->n, s->logits));
            } else if (s->n > 0) {
                HIPCHK(hipMemcpyAsync(s->logits, logits_host, sizeof(float) * (size_t)s->n, hipMemcpyHostToDevice,
                                      st));
            }
        }
        // CP2-CP5: bounds, senses, objective, start (x, 0), new weight and restart state
        HIPCHK(push_setup(s, seed, r, learned ? theta : -1.0));
        s->learned_active = learned;
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        s->in_push = true;
        s->primal_pushed = true;
        s->has_candidate = false;
        s->t_host = 0;
        s->next_check = s->p.push_min_iters;
        // CP6, on the free columns (learned fixes kept), unless the dual half
        // uses the sliced layout of the full matrix
        if (s->p.push_compact && s->kern_a != kSell) HIPCHK(push_compact_begin(s));
        int status = run_phase(s, s->p.push_max_iter, 2, t0);
        HIPCHK(push_compact_end(s, true));
        // CP7: (xhat, y, z)
        if (s->has_candidate) HIPCHK(unscale(s, (const double *)s->xp, nullptr, s->xpush, nullptr));
        else HIPCHK(hipMemcpyAsync(s->xpush, s->xu, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
        HIPCHK(report(s, s->xpush, s->yu, nullptr, &r->after));
        r->status = status;
        r->iters = s->t_host;
        r->restarts = s->st_host->restarts;
        r->rel_p_push = s->st_host->checks > 0 ? s->st_host->rel_p : NAN;
        r->seconds = now_s() - t0;
        if (learned) {
            unsigned cnt[2] = {0, 0};
            HIPCHK(hipMemcpy(cnt, s->lcount, sizeof(cnt), hipMemcpyDeviceToHost));
            r->n_learned_fix = cnt[0];
            r->n_learned_undo = cnt[1];
        }
    } catch (const HipFailure &f) {
        (void)push_compact_end(s, false); // the full model's arrays back in the handle
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_corner_push(pdhg_solver *s, uint64_t seed, pdhg_push_result *r)
{
    return corner_push_common(s, seed, r, nullptr, nullptr, -1.0);
}

int pdhg_corner_push_learned(pdhg_solver *s, pdhg_mlp *net, double theta, uint64_t seed, pdhg_push_result *r)
{
    if (!net) return fail(PDHG_ERR_INVALID_ARG, "NULL network");
    if (!(theta > 0.0 && theta < 1.0)) return fail(PDHG_ERR_INVALID_ARG, "theta must lie in (0, 1)");
    return corner_push_common(s, seed, r, net, nullptr, theta);
}

int pdhg_corner_push_logits(pdhg_solver *s, const float *logits, double theta, uint64_t seed, pdhg_push_result *r)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (!logits && s->n > 0) return fail(PDHG_ERR_INVALID_ARG, "NULL logits");
    if (!(theta > 0.0 && theta < 1.0)) return fail(PDHG_ERR_INVALID_ARG, "theta must lie in (0, 1)");
    return corner_push_common(s, seed, r, nullptr, logits, theta);
}

// The dual corner push: DP1 the solve's answer, x replaced by the corner
// push's xhat when that push came first, and its report (which leaves A x in
// s->ax and A'y in s->aty), DP2-DP5 the dual face of x as a push model
// anchored at the solve's y, with the anchored random right-hand side, start
// (0, y), DP6 PDHG to the dual test, DP7 (x, yhat, zhat).
int pdhg_dual_push(pdhg_solver *s, uint64_t seed, pdhg_dual_push_result *r)
{
    if (!s || !r) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (!s->solved || s->dual_pushed)
        return fail(PDHG_ERR_STATE, "dual push needs a solve first (and runs once)");
    std::memset(r, 0, sizeof(*r));
    const double t0 = now_s();
    try {
        hipStream_t st = s->stream;
        if (!s->ypush) dalloc(&s->ypush, (size_t)(s->m > 0 ? s->m : 1));
        if (!s->zpush) dalloc(&s->zpush, (size_t)(s->n > 0 ? s->n : 1));
        // DP1 (after the corner push, xs, ys, xu, yu already hold the solve's answer)
        if (!s->primal_pushed) {
            HIPCHK(hipMemcpyAsync(s->xs, s->xp, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(s->ys, s->yp, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, st));
            HIPCHK(unscale(s, (const double *)s->xs, (const double *)s->ys, s->xu, s->yu));
        }
        const double *xk = cur_x(s);
        HIPCHK(report(s, xk, s->yu, s->zsol, &r->before));
        // DP2-DP5; ybar on the dropped rows lives in ypush and A_N'ybar_N in
        // zpush until the push writes them
        if (!s->w0) dalloc(&s->w0, (size_t)(s->n > 0 ? s->n : 1));
        HIPCHK(dual_push_setup(s, seed, xk, s->w0, s->ypush, s->zpush, &r->n_cols_free, &r->n_rows_fixed));
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        s->in_push = true;
        s->dual_pushed = true;
        s->has_candidate = false;
        s->t_host = 0;
        s->next_check = s->p.push_min_iters;
        // DP6
        int status = run_phase(s, s->p.push_max_iter, 3, t0);
        // DP7
        if (s->has_candidate) {
            HIPCHK(unscale(s, nullptr, (const double *)s->yp, nullptr, s->ypush));
            HIPCHK(dual_push_finish(s)); // the solve's y on the dropped rows
        } else {
            HIPCHK(hipMemcpyAsync(s->ypush, s->yu, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, st));
        }
        HIPCHK(report(s, xk, s->ypush, s->zpush, &r->after));
        r->status = status;
        r->iters = s->t_host;
        r->restarts = s->st_host->restarts;
        r->rel_d_push = s->st_host->checks > 0 ? s->st_host->rel_d : NAN;
        r->seconds = now_s() - t0;
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_features(pdhg_solver *s, uint64_t seed, float *out)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (!s->solved || s->in_push) return fail(PDHG_ERR_STATE, "features describe a solved LP before its push");
    try {
        const size_t n = (size_t)(s->n > 0 ? s->n : 1);
        if (!s->feat_raw) dalloc(&s->feat_raw, 16 * n);
        if (!s->feat_b) dalloc(&s->feat_b, 16 * n);
        HIPCHK(compute_features(s, seed));
        if (out) HIPCHK(hipMemcpyAsync(out, s->feat_raw, sizeof(float) * 16 * (size_t)s->n, hipMemcpyDeviceToHost,
                                       s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_kkt(pdhg_solver *s, const double *x, const double *y, pdhg_kkt_report *k)
{
    if (!s || !k) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    try {
        hipStream_t st = s->stream;
        double *dx = nullptr, *dy = nullptr;
        if (!s->in_push && (!x || !y)) {
            pdhg_kkt_report tmp;
            solution_report(s, &tmp);
        }
        const double *cx = cur_x(s);
        const double *cy = cur_y(s);
        if (x) {
            dalloc(&dx, (size_t)s->n);
            HIPCHK(hipMemcpyAsync(dx, x, sizeof(double) * (size_t)s->n, hipMemcpyHostToDevice, st));
            cx = dx;
        }
        if (y) {
            dalloc(&dy, (size_t)s->m);
            HIPCHK(hipMemcpyAsync(dy, y, sizeof(double) * (size_t)s->m, hipMemcpyHostToDevice, st));
            cy = dy;
        }
        hipError_t e = report(s, cx, cy, nullptr, k);
        if (dx) (void)hipFree(dx);
        if (dy) (void)hipFree(dy);
        HIPCHK(e);
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_get_solution(pdhg_solver *s, double *x, double *y, double *z)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    try {
        hipStream_t st = s->stream;
        if (!s->in_push) {
            pdhg_kkt_report tmp;
            solution_report(s, &tmp);
        }
        if (x) HIPCHK(hipMemcpyAsync(x, cur_x(s), sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost, st));
        if (y) HIPCHK(hipMemcpyAsync(y, cur_y(s), sizeof(double) * (size_t)s->m, hipMemcpyDeviceToHost, st));
        if (z) HIPCHK(hipMemcpyAsync(z, cur_z(s), sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_get_solve_solution(pdhg_solver *s, double *x, double *y, double *z)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (!s->solved) return fail(PDHG_ERR_STATE, "no solve answer yet");
    try {
        hipStream_t st = s->stream;
        if (!s->in_push) {
            pdhg_kkt_report tmp;
            solution_report(s, &tmp);
        }
        // xu, yu, zsol hold the solve's answer; the push writes its x to xpush
        if (x) HIPCHK(hipMemcpyAsync(x, s->xu, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost, st));
        if (y) HIPCHK(hipMemcpyAsync(y, s->yu, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToHost, st));
        if (z) HIPCHK(hipMemcpyAsync(z, s->zsol, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_get_solution_device(pdhg_solver *s, double *x, double *y, double *z, void *stream)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    try {
        hipStream_t st = s->stream;
        if (!s->in_push) {
            pdhg_kkt_report tmp;
            solution_report(s, &tmp);
        }
        if (x) HIPCHK(hipMemcpyAsync(x, cur_x(s), sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
        if (y) HIPCHK(hipMemcpyAsync(y, cur_y(s), sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, st));
        if (z) HIPCHK(hipMemcpyAsync(z, cur_z(s), sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
        hipStream_t cs = stream ? (hipStream_t)stream : st;
        if (cs != st) { // order the caller's stream after the copies
            hipEvent_t ev = nullptr;
            HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            HIPCHK(hipEventRecord(ev, st));
            HIPCHK(hipStreamWaitEvent(cs, ev, 0));
            HIPCHK(hipEventDestroy(ev));
        }
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_set_start(pdhg_solver *s, const double *x, const double *y)
{
    if (!s || !x || !y) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (s->in_push) return fail(PDHG_ERR_STATE, "the handle is in its push phase");
    for (int j = 0; j < s->n; j++)
        if (!std::isfinite(x[j])) return fail(PDHG_ERR_INVALID_ARG, "non-finite start x");
    for (int i = 0; i < s->m; i++)
        if (!std::isfinite(y[i])) return fail(PDHG_ERR_INVALID_ARG, "non-finite start y");
    try {
        hipStream_t st = s->stream;
        HIPCHK(hipMemcpyAsync(s->xu, x, sizeof(double) * (size_t)s->n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s->yu, y, sizeof(double) * (size_t)s->m, hipMemcpyHostToDevice, st));
        HIPCHK(set_start(s));
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        s->t_host = 0;
        s->next_check = s->p.check_every;
        s->has_candidate = false;
        s->solved = false;
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

// checkpoint layout: header, DevState, x, x_anchor, x+ (working precision),
// y, y_anchor, y+ (float64)
namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, m, n, fp32;
    int64_t t_host, next_check;
    int32_t has_candidate, solved;
    int64_t bytes;
};
constexpr char kCkptMagic[8] = {'P', 'D', 'H', 'G', 'C', 'K', 'P', 'T'};

int64_t ckpt_bytes(const pdhg_solver *s)
{
    // x in the working precision (mixed mode: its difference from x_a), x_a and x+ in float64, y, y_a, y+
    const int64_t vb = s->fp32 ? 4 : 8;
    return (int64_t)sizeof(CkptHeader) + (int64_t)sizeof(DevState) + (vb + 16) * s->n + 3 * 8 * (int64_t)s->m;
}
} // namespace

int pdhg_state_size(pdhg_solver *s, int64_t *bytes)
{
    if (!s || !bytes) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    *bytes = ckpt_bytes(s);
    return PDHG_OK;
}

int pdhg_get_state(pdhg_solver *s, void *buf, int64_t bytes)
{
    if (!s || !buf) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (bytes < ckpt_bytes(s)) return fail(PDHG_ERR_INVALID_ARG, "state buffer smaller than pdhg_state_size");
    if (s->in_push) return fail(PDHG_ERR_STATE, "checkpoints cover the solve phase only");
    try {
        hipStream_t st = s->stream;
        char *p = (char *)buf;
        CkptHeader h{};
        std::memcpy(h.magic, kCkptMagic, 8);
        h.version = 2;
        h.m = s->m;
        h.n = s->n;
        h.fp32 = s->fp32 ? 1 : 0;
        h.t_host = s->t_host;
        h.next_check = s->next_check;
        h.has_candidate = s->has_candidate ? 1 : 0;
        h.solved = s->solved ? 1 : 0;
        h.bytes = ckpt_bytes(s);
        std::memcpy(p, &h, sizeof(h));
        p += sizeof(h);
        HIPCHK(hipMemcpyAsync(p, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        p += sizeof(DevState);
        const size_t vb = (size_t)(s->fp32 ? 4 : 8) * (size_t)s->n, xb = 8 * (size_t)s->n, yb = 8 * (size_t)s->m;
        for (const void *src : {(const void *)s->x, (const void *)s->xa, (const void *)s->xp}) {
            const size_t nb = src == s->x ? vb : xb;
            HIPCHK(hipMemcpyAsync(p, src, nb, hipMemcpyDeviceToHost, st));
            p += nb;
        }
        for (const void *src : {(const void *)s->y, (const void *)s->ya, (const void *)s->yp}) {
            HIPCHK(hipMemcpyAsync(p, src, yb, hipMemcpyDeviceToHost, st));
            p += yb;
        }
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_set_state(pdhg_solver *s, const void *buf, int64_t bytes)
{
    if (!s || !buf) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (s->in_push) return fail(PDHG_ERR_STATE, "checkpoints cover the solve phase only");
    CkptHeader h;
    if (bytes < (int64_t)sizeof(h)) return fail(PDHG_ERR_INVALID_ARG, "state buffer too small");
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 2)
        return fail(PDHG_ERR_INVALID_ARG, "not a checkpoint of this library");
    if (h.m != s->m || h.n != s->n || h.fp32 != (s->fp32 ? 1 : 0) || h.bytes != ckpt_bytes(s) || bytes < h.bytes)
        return fail(PDHG_ERR_INVALID_ARG, "checkpoint of another LP size or precision");
    try {
        hipStream_t st = s->stream;
        const char *p = (const char *)buf + sizeof(h);
        HIPCHK(hipMemcpyAsync(s->st, p, sizeof(DevState), hipMemcpyHostToDevice, st));
        p += sizeof(DevState);
        const size_t vb = (size_t)(s->fp32 ? 4 : 8) * (size_t)s->n, xb = 8 * (size_t)s->n, yb = 8 * (size_t)s->m;
        for (void *dst : {(void *)s->x, (void *)s->xa, (void *)s->xp}) {
            const size_t nb = dst == s->x ? vb : xb;
            HIPCHK(hipMemcpyAsync(dst, p, nb, hipMemcpyHostToDevice, st));
            p += nb;
        }
        for (void *dst : {(void *)s->y, (void *)s->ya, (void *)s->yp}) {
            HIPCHK(hipMemcpyAsync(dst, p, yb, hipMemcpyHostToDevice, st));
            p += yb;
        }
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        s->t_host = h.t_host;
        s->next_check = h.next_check;
        s->defect_stale = true; // the restored anchor's correction (mixed mode)
        s->has_candidate = h.has_candidate != 0;
        s->solved = h.solved != 0;
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_get_iterate(pdhg_solver *s, double *x, double *y)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    try {
        hipStream_t st = s->stream;
        double *dx = nullptr, *dy = nullptr;
        dalloc(&dx, (size_t)s->n);
        dalloc(&dy, (size_t)s->m);
        HIPCHK(unscale_iterate(s, dx, dy));
        if (x) HIPCHK(hipMemcpyAsync(x, dx, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost, st));
        if (y) HIPCHK(hipMemcpyAsync(y, dy, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToHost, st));
        hipError_t e = hipStreamSynchronize(st);
        (void)hipFree(dx);
        (void)hipFree(dy);
        HIPCHK(e);
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_get_scaling(pdhg_solver *s, double *dr, double *dc, double *scalars5)
{
    if (!s) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    try {
        hipStream_t st = s->stream;
        if (dr) HIPCHK(hipMemcpyAsync(dr, s->dr, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToHost, st));
        if (dc) HIPCHK(hipMemcpyAsync(dc, s->dc, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (scalars5) {
            scalars5[0] = s->st_host->eta;
            scalars5[1] = s->st_host->omega;
            scalars5[2] = s->st_host->sigma_est;
            scalars5[3] = (double)s->t_host;
            scalars5[4] = (double)s->power_steps;
        }
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_get_timing(pdhg_solver *s, pdhg_timing *t)
{
    if (!s || !t) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    std::memset(t, 0, sizeof(*t));
    t->samples = s->t_samples;
    if (s->t_samples > 0) {
        t->primal_ms = s->t_primal_ms / (double)s->t_samples;
        t->dual_ms = s->t_dual_ms / (double)s->t_samples;
    }
    if (s->t_samples > 0) { // mean over the timed launches (solve and push models)
        t->bytes_primal = (int64_t)(s->t_bytes_primal / (double)s->t_samples);
        t->bytes_dual = (int64_t)(s->t_bytes_dual / (double)s->t_samples);
    } else {
        model_bytes(s, &t->bytes_primal, &t->bytes_dual);
    }
    t->lanes_at = s->kern_at;
    t->lanes_a = s->kern_a;
    return PDHG_OK;
}

int pdhg_copy_probe(int64_t bytes, int32_t reps, double *gbps)
{
    if (bytes < 16 || reps < 1 || !gbps) return fail(PDHG_ERR_INVALID_ARG, "bad copy-probe arguments");
    hipError_t e = copy_probe(bytes, reps, gbps);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? PDHG_ERR_OOM : PDHG_ERR_HIP, std::string("copy probe: ") + hipGetErrorString(e));
    return PDHG_OK;
}

void pdhg_destroy(pdhg_solver *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
}

static int batch_finish(pdhg_solver *s, int count, const std::vector<int> &roff, const std::vector<int> &coff,
                        const std::vector<int64_t> &nnz_of, const pdhg_params &p, pdhg_batch **out);

int pdhg_batch_create(int32_t count, const pdhg_lp_desc *lps, const pdhg_params *params, pdhg_batch **out)
{
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !lps) return fail(PDHG_ERR_INVALID_ARG, "count must be >= 1 with a descriptor array");
    pdhg_params p;
    if (params) p = *params;
    else pdhg_default_params(&p);
    for (int32_t k : {p.lanes_a, p.lanes_at})
        if (k > 0 || k == kRowBlock || k == kSell || k == kRowSegs)
            return fail(PDHG_ERR_INVALID_ARG, "the batch engine runs tiled kernels only (lanes -32/-64/-128/-256/-1032/-1064)");
    // one block-diagonal model with global column indices
    std::vector<int> roff(1, 0), coff(1, 0);
    int64_t nz_total = 0;
    for (int i = 0; i < count; i++) {
        const pdhg_lp_desc &d = lps[i];
        if (d.m < 1 || d.n < 1 || d.nnz < 0 || !d.row_ptr || !d.b || !d.c || (d.nnz > 0 && (!d.col_idx || !d.val)))
            return fail(PDHG_ERR_INVALID_ARG, "LP " + std::to_string(i) + ": bad dimensions or NULL arrays");
        if (d.row_ptr[0] != 0 || d.row_ptr[d.m] != d.nnz)
            return fail(PDHG_ERR_INVALID_ARG, "LP " + std::to_string(i) + ": row_ptr[0] != 0 or row_ptr[m] != nnz");
        if ((int64_t)roff.back() + d.m >= (int64_t)1 << 31 || (int64_t)coff.back() + d.n >= (int64_t)1 << 31)
            return fail(PDHG_ERR_INVALID_ARG, "batch too large for 32-bit indices");
        roff.push_back(roff.back() + d.m);
        coff.push_back(coff.back() + d.n);
        nz_total += d.nnz;
    }
    if (nz_total >= (int64_t)1 << 31) return fail(PDHG_ERR_INVALID_ARG, "batch nnz must stay below 2^31");
    const int M = roff.back(), N = coff.back();
    std::vector<int64_t> rp((size_t)M + 1, 0);
    std::vector<int32_t> ci((size_t)nz_total);
    std::vector<double> va((size_t)nz_total), bb((size_t)M), cc((size_t)N), ll((size_t)N), uu((size_t)N);
    std::vector<char> sn((size_t)M);
    int64_t w = 0;
    for (int i = 0; i < count; i++) {
        const pdhg_lp_desc &d = lps[i];
        for (int r = 0; r < d.m; r++) {
            for (int64_t e = d.row_ptr[r]; e < d.row_ptr[r + 1]; e++, w++) {
                const int32_t col = d.col_idx[e];
                if (col < 0 || col >= d.n)
                    return fail(PDHG_ERR_INVALID_ARG, "LP " + std::to_string(i) + ": column index out of range");
                ci[w] = col + coff[i];
                va[w] = d.val[e];
            }
            rp[roff[i] + r + 1] = w;
            bb[roff[i] + r] = d.b[r];
            sn[roff[i] + r] = d.sense ? d.sense[r] : '=';
        }
        for (int j = 0; j < d.n; j++) {
            cc[coff[i] + j] = d.c[j];
            ll[coff[i] + j] = d.l ? d.l[j] : 0.0;
            uu[coff[i] + j] = d.u ? d.u[j] : INFINITY;
        }
    }
    pdhg_solver *s = nullptr;
    int rc = create_model(M, N, nz_total, rp.data(), ci.data(), va.data(), bb.data(), cc.data(), ll.data(), uu.data(),
                          sn.data(), &p, false, &s);
    if (rc != PDHG_OK) return rc;
    std::vector<int64_t> nnz_of;
    for (int i = 0; i < count; i++) nnz_of.push_back(lps[i].nnz);
    return batch_finish(s, count, roff, coff, nnz_of, p, out);
}

// The batch around a solver already built on the block-diagonal model: tiles,
// per-LP state, kernel choice, setup and the first phase start.
static int batch_finish(pdhg_solver *s, int count, const std::vector<int> &roff, const std::vector<int> &coff,
                        const std::vector<int64_t> &nnz_of, const pdhg_params &p, pdhg_batch **out)
{
    const int M = roff.back(), N = coff.back();
    int64_t nz_total = 0;
    for (int64_t v : nnz_of) nz_total += v;
    pdhg_batch *b = new (std::nothrow) pdhg_batch();
    if (!b) {
        pdhg_destroy(s);
        return fail(PDHG_ERR_OOM, "host allocation failed");
    }
    b->s = s;
    b->count = count;
    b->roff = roff;
    b->coff = coff;
    b->nnz_of = nnz_of;
    try {
        hipStream_t st = s->stream;
        std::vector<int4> rn, rm;
        std::vector<int> rn_start, rm_start;
        auto tiles = [&](const std::vector<int> &off, std::vector<int4> &t, std::vector<int> &start) {
            t.clear();
            start.assign((size_t)count + 1, 0);
            for (int i = 0; i < count; i++) {
                start[i] = (int)t.size();
                for (int r = off[i]; r < off[i + 1]; r += kBlock) {
                    int4 q;
                    q.x = i;
                    q.y = r;
                    q.z = std::min(kBlock, off[i + 1] - r);
                    q.w = 0;
                    t.push_back(q);
                }
            }
            start[count] = (int)t.size();
        };
        tiles(coff, rn, rn_start);
        tiles(roff, rm, rm_start);
        b->n_rn = (int)rn.size();
        b->n_rm = (int)rm.size();
        dalloc(&b->rn, rn.size());
        dalloc(&b->rm, rm.size());
        dalloc(&b->rn_start, rn_start.size());
        dalloc(&b->rm_start, rm_start.size());
        dalloc(&b->d_coff, coff.size());
        HIPCHK(hipMemcpy(b->rn, rn.data(), sizeof(int4) * rn.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->rm, rm.data(), sizeof(int4) * rm.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->rn_start, rn_start.data(), sizeof(int) * rn_start.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->rm_start, rm_start.data(), sizeof(int) * rm_start.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_coff, coff.data(), sizeof(int) * coff.size(), hipMemcpyHostToDevice));
        dalloc(&b->sts, (size_t)count);
        dalloc(&b->part, (size_t)(Q_COUNT + 1) * (b->n_rm + b->n_rn));
        dalloc(&b->lp_scalar, 4 * (size_t)count);
        dalloc(&b->rep, (size_t)count * R_COUNT);
        dalloc(&b->active, (size_t)count);
        dalloc(&b->seeds, (size_t)count);
        HIPCHK(hipHostMalloc((void **)&b->sts_host, sizeof(DevState) * (size_t)count, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&b->rep_host, sizeof(double) * R_COUNT * (size_t)count, hipHostMallocDefault));
        // every LP starts from the constants of the shared parameters
        for (int i = 0; i < count; i++) b->sts_host[i] = *s->st_host;
        HIPCHK(hipMemcpy(b->sts, b->sts_host, sizeof(DevState) * (size_t)count, hipMemcpyHostToDevice));
        b->active_host.assign((size_t)count, 1);
        HIPCHK(hipMemcpy(b->active, b->active_host.data(), sizeof(int) * (size_t)count, hipMemcpyHostToDevice));
        // tiled kernels from the mean row lengths (tiles only: the batch has no lane-group path)
        auto tiled = [](double mean) {
            const int k = choose_kernel(mean, false);
            if (k == kRowBlock || k > 0) return mean <= 3.0 ? -256 : -32;
            return k;
        };
        const int ka = p.lanes_a ? p.lanes_a : tiled(M > 0 ? (double)nz_total / M : 1.0);
        const int kat = p.lanes_at ? p.lanes_at : tiled(N > 0 ? (double)nz_total / N : 1.0);
        HIPCHK(batch_set_kernels(b, kat, ka));
        HIPCHK(batch_setup(b));
        HIPCHK(batch_phase_begin(b, true));
        if (p.autotune) HIPCHK(batch_autotune(b));
        HIPCHK(hipStreamSynchronize(st));
        b->t_host = 0;
        b->next_check = p.check_every;
    } catch (const HipFailure &f) {
        free_batch(b);
        delete b;
        return fail(f.err == hipErrorOutOfMemory ? PDHG_ERR_OOM : PDHG_ERR_HIP,
                    std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    *out = b;
    set_error("");
    return PDHG_OK;
}

int pdhg_batch_create_device(int32_t count, const pdhg_lp_desc *lps, const pdhg_params *params, pdhg_batch **out)
{
    if (!out) return fail(PDHG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !lps) return fail(PDHG_ERR_INVALID_ARG, "count must be >= 1 with a descriptor array");
    if (count > 65535) return fail(PDHG_ERR_INVALID_ARG, "a batch from device arrays takes at most 65535 LPs");
    pdhg_params p;
    if (int rc = check_params(params, p)) return rc;
    for (int32_t k : {p.lanes_a, p.lanes_at})
        if (k > 0 || k == kRowBlock || k == kSell || k == kRowSegs)
            return fail(PDHG_ERR_INVALID_ARG, "the batch engine runs tiled kernels only (lanes -32/-64/-128/-256/-1032/-1064)");
    std::vector<int> roff(1, 0), coff(1, 0);
    std::vector<int64_t> nnz_of;
    std::vector<BatchPart> parts;
    int64_t nz_total = 0;
    for (int i = 0; i < count; i++) {
        const pdhg_lp_desc &d = lps[i];
        if (d.m < 1 || d.n < 1 || d.nnz < 0 || !d.row_ptr || !d.b || !d.c || (d.nnz > 0 && (!d.col_idx || !d.val)))
            return fail(PDHG_ERR_INVALID_ARG, "LP " + std::to_string(i) + ": bad dimensions or NULL arrays");
        if ((int64_t)roff.back() + d.m >= (int64_t)1 << 31 || (int64_t)coff.back() + d.n >= (int64_t)1 << 31)
            return fail(PDHG_ERR_INVALID_ARG, "batch too large for 32-bit indices");
        parts.push_back(BatchPart{d.row_ptr, d.col_idx, d.val, d.b, d.c, d.l, d.u, d.sense, d.m, d.n, d.nnz,
                                  roff.back(), coff.back(), nz_total});
        roff.push_back(roff.back() + d.m);
        coff.push_back(coff.back() + d.n);
        nz_total += d.nnz;
        nnz_of.push_back(d.nnz);
    }
    if (nz_total >= (int64_t)1 << 31) return fail(PDHG_ERR_INVALID_ARG, "batch nnz must stay below 2^31");
    const int M = roff.back(), N = coff.back();
    // the block-diagonal model assembled on the device, then ingested as pdhg_create_device does
    hipStream_t st = nullptr;
    std::vector<void *> temps;
    auto release = [&]() {
        for (void *q : temps) (void)hipFree(q);
        temps.clear();
        if (st) (void)hipStreamDestroy(st);
        st = nullptr;
    };
    DeviceModel dm{};
    unsigned bad = 0;
    hipError_t e = hipStreamCreate(&st);
    if (e == hipSuccess) e = batch_assemble_device(st, parts, M, N, nz_total, &dm, temps, &bad);
    if (e != hipSuccess) {
        release();
        return fail(e == hipErrorOutOfMemory ? PDHG_ERR_OOM : PDHG_ERR_HIP,
                    std::string("HIP error assembling the batch: ") + hipGetErrorString(e));
    }
    if (bad) {
        release();
        return fail(PDHG_ERR_INVALID_ARG, ingest_error(bad));
    }
    ModelSource src;
    src.dev = &dm;
    pdhg_solver *s = nullptr;
    const int rc = build_solver(M, N, (int)nz_total, p, src, false, &s);
    release(); // the solver holds its own copies
    if (rc != PDHG_OK) return rc;
    return batch_finish(s, count, roff, coff, nnz_of, p, out);
}

int pdhg_batch_solve(pdhg_batch *b, pdhg_result *results)
{
    if (!b || !results) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (b->pushed || b->solved) return fail(PDHG_ERR_STATE, "the batch has already been solved");
    const double t0 = now_s();
    try {
        pdhg_solver *s = b->s;
        const bool time_out = run_batch_phase(b, s->p.max_iter, 1, t0);
        if (b->t_host < s->p.check_every) HIPCHK(candidate_from_iterate(s));
        HIPCHK(unscale(s, (const double *)s->xp, (const double *)s->yp, s->xu, s->yu));
        std::vector<pdhg_kkt_report> k((size_t)b->count);
        HIPCHK(batch_report(b, s->xu, s->yu, s->zsol, k.data()));
        b->solve_seconds = now_s() - t0;
        b->solve_iters_max = b->t_host;
        for (int i = 0; i < b->count; i++) {
            const DevState &d = b->sts_host[i];
            pdhg_result &r = results[i];
            std::memset(&r, 0, sizeof(r));
            r.status = d.done ? d.status : (time_out ? PDHG_TIME_LIMIT : PDHG_ITER_LIMIT);
            r.iters = d.done ? d.t : b->t_host;
            r.restarts = d.restarts;
            r.rel_p = k[i].rel_p;
            r.rel_d = k[i].rel_d;
            r.rel_gap = k[i].rel_gap;
            r.pobj = k[i].pobj;
            r.dobj = k[i].dobj;
            r.seconds = b->solve_seconds;
            b->active_host[i] = (r.status == PDHG_OPTIMAL) ? 1 : 0;
        }
        b->solved = true;
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

// learned-part buffers of a batch (allocated on first use)
static void batch_learned_buffers(pdhg_batch *b)
{
    pdhg_solver *s = b->s;
    const size_t n = (size_t)(s->n > 0 ? s->n : 1);
    if (!s->feat_raw) dalloc(&s->feat_raw, 16 * n);
    if (!s->feat_b) dalloc(&s->feat_b, 16 * n);
    if (!s->logits) dalloc(&s->logits, n);
    if (!s->lfix) dalloc(&s->lfix, n);
    if (!s->lcount) dalloc(&s->lcount, 2 * (size_t)b->count);
    if (!b->fpart) dalloc(&b->fpart, 16 * (size_t)(b->n_rn > 0 ? b->n_rn : 1));
    if (!b->fscale) dalloc(&b->fscale, 16 * (size_t)b->count);
}

static int batch_push_common(pdhg_batch *b, const uint64_t *seeds, pdhg_push_result *results, pdhg_mlp *net,
                             const float *logits_host, double theta)
{
    const bool learned = net != nullptr || logits_host != nullptr;
    if (!b || !seeds || !results) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (!b->solved || b->pushed || b->dual_pushed)
        return fail(PDHG_ERR_STATE, "corner push needs a batch solve first (runs once, and not after a dual push)");
    const double t0 = now_s();
    try {
        pdhg_solver *s = b->s;
        hipStream_t st = s->stream;
        for (int i = 0; i < b->count; i++) std::memset(&results[i], 0, sizeof(pdhg_push_result));
        HIPCHK(hipMemcpyAsync(s->xs, s->xp, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(s->ys, s->yp, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, st));
        HIPCHK(unscale(s, (const double *)s->xs, (const double *)s->ys, s->xu, s->yu));
        std::vector<pdhg_kkt_report> before((size_t)b->count), after((size_t)b->count);
        HIPCHK(batch_report(b, s->xu, s->yu, s->zsol, before.data()));
        std::vector<int> solve_status((size_t)b->count);
        for (int i = 0; i < b->count; i++) solve_status[i] = b->sts_host[i].status;
        // per-LP gate (section 4.2): a gated LP stays at its solve's answer
        std::vector<int> act = b->active_host;
        std::vector<char> gated((size_t)b->count, 0);
        if (s->p.push_gate)
            for (int i = 0; i < b->count; i++)
                if (act[i] && (double)before[i].candidates < gate_threshold(s->p, b->roff[i + 1] - b->roff[i])) {
                    act[i] = 0;
                    gated[i] = 1;
                }
        HIPCHK(hipMemcpy(b->active, act.data(), sizeof(int) * (size_t)b->count, hipMemcpyHostToDevice));
        if (learned) { // predictor on every LP's solve state, before the models change
            batch_learned_buffers(b);
            HIPCHK(hipMemsetAsync(s->lcount, 0, 2 * sizeof(unsigned) * (size_t)b->count, st));
            if (net) {
                HIPCHK(hipMemcpyAsync(b->seeds, seeds, sizeof(uint64_t) * (size_t)b->count, hipMemcpyHostToDevice,
                                      st));
                HIPCHK(batch_compute_features(b));
                HIPCHK(mlp_forward(net, st, s->feat_b, s->n, s->logits));
            } else if (s->n > 0) {
                HIPCHK(hipMemcpyAsync(s->logits, logits_host, sizeof(float) * (size_t)s->n, hipMemcpyHostToDevice,
                                      st));
            }
        }
        HIPCHK(batch_push_setup(b, seeds, results, learned ? theta : -1.0));
        s->learned_active = learned;
        b->t_host = 0;
        b->next_check = s->p.push_min_iters;
        if (s->p.push_compact) HIPCHK(batch_push_compact_begin(b)); // the push on the free columns
        const bool time_out = run_batch_phase(b, s->p.push_max_iter, 2, t0);
        HIPCHK(batch_push_compact_end(b, true));
        HIPCHK(unscale(s, (const double *)s->xp, nullptr, s->xpush, nullptr));
        HIPCHK(batch_keep_unpushed(b));
        HIPCHK(batch_report(b, s->xpush, s->yu, nullptr, after.data()));
        b->push_seconds = now_s() - t0;
        b->push_iters_max = b->t_host;
        for (int i = 0; i < b->count; i++) {
            const DevState &d = b->sts_host[i];
            pdhg_push_result &r = results[i];
            r.before = before[i];
            r.after = after[i];
            r.seconds = b->push_seconds;
            if (!act[i]) { // no push: the solve did not reach the tolerance, or the gate is closed
                r.status = gated[i] ? PDHG_PUSH_SKIPPED : solve_status[i];
                r.iters = 0;
                r.rel_p_push = NAN;
                continue;
            }
            r.status = d.done ? d.status : (time_out ? PDHG_TIME_LIMIT : PDHG_ITER_LIMIT);
            r.iters = d.done ? d.t : b->t_host;
            r.restarts = d.restarts;
            r.rel_p_push = d.checks > 0 ? d.rel_p : NAN;
        }
        if (learned) {
            std::vector<unsigned> cnt(2 * (size_t)b->count);
            HIPCHK(hipMemcpy(cnt.data(), s->lcount, sizeof(unsigned) * cnt.size(), hipMemcpyDeviceToHost));
            for (int i = 0; i < b->count; i++) {
                results[i].n_learned_fix = cnt[2 * (size_t)i];
                results[i].n_learned_undo = cnt[2 * (size_t)i + 1];
            }
        }
        s->learned_active = false;
        b->pushed = true;
    } catch (const HipFailure &f) {
        (void)batch_push_compact_end(b, false); // the full model's structures back in the handle
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_batch_corner_push(pdhg_batch *b, const uint64_t *seeds, pdhg_push_result *results)
{
    return batch_push_common(b, seeds, results, nullptr, nullptr, -1.0);
}

int pdhg_batch_corner_push_learned(pdhg_batch *b, pdhg_mlp *net, double theta, const uint64_t *seeds,
                                   pdhg_push_result *results)
{
    if (!net) return fail(PDHG_ERR_INVALID_ARG, "NULL network");
    if (!(theta > 0.0 && theta < 1.0)) return fail(PDHG_ERR_INVALID_ARG, "theta must lie in (0, 1)");
    return batch_push_common(b, seeds, results, net, nullptr, theta);
}

int pdhg_batch_corner_push_logits(pdhg_batch *b, const float *logits, double theta, const uint64_t *seeds,
                                  pdhg_push_result *results)
{
    if (!b) return fail(PDHG_ERR_INVALID_ARG, "NULL handle");
    if (!logits && b->s->n > 0) return fail(PDHG_ERR_INVALID_ARG, "NULL logits");
    if (!(theta > 0.0 && theta < 1.0)) return fail(PDHG_ERR_INVALID_ARG, "theta must lie in (0, 1)");
    return batch_push_common(b, seeds, results, nullptr, logits, theta);
}

// The dual corner push of every LP that reached the tolerance, each with its
// own seed: the single-LP steps DP1-DP7 over the block-diagonal model, the
// iterations in lockstep cycles.  After a batch corner push each LP's face is
// that of its pushed xhat.
int pdhg_batch_dual_push(pdhg_batch *b, const uint64_t *seeds, pdhg_dual_push_result *results)
{
    if (!b || !seeds || !results) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (!b->solved || b->dual_pushed)
        return fail(PDHG_ERR_STATE, "dual push needs a batch solve first (and runs once)");
    const double t0 = now_s();
    try {
        pdhg_solver *s = b->s;
        hipStream_t st = s->stream;
        for (int i = 0; i < b->count; i++) std::memset(&results[i], 0, sizeof(pdhg_dual_push_result));
        if (!s->ypush) dalloc(&s->ypush, (size_t)(s->m > 0 ? s->m : 1));
        if (!s->zpush) dalloc(&s->zpush, (size_t)(s->n > 0 ? s->n : 1));
        if (!s->w0) dalloc(&s->w0, (size_t)(s->n > 0 ? s->n : 1));
        if (!b->pushed) { // DP1 (after the corner push the solve's answer is already in place)
            HIPCHK(hipMemcpyAsync(s->xs, s->xp, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(s->ys, s->yp, sizeof(double) * (size_t)s->m, hipMemcpyDeviceToDevice, st));
            HIPCHK(unscale(s, (const double *)s->xs, (const double *)s->ys, s->xu, s->yu));
        }
        const double *xk = b->pushed ? s->xpush : s->xu;
        std::vector<pdhg_kkt_report> before((size_t)b->count), after((size_t)b->count);
        HIPCHK(batch_report(b, xk, s->yu, s->zsol, before.data()));
        // the LPs that reached the tolerance take part (the solve's flags; an LP
        // that did not keeps the solve's state and status)
        const std::vector<int> act = b->active_host;
        std::vector<int> solve_status((size_t)b->count);
        for (int i = 0; i < b->count; i++) solve_status[i] = b->sts_host[i].status;
        HIPCHK(hipMemcpy(b->active, act.data(), sizeof(int) * (size_t)b->count, hipMemcpyHostToDevice));
        std::vector<int64_t> cols_free((size_t)b->count), rows_fixed((size_t)b->count);
        HIPCHK(batch_dual_push_setup(b, seeds, xk, cols_free.data(), rows_fixed.data()));
        b->t_host = 0;
        b->next_check = s->p.push_min_iters;
        const bool time_out = run_batch_phase(b, s->p.push_max_iter, 3, t0);
        HIPCHK(unscale(s, nullptr, (const double *)s->yp, nullptr, s->ypush));
        HIPCHK(batch_dual_push_finish(b));
        HIPCHK(batch_report(b, xk, s->ypush, s->zpush, after.data()));
        const double secs = now_s() - t0;
        for (int i = 0; i < b->count; i++) {
            const DevState &d = b->sts_host[i];
            pdhg_dual_push_result &r = results[i];
            r.before = before[i];
            r.after = after[i];
            r.seconds = secs;
            r.n_cols_free = cols_free[i];
            r.n_rows_fixed = rows_fixed[i];
            if (!act[i]) { // the solve did not reach the tolerance: no push
                r.status = solve_status[i];
                r.rel_d_push = NAN;
                continue;
            }
            r.status = d.done ? d.status : (time_out ? PDHG_TIME_LIMIT : PDHG_ITER_LIMIT);
            r.iters = d.done ? d.t : b->t_host;
            r.restarts = d.restarts;
            r.rel_d_push = d.checks > 0 ? d.rel_d : NAN;
        }
        b->dual_pushed = true;
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_batch_features(pdhg_batch *b, const uint64_t *seeds, float *out)
{
    if (!b || !seeds) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    if (!b->solved || b->pushed || b->dual_pushed)
        return fail(PDHG_ERR_STATE, "features describe a solved batch before its push");
    try {
        pdhg_solver *s = b->s;
        batch_learned_buffers(b);
        HIPCHK(hipMemcpyAsync(b->seeds, seeds, sizeof(uint64_t) * (size_t)b->count, hipMemcpyHostToDevice, s->stream));
        HIPCHK(batch_compute_features(b));
        if (out)
            HIPCHK(hipMemcpyAsync(out, s->feat_raw, sizeof(float) * 16 * (size_t)s->n, hipMemcpyDeviceToHost,
                                  s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_batch_get_solution(pdhg_batch *b, int32_t i, double *x, double *y, double *z)
{
    if (!b || i < 0 || i >= b->count) return fail(PDHG_ERR_INVALID_ARG, "bad handle or LP index");
    if (!b->solved) return fail(PDHG_ERR_STATE, "no batch solve yet");
    try {
        pdhg_solver *s = b->s;
        const size_t n0 = (size_t)b->coff[i], nn = (size_t)(b->coff[i + 1] - b->coff[i]);
        const size_t m0 = (size_t)b->roff[i], mm = (size_t)(b->roff[i + 1] - b->roff[i]);
        const double *cx = b->pushed ? s->xpush : s->xu;
        const double *cy = b->dual_pushed ? s->ypush : s->yu;
        const double *cz = b->dual_pushed ? s->zpush : s->zsol;
        if (x) HIPCHK(hipMemcpy(x, cx + n0, sizeof(double) * nn, hipMemcpyDeviceToHost));
        if (y) HIPCHK(hipMemcpy(y, cy + m0, sizeof(double) * mm, hipMemcpyDeviceToHost));
        if (z) HIPCHK(hipMemcpy(z, cz + n0, sizeof(double) * nn, hipMemcpyDeviceToHost));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_batch_get_solve_solution(pdhg_batch *b, int32_t i, double *x, double *y, double *z)
{
    if (!b || i < 0 || i >= b->count) return fail(PDHG_ERR_INVALID_ARG, "bad handle or LP index");
    if (!b->solved) return fail(PDHG_ERR_STATE, "no batch solve yet");
    try {
        pdhg_solver *s = b->s;
        const size_t n0 = (size_t)b->coff[i], nn = (size_t)(b->coff[i + 1] - b->coff[i]);
        const size_t m0 = (size_t)b->roff[i], mm = (size_t)(b->roff[i + 1] - b->roff[i]);
        if (x) HIPCHK(hipMemcpy(x, s->xu + n0, sizeof(double) * nn, hipMemcpyDeviceToHost));
        if (y) HIPCHK(hipMemcpy(y, s->yu + m0, sizeof(double) * mm, hipMemcpyDeviceToHost));
        if (z) HIPCHK(hipMemcpy(z, s->zsol + n0, sizeof(double) * nn, hipMemcpyDeviceToHost));
    } catch (const HipFailure &f) {
        return fail(PDHG_ERR_HIP, std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.err));
    }
    return PDHG_OK;
}

int pdhg_batch_get_report(pdhg_batch *b, pdhg_batch_report *r)
{
    if (!b || !r) return fail(PDHG_ERR_INVALID_ARG, "NULL argument");
    std::memset(r, 0, sizeof(*r));
    pdhg_solver *s = b->s;
    r->count = b->count;
    r->solve_seconds = b->solve_seconds;
    r->push_seconds = b->push_seconds;
    r->solve_lockstep_iters = b->solve_iters_max;
    r->push_lockstep_iters = b->push_iters_max;
    r->lanes_at = b->kern_at;
    r->lanes_a = b->kern_a;
    r->samples = s->t_samples;
    if (s->t_samples > 0) {
        r->primal_ms = s->t_primal_ms / (double)s->t_samples;
        r->dual_ms = s->t_dual_ms / (double)s->t_samples;
    }
    const int64_t m = s->m, n = s->n, nz = s->nnz;
    // mean algorithmic bytes of the timed launches (LPs still iterating)
    if (s->t_samples > 0) {
        r->bytes_primal = (int64_t)(b->timed_bytes_primal / (double)s->t_samples);
        r->bytes_dual = (int64_t)(b->timed_bytes_dual / (double)s->t_samples);
    }
    r->total_m = m;
    r->total_n = n;
    r->total_nnz = nz;
    return PDHG_OK;
}

void pdhg_batch_destroy(pdhg_batch *b)
{
    if (!b) return;
    if (b->s && b->s->stream) (void)hipStreamSynchronize(b->s->stream);
    free_batch(b);
    delete b;
}

} // extern "C"

