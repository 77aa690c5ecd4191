// Internal declarations of the gfx950 PDHG library (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pdhg.h"

// Launch a kernel on STREAM.  With a start/stop event pair the events are
// bound to this one dispatch (hipExtLaunchKernel), so their elapsed time is
// the kernel's own execution, free of the dispatch latency a separate
// hipEventRecord would add.
#define PDHG_LAUNCH(E0, E1, KERNEL, GRID, BLOCK, STREAM, ...)                                                    \
    do {                                                                                                         \
        if (E0) hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, E0, E1, 0, __VA_ARGS__);                    \
        else hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                                    \
    } while (0)

namespace pdhg {

constexpr int kBlock = 256;         // threads per workgroup (4 wave64)
constexpr int kRowBlock = -2256; // kernel code: one row per workgroup of kBlock threads
constexpr int kSell = -3032;     // kernel code (dual half): sliced ELLPACK, 32-row slices
constexpr int kRowSegs = -4000;  // kernel code (dual half): row segments, each with its own lane-group width
constexpr int kMaxRedBlocks = 1024; // cap on per-block partials of a reduction
constexpr int kMaxSegs = 4;         // row segments of the kRowSegs dual half

// Row segments of A for the dual half (kernel code kRowSegs): rows
// [row0[k], row0[k+1]) run in lane groups of lanes[k], on workgroups
// [blk0[k], blk0[k+1]) of one launch.  Every segment's workgroup count is a
// multiple of 8, so a segment spreads over the 8 XCDs as its own launch would.
struct RowSegs {
    int count = 0;
    int row0[kMaxSegs + 1] = {};
    int blk0[kMaxSegs + 1] = {};
    int lanes[kMaxSegs] = {};
};

// Quantities reduced at a check (block partials, then one fixed-order pass).
enum CheckQ {
    Q_PH2 = 0, // sum rP_hat^2           (scaled, current senses)
    Q_P2,      // sum rP^2               (unscaled)
    Q_PINF,    // max |rP|               (unscaled)
    Q_BTY,     // sum bhat_i yhat_i
    Q_DY2,     // sum (yp - ya)^2        (scaled)
    Q_DH2,     // sum rD_hat^2
    Q_D2,      // sum rD^2               (unscaled)
    Q_DINF,    // max |rD|
    Q_CTX,     // sum chat_j xhat_j
    Q_BND,     // sum lhat zhat+ - uhat zhat-
    Q_DX2,     // sum (xp - xa)^2
    Q_NAN,     // count of non-finite candidate entries
    Q_COUNT
};

// Quantities of a KKT report (original model, float64).
enum ReportQ {
    R_P2 = 0, R_PINF, R_BTY, R_D2, R_DINF, R_CTX, R_BND, R_POFF, R_DZERO, R_CAND, R_COUNT
};

// Scalar solver state kept in device memory so that every kernel reads its
// step sizes, Halpern counter and flags without host round trips.
struct DevState {
    double eta, omega, tau, sigma;
    double gamma;                  // reflection
    double eps_rel;
    double r_suff, r_nec, r_art, pw_smooth;
    double nb1, nc1;               // 1 + ||b||_2, 1 + ||c||_2 (original model)
    double sigma_est;              // power-iteration estimate of ||Ahat||_2
    int64_t k0;                    // Halpern counter at the last state update
    int64_t t;                     // iterations of this phase at the last update
    int64_t restarts;
    double anc_p2, anc_d2, anc_g2; // weighted-KKT parts at the anchor
    double kkt_prev;
    // values of the last check (unscaled relative tests, objectives)
    double rel_p, rel_d, rel_gap, pobj, dobj, kkt_c;
    int32_t halpern;
    int32_t restart_flag;
    int32_t done;
    int32_t status;
    int32_t checks;
    int32_t pad_;
};

// Host-side report values read back from the device.
struct ReportOut {
    double v[R_COUNT];
};

} // namespace pdhg

// The opaque handle of the ABI.
struct pdhg_solver {
    int m = 0, n = 0;
    int nnz = 0;
    pdhg_params p{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool fp32 = false;

    // original model, float64, row-compressed A and its explicit transpose
    int *rp = nullptr, *ci = nullptr;
    double *av = nullptr;
    int *tp = nullptr, *ti = nullptr, *tperm = nullptr;
    double *atv = nullptr;
    double *b = nullptr, *c = nullptr, *l = nullptr, *u = nullptr;
    int8_t *sense0 = nullptr;

    // scaling
    double *dr = nullptr, *dc = nullptr;

    // iteration arrays: the matrix, lhat, uhat, x and xbar in the working
    // precision (float or double); in the mixed mode x and xbar hold the
    // differences x - x_a and xbar - x_a from the float64 anchor.  The anchors,
    // the candidate (xp, yp), the solve's solution (xs, ys) and every m-vector
    // are float64 in both precisions.
    void *ahat = nullptr, *ahat_t = nullptr;
    void *x = nullptr, *y = nullptr, *xa = nullptr, *ya = nullptr, *xbar = nullptr;
    void *xp = nullptr, *yp = nullptr;
    double *ch = nullptr;            // scaled objective
    void *bh = nullptr, *lh = nullptr, *uh = nullptr;
    // Mixed precision: the rounding error of the float matrix, E = Ahat -
    // fl32(Ahat), stored as float in A order and transpose order, so that
    // fl32(Ahat) v + E v is the float64 product (ex, ety: the error parts of
    // a product).  The iteration kernels read chc and bhc: in float64 mode
    // the same arrays as ch and bh; in the mixed mode ch - E' y_a and
    // bh - Ahat x_a at the anchor (x_a, y_a) in float64, which the float
    // products of y and of the differences xbar - x_a complete.
    void *aerr = nullptr, *aerr_t = nullptr;
    double *ex = nullptr, *ety = nullptr;
    double *chc = nullptr, *bhc = nullptr;
    bool defect_stale = true; // chc, bhc do not yet follow the current anchor and model
    void *xs = nullptr, *ys = nullptr; // scaled solution of the solve (kept for the push)
    int8_t *sense = nullptr;

    // float64 work: products, unscaled copies, reduced costs, partial sums
    double *ax = nullptr, *aty = nullptr;
    double *xu = nullptr, *yu = nullptr, *zsol = nullptr, *xpush = nullptr;
    double *ypush = nullptr, *zpush = nullptr; // dual push result (allocated by the dual push)
    double *w0 = nullptr;                      // dual push: the anchor point of its right-hand side
    double *partials = nullptr;
    double *redout = nullptr; // small reduction results
    int red_blocks_m = 1, red_blocks_n = 1;
    pdhg::DevState *st = nullptr;
    pdhg::DevState *st_host = nullptr; // pinned mirror
    double *rep_host = nullptr;        // pinned report values
    int64_t *cnt_host = nullptr;       // pinned integer counts

    int lanes_at = 1, lanes_a = 1; // lane-group width of setup / check products
    int udeg_at = 0;               // every column holds this many entries (1..3), else 0
    int kern_at = 1, kern_a = 1;   // iteration kernels: > 0 lane-group width, < 0 LDS tile of -k rows
    pdhg::RowSegs segs;            // the dual half's row segments (kern_a == kRowSegs)
    int64_t t_host = 0;      // iterations of the current phase (mirror of st->t)
    int64_t power_steps = 0; // power-iteration steps taken at create
    int64_t next_check = 0;  // phase iteration count of the next check
    bool in_push = false;
    bool primal_pushed = false; // pdhg_corner_push has run (its x is in xpush)
    bool dual_pushed = false;   // pdhg_dual_push has run (its y and z in ypush, zpush)
    // sliced ELLPACK copy of Ahat for the dual half (kernel code kSell)
    int *sell_idx = nullptr, *sell_len = nullptr, *sell_wi_start = nullptr;
    void *sell_val = nullptr;
    int64_t *sell_soff = nullptr;
    int2 *sell_wi = nullptr;
    double *sell_part = nullptr;
    int n_sell_wi = 0;
    bool model_original = true; // the solve's model is in ch/lh/uh (false once a push rewrote it)
    bool has_candidate = false;   // a check has produced (xp, yp) in this phase
    bool solved = false;          // the solve has a candidate (push allowed)
    bool has_push_candidate = false;

    // captured cycle graphs (K iterations + check) keyed by length
    hipGraphExec_t graph_exec = nullptr;
    int graph_len = 0;
    int graph_mode = -1;

    // learned push: restart history (4 slots of x and z, scaled), features,
    // per-column learned-fix flags (1 lower, 2 upper) and counters
    float *hx = nullptr, *hz = nullptr;
    float *feat_raw = nullptr;   // n x 16
    short *feat_b = nullptr;     // n x 16 bfloat16
    float *logits = nullptr;     // n
    int8_t *lfix = nullptr;      // n
    unsigned *lcount = nullptr;  // [fixed, undone]
    bool learned_active = false;

    // push model without its fixed columns while the push iterates
    // (pdhg_compact.hip): the compact arrays, and the full model's fields they
    // replace in this struct until the push ends
    struct PushCompact {
        bool active = false;
        int nf = 0, nnz = 0;
        int *flag = nullptr, *newid = nullptr, *keep = nullptr; // free flag and index of every full column; full index of each compact one
        int *tp = nullptr, *ti = nullptr, *rp = nullptr, *ci = nullptr;
        void *ahat = nullptr, *ahat_t = nullptr, *lh = nullptr, *uh = nullptr;
        void *x = nullptr, *xa = nullptr, *xbar = nullptr, *xp = nullptr;
        double *ch = nullptr, *dc = nullptr, *bt = nullptr;
        void *aerr = nullptr, *aerr_t = nullptr; // mixed precision: the free columns' matrix errors
        int8_t *lfix = nullptr;             // learned push: its fixes, which an undo may free again
        double *l = nullptr, *u = nullptr;  // learned push: the original bounds an undo restores
        int n0 = 0, nnz0 = 0, red_blocks_n0 = 1, udeg_at0 = 0;
        int8_t *lfix0 = nullptr;
        double *l0 = nullptr, *u0 = nullptr;
        int *tp0 = nullptr, *ti0 = nullptr, *rp0 = nullptr, *ci0 = nullptr;
        void *ahat0 = nullptr, *ahat_t0 = nullptr, *lh0 = nullptr, *uh0 = nullptr, *bh0 = nullptr;
        void *x0 = nullptr, *xa0 = nullptr, *xbar0 = nullptr, *xp0 = nullptr;
        double *ch0 = nullptr, *dc0 = nullptr;
        void *aerr0 = nullptr, *aerr_t0 = nullptr;
        double *chc0 = nullptr, *bhc0 = nullptr;
        pdhg::RowSegs segs0;
    } pc;

    // live kernel timing: events around one primal and one dual launch per cycle
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr}; // primal start/stop, dual start/stop
    double t_primal_ms = 0.0, t_dual_ms = 0.0;
    int64_t t_samples = 0;
    double t_bytes_primal = 0.0, t_bytes_dual = 0.0; // algorithmic bytes of the timed launches
};

// A batch of independent LPs stored as one block-diagonal model: every
// row-space and column-space array of `s` is the concatenation of the LPs'
// arrays, column indices are global, and each LP keeps its own DevState.
struct pdhg_batch {
    pdhg_solver *s = nullptr;
    int count = 0;
    std::vector<int> roff, coff;           // row / column offsets of each LP (count + 1)
    std::vector<int64_t> nnz_of;           // entries of each LP
    int *d_coff = nullptr;                 // device copy of coff
    int4 *ptiles = nullptr, *dtiles = nullptr; // iteration tiles {lp, first row, rows, 0}
    int n_ptiles = 0, n_dtiles = 0;        // tiles in use (only LPs still iterating after a compaction)
    std::vector<int4> ptiles_all, dtiles_all; // every LP's iteration tiles (host copy)
    int kern_at = -64, kern_a = -64;       // tiled-kernel choice, pdhg_params.lanes_* encoding
    int4 *rn = nullptr, *rm = nullptr;     // 256-row reduction tiles of the column / row space
    int n_rn = 0, n_rm = 0;
    int *rn_start = nullptr, *rm_start = nullptr; // first reduction tile of each LP (count + 1)
    pdhg::DevState *sts = nullptr, *sts_host = nullptr;
    double *part = nullptr;                // per-tile partial sums
    double *lp_scalar = nullptr;           // per-LP power iteration {lambda, done, steps, ||v0||} x count
    double *rep = nullptr, *rep_host = nullptr; // per-LP report values
    int *active = nullptr;                 // per-LP flag: takes part in the current phase
    std::vector<int> active_host;
    uint64_t *seeds = nullptr;
    double *fpart = nullptr, *fscale = nullptr; // feature sums per column tile (16 x n_rn), scales per LP (16 x count)
    hipGraphExec_t graph = nullptr;
    int graph_len = 0, graph_mode = -1;
    int64_t t_host = 0, next_check = 0;
    bool solved = false, pushed = false;
    bool dual_pushed = false; // pdhg_batch_dual_push has run (y, z in the solver's ypush, zpush)
    double solve_seconds = 0.0, push_seconds = 0.0;
    double timed_bytes_primal = 0.0, timed_bytes_dual = 0.0; // algorithmic bytes of the timed launches
    int64_t solve_iters_max = 0, push_iters_max = 0;
    // while the push runs on the free columns: the full model's column-side
    // structures, replaced by those of the compact numbering
    struct {
        bool active = false;
        std::vector<int> coff;
        std::vector<int64_t> nnz_of;
        std::vector<int4> ptiles_all;
        int4 *rn = nullptr;
        int n_rn = 0;
        int *rn_start = nullptr, *d_coff = nullptr;
    } full;
};

namespace pdhg {

// error helpers (capi.cpp)
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// a caller's model in device memory (pdhg_create_device)
struct DeviceModel {
    int m, n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val, *b, *c, *l, *u; // l, u may be NULL (0 and +infinity)
    const char *sense;                 // may be NULL (all '=')
};
// ingest bits: what the device found wrong with a DeviceModel
enum IngestBad : unsigned {
    BAD_ROWPTR = 1u, BAD_COL = 2u, BAD_ORDER = 4u, BAD_VAL = 8u, BAD_B = 16u, BAD_C = 32u, BAD_BOUND = 64u,
    BAD_SENSE = 128u
};

// setup kernels (pdhg_setup.hip)
// check a device model and copy it into the solver's arrays (row pointers
// to int32, infinite bounds for |v| >= 1e20, defaults for NULL l, u, sense);
// *bad receives the IngestBad bits (0: accepted)
hipError_t ingest_device(pdhg_solver *s, const DeviceModel &dm, unsigned *bad);
const char *ingest_error(unsigned bad);
// one LP of a batch created from device arrays: its caller-owned arrays and
// its place in the block-diagonal model
struct BatchPart {
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val, *b, *c, *l, *u; // l, u may be NULL (0 and +infinity)
    const char *sense;                 // may be NULL (all '=')
    int m, n;
    int64_t nnz;
    int roff, coff; // first row and column in the block
    int64_t nzoff;  // first entry in the block
};
// Assemble the block-diagonal model of `parts` in new device arrays (kept in
// temps, freed by the caller after the solver has copied them): row pointers
// and column indices shifted by each LP's offsets, every LP's row pointers
// checked at both ends and its column indices against its own n (bad gets
// BAD_ROWPTR / BAD_COL); the rest is checked by ingest_device.
hipError_t batch_assemble_device(hipStream_t st, const std::vector<BatchPart> &parts, int M, int N, int64_t NZ,
                                 DeviceModel *dm, std::vector<void *> &temps, unsigned *bad);
hipError_t build_transpose(pdhg_solver *s);
hipError_t scale_problem(pdhg_solver *s);
hipError_t power_iteration(pdhg_solver *s);
// out = Ahat vec (transpose = false) or Ahat' vec, float64, with the structure of
// the iteration kernel of that half (the kernels must have been chosen)
hipError_t solver_product(pdhg_solver *s, bool transpose, const double *vec, double *out);
// the same product with the float64 matrix: in the mixed mode the float
// matrix's product plus that of its rounding error E
hipError_t exact_product(pdhg_solver *s, bool transpose, const double *vec, double *out);
// mixed precision: chc = ch - E' y_a, bhc = bh - E x_a at the current anchor
// (a no-op in float64 mode, where chc and bhc are ch and bh)
hipError_t defect_refresh(pdhg_solver *s);
// udeg_at: the common entry count of every column (1..3) of the current model, or 0
hipError_t detect_uniform_columns(pdhg_solver *s);
// the primal half runs the uniform-column kernel: columns of 1-3 entries each,
// 256-row tiles chosen by the library (an explicit lanes_at keeps the tiles)
inline bool uses_uniform_kernel(const pdhg_solver *s)
{
    return s->kern_at == -256 && s->p.lanes_at == 0 && s->udeg_at >= 1 && s->udeg_at <= 3;
}
// float64 mode: chc and bhc follow ch and bh (after any swap of those arrays)
inline void defect_alias(pdhg_solver *s)
{
    if (!s->aerr) {
        s->chc = s->ch;
        s->bhc = (double *)s->bh;
    }
}
// sliced ELLPACK dual half: layout (after scaling), iteration half, product Ahat vec
hipError_t sell_build(pdhg_solver *s, const std::vector<int> &rp_host);
void sell_dual(pdhg_solver *s, int i, int store, hipEvent_t e0, hipEvent_t e1);
void sell_product(pdhg_solver *s, const double *vec, double *out);
void sell_product(pdhg_solver *s, const float *vec, double *out);

// iteration, checks, push and reports (pdhg_iter.hip)
hipError_t init_iteration(pdhg_solver *s);
// the dual half's row segments of the current model (kern_a == kRowSegs)
hipError_t plan_row_segments(pdhg_solver *s);
// restart the solve phase from the start point staged (unscaled) in xu, yu
hipError_t set_start(pdhg_solver *s);
hipError_t launch_iterations(pdhg_solver *s, int count, bool check_at_end, int mode, bool timed_launch);
hipError_t launch_check(pdhg_solver *s, int mode, int len);
hipError_t launch_advance(pdhg_solver *s, int len);
hipError_t candidate_from_iterate(pdhg_solver *s);
hipError_t launch_start_vectors(pdhg_solver *s, bool fresh_start);
hipError_t unscale(pdhg_solver *s, const double *xh, const double *yh, double *xo, double *yo);
hipError_t unscale_iterate(pdhg_solver *s, double *xo, double *yo); // the current iterate (x, y), unscaled
hipError_t report(pdhg_solver *s, const double *x, const double *y, double *z, pdhg_kkt_report *k);
hipError_t push_setup(pdhg_solver *s, uint64_t seed, pdhg_push_result *r, double theta);
hipError_t dual_push_setup(pdhg_solver *s, uint64_t seed, const double *xk, double *w0, double *yn, double *atyn,
                           int64_t *n_cols_free, int64_t *n_rows_fixed);
hipError_t dual_push_finish(pdhg_solver *s);
// push on the free columns only: build the compact model and put it in place,
// or (end) put x and x+ back into the full vectors and restore the full model
hipError_t push_compact_begin(pdhg_solver *s);
hipError_t push_compact_end(pdhg_solver *s, bool scatter);
// algorithmic bytes of one primal and one dual launch on the current model
void model_bytes(const pdhg_solver *s, int64_t *bytes_primal, int64_t *bytes_dual);
// the batch push on its free columns (per-LP offsets and tiles of the compact
// numbering), and back
hipError_t batch_push_compact_begin(pdhg_batch *b);
hipError_t batch_push_compact_end(pdhg_batch *b, bool scatter);
hipError_t capture_cycle(pdhg_solver *s, int len, int mode);
hipError_t copy_probe(int64_t bytes, int reps, double *gbps);

// batch engine (pdhg_batch.hip)
hipError_t batch_setup(pdhg_batch *b);
hipError_t batch_autotune(pdhg_batch *b);
hipError_t batch_compact_tiles(pdhg_batch *b, bool all);
hipError_t batch_set_kernels(pdhg_batch *b, int kern_at, int kern_a);
hipError_t batch_phase_begin(pdhg_batch *b, bool fresh);
hipError_t batch_defect_refresh(pdhg_batch *b);
hipError_t batch_iterations(pdhg_batch *b, int count, bool check_at_end, int mode, bool timed);
hipError_t batch_capture_cycle(pdhg_batch *b, int len, int mode);
hipError_t batch_report(pdhg_batch *b, const double *x, const double *y, double *z, pdhg_kkt_report *out);
hipError_t batch_push_setup(pdhg_batch *b, const uint64_t *seeds, pdhg_push_result *out, double theta);
hipError_t batch_dual_push_setup(pdhg_batch *b, const uint64_t *seeds, const double *xk, int64_t *cols_free,
                                 int64_t *rows_fixed);
hipError_t batch_dual_push_finish(pdhg_batch *b);
hipError_t batch_keep_unpushed(pdhg_batch *b);

// learned push (pdhg_learned.hip)
hipError_t launch_record_history(pdhg_solver *s);
hipError_t launch_learned_undo(pdhg_solver *s);
hipError_t compute_features(pdhg_solver *s, uint64_t seed);
hipError_t launch_learned_fix(pdhg_solver *s, double theta);
// the learned warm start for every LP of a batch (per-LP history, features,
// scales and counters over the column reduction tiles)
hipError_t batch_record_history(pdhg_batch *b);
hipError_t batch_compute_features(pdhg_batch *b);
hipError_t batch_learned_fix(pdhg_batch *b, double theta);
hipError_t batch_learned_undo(pdhg_batch *b);
int choose_kernel(double mean_row, bool dual_half);
hipError_t autotune(pdhg_solver *s);

// launch-shape helpers
// Lane count for a given mean row length: the power of two at or above the
// mean, between 1 and 64.
inline int lanes_for_mean(double mean)
{
    int l = 1;
    while (l < 64 && l < mean) l <<= 1;
    return l;
}

inline int grid_for(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

} // namespace pdhg
