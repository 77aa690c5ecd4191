/*
 * pdhg.h -- C ABI of the MI355X (gfx950) PDHG + corner-push library.
 *
 * Problem (paper, section 2, with bounds and inequalities handled implicitly):
 *     min c'x   s.t.  a_i'x (=, <=, >=) b_i  (i < m),   l <= x <= u   (x in R^n)
 * Dual: y_i free on '=' rows, y_i <= 0 on '<=' rows, y_i >= 0 on '>=' rows;
 * reduced costs z = c - A'y, of which a finite lower bound absorbs the
 * positive part and a finite upper bound the negative part.  Residuals
 * r_P = b - Ax (only violations count on inequality rows), r_D = c - A'y - z,
 * and the relative l2 termination tests of section 2:
 *     ||r_P|| <= eps (1 + ||b||),  ||r_D|| <= eps (1 + ||c||),
 *     |c'x - b'y| <= eps (1 + |c'x| + |b'y|)   (b'y including bound terms).
 *
 * Method: restarted PDHG with a reflected Halpern average (the paper uses a
 * PDHG "closely following cuPDLP+", section 4.1, and describes nothing
 * more), then the corner push of section 3, Algorithm 1: bounds fixed at the
 * current x where |z_j| > eps_abs, inequality rows with a non-trivial slack
 * reduced cost turned into equalities, a Uniform[0,1)^n objective, PDHG
 * restarted from (x, 0) and stopped as soon as the primal residual of the
 * modified model is back at the original tolerance after at least
 * push_min_iters iterations (section 3.1).
 *
 * Conventions for every entry point:
 *   - Host arrays are read-only and stay owned by the caller; the library
 *     copies what it needs.  Output arrays are caller-allocated.
 *   - Dense vectors are contiguous float64.  The matrix is row-compressed:
 *     row_ptr[m+1] (int64, row_ptr[0] = 0, row_ptr[m] = nnz), col_idx[nnz]
 *     (int32, 0 <= col < n, any order inside a row, duplicates are summed),
 *     val[nnz] (float64, finite).  nnz must stay below 2^31.
 *   - Infinite bounds are +-INFINITY; |bound| >= 1e20 is treated as infinite.
 *   - sense[m] holds '=', '<' (a_i'x <= b_i) or '>' (a_i'x >= b_i); NULL
 *     means all '='.  l == NULL means 0, u == NULL means +INFINITY.
 *   - Every function returns PDHG_OK (0) or a negative pdhg_error; no C++
 *     exception crosses the ABI.  pdhg_last_error() returns a thread-local
 *     description of the last failure.
 *   - All device work runs on params.stream (a hipStream_t passed as void*;
 *     NULL makes the library create its own stream at default priority).
 *     Calls on one handle must not overlap; distinct handles are independent.
 */
#ifndef PDHG_H
#define PDHG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdhg_solver pdhg_solver;
typedef struct pdhg_mlp pdhg_mlp;

/* solve / push outcome */
enum pdhg_status {
    PDHG_OPTIMAL = 0,    /* the three relative tests hold at a check           */
    PDHG_ITER_LIMIT = 1, /* max_iter (push: push_max_iter) reached              */
    PDHG_NUMERICAL = 2,  /* a non-finite value appeared in the candidate        */
    PDHG_PUSH_DONE = 3,  /* push: primal residual back at eps_rel (section 3.1) */
    PDHG_TIME_LIMIT = 4, /* time_limit seconds elapsed (checked between cycles) */
    PDHG_PUSH_SKIPPED = 5 /* push gate closed: too few candidates (section 4.2)  */
};

/* return codes */
enum pdhg_error {
    PDHG_OK = 0,
    PDHG_ERR_INVALID_ARG = -1, /* bad pointer, dimension, NaN/Inf data, l > u, bad sense */
    PDHG_ERR_STATE = -2,       /* call out of order (e.g. push before solve)         */
    PDHG_ERR_OOM = -3,         /* device or host allocation failed                    */
    PDHG_ERR_HIP = -4          /* a HIP runtime call failed                           */
};

enum pdhg_precision {
    PDHG_FP64 = 0,      /* matrix, vectors and updates in float64                         */
    PDHG_FP32_MIXED = 1 /* matrix, bounds, x and xbar in float32, x and xbar stored as
                           differences from the float64 restart anchor; anchors, objective,
                           dual vectors, arithmetic, residual norms, restart test,
                           termination and the push fixing test in float64                */
};

/* Parameters.  Every constant the paper leaves open lives here. */
typedef struct pdhg_params {
    double eps_rel;        /* relative l2 tolerance (section 2); default 1e-6          */
    double eps_abs;        /* fixing threshold of Algorithm 1; default 1e-6            */
    int64_t max_iter;      /* iteration cap of a solve; default 1e6                     */
    int32_t check_every;   /* iterations between checks K; default 64                   */
    int32_t ruiz_iters;    /* Ruiz equilibration passes; default 10                     */
    double restart_suff;   /* restart if KKT_c <= suff * KKT_anchor; default 0.2        */
    double restart_nec;    /* ... or KKT_c <= nec * KKT_anchor and no progress; 0.8     */
    double restart_art;    /* ... or k >= art * t (artificial); default 0.36            */
    double pw_smooth;      /* primal-weight log-smoothing; default 0.5                  */
    double pc_alpha;       /* Pock-Chambolle exponent; default 1; < 0 disables the pass */
    int32_t power_iters;   /* cap on power-iteration steps for ||Ahat||_2; default 4000 */
    int32_t halpern;       /* 1: reflected Halpern average (default), 0: plain PDHG     */
    double eta_safety;     /* step = eta_safety / ||Ahat||_2 estimate; default 0.99     */
    double reflect_gamma;  /* reflection gamma in [0,1]; default 1                      */
    double power_tol;      /* the power iteration on Ahat'Ahat stops at the first step
                              whose eigen-residual ||Mv - rho v|| <= power_tol * rho
                              (rho the Rayleigh quotient of the unit v); default 1e-3  */
    int32_t push_min_iters;/* push iterations before the first push check; default 100  */
    int32_t precision;     /* enum pdhg_precision; default PDHG_FP64                    */
    double push_obj_scale; /* push objective = scale * Uniform[0,1); default 1          */
    int64_t push_max_iter; /* iteration cap of a push; default 1e6                      */
    double time_limit;     /* seconds per solve / push call; <= 0: none (default)       */
    void *stream;          /* hipStream_t; NULL: library-owned stream                   */
    int32_t verbosity;     /* 0 silent (default); > 0: kernel plans on stderr          */
    int32_t lanes_at;      /* primal-half kernel: 1..64 (power of 2) lanes per row;
                              -32/-64/-128/-256: LDS tile of that many rows, 256
                              threads; -1032/-1064: tile of 32/64 rows, 64 threads;
                              -2256: one row per workgroup of 256 threads (long rows);
                              -3032 (lanes_a only): sliced ELLPACK, 32-row slices with
                              interleaved entries (long rows whose columns advance
                              together, e.g. the sinks of a transportation model);
                              -4000 (lanes_a only): row segments, runs of rows whose
                              columns are contiguous or spread out, each with its own
                              lane-group width (the default for rows of more than 48
                              entries; a batch takes tiled kernels only);
                              0 = chosen from the mean row length                      */
    int32_t lanes_a;       /* dual-half kernel, same encoding                           */
    int32_t use_graph;     /* 1: replay check cycles from a captured hipGraph (default) */
    int32_t timing;        /* 1: time one primal and one dual launch per cycle with HIP
                              events on the solver's stream (read by pdhg_get_timing)  */
    int32_t autotune;      /* 1: at create, time every kernel choice of each half on
                              scratch vectors and keep the fastest (0 = default: the
                              mean-row-length rule, reproducible run to run)          */
    int32_t record_history;/* 1: keep x and z of the last 4 restarts of the solve (the
                              learned push's trend features); default 0               */
    int32_t push_compact;  /* 1 (default): the push iterates on its free columns only
                              (per LP in a batch).  A column Algorithm 1 fixes (lower bound =
                              upper bound) keeps its value, so it enters only as the
                              constant Ahat_j x_j of the dual product, folded into the
                              right-hand side; residuals, gap, restarts and the stop
                              test are those of the full push model up to rounding.
                              The learned push keeps its learned fixes (an undo may
                              free them again) and drops only the plain rule's.  Not
                              used with the sliced ELLPACK dual.
                              0: iterate on the full push model                       */
    int32_t push_gate;     /* 1: push only when the solve's answer has at least
                              max(push_gate_rows * m, push_gate_min) candidates (off
                              bound, |z| < 1e-6): the selection rule of section 4.2,
                              which asks for a substantial number of primal push steps
                              and enough freedom to reduce them.  Otherwise the push
                              returns PDHG_PUSH_SKIPPED with the solve's point.  0
                              (default): always push                                   */
    double push_gate_rows; /* 2.0 */
    int64_t push_gate_min; /* 100000 */
} pdhg_params;

/* outcome of pdhg_solve / pdhg_iterate, evaluated on the original model */
typedef struct pdhg_result {
    int32_t status;       /* enum pdhg_status                                          */
    int32_t pad_;
    int64_t iters;        /* iterations done in this phase (the passing check's count) */
    int64_t restarts;
    double rel_p, rel_d, rel_gap;
    double pobj, dobj;
    double seconds;       /* wall time of the call                                     */
} pdhg_result;

/* KKT and corner statistics of a primal/dual pair on the original model */
typedef struct pdhg_kkt_report {
    double rp2, rd2;      /* ||r_P||_2, ||r_D||_2 (unscaled)                           */
    double rpinf, rdinf;  /* ||r_P||_inf, ||r_D||_inf (absolute test of section 2.1)   */
    double pobj, dobj, gap;
    double rel_p, rel_d, rel_gap;
    int64_t p_off;        /* columns and implicit slacks off their bounds by > 1e-6   */
    int64_t d_zero;       /* reduced costs (columns, slacks) with |z| <= 1e-6          */
    int64_t candidates;   /* off bound and |z| < 1e-6 (section 4.2 selection count)    */
    int64_t est_primal;   /* max(p_off - m, 0): primal push estimate (section 2.1)     */
    int64_t est_dual;     /* max(m - d_zero, 0): dual push estimate                    */
} pdhg_kkt_report;

typedef struct pdhg_push_result {
    int32_t status;       /* PDHG_PUSH_DONE, ITER_LIMIT, TIME_LIMIT, NUMERICAL or
                             PUSH_SKIPPED (gate closed: after = before, 0 iterations) */
    int32_t pad_;
    int64_t iters;        /* push iterations                                          */
    int64_t restarts;
    int64_t n_fix_lower;  /* columns with lb <- x (z_j < -eps_abs)                    */
    int64_t n_fix_upper;  /* columns with ub <- x (z_j >  eps_abs)                    */
    int64_t n_rows_to_eq; /* inequality rows turned into equalities                   */
    double rel_p_push;    /* relative primal residual of the push model at the stop   */
    double seconds;
    pdhg_kkt_report before; /* (x, y, z) of the solve, original model                 */
    pdhg_kkt_report after;  /* (xhat, y, z): pushed x with the solve's y and z         */
    int64_t n_learned_fix;  /* learned push: columns fixed from the predictor          */
    int64_t n_learned_undo; /* learned push: fixes undone at push checks               */
} pdhg_push_result;

/* Outcome of the dual corner push (pdhg_dual_push). */
typedef struct pdhg_dual_push_result {
    int32_t status;       /* PDHG_PUSH_DONE, ITER_LIMIT, TIME_LIMIT or NUMERICAL       */
    int32_t pad_;
    int64_t iters;        /* push iterations                                          */
    int64_t restarts;
    int64_t n_cols_free;  /* columns off both bounds by more than eps_abs (z_j = 0)   */
    int64_t n_rows_fixed; /* inequality rows with slack beyond eps_abs: y_i held at
                             the solve's value (dropped from the push model)          */
    double rel_d_push;    /* relative dual residual of the push model at the stop     */
    double seconds;
    pdhg_kkt_report before; /* (x, y, z) of the solve, original model                 */
    pdhg_kkt_report after;  /* (x, yhat, zhat): the solve's x with the pushed y       */
} pdhg_dual_push_result;

/* Live kernel timing (params.timing = 1): average durations of the two
 * iteration kernels over the sampled launches of every solve and push call
 * since pdhg_create, and their algorithmic bytes per launch (matrix values,
 * indices and row pointers, one read of every vector the kernel reads, one
 * write of every vector it writes; gathers counted once). */
typedef struct pdhg_timing {
    double primal_ms;      /* mean duration of one primal-half launch (A'y + update) */
    double dual_ms;        /* mean duration of one dual-half launch (A xbar + update) */
    int64_t samples;       /* sampled launches of each kernel                          */
    int64_t bytes_primal;  /* algorithmic bytes of one primal-half launch: the mean
                              over the sampled launches, each counted on the model it
                              ran on (the push may iterate on fewer columns); the
                              current model's count when nothing was sampled           */
    int64_t bytes_dual;    /* the same for the dual half                              */
    int32_t lanes_at;      /* primal-half kernel in use (lanes_at encoding)           */
    int32_t lanes_a;       /* dual-half kernel in use                                  */
} pdhg_timing;

/* Fill *p with the defaults listed above. */
void pdhg_default_params(pdhg_params *p);

/* Copy the LP to the device, build the explicit transpose, scale it (Ruiz,
 * then Pock-Chambolle), estimate ||Ahat||_2 by power iteration and set up the
 * iteration at x = clamp(0, l, u), y = 0.  p == NULL uses the defaults.  On
 * success *out owns all device memory of the solver.  Errors: INVALID_ARG
 * (NULL pointers, m or n < 0, nnz mismatch, column out of range, non-finite
 * val/b/c, NaN bound, l > u, unknown sense), OOM, HIP. */
int pdhg_create(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                const double *val, const double *b, const double *c, const double *l, const double *u,
                const char *sense, const pdhg_params *p, pdhg_solver **out);

/* pdhg_create on a model already in device memory (the same meaning and
 * layout; every pointer is a device address on the current device): the
 * inputs stay where they are and are copied device to device, so a caller
 * whose data lives in HBM never crosses PCIe.  The device checks the model:
 * row_ptr as above, columns in range and strictly ascending within each row
 * (this entry point does not sort or merge duplicates), finite val, b and c,
 * bounds not NaN with l <= u, senses '=', '<' or '>' (l, u, sense may be
 * NULL: 0, +infinity, all '=').  The caller keeps ownership and may free its
 * arrays once this returns.  Errors: as pdhg_create (INVALID_ARG names the
 * first failed check), OOM, HIP. */
int pdhg_create_device(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                       const double *val, const double *b, const double *c, const double *l, const double *u,
                       const char *sense, const pdhg_params *p, pdhg_solver **out);

/* Iterate until the relative tests hold (PDHG_OPTIMAL), max_iter, the time
 * limit or a non-finite value.  Re-callable: continues from the current
 * state.  *r may be NULL.  Errors: INVALID_ARG, STATE (after a push), HIP. */
int pdhg_solve(pdhg_solver *s, pdhg_result *r);

/* Exactly `iters` further iterations of the solve (fewer only if it
 * terminates), with checks every check_every iterations as in pdhg_solve. */
int pdhg_iterate(pdhg_solver *s, int64_t iters, pdhg_result *r);

/* Algorithm 1 of section 3 on the solve's (x, y, z), in place, continued by
 * PDHG; seed selects the Uniform[0,1) objective (splitmix64 of seed xor
 * j * 0x9E3779B97F4A7C15, top 53 bits).  Requires a prior solve (STATE). */
int pdhg_corner_push(pdhg_solver *s, uint64_t seed, pdhg_push_result *r);

/* Dual corner push: the mirror image of Algorithm 1 for the dual superbasics
 * that section 6 says the same technique could reduce (the paper gives no
 * construction; this is the library's reading).  Keeps the solve's x and
 * restricts (y, z) to the dual optimal face that complementary slackness with
 * x defines: z_j = 0 for a column off both bounds by more than eps_abs,
 * z_j >= 0 (<= 0) for one within eps_abs of its lower (upper) bound only, and
 * an inequality row whose slack exceeds eps_abs keeps its dual.  Like
 * Algorithm 1, which fixes bounds at the solve's x so that x stays feasible,
 * the face is anchored at the solve's ybar: a dropped row keeps y_i = ybar_i,
 * and each column's objective is shifted by the part of its reduced cost at
 * ybar that its sign rule rejects.  On that face PDHG maximises g'y,
 * g = push_obj_scale * (A w0 - s.v): w0_j = U_j inside the column's cone (-U_j
 * for an upper-bound cone, 0 for a column at both bounds), v_i = U_(n+i) on
 * inequality rows (s_i = +1 for '>', -1 for '<'), U_k the uniform draw of
 * pdhg_corner_push's generator at index k; w0 keeps the push model feasible,
 * so the push is bounded.  Starts from (0, ybar), stops as soon as the push
 * model's dual residual over (1 + ||c||) is back at eps_rel (after at least
 * push_min_iters iterations; checks at push_min_iters + k K).  Afterwards
 * pdhg_get_solution gives (x, yhat, zhat), zhat the reduced costs of yhat on
 * the original model.  Runs once per solve, right after it or after
 * pdhg_corner_push (the primal phase first, as in crossover): then x is the
 * pushed xhat, ybar is still the solve's y, and the answer is (xhat, yhat,
 * zhat).  pdhg_corner_push is refused after it.  pdhg_batch_dual_push is the
 * batch form.  The push runs on the full model (push_compact applies to
 * pdhg_corner_push).
 * Errors: INVALID_ARG, STATE (no solve yet, or a second dual push), HIP. */
int pdhg_dual_push(pdhg_solver *s, uint64_t seed, pdhg_dual_push_result *r);

/* KKT report of (x, y) on the original model, in float64.  x (n) and y (m)
 * are host arrays; NULL selects the current solution.  Errors: INVALID_ARG. */
int pdhg_kkt(pdhg_solver *s, const double *x, const double *y, pdhg_kkt_report *k);

/* Current solution, unscaled: after a solve the last checked candidate
 * (x, y) and z = reduced costs; after a push (xhat, y, z) with the solve's y
 * and z (Algorithm 1 returns them unchanged); after a dual push (x, yhat,
 * zhat), x the solve's or, after both pushes, the corner push's xhat.  Any
 * pointer may be NULL. */
int pdhg_get_solution(pdhg_solver *s, double *x, double *y, double *z);

/* The solve's own answer (x, y, z), unscaled, also after a push: the point a
 * crossover started before the push would take, where pdhg_get_solution then
 * gives the pushed one.  Errors: STATE before a solve has a candidate. */
int pdhg_get_solve_solution(pdhg_solver *s, double *x, double *y, double *z);

/* Current PDHG iterate (x, y) of the running phase, unscaled. */
int pdhg_get_iterate(pdhg_solver *s, double *x, double *y);

/* pdhg_get_solution into caller-owned device buffers (n, m, n doubles, any
 * may be NULL), copied on the solver's stream; `stream` (a hipStream_t, or
 * NULL for the solver's) is ordered after the copies.  No host sync. */
int pdhg_get_solution_device(pdhg_solver *s, double *x, double *y, double *z, void *stream);

/* Warm start: restart the solve phase from the caller's (x, y) (host,
 * unscaled; x is clamped to the bounds and y projected on the signs of its
 * rows, the projections of section 2), with the anchors at that point, the
 * primal weight re-initialised and the restart state reset (the iteration
 * count starts at 0).  Errors: INVALID_ARG (NULL or non-finite entries),
 * STATE during a push. */
int pdhg_set_start(pdhg_solver *s, const double *x, const double *y);

/* Checkpoint and resume of the solve phase: pdhg_state_size gives the
 * buffer size; pdhg_get_state writes the iteration state (iterate, anchors,
 * candidate, step sizes, primal weight, restart state, counters) into the
 * caller's host buffer; pdhg_set_state loads such a buffer into a handle
 * created from the same LP and parameters, after which pdhg_iterate /
 * pdhg_solve continue exactly as the checkpointed run would have.  Errors:
 * INVALID_ARG (NULL, buffer too small, not a checkpoint of this layout,
 * another size or precision), STATE during a push. */
int pdhg_state_size(pdhg_solver *s, int64_t *bytes);
int pdhg_get_state(pdhg_solver *s, void *buf, int64_t bytes);
int pdhg_set_state(pdhg_solver *s, const void *buf, int64_t bytes);

/* Scaling vectors Dr (m), Dc (n) (Ahat = diag(Dr) A diag(Dc)) and
 * scalars5 = {eta, omega, sigma_estimate, iterations of the phase,
 * power-iteration steps taken}.  Any pointer may be NULL. */
int pdhg_get_scaling(pdhg_solver *s, double *dr, double *dc, double *scalars5);

/* Kernel timing and byte model (see pdhg_timing).  Errors: INVALID_ARG. */
int pdhg_get_timing(pdhg_solver *s, pdhg_timing *t);

/* Device copy probe: copies `bytes` (rounded down to 16-byte units) between
 * two device buffers `reps` times with a plain streaming kernel and returns
 * the achieved bandwidth (read + write bytes / time) in *gbps; the HBM
 * ceiling that the iteration kernels are measured against.  Allocates and
 * frees its own buffers.  Errors: INVALID_ARG, OOM, HIP. */
int pdhg_copy_probe(int64_t bytes, int32_t reps, double *gbps);

/* ------------------------------------------------------------------------
 * Batch engine: many independent LPs of uneven sizes, solved and then
 * corner-pushed together (the same method as above for each LP).  The LPs
 * form one block-diagonal model; every half-iteration is one launch over
 * instance-aligned row tiles of all LPs; each LP keeps its own scaling, step
 * size, primal weight, restart state and termination.  LPs advance in
 * lockstep cycles of check_every iterations; an LP that terminates stops
 * changing while the others continue.  The push phase starts for every LP
 * whose solve reached PDHG_OPTIMAL; its checks come at push iterations
 * push_min_iters, +check_every, ...  params as for pdhg_create (the iteration
 * kernels are the tiled ones: lanes_* must be 0 or a tile encoding).
 * ------------------------------------------------------------------------ */
typedef struct pdhg_batch pdhg_batch;

typedef struct pdhg_lp_desc { /* one LP, same layout and conventions as pdhg_create */
    int32_t m, n;            /* m >= 1, n >= 1                                      */
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    const double *b, *c, *l, *u; /* l, u may be NULL (0 and +INFINITY)              */
    const char *sense;           /* may be NULL (all '=')                          */
} pdhg_lp_desc;

typedef struct pdhg_batch_report {
    int32_t count;
    int32_t lanes_at, lanes_a;   /* tiled kernels in use (pdhg_params encoding)     */
    int32_t pad_;
    double solve_seconds, push_seconds;
    int64_t solve_lockstep_iters; /* iterations the batch ran in the solve phase   */
    int64_t push_lockstep_iters;
    double primal_ms, dual_ms;   /* mean launch time of the batched halves (timing) */
    int64_t samples;
    int64_t bytes_primal, bytes_dual; /* mean algorithmic bytes of the timed launches,
                                         counting only LPs still iterating          */
    int64_t total_m, total_n, total_nnz;
} pdhg_batch_report;

/* Copy `count` LPs (host arrays, caller keeps ownership) and set each up as
 * pdhg_create does.  Errors: INVALID_ARG (any LP invalid, or sizes beyond
 * 32-bit indices), OOM, HIP. */
int pdhg_batch_create(int32_t count, const pdhg_lp_desc *lps, const pdhg_params *p, pdhg_batch **out);

/* pdhg_batch_create on LPs already in device memory: the descriptors are a
 * host array (count <= 65535), every array they point to is device memory
 * of this GPU, owned by the caller and only read (it may be freed once the
 * call returns).  The block-diagonal model is assembled and checked on the
 * device as pdhg_create_device checks one LP, rows needing ascending,
 * unique column indices; each LP's row_ptr must start at 0 and end at its
 * nnz, and its column indices stay below its own n.  Errors: INVALID_ARG
 * (bad sizes or pointers, an invalid LP), OOM, HIP. */
int pdhg_batch_create_device(int32_t count, const pdhg_lp_desc *lps, const pdhg_params *p, pdhg_batch **out);

/* Solve every LP (results[count]); STATE if called twice. */
int pdhg_batch_solve(pdhg_batch *b, pdhg_result *results);

/* Algorithm 1 for every LP whose solve is optimal, seeds[i] selecting LP i's
 * random objective (results[count]; LPs without a push report their solve
 * status and 0 push iterations).  Requires pdhg_batch_solve (STATE). */
int pdhg_batch_corner_push(pdhg_batch *b, const uint64_t *seeds, pdhg_push_result *results);

/* pdhg_dual_push for every LP whose solve is optimal, seeds[i] selecting LP
 * i's draws (U_k at LP i's own column and row numbering), in lockstep cycles
 * over the block-diagonal model (results[count]; an LP without a push reports
 * its solve status and 0 iterations).  After pdhg_batch_corner_push each LP's
 * face is that of its pushed xhat; pdhg_batch_corner_push is refused after
 * it.  Afterwards pdhg_batch_get_solution gives (x, yhat, zhat).  Errors:
 * INVALID_ARG, STATE (no batch solve, or a second dual push), HIP. */
int pdhg_batch_dual_push(pdhg_batch *b, const uint64_t *seeds, pdhg_dual_push_result *results);

/* Solution of LP i, unscaled (x: n_i, y: m_i, z: n_i; any may be NULL);
 * after the push x is the pushed x. */
int pdhg_batch_get_solution(pdhg_batch *b, int32_t i, double *x, double *y, double *z);

/* LP i's solve answer, also after the push (see pdhg_get_solve_solution). */
int pdhg_batch_get_solve_solution(pdhg_batch *b, int32_t i, double *x, double *y, double *z);

/* Aggregate timings and sizes of the batch. */
int pdhg_batch_get_report(pdhg_batch *b, pdhg_batch_report *r);

void pdhg_batch_destroy(pdhg_batch *b);

/* ------------------------------------------------------------------------
 * Learned fix predictor: a per-variable network 16 -> 64 -> 64 -> 1 (12
 * features padded to 16) on bfloat16 matrix cores with float32 accumulation
 * and float32 master weights:  h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2),
 * logit = w3 . h2 + b3, probability = 1 / (1 + exp(-logit)).  It predicts
 * which variables end at a bound after the corner push (Algorithm 1 of
 * section 3), so that the push can start with them fixed; the paper itself
 * has no learned component.  Parameters are a flat float32 vector of
 * PDHG_MLP_NPARAMS values in the order w1 (64 x 16, row-major), b1 (64),
 * w2 (64 x 64), b2 (64), w3 (64), b3 (1).  Features are float32, 16 per
 * variable, row-major, rounded to bfloat16 on the device.
 * ------------------------------------------------------------------------ */
#define PDHG_MLP_NPARAMS 5313
#define PDHG_MLP_FEATURES 16

typedef struct pdhg_train_params {
    int32_t epochs;     /* passes over the data; default 4                          */
    int32_t batch;      /* minibatch size, 1..65536; default 4096                   */
    double lr, beta1, beta2, eps; /* Adam; defaults 1e-3, 0.9, 0.999, 1e-8          */
    double pos_weight;  /* weight of positive samples in the loss; <= 0: N_neg/N_pos */
    uint64_t seed;      /* shuffling seed                                           */
} pdhg_train_params;

typedef struct pdhg_train_report {
    double loss_first, loss_last; /* mean weighted BCE of the first and last epoch    */
    double seconds;
    int64_t steps;      /* Adam steps                                               */
    double samples_per_s;
    double pos_weight;  /* the weight used                                          */
} pdhg_train_report;

/* New network with Kaiming-uniform weights (bound sqrt(6 / fan_in), drawn
 * from splitmix64 of seed xor parameter index) and zero biases. */
int pdhg_mlp_create(uint64_t seed, pdhg_mlp **out);
void pdhg_mlp_destroy(pdhg_mlp *net);
/* Copy parameters in / out (host, PDHG_MLP_NPARAMS floats); setting them
 * resets the Adam state. */
int pdhg_mlp_set_params(pdhg_mlp *net, const float *params);
int pdhg_mlp_get_params(pdhg_mlp *net, float *params);
/* logits[n] of features[n x 16] (host arrays). */
int pdhg_mlp_forward(pdhg_mlp *net, const float *features, int64_t n, float *logits);
/* pdhg_mlp_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops): features[n x 16] and
 * logits[n] are the caller's device buffers, on the device the network was
 * created on; the work is enqueued on `stream` (a hipStream_t, NULL: the
 * network's own stream) and the call returns without waiting.  The bfloat16
 * staging copy of the features lives in a fixed 2 MiB device array per GPU,
 * so n is at most 65536 per call (INVALID_ARG beyond); no allocation, no
 * synchronisation.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  Errors: INVALID_ARG, HIP. */
int pdhg_mlp_forward_noalloc(pdhg_mlp *net, const float *features, int64_t n, float *logits, void *stream);
/* Gradient of the mean weighted binary cross-entropy over n <= 65536
 * samples (labels 0/1) into grad[PDHG_MLP_NPARAMS]; *loss = the mean loss. */
int pdhg_mlp_gradient(pdhg_mlp *net, const float *features, const float *labels, int64_t n, double pos_weight,
                      float *grad, double *loss);
void pdhg_default_train_params(pdhg_train_params *t);
/* Adam training over n samples (features n x 16, labels n), shuffled per
 * epoch; t == NULL uses the defaults. */
int pdhg_mlp_train(pdhg_mlp *net, const float *features, const float *labels, int64_t n, const pdhg_train_params *t,
                   pdhg_train_report *r);

/* The 16 predictor features of every column of a solved LP (before its
 * push), normalised as the network sees them, into out[n x 16] (float32
 * host array, row j = column j), or NULL to only compute them:
 *   0..3  x_j, z_j, |c_j|, ||A_{:,j}||_2 on the scaled model;
 *   4..11 x_j, then z_j, at each of the last 4 restarts minus the current
 *         value (0 where fewer restarts happened, and all 0 unless
 *         params.record_history = 1);
 *   12    the push objective coefficient that pdhg_corner_push(seed) draws;
 *   13-15 distance to the lower and the upper bound, relative position
 *         between them (-1 where not defined);
 * each mapped to sign(v) ln(1 + |v|/s), s its root mean square over the LP.
 * The learned predictor of the push and its training data are built on
 * these (the paper does not fix them).  Errors: STATE before a solve or
 * after a push. */
int pdhg_features(pdhg_solver *s, uint64_t seed, float *out);

/* Corner push with a learned warm start: the plain fixes of Algorithm 1,
 * then every column the plain rule leaves free whose predicted probability
 * is >= theta is fixed at its nearer finite bound if the sign of its reduced
 * cost allows it; at each push check a learned fix whose push-model reduced
 * cost has the wrong sign (beyond eps_abs) is undone.  r->n_learned_fix and
 * r->n_learned_undo count them.  Errors as pdhg_corner_push, and INVALID_ARG
 * for theta outside (0, 1). */
int pdhg_corner_push_learned(pdhg_solver *s, pdhg_mlp *net, double theta, uint64_t seed, pdhg_push_result *r);

/* pdhg_corner_push_learned with the predictor's output supplied by the
 * caller: logits[n] (host float32, column j's logit; copied before the
 * call returns, the caller keeps ownership) take the place of the network
 * on the handle's features.  A column is predicted fixed when its logit is
 * >= ln(theta / (1 - theta)), compared in float32; a NaN logit never fixes.
 * The same fixes, undo rule and counts follow.  For callers with their own
 * predictor (the paper has none: a warm start of Algorithm 1's fixing set).
 * Errors as pdhg_corner_push_learned, INVALID_ARG for NULL logits. */
int pdhg_corner_push_logits(pdhg_solver *s, const float *logits, double theta, uint64_t seed, pdhg_push_result *r);

/* The features of pdhg_features for every LP of a solved batch (before its
 * push), each LP normalised over its own columns and drawing the push
 * objective of seeds[i] (count seeds, host): out[total_n x 16] (host),
 * LPs in batch order, or NULL to only compute them.  The trend features
 * need params.record_history = 1 at pdhg_batch_create.  Errors: INVALID_ARG
 * (NULL seeds), STATE before the solve or after the push. */
int pdhg_batch_features(pdhg_batch *b, const uint64_t *seeds, float *out);

/* pdhg_batch_corner_push with the learned warm start of
 * pdhg_corner_push_learned applied to every LP of the batch (the same
 * rules, per LP); results[i].n_learned_fix / n_learned_undo count LP i's
 * fixes and undos.  Errors as pdhg_batch_corner_push, and INVALID_ARG for
 * theta outside (0, 1) or a NULL network. */
int pdhg_batch_corner_push_learned(pdhg_batch *b, pdhg_mlp *net, double theta, const uint64_t *seeds,
                                   pdhg_push_result *results);

/* pdhg_batch_corner_push_learned with caller logits: logits[total_n] (host
 * float32, the LPs' columns in batch order), as pdhg_corner_push_logits. */
int pdhg_batch_corner_push_logits(pdhg_batch *b, const float *logits, double theta, const uint64_t *seeds,
                                  pdhg_push_result *results);

/* Release all device memory of the handle (NULL is a no-op). */
void pdhg_destroy(pdhg_solver *s);

/* Thread-local text of the last error ("" if none). */
const char *pdhg_last_error(void);

/* Size checks for bindings: sizeof of each public struct. */
int32_t pdhg_struct_size(int32_t which); /* 0 params, 1 result, 2 kkt, 3 push, 4 timing,
                                             5 lp desc, 6 batch report, 7 dual push */

#ifdef __cplusplus
}
#endif
#endif /* PDHG_H */
