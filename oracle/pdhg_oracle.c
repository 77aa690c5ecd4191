/*
 * pdhg_oracle.c -- plain FP64 CPU reference for restarted Halpern PDHG on LPs
 * and for the corner-push phase of "Backing PDHG into a Corner" (Rothberg,
 * arXiv 2511.13894).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU leg of the
 * benchmark do.  It shares no code, header, table or constant generator with
 * the HIP path.
 *
 * What it computes, in the paper's notation (section 2, "Background"):
 *   primal  min c'x  s.t.  a_i'x (=, <=, >=) b_i,  l <= x <= u
 *   dual    y (free for '=', y_i <= 0 for '<=', y_i >= 0 for '>='), reduced
 *           costs z = c - A'y split into the parts that bounds can absorb.
 * Residuals r_P = b - Ax, r_D = c - A'y - z and the relative l2 termination
 * tests are the ones of section 2.  Inequalities and bounds are handled
 * implicitly (section 2, last paragraph before the restated objective).
 *
 * The paper names its PDHG only as "closely following cuPDLP+" (section 4.1)
 * and says nothing of scaling, step size, restarts or primal weight.  The
 * readings used for those silent parts are:
 *   scaling   : 10 Ruiz passes (inf-norm, rows and columns from the same
 *               matrix), then one Pock-Chambolle pass with alpha = 1;
 *   step size : power iteration on M = Ahat'Ahat from v0 proportional to
 *               1 + U_j (U_j the counter-based uniform draw of column j with
 *               a fixed seed, OR_POWER_SEED), scaled to unit length; a
 *               constant start lies in the null space of any matrix whose
 *               scaled rows sum to zero, such as [1, -1].  Each
 *               step forms u = Ahat v, w = Ahat'u, rho = u'u (the Rayleigh
 *               quotient of the unit v) and lambda = ||w||, and stops at the
 *               first step whose eigen-residual ||w - rho v|| =
 *               sqrt(w'w - rho^2) is at most tol * rho (else after P steps);
 *               eta = safety / sqrt(lambda);
 *   iteration : PDHG step T followed by a reflected Halpern average with the
 *               restart anchor (halpern = 0 gives vanilla PDHG);
 *   checks    : every K iterations on the candidate T(z); termination on the
 *               unscaled model, restart on a weighted KKT of the scaled model
 *               (sufficient / necessary-without-progress / artificial rules);
 *   weight    : log-smoothed primal weight update at restarts.
 * Corner push (section 3, Algorithm 1; implicit slacks in the paragraph after
 * it; option 1 "modify in place and continue"; termination in section 3.1):
 *   ub_j <- x_j if z_j > eps_abs, lb_j <- x_j if z_j < -eps_abs; an inequality
 *   row whose slack has a reduced cost beyond eps_abs becomes an equality;
 *   objective Uniform[0,1)^n; restart from (x, 0); stop as soon as the primal
 *   residual of the modified model is back at the original tolerance, after at
 *   least push_min_iters push iterations.  Returns (xhat, y, z) with y and z
 *   those of the input.
 * Dual corner push (section 6 names the idea of cutting dual superbasics the
 * same way, and nothing more; the construction is this library's reading,
 * the mirror image of Algorithm 1):
 *   keep the solve's x and restrict (y, z) to the dual optimal face that
 *   complementary slackness with x defines: a column further than eps_abs
 *   from both bounds gets z_j = 0, one within eps_abs of its lower bound only
 *   z_j >= 0, of its upper bound only z_j <= 0, of both z_j free; an
 *   inequality row whose slack exceeds eps_abs keeps its dual fixed (sense
 *   'N'), every other row keeps its sign rule.  As Algorithm 1 fixes bounds
 *   at the solve's x rather than at the bound, so that x stays feasible, the
 *   dual push fixes at the solve's point ybar: a dropped row's y_i stays
 *   ybar_i (its term moves into the objective), and each column's objective
 *   is shifted by r_j, the part of its reduced cost at ybar that its cone
 *   rejects (all of it off both bounds, the negative part at the lower bound
 *   only, the positive part at the upper bound only), so that ybar is a point
 *   of the face.  The face is then the dual feasible set of the push model
 *     min c~'w  s.t.  a_i'w (sense_i) g_i (rows kept),  w_j in the cone of
 *     column j (R, R+, R-, {0}),  c~ = c - A_N' ybar_N - r,
 *   whose right-hand side is random but anchored:
 *   g = scale * (A w0 - s.v), w0 a random point of the cones (w0_j = U_j on
 *   R and R+, -U_j on R-, 0 on {0}), v_i = U_(n+i) a random slack with
 *   s_i = +1 on '>' rows, -1 on '<' rows, 0 on '=' rows.  w0 is feasible for
 *   the push model, so the random dual objective g'y is bounded on the face
 *   (the mirror of the primal push, whose model keeps the solve's x
 *   feasible); a random g alone is unbounded wherever A has dependent
 *   equality rows.  PDHG restarts from (0, ybar) and stops
 *   as soon as the dual residual of the push model, relative to 1 + ||c||,
 *   is back at the original tolerance, after at least push_min_iters
 *   iterations.  Returns (x, yhat, zhat): the solve's x, the pushed y (ybar
 *   on the dropped rows) and its reduced costs on the original model.  Run
 *   after the corner push (the primal phase first, as in crossover), x is the
 *   pushed xhat and ybar still the solve's y.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BIG 1e20 /* |bound| >= 1e20 counts as infinite */

/* status codes (numeric values documented in the test suite) */
enum {
    OR_OPTIMAL = 0,
    OR_ITER_LIMIT = 1,
    OR_NUMERICAL = 2,
    OR_PUSH_DONE = 3,
    OR_PUSH_SKIPPED = 5, /* gate of section 4.2 closed: too few candidates */
    OR_ERR_ARG = -1,
    OR_ERR_STATE = -2
};

typedef struct {
    double eps_rel, eps_abs;
    int64_t max_iter;
    int32_t check_every;
    int32_t ruiz_iters;
    double restart_suff, restart_nec, restart_art;
    double pw_smooth;
    double pc_alpha;
    int32_t power_iters;
    int32_t halpern;
    double eta_safety;
    double reflect_gamma;
    double power_tol;
    int32_t push_min_iters;
    int32_t pad_;
    double push_obj_scale;
    int64_t push_max_iter;
    /* selection rule of section 4.2 (off by default): push only when the
       solve's answer has at least max(push_gate_rows * m, push_gate_min)
       candidates (off bound with |z| < tol) */
    int32_t push_gate;
    /* keep x and z of the solve's candidate at its last 4 restarts (float32
       values), for the trend features of the learned warm start */
    int32_t record_history;
    double push_gate_rows;
    int64_t push_gate_min;
} or_params;

typedef struct {
    double rp2, rd2, rpinf, rdinf; /* unscaled residual norms */
    double pobj, dobj, gap;
    double rel_p, rel_d, rel_gap;
    int64_t p_off;       /* variables off their bounds (structural + slack)  */
    int64_t d_zero;      /* reduced costs at zero (structural + slack)      */
    int64_t candidates;  /* off bound and |z| < tol                         */
    int64_t est_primal;  /* max(p - m, 0)                                    */
    int64_t est_dual;    /* max(m - d, 0)                                    */
} or_kkt;

typedef struct {
    int32_t status;
    int32_t pad_;
    int64_t iters, restarts;
    double rel_p, rel_d, rel_gap, pobj, dobj;
} or_result;

typedef struct {
    int32_t status;
    int32_t pad_;
    int64_t iters, restarts;
    int64_t n_fix_lower, n_fix_upper, n_rows_to_eq;
    double rel_p_push; /* relative primal residual of the push model at stop */
    or_kkt before, after;
    int64_t n_learned_fix;  /* learned warm start: columns fixed from the predictor */
    int64_t n_learned_undo; /* learned fixes undone at push checks                  */
} or_push_result;

typedef struct {
    int32_t status;
    int32_t pad_;
    int64_t iters, restarts;
    int64_t n_cols_free;  /* columns off both bounds: reduced cost held at ybar's */
    int64_t n_rows_fixed; /* inequality rows with slack: y_i held at ybar_i        */
    double rel_d_push;   /* relative dual residual of the push model at the stop */
    or_kkt before, after;
} or_dual_push_result;

typedef struct {
    int m, n;
    int64_t nnz;
    /* original model (unscaled), A row-compressed with sorted, summed rows */
    int64_t *rp;
    int32_t *ci;
    double *av;
    /* explicit transpose: row j of T is column j of A, entries by ascending i */
    int64_t *tp;
    int32_t *ti;
    int64_t *tpos; /* index into the CSR value arrays of each transpose entry */
    double *b, *c, *l, *u;
    char *sense0;
    /* scaled operator */
    double *ahat, *ahat_t; /* Ahat values in CSR order and in transpose order */
    double *dr, *dc;
    double eta, sigma_est;
    int64_t power_steps; /* power-iteration steps taken */
    /* current (scaled) model: solve model or push model */
    double *bh, *ch, *lh, *uh;
    char *sense;
    /* iterate state (scaled) */
    double *x, *y, *xa, *ya, *xp, *yp, *xbar, *g, *hv;
    double omega;
    int64_t k, t, restarts, next_check;
    double kkt_anchor_p2, kkt_anchor_d2, kkt_anchor_gap2; /* at the anchor */
    double kkt_prev;
    int solved;   /* a solve has produced a checked candidate */
    int in_push;  /* bits: 1 corner push done, 2 dual corner push done (0: solve) */
    /* solution of the original solve, unscaled, kept for the push */
    double *xs_hat, *ys_hat; /* scaled candidate accepted by the solve */
    double *xsol, *ysol, *zsol;
    double *xpush;         /* unscaled push result */
    double *ypush, *zpush; /* unscaled dual push result and its reduced costs */
    double *cpush;         /* unscaled objective of the dual push model        */
    /* learned warm start: restart history of the solve (slot (r - 1) mod 4
       holds the candidate of restart r, rounded to float32) and the fixes */
    double *hx, *hz;
    signed char *lfix; /* 0 none, 1 fixed at its lower bound, 2 at its upper */
    int learned;       /* the push runs with learned fixes                    */
    int64_t n_lfix, n_lundo;
    or_params p;
} or_solver;

/* ------------------------------------------------------------------------ */
static int is_inf_lo(double v) { return v <= -OR_BIG; }
static int is_inf_up(double v) { return v >= OR_BIG; }

static double clampd(double v, double lo, double hi)
{
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* projection of one dual entry onto its cone: '=' free, '<' y <= 0, '>' y >= 0,
 * 'N' (a row the dual push drops) y = 0 */
static double proj_dual(double v, char s)
{
    if (s == '<') return v < 0.0 ? v : 0.0;
    if (s == '>') return v > 0.0 ? v : 0.0;
    if (s == 'N') return 0.0;
    return v;
}

/* splitmix64 (Steele, Lea and Flood 2014), counter-based uniform draw */
uint64_t or_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform[0,1) value number j of the push objective for a given seed */
double or_push_uniform(uint64_t seed, int64_t j)
{
    uint64_t h = or_splitmix64(seed ^ ((uint64_t)j * 0x9E3779B97F4A7C15ULL));
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* seed of the power iteration's start vector (any fixed value) */
#define OR_POWER_SEED 0x5DEECE66DULL

/* ------------------------------------------------------------------------ */
/* plain products with the unscaled and the scaled operator                 */
static void mv_A(const or_solver *s, const double *val, const double *x, double *out)
{
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < s->m; i++) {
        double acc = 0.0;
        for (int64_t e = s->rp[i]; e < s->rp[i + 1]; e++) acc += val[e] * x[s->ci[e]];
        out[i] = acc;
    }
}

static void mv_At(const or_solver *s, const double *tval, const double *y, double *out)
{
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < s->n; j++) {
        double acc = 0.0;
        for (int64_t e = s->tp[j]; e < s->tp[j + 1]; e++) acc += tval[e] * y[s->ti[e]];
        out[j] = acc;
    }
}

/* transpose values in transpose order, gathered from row order */
static void gather_t(const or_solver *s, const double *val, double *tval)
{
    for (int64_t e = 0; e < s->nnz; e++) tval[e] = val[s->tpos[e]];
}

/* Compensated summation (Neumaier's improvement of Kahan's method): the
 * rounding error of a sum stays within a few units in the last place of the
 * result whatever the number of terms.  Every reduction over all rows or all
 * columns uses it, so that at 10^7 terms the reference is at least as exact
 * as any summation order a parallel implementation may use (a plain
 * left-to-right sum can drift by n*eps, 1e-9 at that size). */
typedef struct {
    double s, c;
} csum;

static void cadd(csum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

static double cval(const csum *a) { return a->s + a->c; }

static double norm2(const double *v, int64_t n)
{
    csum acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; i++) cadd(&acc, v[i] * v[i]);
    return sqrt(cval(&acc));
}

/* ------------------------------------------------------------------------ */
/* KKT of (x, y) on an unscaled model (section 2 residuals, relative l2 tests;
 * bounds and inequalities handled implicitly).  sense may differ from the
 * original model (push model).  With l = 0, u = inf and '=' rows this is
 * exactly r_P = b - Ax, r_D = c - A'y - z, gap = c'x - b'y. */
static void kkt_unscaled(const or_solver *s, const double *c, const double *l, const double *u,
                         const char *sense, const double *x, const double *y, double *ax,
                         double *aty, double *zout, or_kkt *k)
{
    int m = s->m, n = s->n;
    double *tv = (double *)malloc(sizeof(double) * (size_t)(s->nnz > 0 ? s->nnz : 1));
    gather_t(s, s->av, tv);
    mv_A(s, s->av, x, ax);
    mv_At(s, tv, y, aty);
    free(tv);
    double rpinf = 0, rdinf = 0;
    csum rp2 = {0, 0}, rd2 = {0, 0}, cx = {0, 0}, by = {0, 0};
    for (int i = 0; i < m; i++) {
        double r = s->b[i] - ax[i];
        if (sense[i] == '<') r = r < 0.0 ? r : 0.0;
        else if (sense[i] == '>') r = r > 0.0 ? r : 0.0;
        else if (sense[i] == 'N') r = 0.0;
        cadd(&rp2, r * r);
        if (fabs(r) > rpinf) rpinf = fabs(r);
        cadd(&by, s->b[i] * y[i]);
    }
    for (int j = 0; j < n; j++) {
        double lam = c[j] - aty[j];
        double zp = (!is_inf_lo(l[j]) && lam > 0.0) ? lam : 0.0;
        double zm = (!is_inf_up(u[j]) && lam < 0.0) ? -lam : 0.0;
        double z = zp - zm;
        double rd = lam - z;
        cadd(&rd2, rd * rd);
        if (fabs(rd) > rdinf) rdinf = fabs(rd);
        cadd(&cx, c[j] * x[j]);
        if (zp > 0.0) cadd(&by, l[j] * zp);
        if (zm > 0.0) cadd(&by, -(u[j] * zm));
        if (zout) zout[j] = z;
    }
    double pobj = cval(&cx), dobj = cval(&by);
    double nb = norm2(s->b, m), nc = norm2(c, n);
    k->rp2 = sqrt(cval(&rp2));
    k->rd2 = sqrt(cval(&rd2));
    k->rpinf = rpinf;
    k->rdinf = rdinf;
    k->pobj = pobj;
    k->dobj = dobj;
    k->gap = pobj - dobj;
    k->rel_p = k->rp2 / (1.0 + nb);
    k->rel_d = k->rd2 / (1.0 + nc);
    k->rel_gap = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
}

/* push-estimate counts of section 2.1 and the selection count of section 4.2,
 * for x (unscaled) against the original bounds and z (unscaled). */
static void corner_counts(const or_solver *s, const double *x, const double *ax, const double *y,
                          const double *z, or_kkt *k)
{
    const double tol = 1e-6;
    int64_t p = 0, d = 0, cand = 0;
    for (int j = 0; j < s->n; j++) {
        int off = (x[j] - s->l[j] > tol) && (s->u[j] - x[j] > tol);
        int zz = fabs(z[j]) <= tol;
        p += off;
        d += zz;
        cand += off && (fabs(z[j]) < tol);
    }
    for (int i = 0; i < s->m; i++) {
        char sn = s->sense0[i];
        if (sn == '=') continue;
        double slack = (sn == '<') ? (s->b[i] - ax[i]) : (ax[i] - s->b[i]);
        double zs = (sn == '<') ? -y[i] : y[i];
        int off = slack > tol;
        p += off;
        d += fabs(zs) <= tol;
        cand += off && (fabs(zs) < tol);
    }
    k->p_off = p;
    k->d_zero = d;
    k->candidates = cand;
    k->est_primal = p > s->m ? p - s->m : 0;
    k->est_dual = s->m > d ? s->m - d : 0;
}

/* ------------------------------------------------------------------------ */
/* weighted KKT of the scaled current model at (x, y):
 * returns squared ||rP_hat||, ||rD_hat|| and gap^2 through the pointers. */
static void kkt_scaled_parts(or_solver *s, const double *x, const double *y, double *p2, double *d2,
                             double *gap2)
{
    int m = s->m, n = s->n;
    double *ax = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *aty = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    mv_A(s, s->ahat, x, ax);
    mv_At(s, s->ahat_t, y, aty);
    csum rp = {0, 0}, rd = {0, 0}, cx = {0, 0}, by = {0, 0};
    for (int i = 0; i < m; i++) {
        double r = s->bh[i] - ax[i];
        if (s->sense[i] == '<') r = r < 0.0 ? r : 0.0;
        else if (s->sense[i] == '>') r = r > 0.0 ? r : 0.0;
        else if (s->sense[i] == 'N') r = 0.0;
        cadd(&rp, r * r);
        cadd(&by, s->bh[i] * y[i]);
    }
    for (int j = 0; j < n; j++) {
        double lam = s->ch[j] - aty[j];
        double zp = (!is_inf_lo(s->lh[j]) && lam > 0.0) ? lam : 0.0;
        double zm = (!is_inf_up(s->uh[j]) && lam < 0.0) ? -lam : 0.0;
        double rdj = lam - (zp - zm);
        cadd(&rd, rdj * rdj);
        cadd(&cx, s->ch[j] * x[j]);
        if (zp > 0.0) cadd(&by, s->lh[j] * zp);
        if (zm > 0.0) cadd(&by, -(s->uh[j] * zm));
    }
    double pobj = cval(&cx), dobj = cval(&by);
    *p2 = cval(&rp);
    *d2 = cval(&rd);
    *gap2 = (pobj - dobj) * (pobj - dobj);
    free(ax);
    free(aty);
}

/* KKT_omega = sqrt(omega^2 ||rP||^2 + ||rD||^2 / omega^2 + gap^2): the primal
 * part weighted up and the dual part down by the primal weight omega. */
double or_kkt_weighted(double omega, double p2, double d2, double gap2)
{
    return sqrt(omega * omega * p2 + d2 / (omega * omega) + gap2);
}

/* Restart decision at a check from the weighted KKT of the candidate (kc),
 * of the anchor (ka) and of the previous check's candidate (kprev), the
 * iterations since the last restart (k) and in the phase (t): restart on
 * sufficient decay, on necessary decay without progress since the last
 * check, or when the inner run is long against the whole phase. */
int or_restart_decision(const or_params *p, double kc, double ka, double kprev, int64_t k, int64_t t)
{
    return (kc <= p->restart_suff * ka) || (kc <= p->restart_nec * ka && kc > kprev) ||
           ((double)k >= p->restart_art * (double)t);
}

/* Primal weight after a restart whose anchors moved by dx (primal) and dy
 * (dual): log-space smoothing of dy/dx with the old weight,
 * exp(th ln(dy/dx) + (1 - th) ln omega); kept when either move is below 1e-10. */
double or_weight_update(const or_params *p, double omega, double dx, double dy)
{
    if (!(dx > 1e-10 && dy > 1e-10)) return omega;
    double th = p->pw_smooth;
    return exp(th * log(dy / dx) + (1.0 - th) * log(omega));
}

/* ------------------------------------------------------------------------ */
static void set_defaults(or_params *p)
{
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
    p->pad_ = 0;
    p->push_obj_scale = 1.0;
    p->push_gate = 0;
    p->record_history = 0;
    p->push_gate_rows = 2.0;
    p->push_gate_min = 100000;
    p->push_max_iter = 1000000;
}

void or_default_params(or_params *p) { set_defaults(p); }

/* row-compress (sort each row by column, sum duplicates) */
static int canonical_rows(int m, const int64_t *rp, const int32_t *ci, const double *v, int64_t **orp,
                          int32_t **oci, double **ov, int64_t *onnz)
{
    int64_t nnz = rp[m];
    int64_t *nrp = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    int32_t *nci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *nv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!nrp || !nci || !nv) return -1;
    int64_t w = 0;
    for (int i = 0; i < m; i++) {
        int64_t a = rp[i], e = rp[i + 1];
        int64_t start = w;
        for (int64_t q = a; q < e; q++) { /* insertion into the sorted run */
            int32_t col = ci[q];
            double val = v[q];
            int64_t pos = w;
            int dup = 0;
            for (int64_t r = start; r < w; r++) {
                if (nci[r] == col) { nv[r] += val; dup = 1; break; }
            }
            if (dup) continue;
            while (pos > start && nci[pos - 1] > col) {
                nci[pos] = nci[pos - 1];
                nv[pos] = nv[pos - 1];
                pos--;
            }
            nci[pos] = col;
            nv[pos] = val;
            w++;
        }
        nrp[i + 1] = w;
    }
    *orp = nrp;
    *oci = nci;
    *ov = nv;
    *onnz = w;
    return 0;
}

void or_destroy(or_solver *s)
{
    if (!s) return;
    void *ptrs[] = {s->rp, s->ci, s->av, s->tp, s->ti, s->tpos, s->b, s->c, s->l, s->u, s->sense0,
                    s->ahat, s->ahat_t, s->dr, s->dc, s->bh, s->ch, s->lh, s->uh, s->sense, s->x,
                    s->y, s->xa, s->ya, s->xp, s->yp, s->xbar, s->g, s->hv, s->xs_hat, s->xsol,
                    s->ysol, s->zsol, s->xpush, s->ys_hat, s->ypush, s->zpush, s->cpush,
                    s->hx, s->hz, s->lfix};
    for (size_t q = 0; q < sizeof(ptrs) / sizeof(ptrs[0]); q++) free(ptrs[q]);
    free(s);
}

static double *dalloc(int64_t n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* scaling (Ruiz then Pock-Chambolle), power iteration and step size */
static void scale_and_step(or_solver *s)
{
    int m = s->m, n = s->n;
    double *r = dalloc(m), *q = dalloc(n);
    for (int i = 0; i < m; i++) s->dr[i] = 1.0;
    for (int j = 0; j < n; j++) s->dc[j] = 1.0;
    memcpy(s->ahat, s->av, sizeof(double) * (size_t)s->nnz);

    for (int pass = 0; pass < s->p.ruiz_iters; pass++) {
        for (int i = 0; i < m; i++) r[i] = 0.0;
        for (int j = 0; j < n; j++) q[j] = 0.0;
        for (int i = 0; i < m; i++)
            for (int64_t e = s->rp[i]; e < s->rp[i + 1]; e++) {
                double a = fabs(s->ahat[e]);
                if (a > r[i]) r[i] = a;
                if (a > q[s->ci[e]]) q[s->ci[e]] = a;
            }
        for (int i = 0; i < m; i++) r[i] = r[i] > 0.0 ? sqrt(r[i]) : 1.0;
        for (int j = 0; j < n; j++) q[j] = q[j] > 0.0 ? sqrt(q[j]) : 1.0;
        for (int i = 0; i < m; i++)
            for (int64_t e = s->rp[i]; e < s->rp[i + 1]; e++) s->ahat[e] = s->ahat[e] / (r[i] * q[s->ci[e]]);
        for (int i = 0; i < m; i++) s->dr[i] = s->dr[i] / r[i];
        for (int j = 0; j < n; j++) s->dc[j] = s->dc[j] / q[j];
    }
    if (s->p.pc_alpha >= 0.0) { /* one Pock-Chambolle pass (pc_alpha < 0 disables it) */
        double al = s->p.pc_alpha;
        for (int i = 0; i < m; i++) r[i] = 0.0;
        for (int j = 0; j < n; j++) q[j] = 0.0;
        for (int i = 0; i < m; i++)
            for (int64_t e = s->rp[i]; e < s->rp[i + 1]; e++) {
                double a = fabs(s->ahat[e]);
                r[i] += pow(a, 2.0 - al);
                q[s->ci[e]] += pow(a, al);
            }
        for (int i = 0; i < m; i++) r[i] = r[i] > 0.0 ? sqrt(r[i]) : 1.0;
        for (int j = 0; j < n; j++) q[j] = q[j] > 0.0 ? sqrt(q[j]) : 1.0;
        for (int i = 0; i < m; i++)
            for (int64_t e = s->rp[i]; e < s->rp[i + 1]; e++) s->ahat[e] = s->ahat[e] / (r[i] * q[s->ci[e]]);
        for (int i = 0; i < m; i++) s->dr[i] = s->dr[i] / r[i];
        for (int j = 0; j < n; j++) s->dc[j] = s->dc[j] / q[j];
    }
    gather_t(s, s->ahat, s->ahat_t);

    /* power iteration for the largest eigenvalue of Ahat'Ahat */
    double *v = dalloc(n), *w = dalloc(n), *av = dalloc(m);
    {
        csum vs = {0, 0};
        for (int j = 0; j < n; j++) {
            v[j] = 1.0 + or_push_uniform(OR_POWER_SEED, j);
            cadd(&vs, v[j] * v[j]);
        }
        const double nv = sqrt(cval(&vs));
        for (int j = 0; j < n; j++) v[j] = v[j] / nv;
    }
    double lam = 0.0;
    s->power_steps = 0;
    for (int it = 0; it < s->p.power_iters; it++) {
        mv_A(s, s->ahat, v, av);
        mv_At(s, s->ahat_t, av, w);
        csum rs = {0, 0}, ws = {0, 0};
        for (int i = 0; i < m; i++) cadd(&rs, av[i] * av[i]);
        for (int j = 0; j < n; j++) cadd(&ws, w[j] * w[j]);
        double rho = cval(&rs), ww = cval(&ws);
        lam = sqrt(ww);
        s->power_steps = it + 1;
        if (!(lam > 0.0)) break;
        if (sqrt(fmax(ww - rho * rho, 0.0)) <= s->p.power_tol * rho) break;
        for (int j = 0; j < n; j++) v[j] = w[j] / lam;
    }
    s->sigma_est = lam > 0.0 ? sqrt(lam) : 0.0;
    s->eta = s->sigma_est > 1e-12 ? s->p.eta_safety / s->sigma_est : s->p.eta_safety;
    free(v);
    free(w);
    free(av);
    free(r);
    free(q);
}

/* primal weight from the norms of the scaled objective and right-hand side */
static double initial_omega(const double *ch, int n, const double *bh, int m)
{
    double nc = norm2(ch, n), nb = norm2(bh, m);
    if (nc > 1e-10 && nb > 1e-10) return nc / nb;
    return 1.0;
}

/* start (or restart from scratch) the iteration at (x0, y0), scaled */
static void reset_iteration(or_solver *s, int64_t first_check)
{
    memcpy(s->xa, s->x, sizeof(double) * (size_t)s->n);
    memcpy(s->ya, s->y, sizeof(double) * (size_t)s->m);
    memcpy(s->xp, s->x, sizeof(double) * (size_t)s->n);
    memcpy(s->yp, s->y, sizeof(double) * (size_t)s->m);
    s->k = 0;
    s->t = 0;
    s->restarts = 0;
    s->next_check = first_check;
    kkt_scaled_parts(s, s->x, s->y, &s->kkt_anchor_p2, &s->kkt_anchor_d2, &s->kkt_anchor_gap2);
    s->kkt_prev = or_kkt_weighted(s->omega, s->kkt_anchor_p2, s->kkt_anchor_d2, s->kkt_anchor_gap2);
}

or_solver *or_create(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                     const double *val, const double *b, const double *c, const double *l,
                     const double *u, const char *sense, const or_params *params)
{
    if (m < 0 || n < 0 || nnz < 0 || !row_ptr) return NULL;
    if (row_ptr[0] != 0 || row_ptr[m] != nnz) return NULL;
    for (int64_t e = 0; e < nnz; e++)
        if (col[e] < 0 || col[e] >= n || !isfinite(val[e])) return NULL;
    for (int j = 0; j < n; j++) {
        double lo = l ? l[j] : 0.0, hi = u ? u[j] : INFINITY;
        if (isnan(lo) || isnan(hi) || lo > hi || !isfinite(c[j])) return NULL;
    }
    for (int i = 0; i < m; i++) {
        if (!isfinite(b[i])) return NULL;
        if (sense && sense[i] != '=' && sense[i] != '<' && sense[i] != '>') return NULL;
    }
    or_solver *s = (or_solver *)calloc(1, sizeof(or_solver));
    if (!s) return NULL;
    if (params) s->p = *params;
    else set_defaults(&s->p);
    s->m = m;
    s->n = n;
    if (canonical_rows(m, row_ptr, col, val, &s->rp, &s->ci, &s->av, &s->nnz) != 0) {
        or_destroy(s);
        return NULL;
    }
    /* explicit transpose by a stable counting sort over columns */
    s->tp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    s->ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s->nnz > 0 ? s->nnz : 1));
    s->tpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->nnz > 0 ? s->nnz : 1));
    for (int64_t e = 0; e < s->nnz; e++) s->tp[s->ci[e] + 1]++;
    for (int j = 0; j < n; j++) s->tp[j + 1] += s->tp[j];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; j++) cur[j] = s->tp[j];
    for (int i = 0; i < m; i++)
        for (int64_t e = s->rp[i]; e < s->rp[i + 1]; e++) {
            int64_t dst = cur[s->ci[e]]++;
            s->ti[dst] = i;
            s->tpos[dst] = e;
        }
    free(cur);

    s->b = dalloc(m);
    s->c = dalloc(n);
    s->l = dalloc(n);
    s->u = dalloc(n);
    s->sense0 = (char *)malloc((size_t)m + 1);
    s->sense = (char *)malloc((size_t)m + 1);
    for (int i = 0; i < m; i++) {
        s->b[i] = b[i];
        s->sense0[i] = sense ? sense[i] : '=';
    }
    for (int j = 0; j < n; j++) {
        s->c[j] = c[j];
        double lo = l ? l[j] : 0.0, hi = u ? u[j] : INFINITY;
        s->l[j] = lo <= -OR_BIG ? -INFINITY : lo;
        s->u[j] = hi >= OR_BIG ? INFINITY : hi;
    }
    s->ahat = dalloc(s->nnz);
    s->ahat_t = dalloc(s->nnz);
    s->dr = dalloc(m);
    s->dc = dalloc(n);
    s->bh = dalloc(m);
    s->ch = dalloc(n);
    s->lh = dalloc(n);
    s->uh = dalloc(n);
    s->x = dalloc(n);
    s->y = dalloc(m);
    s->xa = dalloc(n);
    s->ya = dalloc(m);
    s->xp = dalloc(n);
    s->yp = dalloc(m);
    s->xbar = dalloc(n);
    s->g = dalloc(n);
    s->hv = dalloc(m);
    s->xs_hat = dalloc(n);
    s->xsol = dalloc(n);
    s->ysol = dalloc(m);
    s->zsol = dalloc(n);
    s->xpush = dalloc(n);
    s->ys_hat = dalloc(m);
    s->ypush = dalloc(m);
    s->zpush = dalloc(n);
    s->cpush = dalloc(n);
    s->lfix = (signed char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (s->p.record_history) {
        s->hx = dalloc(4 * (int64_t)n);
        s->hz = dalloc(4 * (int64_t)n);
    }

    scale_and_step(s);
    for (int i = 0; i < m; i++) {
        s->bh[i] = s->dr[i] * s->b[i];
        s->sense[i] = s->sense0[i];
    }
    for (int j = 0; j < n; j++) {
        s->ch[j] = s->dc[j] * s->c[j];
        s->lh[j] = s->l[j] / s->dc[j];
        s->uh[j] = s->u[j] / s->dc[j];
    }
    s->omega = initial_omega(s->ch, n, s->bh, m);
    for (int j = 0; j < n; j++) s->x[j] = clampd(0.0, s->lh[j], s->uh[j]);
    for (int i = 0; i < m; i++) s->y[i] = 0.0;
    reset_iteration(s, s->p.check_every);
    return s;
}

/* one PDHG step T and the Halpern average with the anchor (scaled space) */
static void pdhg_step(or_solver *s)
{
    int m = s->m, n = s->n;
    double tau = s->eta / s->omega, sig = s->eta * s->omega;
    mv_At(s, s->ahat_t, s->y, s->g);
    for (int j = 0; j < n; j++) {
        s->xp[j] = clampd(s->x[j] - tau * (s->ch[j] - s->g[j]), s->lh[j], s->uh[j]);
        s->xbar[j] = 2.0 * s->xp[j] - s->x[j];
    }
    mv_A(s, s->ahat, s->xbar, s->hv);
    for (int i = 0; i < m; i++) s->yp[i] = proj_dual(s->y[i] + sig * (s->bh[i] - s->hv[i]), s->sense[i]);
    if (s->p.halpern) {
        double kk = (double)s->k;
        double wgt = (kk + 1.0) / (kk + 2.0), wa = 1.0 / (kk + 2.0), gm = s->p.reflect_gamma;
        for (int j = 0; j < n; j++)
            s->x[j] = wgt * ((1.0 + gm) * s->xp[j] - gm * s->x[j]) + wa * s->xa[j];
        for (int i = 0; i < m; i++)
            s->y[i] = wgt * ((1.0 + gm) * s->yp[i] - gm * s->y[i]) + wa * s->ya[i];
    } else {
        memcpy(s->x, s->xp, sizeof(double) * (size_t)n);
        memcpy(s->y, s->yp, sizeof(double) * (size_t)m);
    }
    s->k++;
    s->t++;
}

/* unscaled copies of a scaled primal/dual pair */
static void unscale(const or_solver *s, const double *xh, const double *yh, double *x, double *y)
{
    if (x)
        for (int j = 0; j < s->n; j++) x[j] = s->dc[j] * xh[j];
    if (y)
        for (int i = 0; i < s->m; i++) y[i] = s->dr[i] * yh[i];
}

/* zsplit: the part of the reduced cost lam that finite bounds absorb */
static double zsplit(double lam, double lo, double hi)
{
    double zp = (!is_inf_lo(lo) && lam > 0.0) ? lam : 0.0;
    double zm = (!is_inf_up(hi) && lam < 0.0) ? -lam : 0.0;
    return zp - zm;
}

/* the solve's candidate (x+, y+) at restart number s->restarts, rounded to
 * float32, into slot (restarts - 1) mod 4 of the history */
static void record_history(or_solver *s)
{
    int n = s->n;
    double *aty = dalloc(n);
    mv_At(s, s->ahat_t, s->yp, aty);
    int64_t slot = (s->restarts - 1) % 4;
    for (int j = 0; j < n; j++) {
        s->hx[slot * n + j] = (double)(float)s->xp[j];
        s->hz[slot * n + j] = (double)(float)zsplit(s->ch[j] - aty[j], s->lh[j], s->uh[j]);
    }
    free(aty);
}

/* restart test and primal-weight update at a check; candidate = (xp, yp) */
static void restart_check(or_solver *s)
{
    double p2, d2, g2;
    kkt_scaled_parts(s, s->xp, s->yp, &p2, &d2, &g2);
    double kc = or_kkt_weighted(s->omega, p2, d2, g2);
    double ka = or_kkt_weighted(s->omega, s->kkt_anchor_p2, s->kkt_anchor_d2, s->kkt_anchor_gap2);
    int do_restart = or_restart_decision(&s->p, kc, ka, s->kkt_prev, s->k, s->t);
    s->kkt_prev = kc;
    if (!do_restart) return;
    csum sx = {0, 0}, sy = {0, 0};
    for (int j = 0; j < s->n; j++) cadd(&sx, (s->xp[j] - s->xa[j]) * (s->xp[j] - s->xa[j]));
    for (int i = 0; i < s->m; i++) cadd(&sy, (s->yp[i] - s->ya[i]) * (s->yp[i] - s->ya[i]));
    s->omega = or_weight_update(&s->p, s->omega, sqrt(cval(&sx)), sqrt(cval(&sy)));
    s->restarts++;
    if (!s->in_push && s->p.record_history) record_history(s);
    memcpy(s->x, s->xp, sizeof(double) * (size_t)s->n);
    memcpy(s->xa, s->xp, sizeof(double) * (size_t)s->n);
    memcpy(s->y, s->yp, sizeof(double) * (size_t)s->m);
    memcpy(s->ya, s->yp, sizeof(double) * (size_t)s->m);
    s->kkt_anchor_p2 = p2;
    s->kkt_anchor_d2 = d2;
    s->kkt_anchor_gap2 = g2;
    s->kkt_prev = or_kkt_weighted(s->omega, p2, d2, g2);
    s->k = 0;
}

/* learned warm start, undo rule: a learned fix whose push-model reduced cost
 * (unscaled: the push objective minus A'y of the check's candidate, aty
 * unscaled) has the wrong sign beyond eps_abs goes back to the bounds the
 * plain rule left it (the original ones) */
static void learned_undo(or_solver *s, const double *aty)
{
    double ea = s->p.eps_abs;
    for (int j = 0; j < s->n; j++) {
        if (!s->lfix[j]) continue;
        double lam = s->ch[j] / s->dc[j] - aty[j];
        if ((s->lfix[j] == 1 && lam < -ea) || (s->lfix[j] == 2 && lam > ea)) {
            s->lh[j] = s->l[j] / s->dc[j];
            s->uh[j] = s->u[j] / s->dc[j];
            s->lfix[j] = 0;
            s->n_lundo++;
        }
    }
}

static int all_finite(const double *v, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* run up to `iters` further iterations of the current phase; returns status.
 * Each check evaluates the candidate T(z): termination first, then restart. */
static int run_phase(or_solver *s, int64_t iters, double *out_relp)
{
    int m = s->m, n = s->n;
    double *x = dalloc(n), *y = dalloc(m), *ax = dalloc(m), *aty = dalloc(n);
    int status = OR_ITER_LIMIT;
    for (int64_t it = 0; it < iters; it++) {
        pdhg_step(s);
        if (s->t != s->next_check) continue;
        s->next_check += s->p.check_every;
        if (!all_finite(s->xp, n) || !all_finite(s->yp, m)) {
            status = OR_NUMERICAL;
            break;
        }
        unscale(s, s->xp, s->yp, x, y);
        or_kkt k;
        if (!s->in_push) {
            kkt_unscaled(s, s->c, s->l, s->u, s->sense, x, y, ax, aty, s->zsol, &k);
            memcpy(s->xs_hat, s->xp, sizeof(double) * (size_t)n);
            memcpy(s->ys_hat, s->yp, sizeof(double) * (size_t)m);
            memcpy(s->xsol, x, sizeof(double) * (size_t)n);
            memcpy(s->ysol, y, sizeof(double) * (size_t)m);
            s->solved = 1;
            if (k.rel_p <= s->p.eps_rel && k.rel_d <= s->p.eps_rel && k.rel_gap <= s->p.eps_rel) {
                status = OR_OPTIMAL;
                if (out_relp) *out_relp = k.rel_p;
                break;
            }
        } else if (s->in_push & 2) {
            /* dual residual of the dual push model: its cones (0 or infinite,
               the same scaled and unscaled) decide what the bounds absorb */
            kkt_unscaled(s, s->cpush, s->lh, s->uh, s->sense, x, y, ax, aty, NULL, &k);
            double reld = k.rd2 / (1.0 + norm2(s->c, n));
            for (int i = 0; i < m; i++) s->ypush[i] = s->sense[i] == 'N' ? s->ysol[i] : y[i];
            if (out_relp) *out_relp = reld;
            if (reld <= s->p.eps_rel) {
                status = OR_PUSH_DONE;
                break;
            }
        } else {
            /* primal residual of the push model (its senses), unscaled */
            kkt_unscaled(s, s->c, s->l, s->u, s->sense, x, y, ax, aty, NULL, &k);
            memcpy(s->xpush, x, sizeof(double) * (size_t)n);
            if (out_relp) *out_relp = k.rel_p;
            if (k.rel_p <= s->p.eps_rel) {
                status = OR_PUSH_DONE;
                /* the check's tests saw the model the candidate came from;
                   the undo follows them, at the terminating check too */
                if (s->learned) learned_undo(s, aty);
                break;
            }
        }
        restart_check(s);
        if (s->in_push == 1 && s->learned) learned_undo(s, aty);
    }
    free(x);
    free(y);
    free(ax);
    free(aty);
    return status;
}

static void fill_result(const or_solver *s, int status, or_result *r)
{
    double *ax = dalloc(s->m), *aty = dalloc(s->n);
    or_kkt k;
    kkt_unscaled(s, s->c, s->l, s->u, s->sense0, s->xsol, s->ysol, ax, aty, NULL, &k);
    r->status = status;
    r->iters = s->t;
    r->restarts = s->restarts;
    r->rel_p = k.rel_p;
    r->rel_d = k.rel_d;
    r->rel_gap = k.rel_gap;
    r->pobj = k.pobj;
    r->dobj = k.dobj;
    free(ax);
    free(aty);
}

/* exactly `iters` more iterations of the solve (fewer if it terminates) */
int or_iterate(or_solver *s, int64_t iters, or_result *r)
{
    if (!s || s->in_push) return OR_ERR_STATE;
    int st = run_phase(s, iters, NULL);
    if (!s->solved) { /* no check yet: report the current iterate */
        or_kkt k;
        double *ax = dalloc(s->m), *aty = dalloc(s->n);
        unscale(s, s->x, s->y, s->xsol, s->ysol);
        memcpy(s->xs_hat, s->x, sizeof(double) * (size_t)s->n);
        memcpy(s->ys_hat, s->y, sizeof(double) * (size_t)s->m);
        kkt_unscaled(s, s->c, s->l, s->u, s->sense0, s->xsol, s->ysol, ax, aty, s->zsol, &k);
        free(ax);
        free(aty);
    }
    if (r) fill_result(s, st, r);
    return st;
}

int or_solve(or_solver *s, or_result *r)
{
    if (!s || s->in_push) return OR_ERR_STATE;
    int64_t left = s->p.max_iter - s->t;
    return or_iterate(s, left > 0 ? left : 0, r);
}

/* reduced costs z of the original model at y (unscaled), section 2 split */
static void reduced_costs(const or_solver *s, const double *x, const double *y, double *z, double *ax,
                          or_kkt *k)
{
    double *aty = dalloc(s->n);
    kkt_unscaled(s, s->c, s->l, s->u, s->sense0, x, y, ax, aty, z, k);
    free(aty);
}

/* learned warm start, fixes at the push start (after the plain rule): a
 * column the plain rule leaves free (|z_j| <= eps_abs) whose logit is at
 * least logit(theta) (the comparison in float32, the predictor's precision)
 * is fixed at its nearer finite bound (distances to the scaled bounds, a tie
 * going to the lower one) when the sign of z_j allows that bound (z_j >=
 * -eps_abs at the lower, z_j <= eps_abs at the upper); the push starts with
 * x_j at that bound.  A column with no finite bound is left free. */
static void learned_fix(or_solver *s, const float *logits, double theta)
{
    const float tl = (float)log(theta / (1.0 - theta));
    double ea = s->p.eps_abs;
    s->n_lfix = 0;
    s->n_lundo = 0;
    for (int j = 0; j < s->n; j++) {
        s->lfix[j] = 0;
        if (fabs(s->zsol[j]) > ea || !(logits[j] >= tl)) continue;
        double lo = s->l[j] / s->dc[j], hi = s->u[j] / s->dc[j], xv = s->xs_hat[j];
        double dl = is_inf_lo(lo) ? INFINITY : xv - lo;
        double du = is_inf_up(hi) ? INFINITY : hi - xv;
        if (isinf(dl) && isinf(du)) continue;
        if (dl <= du) {
            if (s->zsol[j] < -ea) continue;
            s->lh[j] = s->uh[j] = s->x[j] = lo;
            s->lfix[j] = 1;
        } else {
            if (s->zsol[j] > ea) continue;
            s->lh[j] = s->uh[j] = s->x[j] = hi;
            s->lfix[j] = 2;
        }
        s->n_lfix++;
    }
}

/* Algorithm 1 with implicit slacks, modified in place, continued by PDHG;
 * with logits, the learned warm start on top of the plain rule */
static int corner_push_impl(or_solver *s, uint64_t seed, or_push_result *r, const float *logits, double theta)
{
    if (!s || !s->solved || s->in_push) return OR_ERR_STATE;
    int m = s->m, n = s->n;
    double *ax = dalloc(m);
    memset(r, 0, sizeof(*r));
    /* CP1: (x, y, z) of the solve on M */
    reduced_costs(s, s->xsol, s->ysol, s->zsol, ax, &r->before);
    corner_counts(s, s->xsol, ax, s->ysol, s->zsol, &r->before);
    if (s->p.push_gate &&
        (double)r->before.candidates < fmax(s->p.push_gate_rows * (double)m, (double)s->p.push_gate_min)) {
        /* too few candidates: no push, the solve's point is the answer */
        r->status = OR_PUSH_SKIPPED;
        r->rel_p_push = NAN;
        r->after = r->before;
        memcpy(s->xpush, s->xsol, sizeof(double) * (size_t)n);
        s->in_push = 1;
        free(ax);
        return OR_PUSH_SKIPPED;
    }
    double ea = s->p.eps_abs;
    /* CP2: bounds (stored scaled: the scaled candidate itself) */
    for (int j = 0; j < n; j++) {
        if (s->zsol[j] > ea) { s->uh[j] = s->xs_hat[j]; r->n_fix_upper++; }
        else if (s->zsol[j] < -ea) { s->lh[j] = s->xs_hat[j]; r->n_fix_lower++; }
    }
    /* CP3: inequality rows whose slack has a non-trivial reduced cost */
    for (int i = 0; i < m; i++) {
        if ((s->sense[i] == '<' && s->ysol[i] < -ea) || (s->sense[i] == '>' && s->ysol[i] > ea)) {
            s->sense[i] = '=';
            r->n_rows_to_eq++;
        }
    }
    /* CP4: random objective Uniform[0,1)^n, scaled like c */
    for (int j = 0; j < n; j++) s->ch[j] = s->dc[j] * (s->p.push_obj_scale * or_push_uniform(seed, j));
    /* CP5: start from (x, 0); keep scaling and eta; new weight and restart state */
    memcpy(s->x, s->xs_hat, sizeof(double) * (size_t)n);
    for (int i = 0; i < m; i++) s->y[i] = 0.0;
    s->learned = logits != NULL;
    if (logits) learned_fix(s, logits, theta);
    s->omega = initial_omega(s->ch, n, s->bh, m);
    s->in_push = 1;
    reset_iteration(s, s->p.push_min_iters);
    memcpy(s->xpush, s->xsol, sizeof(double) * (size_t)n);
    /* CP6 */
    double relp = NAN;
    int st = run_phase(s, s->p.push_max_iter, &relp);
    r->status = st;
    r->iters = s->t;
    r->restarts = s->restarts;
    r->rel_p_push = relp;
    /* CP7: (xhat, y, z); counts after against the original model */
    double *z2 = dalloc(n);
    reduced_costs(s, s->xpush, s->ysol, z2, ax, &r->after);
    corner_counts(s, s->xpush, ax, s->ysol, s->zsol, &r->after);
    r->n_learned_fix = s->learned ? s->n_lfix : 0;
    r->n_learned_undo = s->learned ? s->n_lundo : 0;
    s->learned = 0;
    free(z2);
    free(ax);
    return st;
}

int or_corner_push(or_solver *s, uint64_t seed, or_push_result *r)
{
    return corner_push_impl(s, seed, r, NULL, -1.0);
}

/* the corner push with the learned warm start from per-column logits (n
 * float32 values: the predictor's output on the solve's state) */
int or_corner_push_learned(or_solver *s, const float *logits, double theta, uint64_t seed, or_push_result *r)
{
    if (!logits || !(theta > 0.0 && theta < 1.0)) return OR_ERR_ARG;
    return corner_push_impl(s, seed, r, logits, theta);
}

/* The 16 features of the learned warm start for every column of a solved LP
 * (before its push), on the scaled model at the solve's last checked
 * candidate (x+, y+), z = the bound-absorbed part of c - A'y+:
 *   0..3   x_j, z_j, |c_j|, ||A_{:,j}||_2;
 *   4..7   x_j at the last, second-last, ... 4th-last restart minus x_j (0
 *          where fewer restarts happened or no history was kept);
 *   8..11  the same for z_j;
 *   12     the push objective coefficient of column j for the push seed;
 *   13, 14 x_j - l_j and u_j - x_j (-1 where that bound is infinite);
 *   15     (x_j - l_j) / (u_j - l_j) where both bounds are finite and
 *          distinct, else -1;
 * a non-finite value counts as 0.  Each feature v is then mapped to
 * sign(v) ln(1 + |v| / s), s the root mean square of that feature over the
 * LP's columns (1 if it is 0).  out is n x 16, row j = column j; scale
 * (16 values, or NULL) receives the s of each feature. */
int or_features(or_solver *s, uint64_t seed, double *out, double *scale)
{
    if (!s || !out) return OR_ERR_ARG;
    if (!s->solved || s->in_push) return OR_ERR_STATE;
    int n = s->n;
    double *aty = dalloc(n);
    mv_At(s, s->ahat_t, s->ys_hat, aty);
    int64_t rest = s->restarts, have = rest < 4 ? rest : 4;
    double sq[16];
    for (int q = 0; q < 16; q++) sq[q] = 0.0;
    for (int j = 0; j < n; j++) {
        double v[16];
        double xj = s->xs_hat[j];
        double zj = zsplit(s->ch[j] - aty[j], s->lh[j], s->uh[j]);
        double cn = 0.0;
        for (int64_t e = s->tp[j]; e < s->tp[j + 1]; e++) cn += s->ahat_t[e] * s->ahat_t[e];
        v[0] = xj;
        v[1] = zj;
        v[2] = fabs(s->ch[j]);
        v[3] = sqrt(cn);
        for (int k = 1; k <= 4; k++) {
            int use = k <= have && s->hx;
            int64_t slot = use ? (rest - k) % 4 : 0;
            v[3 + k] = use ? s->hx[slot * n + j] - xj : 0.0;
            v[7 + k] = use ? s->hz[slot * n + j] - zj : 0.0;
        }
        double lo = s->lh[j], hi = s->uh[j];
        int flo = !is_inf_lo(lo), fhi = !is_inf_up(hi);
        v[12] = s->dc[j] * (s->p.push_obj_scale * or_push_uniform(seed, j));
        v[13] = flo ? xj - lo : -1.0;
        v[14] = fhi ? hi - xj : -1.0;
        v[15] = (flo && fhi && hi > lo) ? (xj - lo) / (hi - lo) : -1.0;
        for (int q = 0; q < 16; q++) {
            if (!isfinite(v[q])) v[q] = 0.0;
            out[(int64_t)j * 16 + q] = v[q];
            sq[q] += v[q] * v[q];
        }
    }
    for (int q = 0; q < 16; q++) {
        double rms = n > 0 ? sqrt(sq[q] / n) : 0.0;
        double sc = rms > 0.0 ? rms : 1.0;
        if (scale) scale[q] = sc;
        for (int j = 0; j < n; j++) {
            double v = out[(int64_t)j * 16 + q];
            double t = log1p(fabs(v) / sc);
            out[(int64_t)j * 16 + q] = v < 0.0 ? -t : t;
        }
    }
    free(aty);
    return 0;
}

/* Dual corner push (reading in the file header).  Runs once, after the solve
 * or after the corner push; in the second case its face is that of the
 * pushed xhat, and (xhat, yhat, zhat) is returned. */
int or_dual_push(or_solver *s, uint64_t seed, or_dual_push_result *r)
{
    if (!s || !r || !s->solved || (s->in_push & 2)) return OR_ERR_STATE;
    int m = s->m, n = s->n;
    double *ax = dalloc(m);
    /* x: the solve's, or the corner push's xhat when that push came first */
    const double *xk = (s->in_push & 1) ? s->xpush : s->xsol;
    memset(r, 0, sizeof(*r));
    /* DP1: (x, y, z) on M, y and z the solve's; ax = A x */
    reduced_costs(s, xk, s->ysol, s->zsol, ax, &r->before);
    corner_counts(s, xk, ax, s->ysol, s->zsol, &r->before);
    double ea = s->p.eps_abs, sc = s->p.push_obj_scale;
    double *w0 = dalloc(n), *aw = dalloc(m), *yn = dalloc(m), *atyn = dalloc(n), *aty = dalloc(n);
    double *tv = dalloc(s->nnz);
    gather_t(s, s->av, tv);
    /* DP3: rows with slack beyond eps_abs leave the push model, their dual
       fixed at the solve's value */
    for (int i = 0; i < m; i++) {
        char sn = s->sense0[i];
        double slack = sn == '<' ? s->b[i] - ax[i] : (sn == '>' ? ax[i] - s->b[i] : 0.0);
        int drop = sn != '=' && slack > ea;
        s->sense[i] = drop ? 'N' : sn;
        yn[i] = drop ? s->ysol[i] : 0.0;
        r->n_rows_fixed += drop;
    }
    mv_At(s, tv, s->ysol, aty); /* A'ybar */
    mv_At(s, tv, yn, atyn);     /* A_N'ybar_N */
    /* DP2: the cone of each push column from where x sits against its bounds,
       the objective c~ = c - A_N'ybar_N - r, and the anchor point w0 */
    for (int j = 0; j < n; j++) {
        int at_lo = !is_inf_lo(s->l[j]) && xk[j] - s->l[j] <= ea;
        int at_up = !is_inf_up(s->u[j]) && s->u[j] - xk[j] <= ea;
        s->lh[j] = at_lo ? 0.0 : -INFINITY;
        s->uh[j] = at_up ? 0.0 : INFINITY;
        if (!at_lo && !at_up) r->n_cols_free++;
        double lam = s->c[j] - aty[j];
        double rj = (at_lo && at_up) ? 0.0 : at_lo ? fmin(lam, 0.0) : at_up ? fmax(lam, 0.0) : lam;
        s->cpush[j] = s->c[j] - atyn[j] - rj;
        s->ch[j] = s->dc[j] * s->cpush[j];
        double uj = or_push_uniform(seed, j);
        w0[j] = (at_lo && at_up) ? 0.0 : (at_up ? -uj : uj);
        s->x[j] = 0.0; /* DP5: w = 0 */
    }
    mv_A(s, s->av, w0, aw);
    /* DP4: the anchored random right-hand side (scaled like b) on the rows
       kept; y starts at the solve's there (and is 0 on dropped rows) */
    for (int i = 0; i < m; i++) {
        char sn = s->sense[i];
        if (sn == 'N') {
            s->bh[i] = 0.0;
            s->y[i] = 0.0;
        } else {
            double v = or_push_uniform(seed, (int64_t)n + i);
            double g = sn == '>' ? aw[i] - v : (sn == '<' ? aw[i] + v : aw[i]);
            s->bh[i] = s->dr[i] * (sc * g);
            s->y[i] = s->ys_hat[i];
        }
    }
    free(w0);
    free(aw);
    free(yn);
    free(atyn);
    free(aty);
    free(tv);
    /* DP5: new weight and restart state */
    s->omega = initial_omega(s->ch, n, s->bh, m);
    s->in_push |= 2;
    reset_iteration(s, s->p.push_min_iters);
    memcpy(s->ypush, s->ysol, sizeof(double) * (size_t)m);
    /* DP6 */
    double reld = NAN;
    int st = run_phase(s, s->p.push_max_iter, &reld);
    r->status = st;
    r->iters = s->t;
    r->restarts = s->restarts;
    r->rel_d_push = reld;
    /* DP7: (x, yhat, zhat), counts against the original model */
    reduced_costs(s, xk, s->ypush, s->zpush, ax, &r->after);
    corner_counts(s, xk, ax, s->ypush, s->zpush, &r->after);
    free(ax);
    return st;
}

/* KKT report of (x, y) on the original model M (unscaled host vectors) */
int or_kkt_report(or_solver *s, const double *x, const double *y, or_kkt *k)
{
    if (!s || !k) return OR_ERR_ARG;
    const double *xx = x ? x : ((s->in_push & 1) ? s->xpush : s->xsol);
    const double *yy = y ? y : ((s->in_push & 2) ? s->ypush : s->ysol);
    double *ax = dalloc(s->m), *z = dalloc(s->n);
    reduced_costs(s, xx, yy, z, ax, k);
    corner_counts(s, xx, ax, yy, z, k);
    free(ax);
    free(z);
    return 0;
}

/* ---- accessors (unscaled unless stated) ---------------------------------- */
void or_get_iterate(const or_solver *s, double *x, double *y) { unscale(s, s->x, s->y, x, y); }
void or_get_iterate_scaled(const or_solver *s, double *x, double *y)
{
    if (x) memcpy(x, s->x, sizeof(double) * (size_t)s->n);
    if (y) memcpy(y, s->y, sizeof(double) * (size_t)s->m);
}
void or_get_solution(const or_solver *s, double *x, double *y, double *z)
{
    /* after a dual push: the solve's x, the pushed y and its reduced costs */
    const int dual = (s->in_push & 2) != 0;
    if (x) memcpy(x, (s->in_push & 1) ? s->xpush : s->xsol, sizeof(double) * (size_t)s->n);
    if (y) memcpy(y, dual ? s->ypush : s->ysol, sizeof(double) * (size_t)s->m);
    if (z) memcpy(z, dual ? s->zpush : s->zsol, sizeof(double) * (size_t)s->n);
}
void or_get_scaling(const or_solver *s, double *dr, double *dc, double *out5)
{
    if (dr) memcpy(dr, s->dr, sizeof(double) * (size_t)s->m);
    if (dc) memcpy(dc, s->dc, sizeof(double) * (size_t)s->n);
    if (out5) {
        out5[0] = s->eta;
        out5[1] = s->omega;
        out5[2] = s->sigma_est;
        out5[3] = (double)s->t;
        out5[4] = (double)s->power_steps;
    }
}
/* scaled right-hand side of the current phase */
void or_get_rhs_scaled(const or_solver *s, double *bh)
{
    if (bh) memcpy(bh, s->bh, sizeof(double) * (size_t)s->m);
}
/* scaled model of the current phase (bounds, objective, senses) */
void or_get_model_scaled(const or_solver *s, double *lh, double *uh, double *ch, char *sense)
{
    if (lh) memcpy(lh, s->lh, sizeof(double) * (size_t)s->n);
    if (uh) memcpy(uh, s->uh, sizeof(double) * (size_t)s->n);
    if (ch) memcpy(ch, s->ch, sizeof(double) * (size_t)s->n);
    if (sense) memcpy(sense, s->sense, (size_t)s->m);
}
/* scaled matrix values in canonical row order (sorted, summed rows) */
int64_t or_get_nnz(const or_solver *s) { return s->nnz; }
void or_get_ahat(const or_solver *s, int64_t *rp, int32_t *ci, double *v)
{
    if (rp) memcpy(rp, s->rp, sizeof(int64_t) * ((size_t)s->m + 1));
    if (ci) memcpy(ci, s->ci, sizeof(int32_t) * (size_t)s->nnz);
    if (v) memcpy(v, s->ahat, sizeof(double) * (size_t)s->nnz);
}
#ifdef _OPENMP
#include <omp.h>
#endif
/* threads the row-parallel products use */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
/* thread count of the row-parallel products (the CPU leg's 1-thread timing) */
void or_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
int or_params_size(void) { return (int)sizeof(or_params); }
int or_kkt_size(void) { return (int)sizeof(or_kkt); }
int or_push_result_size(void) { return (int)sizeof(or_push_result); }
int or_dual_push_result_size(void) { return (int)sizeof(or_dual_push_result); }
