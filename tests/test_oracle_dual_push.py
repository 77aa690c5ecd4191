"""Pins of the oracle's dual corner push.

Section 6 of the paper names the idea (cut dual superbasics the way the push of
Algorithm 1 cuts primal ones) and nothing more.  The reading implemented here
restricts (y, z) to the dual optimal face that complementary slackness with the
solve's x defines, and maximises an anchored random objective over it with
PDHG.  These tests pin that reading against things other than the oracle:
* the face itself, checked with HiGHS: every maximiser of a random objective
  over it is dual optimal for the original LP;
* a closed form: on a degenerate 2-column LP the face is a segment whose end
  points are known, and the converged push lands on the one the objective picks;
* HiGHS's maximiser of the push objective over the face, on random degenerate LPs;
* invariants: x unchanged, y dual feasible and optimal, the dual superbasic
  estimate max(m - #zero reduced costs, 0) driven to 0 on planted degenerate LPs.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import lp_ref
from oracle import OracleSolver, push_uniform
from paper_2511_13894_amd import lpgen


def _face_bounds(lp, x, eps_abs):
    """Row cones and reduced-cost sign rules of the dual face at x (complementary slackness)."""
    a = lp.dense()
    ax = a @ x
    sense = [chr(v) for v in np.asarray(lp.sense, dtype=np.uint8)]
    yb = []
    for i, sn in enumerate(sense):
        slack = lp.b[i] - ax[i] if sn == "<" else (ax[i] - lp.b[i] if sn == ">" else 0.0)
        if sn != "=" and slack > eps_abs:
            yb.append((0.0, 0.0))
        elif sn == "<":
            yb.append((None, 0.0))
        elif sn == ">":
            yb.append((0.0, None))
        else:
            yb.append((None, None))
    at_lo = np.isfinite(lp.l) & (x - lp.l <= eps_abs)
    at_up = np.isfinite(lp.u) & (lp.u - x <= eps_abs)
    return a, yb, at_lo, at_up


def face_argmax(lp, x, g, eps_abs=1e-6):
    """HiGHS: maximise g'y over the dual face at x (z = c - A'y: 0 off both
    bounds, >= 0 at the lower bound only, <= 0 at the upper bound only)."""
    a, yb, at_lo, at_up = _face_bounds(lp, x, eps_abs)
    free = ~at_lo & ~at_up
    lo_only = at_lo & ~at_up
    up_only = at_up & ~at_lo
    a_ub = np.vstack([a[:, lo_only].T, -a[:, up_only].T])
    b_ub = np.concatenate([lp.c[lo_only], -lp.c[up_only]])
    res = linprog(-g, A_ub=a_ub if a_ub.size else None, b_ub=b_ub if a_ub.size else None,
                  A_eq=a[:, free].T if free.any() else None, b_eq=lp.c[free] if free.any() else None,
                  bounds=yb, method="highs")
    assert res.status == 0, res.message
    return res.x


def dual_objective(lp, y):
    """b'y + l'z+ - u'z- with z = c - A'y split by the finite bounds (section 2)."""
    lam = lp.c - lp.dense().T @ y
    zp = np.where(np.isfinite(lp.l) & (lam > 0), lam, 0.0)
    zm = np.where(np.isfinite(lp.u) & (lam < 0), -lam, 0.0)
    lf = np.where(np.isfinite(lp.l), lp.l, 0.0)
    uf = np.where(np.isfinite(lp.u), lp.u, 0.0)
    return lp.b @ y + (lf * zp).sum() - (uf * zm).sum()


def anchored_rhs(lp, x, seed, eps_abs=1e-6, scale=1.0):
    """g = scale (A w0 - s.v): w0_j = U_j in the column's cone, v_i = U_(n+i) a slack on inequality rows."""
    a, yb, at_lo, at_up = _face_bounds(lp, x, eps_abs)
    u = np.array([push_uniform(seed, j) for j in range(lp.n + lp.m)])
    w0 = np.where(at_lo & at_up, 0.0, np.where(at_up & ~at_lo, -u[: lp.n], u[: lp.n]))
    sense = np.asarray(lp.sense, dtype=np.uint8)
    s = np.where(sense == ord(">"), 1.0, np.where(sense == ord("<"), -1.0, 0.0))
    g = scale * (a @ w0 - s * u[lp.n:])
    dropped = np.array([b == (0.0, 0.0) for b in yb])
    g[dropped] = 0.0
    return g


@pytest.mark.parametrize("seed", range(5))
def test_every_point_of_the_dual_push_face_is_dual_optimal(seed):
    """Mirror of the lemma behind Algorithm 1: the dual push model's feasible
    set (its face, built from the oracle's own push cones and senses) holds only
    dual optimal points; HiGHS maximises random objectives over it and every
    maximiser has the original optimal objective."""
    lp = lpgen.tiny(300 + seed, m=4, n=9)
    opt, _ = lp_ref.highs(lp)
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_max_iter=1)
    s.solve()
    x = s.solution()[0]
    pr = s.dual_push(seed)
    lh, uh, _, sense = s.model_scaled()
    # the oracle's push model is the face of complementary slackness at x
    a, yb, at_lo, at_up = _face_bounds(lp, x, 1e-6)
    np.testing.assert_array_equal(lh == 0.0, at_lo)
    np.testing.assert_array_equal(uh == 0.0, at_up)
    assert np.all(np.isinf(lh[~at_lo])) and np.all(np.isinf(uh[~at_up]))
    np.testing.assert_array_equal(np.frombuffer(sense, dtype=np.uint8) == ord("N"),
                                  np.array([b == (0.0, 0.0) for b in yb]))
    assert pr.n_cols_free == int((~at_lo & ~at_up).sum())
    rng = np.random.default_rng(seed)
    for _ in range(6):
        y = face_argmax(lp, x, rng.standard_normal(lp.m))
        assert abs(dual_objective(lp, y) - opt) <= 1e-7 * (1 + abs(opt))


def test_converged_dual_push_lands_on_the_closed_form_vertex():
    """min x1 + x2 s.t. x1 + 2 x2 >= 1, 2 x1 + x2 >= 1, x1 + x2 >= 2/3, x >= 0:
    x* = (1/3, 1/3) with all three rows active (primal degenerate).  Both columns
    are off their bounds, so the dual face is y = (t, t, 1 - 3t), t in [0, 1/3],
    and g'y = g3 + t (g1 + g2 - 3 g3) picks t = 1/3 or t = 0 by its sign."""
    lp = lpgen.from_dense([[1, 2], [2, 1], [1, 1]], [1, 1, 2 / 3], [1, 1], [0, 0], [np.inf, np.inf], ">>>")
    for seed in range(6):
        s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=20000)
        s.solve()
        x0, y0, _ = s.solution()
        np.testing.assert_allclose(x0, [1 / 3, 1 / 3], atol=1e-8)
        pr = s.dual_push(seed)
        assert pr.status == 3
        x1, y1, z1 = s.solution()
        np.testing.assert_array_equal(x1, x0)
        g = anchored_rhs(lp, x0, seed)
        # the oracle's right-hand side is the anchored one, scaled like b
        np.testing.assert_allclose(s.rhs_scaled() / s.scaling()["dr"], g, rtol=1e-13)
        t = 1 / 3 if g[0] + g[1] - 3 * g[2] > 0 else 0.0
        np.testing.assert_allclose(y1, [t, t, 1 - 3 * t], atol=1e-6)
        assert pr.after.est_dual == 0 and pr.before.est_dual == 1


@pytest.mark.parametrize("seed", range(4))
def test_converged_dual_push_matches_highs_on_the_face(seed):
    """Random primal-degenerate LPs: driven to convergence, the pushed y is
    HiGHS's maximiser of the same anchored objective over the same face."""
    lp = lpgen.planted(12, 30, seed=40 + seed, zero_frac=0.8, degen_frac=0.0, ineq_frac=0.25)
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=60000)
    s.solve()
    x0 = s.solution()[0]
    pr = s.dual_push(7)
    assert pr.status == 3
    y1 = s.solution()[1]
    want = face_argmax(lp, x0, anchored_rhs(lp, x0, 7))
    np.testing.assert_allclose(y1, want, atol=1e-5 * (1 + np.abs(want).max()))


@pytest.mark.parametrize("name,make", [
    ("free_columns_10x30", lambda: lpgen.tiny(209, m=10, n=30, with_free=True)),
    ("upper_bounds_ineq_14x40",
     lambda: lpgen.planted(14, 40, seed=77, zero_frac=0.75, degen_frac=0.0, ineq_frac=0.4, upper_frac=0.3)),
    ("transport_4x5", lambda: lpgen.transportation(4, 5, seed=6)),
], ids=["free_columns_10x30", "upper_bounds_ineq_14x40", "transport_4x5"])
def test_converged_dual_push_reaches_highs_optimum_on_the_face(name, make):
    """Driven to convergence, the push attains HiGHS's optimal value of the
    anchored objective over the face, and its reduced costs A'y are HiGHS's.
    A transportation LP's face contains a line (dependent equality rows), so
    its maximiser is unique only up to that line: the value and A'y are."""
    lp = make()
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=60000)
    s.solve()
    x0 = s.solution()[0]
    pr = s.dual_push(11)
    assert pr.status == 3
    y1 = s.solution()[1]
    g = anchored_rhs(lp, x0, 11)
    want = face_argmax(lp, x0, g)
    a = lp.dense()
    assert abs(g @ y1 - g @ want) <= 1e-6 * (1 + abs(g @ want)), (g @ y1, g @ want)
    np.testing.assert_allclose(a.T @ y1, a.T @ want, atol=1e-5 * (1 + np.abs(a.T @ want).max()))


@pytest.mark.parametrize("eps,max_after", [(1e-8, 0), (1e-6, None)])
def test_dual_push_removes_dual_superbasics_on_planted_degenerate_lps(eps, max_after):
    """Planted optimum with 100 of 500 columns off their bounds and m = 200 rows:
    the dual optimal face has dimension >= 100 and the solve lands inside it.
    The push keeps x, keeps y dual feasible and optimal, and cuts the estimate
    max(m - #zero reduced costs, 0); at eps 1e-8 to zero (a dual vertex)."""
    lp = lpgen.planted(200, 500, seed=1, zero_frac=0.8, degen_frac=0.0)
    s = OracleSolver(lp, eps_rel=eps, max_iter=400000)
    r = s.solve()
    assert r.status == 0
    x0, y0, z0 = s.solution()
    pr = s.dual_push(5)
    assert pr.status == 3 and pr.iters >= 100
    assert pr.rel_d_push <= eps
    x1, y1, z1 = s.solution()
    np.testing.assert_array_equal(x1, x0)
    k = s.kkt(x1, y1)
    assert k.rel_d <= 2 * eps and k.rel_gap <= 10 * eps
    assert pr.n_cols_free == 100 and pr.n_rows_fixed == 0
    assert pr.before.est_dual >= 80
    assert pr.after.est_dual < pr.before.est_dual / 2
    if max_after is not None:
        assert pr.after.est_dual <= max_after
    # on an off-bound column the push model's dual residual is the whole
    # reduced cost, so the stop test bounds them: ||z_off|| <= rel_d (1 + ||c||)
    off = (x0 - lp.l > 1e-6) & (lp.u - x0 > 1e-6)
    assert np.linalg.norm(z1[off]) <= pr.rel_d_push * (1 + np.linalg.norm(lp.c)) * (1 + 1e-9)


def test_dual_push_is_bounded_with_dependent_equality_rows():
    """A transportation LP's equality rows are dependent (A'd = 0 for d = +1 on
    sources, -1 on sinks): an unanchored random objective would be unbounded on
    the face; the anchored one stops, with the solve's optimal objective."""
    lp = lpgen.transportation(12, 30, seed=3)
    opt, _ = lp_ref.highs(lp)
    s = OracleSolver(lp, eps_rel=1e-8, max_iter=400000)
    s.solve()
    pr = s.dual_push(5)
    assert pr.status == 3
    x1, y1, _ = s.solution()
    assert abs(dual_objective(lp, y1) - opt) <= 1e-6 * (1 + abs(opt))


def test_dual_push_after_the_corner_push_works_from_xhat():
    """Crossover's order, primal phase first: after Algorithm 1 the dual push
    takes its face from the pushed xhat (its column cones are xhat's), keeps
    xhat, and cuts the dual superbasic estimate of (xhat, y) to zero; the
    pair stays primal and dual feasible with a vanishing gap."""
    lp = lpgen.planted(300, 900, seed=2, zero_frac=0.85, degen_frac=0.0, ineq_frac=0.3, upper_frac=0.2)
    s = OracleSolver(lp, eps_rel=1e-8, max_iter=400000)
    s.solve()
    pp = s.corner_push(3)
    assert pp.status == 3
    xh, y0, _ = s.solution()
    pd = s.dual_push(5)
    assert pd.status == 3
    x2, y2, z2 = s.solution()
    np.testing.assert_array_equal(x2, xh)
    lh, uh, _, _ = s.model_scaled()
    _, _, at_lo, at_up = _face_bounds(lp, xh, 1e-6)
    np.testing.assert_array_equal(lh == 0.0, at_lo)
    np.testing.assert_array_equal(uh == 0.0, at_up)
    assert pd.before.est_dual > 50 and pd.after.est_dual == 0
    k = s.kkt(x2, y2)
    assert k.rel_p <= 1e-8 and k.rel_d <= 2e-8 and k.rel_gap <= 1e-6


def test_dual_push_edge_cases_fixed_and_empty():
    """A fixed column (l = u: both bounds, so z free and w in {0}), an empty
    column (at its lower bound: w >= 0), an empty '<' row and a loose '>' row
    (both dropped, y held at 0): the push keeps HiGHS's optimal objective."""
    lp = lpgen.from_dense([[1, 1, 0, 1], [0, 0, 0, 0], [1, -1, 0, 2]], [3, 5, 1], [1, 2, 3, 0.5], [0, 0, 0, 1],
                          [np.inf, np.inf, np.inf, 1], "=<>")
    opt, _ = lp_ref.highs(lp)
    s = OracleSolver(lp, eps_rel=1e-8, max_iter=400000)
    s.solve()
    pd = s.dual_push(3)
    assert pd.status == 3 and pd.n_cols_free == 1 and pd.n_rows_fixed == 2
    lh, uh, _, sense = s.model_scaled()
    assert sense == b"=NN"
    np.testing.assert_array_equal(lh, [-np.inf, 0.0, 0.0, 0.0])
    np.testing.assert_array_equal(uh, [np.inf, np.inf, np.inf, 0.0])
    x, y, z = s.solution()
    assert y[1] == 0.0 and y[2] == 0.0
    assert abs(dual_objective(lp, y) - opt) <= 1e-7 * (1 + abs(opt))


def test_push_order_rules():
    """One dual push per solve, after the solve or after the corner push; no
    corner push after a dual push."""
    lp = lpgen.config0(0)
    s = OracleSolver(lp, eps_rel=1e-6)
    with pytest.raises(RuntimeError):
        s.dual_push(1)
    s.solve()
    s.dual_push(1)
    with pytest.raises(RuntimeError):
        s.dual_push(1)
    with pytest.raises(RuntimeError):
        s.corner_push(1)
    s2 = OracleSolver(lp, eps_rel=1e-6)
    s2.solve()
    s2.corner_push(1)
    s2.dual_push(1)
    with pytest.raises(RuntimeError):
        s2.dual_push(1)
