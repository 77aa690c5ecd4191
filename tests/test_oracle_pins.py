"""Pins of the CPU reference against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
numbers (tests/golden), brute-force vertex enumeration, a planted optimum, an
independent LP solver (HiGHS), closed forms, and invariants of the method.
"""
import json
import os

import numpy as np
import pytest

import lp_ref
from oracle import OracleSolver, push_uniform, splitmix64
from paper_2511_13894_amd import lpgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lp_from_case(case):
    inf = np.inf
    l = [(-inf if v is None else v) for v in case["l"]]
    u = [(inf if v is None else v) for v in case["u"]]
    return lpgen.from_dense(case["A"], case["b"], case["c"], l, u, case["sense"], name=case["name"])


# ---------------------------------------------------------------- formulas --
@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "kkt_hand.json")))["cases"],
                         ids=lambda c: c["name"])
def test_kkt_report_matches_hand_values(case):
    """Residuals, objectives, relative tests and corner counts (section 2, 2.1, 4.2)."""
    lp = _lp_from_case(case)
    s = OracleSolver(lp)
    k = s.kkt(np.array(case["x"], float), np.array(case["y"], float)).as_dict()
    for key, want in case["expect"].items():
        assert k[key] == pytest.approx(want, rel=1e-12, abs=1e-14), key


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "lps_hand.json")))["cases"],
                         ids=lambda c: c["name"])
def test_hand_solved_lps(case):
    lp = _lp_from_case(case)
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=200000)
    r = s.solve()
    assert r.status == 0
    x, y, z = s.solution()
    assert r.pobj == pytest.approx(case["opt"], abs=1e-7)
    if case.get("x") is not None:
        np.testing.assert_allclose(x, case["x"], atol=1e-6)
    np.testing.assert_allclose(y, case["y"], atol=1e-6)
    if case.get("z") is not None:
        k = s.kkt()
        zz = lp.c - lp.dense().T @ y
        np.testing.assert_allclose(zz, case["z"], atol=1e-6)
        assert k.rd2 < 1e-8


# ---------------------------------------------------------- brute force -----
@pytest.mark.parametrize("seed", range(12))
def test_tiny_lps_vs_vertex_enumeration(seed):
    """Optimal objective of general-form tiny LPs equals the best vertex."""
    lp = lpgen.tiny(seed, m=3, n=6)
    opt, _ = lp_ref.vertex_enumeration(lp)
    assert opt is not None
    s = OracleSolver(lp, eps_rel=1e-9, max_iter=400000)
    r = s.solve()
    assert r.status == 0, (r.status, r.iters)
    assert abs(r.pobj - opt) <= 1e-6 * (1 + abs(opt))
    x, y, _ = s.solution()
    # primal point inside the bounds, duals in their cones (section 2 with implicit inequalities)
    assert np.all(x >= lp.l - 1e-12) and np.all(x <= lp.u + 1e-12)
    sense = lp.sense_str()
    for i, sn in enumerate(sense):
        if sn == "<":
            assert y[i] <= 0.0
        elif sn == ">":
            assert y[i] >= 0.0


@pytest.mark.parametrize("seed,m,n", [(200 + s, 3, 7) for s in range(6)] + [(207, 40, 120)])
def test_free_columns_vs_highs(seed, m, n):
    """Columns with no finite bound (section 2: z_j = 0 there, so the reduced
    cost itself must vanish): the oracle's optimum equals HiGHS's, its free
    columns carry z = 0 and a reduced cost within the dual tolerance."""
    lp = lpgen.tiny(seed, m=m, n=n, with_free=True)
    free = np.isinf(lp.l) & np.isinf(lp.u)
    opt, _ = lp_ref.highs(lp)
    s = OracleSolver(lp, eps_rel=1e-9, max_iter=400000)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-6 * (1 + abs(opt))
    x, y, z = s.solution()
    assert np.all(z[free] == 0.0)
    lam = lp.c - lp.dense().T @ y
    assert np.abs(lam[free]).max(initial=0.0) <= 1e-6 * (1 + np.abs(lp.c).max())


def test_push_gate_follows_the_selection_rule():
    """Section 4.2's selection rule as a push gate: with fewer candidates than
    max(rows * m, min) the push is skipped and the solve's point is the
    answer; at a threshold the count meets ("at least") the push runs exactly
    as without the gate."""
    lp = lpgen.config0(0)
    plain = OracleSolver(lp, eps_rel=1e-8)
    plain.solve()
    pp = plain.corner_push(3)
    cand = pp.before.candidates
    assert cand > 0 and pp.iters > 0
    closed = OracleSolver(lp, eps_rel=1e-8, push_gate=1, push_gate_rows=0.0, push_gate_min=cand + 1)
    closed.solve()
    x0 = closed.solution()[0]
    r = closed.corner_push(3)
    assert r.status == 5 and r.iters == 0
    assert (r.after.p_off, r.after.candidates) == (r.before.p_off, r.before.candidates)
    np.testing.assert_array_equal(closed.solution()[0], x0)
    opened = OracleSolver(lp, eps_rel=1e-8, push_gate=1, push_gate_rows=0.0, push_gate_min=cand)
    opened.solve()
    ro = opened.corner_push(3)
    assert (ro.status, ro.iters) == (pp.status, pp.iters)
    np.testing.assert_array_equal(opened.solution()[0], plain.solution()[0])
    by_rows = OracleSolver(lp, eps_rel=1e-8, push_gate=1, push_gate_rows=(cand + 1) / lp.m, push_gate_min=0)
    by_rows.solve()
    assert by_rows.corner_push(3).status == 5


@pytest.mark.parametrize("seed", range(4))
def test_vanilla_pdhg_also_converges(seed):
    """halpern = 0 (plain PDHG with restarts) reaches the same vertex optimum."""
    lp = lpgen.tiny(100 + seed, m=2, n=5)
    opt, _ = lp_ref.vertex_enumeration(lp)
    s = OracleSolver(lp, eps_rel=1e-9, halpern=0, max_iter=400000)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-6 * (1 + abs(opt))


# ------------------------------------------------------------- planted ------
def test_planted_config0_objective_duals_and_fix_set():
    """Config 0: c'x* = b'y* is the optimum; y* is unique (support of x* has
    more than m columns), so the converged y must be y*; the corner-push fix
    set must be exactly {j : z*_j > 0}."""
    lp = lpgen.config0(0)
    opt = float(lp.c @ lp.x_star)
    assert opt == pytest.approx(float(lp.b @ lp.y_star), rel=1e-12)
    s = OracleSolver(lp, eps_rel=1e-8)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-6 * (1 + abs(opt))
    x, y, z = s.solution()
    np.testing.assert_allclose(y, lp.y_star, atol=1e-5)
    pr = s.corner_push(seed=11)
    zs = lp.z_star
    assert pr.n_fix_upper == int((zs > 0).sum())
    assert pr.n_fix_lower == 0
    _, _, z_sol = s.solution()
    assert set(np.nonzero(z_sol > 1e-6)[0]) == set(np.nonzero(zs > 0)[0])


def test_planted_with_inequalities_and_upper_bounds():
    """Config-1 recipe at small size: '<' rows with implicit slacks and
    finite upper bounds; planted optimum is recovered."""
    lp = lpgen.config1(seed=5, m=300, n=1200)
    opt = float(lp.c @ lp.x_star)
    s = OracleSolver(lp, eps_rel=1e-7, max_iter=500000)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-5 * (1 + abs(opt))
    assert abs(r.dobj - opt) <= 1e-5 * (1 + abs(opt))


# ---------------------------------------------------------------- HiGHS -----
def test_against_highs_on_batched_family_instance():
    lp = lpgen.planted(500, 1250, seed=77, deg_range=(4, 8), degen_frac=0.1)
    opt, _ = lp_ref.highs(lp)
    s = OracleSolver(lp, eps_rel=1e-7)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-5 * (1 + abs(opt))


def test_transportation_integer_optimum():
    """Small transportation LP: integral data give an integral optimum
    (total unimodularity); HiGHS gives it independently."""
    lp = lpgen.transportation(12, 30, seed=3)
    opt, _ = lp_ref.highs(lp)
    assert abs(opt - round(opt)) < 1e-6
    s = OracleSolver(lp, eps_rel=1e-8, max_iter=2_000_000)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-6 * (1 + abs(opt))


# ----------------------------------------------------------- closed forms ---
def test_continuous_knapsack_closed_form_and_corner():
    """One equality row with positive weights and boxes: the greedy fill is
    optimal, and a corner of the optimal face has at most one column strictly
    inside its box (m = 1)."""
    rng = np.random.default_rng(4)
    n = 12
    a = rng.uniform(0.5, 2.0, n)
    u = rng.uniform(1.0, 3.0, n)
    c = rng.uniform(-1.0, 1.0, n)
    c[3] = c[7] * a[3] / a[7]  # a tie in c_j / a_j makes the optimal face an edge
    b = 0.5 * float(a @ u)
    lp = lpgen.from_dense(a[None, :], [b], c, np.zeros(n), u, "=")
    opt, _ = lp_ref.knapsack_greedy(a, b, c, u)
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=20000)
    r = s.solve()
    assert r.status == 0
    assert abs(r.pobj - opt) <= 1e-7 * (1 + abs(opt))
    pr = s.corner_push(seed=3)
    assert pr.status == 3
    assert pr.after.p_off <= 1
    assert abs(pr.after.pobj - opt) <= 1e-5 * (1 + abs(opt))


def test_identity_matrix_closed_form():
    """A = I with '=' rows: x = b, y = c (all columns strictly inside x > 0)."""
    n = 7
    b = np.arange(1.0, n + 1)
    c = np.linspace(-1, 1, n)
    lp = lpgen.from_dense(np.eye(n), b, c)
    s = OracleSolver(lp, eps_rel=1e-11, max_iter=100000)
    r = s.solve()
    assert r.status == 0
    x, y, _ = s.solution()
    np.testing.assert_allclose(x, b, atol=1e-9)
    np.testing.assert_allclose(y, c, atol=1e-9)


def test_empty_row_and_column():
    """An empty column sits at the bound its cost points to; an empty row with
    b = 0 is harmless."""
    a = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    lp = lpgen.from_dense(a, [2.0, 0.0], [1.0, 2.0, -1.0], [0, 0, 0], [np.inf, np.inf, 4.0], "==")
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=100000)
    r = s.solve()
    assert r.status == 0
    x, _, _ = s.solution()
    assert x[2] == pytest.approx(4.0, abs=1e-9)
    assert r.pobj == pytest.approx(2.0 - 4.0, abs=1e-7)


# ---------------------------------------------------------------- scaling ---
def test_scaling_reconstructs_matrix_and_step_bound():
    """Ahat = diag(Dr) A diag(Dc) entrywise; Pock-Chambolle (alpha = 1) leaves
    ||Ahat||_2 <= 1; the power-iteration estimate lies below the true norm and
    within 0.5% of it; the rows of Ahat approach unit inf-norm after Ruiz."""
    lp = lpgen.config0(3)
    s = OracleSolver(lp)
    sc = s.scaling()
    rp, ci, v = s.ahat()
    rows = np.repeat(np.arange(lp.m), np.diff(rp))
    a = lp.dense()
    np.testing.assert_allclose(v, sc["dr"][rows] * a[rows, ci] * sc["dc"][ci], rtol=1e-13)
    ah = np.zeros_like(a)
    ah[rows, ci] = v
    smax = np.linalg.norm(ah, 2)
    assert smax <= 1.0 + 1e-12
    assert sc["sigma_est"] <= smax * (1 + 1e-12)
    assert sc["sigma_est"] >= 0.995 * smax
    assert sc["eta"] == pytest.approx(0.99 / sc["sigma_est"], rel=1e-15)


def test_power_iteration_stops_on_its_residual_and_keeps_the_step_below_one_over_the_norm():
    """On a batched-family LP whose top singular value stands apart from a
    dense cluster just below it, 32 fixed steps from 1/sqrt(n) stop inside
    the cluster (about 2% low, so eta ||Ahat|| > 1 and PDHG diverges); the
    residual rule runs until the estimate is within 0.5% of the true norm
    (scipy's sparse SVD) and below it."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    lp = lpgen.config3_instance(157)
    a = sp.csr_matrix((lp.val, lp.col, lp.row_ptr), shape=(lp.m, lp.n))
    fixed = OracleSolver(lp, power_iters=32, power_tol=0.0)
    rule = OracleSolver(lp)
    sc_f, sc_r = fixed.scaling(), rule.scaling()
    ah = (sp.diags(sc_r["dr"]) @ a @ sp.diags(sc_r["dc"])).tocsr()
    smax = float(sla.svds(ah, k=1, return_singular_vectors=False, tol=1e-12)[0])
    assert sc_f["power_steps"] == 32 and sc_f["sigma_est"] < 0.99 * smax
    assert 32 < sc_r["power_steps"] < 4000
    assert 0.995 * smax <= sc_r["sigma_est"] <= smax * (1 + 1e-12)
    assert sc_r["eta"] * smax < 1.0


def test_ruiz_only_equilibrates_inf_norms():
    lp = lpgen.planted(60, 150, seed=9, deg=4)
    lp.val = lp.val * np.exp(np.random.default_rng(0).uniform(-6, 6, lp.val.size))
    s = OracleSolver(lp, pc_alpha=-1.0, ruiz_iters=30)
    rp, ci, v = s.ahat()
    rows = np.repeat(np.arange(lp.m), np.diff(rp))
    rmax = np.zeros(lp.m)
    np.maximum.at(rmax, rows, np.abs(v))
    cmax = np.zeros(lp.n)
    np.maximum.at(cmax, ci, np.abs(v))
    np.testing.assert_allclose(rmax, 1.0, atol=1e-3)
    np.testing.assert_allclose(cmax, 1.0, atol=1e-3)


# ------------------------------------------------------------ corner push ---
@pytest.mark.parametrize("seed", range(6))
def test_push_model_keeps_every_feasible_point_optimal(seed):
    """Section 2 lemma behind Algorithm 1: with the bounds fixed where the
    reduced cost is non-trivial (and slack-active rows made equalities), every
    vertex of the push model has the original optimal objective."""
    lp = lpgen.tiny(200 + seed, m=3, n=6)
    opt, _ = lp_ref.vertex_enumeration(lp)
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_max_iter=1)
    s.solve()
    pr = s.corner_push(seed=5)
    lh, uh, _, sense = s.model_scaled()
    dc = s.scaling()["dc"]
    vs = lp_ref.vertices(lp, l=lh * dc, u=uh * dc, sense=sense, tol=1e-7)
    assert len(vs) > 0
    objs = np.array([lp.c @ v for v in vs])
    assert np.all(np.abs(objs - opt) <= 1e-5 * (1 + abs(opt))), (objs, opt)
    assert pr.n_fix_lower + pr.n_fix_upper + pr.n_rows_to_eq > 0


def test_push_objective_is_uniform_and_bit_exact_generator():
    # splitmix64 started from state 0 has a well-known first output
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    u = np.array([push_uniform(12345, j) for j in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    from scipy.stats import kstest

    assert kstest(u, "uniform").pvalue > 1e-3
    assert len(np.unique(u)) == u.size


def test_push_on_config0_reaches_a_corner_and_keeps_the_objective():
    """Config 0: the push returns a primal point back at the original tolerance,
    with no more than m structural columns off their bounds (a basic point of the
    optimal face), the original y and z, and the original objective within the
    bound that follows from the fixed terms (z_j (xhat_j - x_j) <= 0)."""
    lp = lpgen.config0(0)
    s = OracleSolver(lp, eps_rel=1e-8)
    r = s.solve()
    x0, y0, z0 = s.solution()
    pr = s.corner_push(seed=7)
    assert pr.status == 3
    assert pr.iters >= 100
    xh, y1, z1 = s.solution()
    np.testing.assert_array_equal(y1, y0)
    np.testing.assert_array_equal(z1, z0)
    assert pr.after.rel_p <= 1e-8
    assert pr.before.p_off > lp.m
    assert pr.after.p_off <= lp.m + 2
    assert pr.after.est_primal <= 2
    a = lp.dense()
    d = xh - x0
    ra = lp.c - a.T @ y0 - z0
    bound = 1e-6 * np.abs(d).sum() + abs(y0 @ (a @ d)) + abs(ra @ d)
    assert lp.c @ xh - lp.c @ x0 <= bound + 1e-12
    # fixed columns never leave their fixed value
    fixed = z0 > 1e-6
    lh, uh, _, _ = s.model_scaled()
    np.testing.assert_allclose(xh[fixed], x0[fixed], atol=1e-12)
    assert np.all(xh >= lp.l - 1e-12)


def test_push_converged_corner_matches_vertex_of_restricted_model():
    """With the push driven to full convergence on a tiny LP, its point is the
    unique minimiser of the random objective over the push model."""
    lp = lpgen.from_dense([[1.0, 1.0, 1.0, 1.0]], [2.0], [0.0, 0.0, 0.0, 1.0], [0, 0, 0, 0], [1, 1, 1, 1], "=")
    s = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=50000)
    s.solve()
    pr = s.corner_push(seed=21)
    xh, _, _ = s.solution()
    lh, uh, ch, sense = s.model_scaled()
    sc = s.scaling()
    cpush = ch / sc["dc"]
    want = np.array([push_uniform(21, j) for j in range(4)])
    np.testing.assert_allclose(cpush, want, rtol=1e-15)
    opt, v = lp_ref.vertex_enumeration(lp, c=cpush, l=lh * sc["dc"], u=uh * sc["dc"], sense=sense, tol=1e-7)
    np.testing.assert_allclose(xh, v, atol=1e-4)
    assert pr.after.p_off <= 1


# ---------------------------------------------------------- failure paths ---
def test_invalid_inputs_are_rejected():
    good = lpgen.config0(0)
    bad = lpgen.config0(0)
    bad.c = bad.c.copy()
    bad.c[3] = np.nan
    with pytest.raises(ValueError):
        OracleSolver(bad)
    bad = lpgen.config0(0)
    bad.l = bad.l.copy()
    bad.l[0] = 5.0
    bad.u = bad.u.copy()
    bad.u[0] = 1.0
    with pytest.raises(ValueError):
        OracleSolver(bad)
    bad = lpgen.config0(0)
    bad.col = bad.col.copy()
    bad.col[0] = good.n + 3
    with pytest.raises(ValueError):
        OracleSolver(bad)


def test_iteration_limit_status_and_push_requires_solve():
    lp = lpgen.config0(0)
    s = OracleSolver(lp, max_iter=100)
    with pytest.raises(RuntimeError):
        s.corner_push(1)
    r = s.solve()
    assert r.status == 1 and r.iters == 100


def test_duplicates_are_summed_and_column_order_is_free():
    lp = lpgen.config0(2)
    s1 = OracleSolver(lp)
    s1.iterate(40)
    # split every entry into two halves and reverse the order inside rows
    rp = lp.row_ptr
    cols, vals, nrp = [], [], [0]
    for i in range(lp.m):
        cc = lp.col[rp[i]:rp[i + 1]][::-1]
        vv = lp.val[rp[i]:rp[i + 1]][::-1]
        cols += list(cc) + list(cc)
        vals += list(0.5 * vv) + list(0.5 * vv)
        nrp.append(len(cols))
    lp2 = lpgen.LP(lp.m, lp.n, np.array(nrp, np.int64), np.array(cols, np.int32), np.array(vals), lp.b, lp.c, lp.l,
                   lp.u, lp.sense)
    s2 = OracleSolver(lp2)
    s2.iterate(40)
    x1, y1 = s1.iterate_state()
    x2, y2 = s2.iterate_state()
    np.testing.assert_allclose(x1, x2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(y1, y2, rtol=1e-12, atol=1e-14)


def test_iterate_is_resumable():
    """Running 30 + 70 iterations equals running 100 at once, bit for bit."""
    lp = lpgen.config0(1)
    a = OracleSolver(lp)
    a.iterate(100)
    b = OracleSolver(lp)
    b.iterate(30)
    b.iterate(70)
    xa, ya = a.iterate_state()
    xb, yb = b.iterate_state()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(ya, yb)
