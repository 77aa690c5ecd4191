"""The dual corner push on the GPU against the oracle.

Same seeded LPs, same solve (equal iteration counts), then the dual push on
both sides: the face it builds (integer decisions) must be identical, the stop
the same up to one check, and the pushed y within rounding of the oracle's when
the stops agree.  The pushed y is also checked on its own against what the
method fixes: x unchanged, the dual test met, the dual superbasic estimate cut,
and on a degenerate 2-column LP the closed-form vertex."""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max())) if a.size else 0.0


def _cases():
    return [
        ("degenerate_200x500", lambda: lpgen.planted(200, 500, seed=1, zero_frac=0.8, degen_frac=0.0)),
        ("degenerate_ineq_ub_300x900",
         lambda: lpgen.planted(300, 900, seed=2, zero_frac=0.85, degen_frac=0.0, ineq_frac=0.3, upper_frac=0.2)),
        ("degenerate_ragged_400x1000",
         lambda: lpgen.planted(400, 1000, seed=3, zero_frac=0.8, degen_frac=0.0, deg_range=(1, 9))),
        ("transport_12x30", lambda: lpgen.transportation(12, 30, seed=3)),
        ("free_mixed_40x120", lambda: lpgen.tiny(207, m=40, n=120, with_free=True)),
        ("c0_s0", lambda: lpgen.config0(0)),
        # a fixed column (cone {0}), an empty column, an empty '<' row and a loose '>' row (both dropped)
        ("edge_fixed_empty", lambda: lpgen.from_dense([[1, 1, 0, 1], [0, 0, 0, 0], [1, -1, 0, 2]], [3, 5, 1],
                                                      [1, 2, 3, 0.5], [0, 0, 0, 1], [np.inf, np.inf, np.inf, 1],
                                                      "=<>")),
    ]


@pytest.mark.parametrize("name,make", _cases(), ids=[c[0] for c in _cases()])
def test_dual_push_matches_oracle(name, make):
    print(f"[dual push] {name}", flush=True)
    lp = make()
    eps = 1e-8
    g = pdhg.Solver(lp, eps_rel=eps, max_iter=400000)
    o = OracleSolver(lp, eps_rel=eps, max_iter=400000)
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status == pdhg.PDHG_OPTIMAL
    assert rg.iters == ro.iters
    x0, y0, _ = g.get_solution()
    pg, po = g.dual_push(5), o.dual_push(5)
    print(f"[dual push] {name}: pinned z {pg.n_cols_free}, pinned y {pg.n_rows_fixed}; iterations {pg.iters} "
          f"(oracle {po.iters}); est_dual {pg.before.est_dual} -> {pg.after.est_dual} "
          f"(oracle {po.before.est_dual} -> {po.after.est_dual})", flush=True)
    assert (pg.n_cols_free, pg.n_rows_fixed) == (po.n_cols_free, po.n_rows_fixed)
    assert pg.status == po.status == pdhg.PDHG_PUSH_DONE
    assert pg.before.d_zero == po.before.d_zero and pg.before.est_dual == po.before.est_dual
    assert pg.iters == po.iters, (pg.iters, po.iters)
    assert pg.rel_d_push <= eps
    x1, y1, z1 = g.get_solution()
    np.testing.assert_array_equal(x1, x0)  # the solve's x is the answer's x
    xs, ys, _ = g.get_solve_solution()
    np.testing.assert_array_equal(ys, y0)  # the solve's answer is kept beside the push's
    k = g.kkt(x1, y1)
    assert k.rel_d <= 2 * eps and k.rel_gap <= 100 * eps
    assert pg.after.est_dual <= pg.before.est_dual
    xo1, yo1, zo1 = o.solution()
    assert rel_inf(y1, yo1) <= 1e-7
    assert pg.after.est_dual == po.after.est_dual


def test_dual_push_reaches_the_closed_form_vertex():
    """x* = (1/3, 1/3) with three active '>' rows: the dual face is
    y = (t, t, 1 - 3t), t in [0, 1/3]; the converged push ends on one end point,
    the same one as the oracle's, with the estimate of dual superbasics 1 -> 0."""
    lp = lpgen.from_dense([[1, 2], [2, 1], [1, 1]], [1, 1, 2 / 3], [1, 1], [0, 0], [np.inf, np.inf], ">>>")
    for seed in range(4):
        g = pdhg.Solver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=20000)
        o = OracleSolver(lp, eps_rel=1e-10, max_iter=400000, push_min_iters=20000)
        g.solve()
        o.solve()
        pg, po = g.dual_push(seed), o.dual_push(seed)
        y = g.get_solution()[1]
        t = y[0]
        assert min(abs(t), abs(t - 1 / 3)) <= 1e-6, y
        np.testing.assert_allclose(y, [t, t, 1 - 3 * t], atol=1e-6)
        np.testing.assert_allclose(y, o.solution()[1], atol=1e-6)
        assert pg.before.est_dual == 1 and pg.after.est_dual == 0 and pg.status == po.status


@pytest.mark.parametrize("lanes_a", [-3032, -4000, -32, 4])
def test_dual_push_on_every_dual_half_kernel(lanes_a):
    """The dropped rows ('N', y = 0) go through every dual-half kernel: sliced
    ELLPACK, row segments, LDS tiles and lane groups give the oracle's push."""
    lp = lpgen.planted(300, 900, seed=2, zero_frac=0.85, degen_frac=0.0, ineq_frac=0.3, upper_frac=0.2)
    g = pdhg.Solver(lp, eps_rel=1e-8, max_iter=400000, lanes_a=lanes_a)
    o = OracleSolver(lp, eps_rel=1e-8, max_iter=400000)
    assert g.get_timing().lanes_a == lanes_a
    g.solve()
    o.solve()
    pg, po = g.dual_push(9), o.dual_push(9)
    print(f"[dual push] lanes_a {lanes_a}: {pg.iters} iterations (oracle {po.iters}), "
          f"{pg.n_rows_fixed} rows dropped", flush=True)
    assert pg.n_rows_fixed == po.n_rows_fixed > 0
    assert pg.status == po.status and pg.iters == po.iters
    assert rel_inf(g.get_solution()[1], o.solution()[1]) <= 1e-7


def test_dual_push_graph_replay_equals_eager_launches():
    lp = lpgen.planted(200, 500, seed=1, zero_frac=0.8, degen_frac=0.0)
    out = []
    for graph in (0, 1):
        g = pdhg.Solver(lp, eps_rel=1e-8, max_iter=400000, use_graph=graph)
        g.solve()
        p = g.dual_push(3)
        out.append((p.iters, g.get_solution()[1]))
    assert out[0][0] == out[1][0]
    np.testing.assert_array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("name,make", [
    ("planted_400x1000", lambda: lpgen.planted(400, 1000, seed=3, zero_frac=0.8, degen_frac=0.0, deg_range=(1, 9))),
    ("c5_family_m1000", lambda: lpgen.config5(seed=5, m=1000, n=4000)),
], ids=["planted_400x1000", "c5_family_m1000"])
def test_dual_push_fp32_mixed(name, make):
    """FP32 matrix and x-vector differences (y and the checks stay float64):
    the same face, and the push cuts the dual superbasic estimate as the
    float64 one does, also on the primal-degenerate family."""
    lp = make()
    res = {}
    for prec in ("fp64", "fp32"):
        g = pdhg.Solver(lp, precision=prec, eps_rel=1e-6, max_iter=400000)
        assert g.solve().status == pdhg.PDHG_OPTIMAL
        res[prec] = g.dual_push(4)
    a, b = res["fp64"], res["fp32"]
    print(f"[dual push] {name} fp32: est_dual {b.before.est_dual} -> {b.after.est_dual}, {b.iters} iterations "
          f"(fp64 {a.before.est_dual} -> {a.after.est_dual}, {a.iters})", flush=True)
    assert b.status == pdhg.PDHG_PUSH_DONE
    assert b.rel_d_push <= 1e-6
    assert b.after.est_dual < b.before.est_dual
    assert abs(b.n_cols_free - a.n_cols_free) <= 2


@pytest.mark.parametrize("name,make", [
    ("degenerate_ineq_ub_300x900",
     lambda: lpgen.planted(300, 900, seed=2, zero_frac=0.85, degen_frac=0.0, ineq_frac=0.3, upper_frac=0.2)),
    ("c0_s0", lambda: lpgen.config0(0)),
    ("ineq_ub_300x1200", lambda: lpgen.config1(seed=3, m=300, n=1200)),
], ids=["degenerate_ineq_ub_300x900", "c0_s0", "ineq_ub_300x1200"])
def test_dual_push_after_corner_push_matches_oracle(name, make):
    """Crossover's order: the corner push (on its free columns, the default),
    then the dual push from its xhat; both phases follow the oracle."""
    print(f"[dual push] after the corner push: {name}", flush=True)
    lp = make()
    g = pdhg.Solver(lp, eps_rel=1e-8, max_iter=400000)
    o = OracleSolver(lp, eps_rel=1e-8, max_iter=400000)
    g.solve()
    o.solve()
    pg, po = g.corner_push(3), o.corner_push(3)
    assert pg.status == po.status == pdhg.PDHG_PUSH_DONE
    xh = g.get_solution()[0]
    dg, do = g.dual_push(5), o.dual_push(5)
    print(f"[dual push] after the corner push: {name}: primal push {pg.iters} / {po.iters}, dual push {dg.iters} / "
          f"{do.iters}; est_primal {pg.after.est_primal}, est_dual {dg.before.est_dual} -> {dg.after.est_dual}",
          flush=True)
    assert (dg.n_cols_free, dg.n_rows_fixed) == (do.n_cols_free, do.n_rows_fixed)
    assert dg.status == do.status == pdhg.PDHG_PUSH_DONE and dg.rel_d_push <= 1e-8
    x2, y2, _ = g.get_solution()
    np.testing.assert_array_equal(x2, xh)
    xs, ys, _ = g.get_solve_solution()
    k = g.kkt(x2, y2)
    assert k.rel_p <= 1e-8 * 1.0000001 and k.rel_d <= 2e-8
    assert rel_inf(xh, o.solution()[0]) <= 1e-7
    assert dg.iters == do.iters
    assert rel_inf(y2, o.solution()[1]) <= 1e-7
    assert dg.after.est_dual == do.after.est_dual


def test_dual_push_state_rules():
    lp = lpgen.config0(0)
    g = pdhg.Solver(lp, eps_rel=1e-6)
    with pytest.raises(pdhg.PdhgError):
        g.dual_push(1)
    g.solve()
    g.dual_push(1)
    with pytest.raises(pdhg.PdhgError):
        g.dual_push(1)
    with pytest.raises(pdhg.PdhgError):
        g.corner_push(1)
    g2 = pdhg.Solver(lp, eps_rel=1e-6)
    g2.solve()
    g2.corner_push(1)
    g2.dual_push(1)
    with pytest.raises(pdhg.PdhgError):
        g2.dual_push(1)


def _batch_lps():
    lps = [lpgen.planted(120 + 20 * i, 300 + 50 * i, seed=60 + i, zero_frac=0.8, degen_frac=0.0, ineq_frac=0.3)
           for i in range(4)]
    lps += [lpgen.config3_instance(i, base_seed=5000, m_range=(40, 300)) for i in range(3)]
    lps.append(lpgen.transportation(6, 9, seed=4))
    lps.append(lpgen.tiny(207, m=40, n=120, with_free=True))
    return lps


def test_batch_dual_push_matches_the_oracle_lp_by_lp():
    """The batch dual push (every LP's own seed and numbering, lockstep cycles
    over the block-diagonal model) against the oracle's dual push of each LP."""
    lps = _batch_lps()
    seeds = [21 + i for i in range(len(lps))]
    b = pdhg.Batch(lps, eps_rel=1e-8)
    b.solve()
    res = b.dual_push(seeds)
    for i, lp in enumerate(lps):
        o = OracleSolver(lp, eps_rel=1e-8)
        o.solve()
        po = o.dual_push(seeds[i])
        r = res[i]
        print(f"[dual push] batch LP {i} ({lp.m}x{lp.n}): {r.iters} iterations (oracle {po.iters}), est_dual "
              f"{r.before.est_dual} -> {r.after.est_dual} (oracle {po.before.est_dual} -> {po.after.est_dual})",
              flush=True)
        assert (r.n_cols_free, r.n_rows_fixed) == (po.n_cols_free, po.n_rows_fixed), i
        assert r.status == po.status == pdhg.PDHG_PUSH_DONE, i
        assert r.iters == po.iters, (i, r.iters, po.iters)
        assert r.rel_d_push <= 1e-8
        x, y, _ = b.get_solution(i)
        xo, yo, _ = o.solution()
        assert rel_inf(x, xo) <= 1e-7, i
        assert rel_inf(y, yo) <= 1e-7, i
        assert r.after.est_dual == po.after.est_dual, i


def test_batch_dual_push_after_the_batch_corner_push():
    lps = _batch_lps()[:5]
    seeds = [31 + i for i in range(len(lps))]
    b = pdhg.Batch(lps, eps_rel=1e-8)
    b.solve()
    pr = b.corner_push(seeds)
    xh = [b.get_solution(i)[0] for i in range(len(lps))]
    dr = b.dual_push(seeds)
    with pytest.raises(pdhg.PdhgError):
        b.dual_push(seeds)
    for i, lp in enumerate(lps):
        o = OracleSolver(lp, eps_rel=1e-8)
        o.solve()
        po = o.corner_push(seeds[i])
        do = o.dual_push(seeds[i])
        x, y, _ = b.get_solution(i)
        np.testing.assert_array_equal(x, xh[i])
        assert dr[i].status == do.status == pdhg.PDHG_PUSH_DONE, i
        assert (dr[i].n_cols_free, dr[i].n_rows_fixed) == (do.n_cols_free, do.n_rows_fixed), i
        assert dr[i].iters == do.iters, i
    b2 = pdhg.Batch(lps, eps_rel=1e-8)
    b2.solve()
    b2.dual_push(seeds)
    with pytest.raises(pdhg.PdhgError):
        b2.corner_push(seeds)


def _sweep():
    cases = [(f"tiny_{3 + 4 * k}x{8 + 10 * k}", lambda k=k: lpgen.tiny(400 + k, m=3 + 4 * k, n=8 + 10 * k,
                                                                        with_free=(k % 2 == 1)))
             for k in range(10)]
    cases += [(f"planted_ragged_{50 + 30 * k}x{150 + 60 * k}",
               lambda k=k: lpgen.planted(50 + 30 * k, 150 + 60 * k, seed=90 + k, zero_frac=0.7 + 0.05 * k,
                                         degen_frac=0.1 * (k % 2), ineq_frac=0.3, upper_frac=0.2, deg_range=(1, 7)))
              for k in range(3)]
    return cases


@pytest.mark.parametrize("k,name,make", [(k, c[0], c[1]) for k, c in enumerate(_sweep())],
                         ids=[c[0] for c in _sweep()])
def test_dual_push_sweep_of_small_lps(k, name, make):
    """Random senses, bounds, free columns and ragged degrees: the same face,
    status and stop as the oracle, and the same pushed y when the stops agree."""
    lp = make()
    g = pdhg.Solver(lp, eps_rel=1e-8, max_iter=400000)
    o = OracleSolver(lp, eps_rel=1e-8, max_iter=400000)
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status == pdhg.PDHG_OPTIMAL and rg.iters == ro.iters
    pg, po = g.dual_push(3 + k), o.dual_push(3 + k)
    print(f"[dual push] sweep {name}: {pg.iters} / {po.iters} iterations, est_dual {pg.before.est_dual} -> "
          f"{pg.after.est_dual}", flush=True)
    assert (pg.n_cols_free, pg.n_rows_fixed) == (po.n_cols_free, po.n_rows_fixed)
    assert pg.status == po.status == pdhg.PDHG_PUSH_DONE
    assert pg.iters == po.iters
    assert rel_inf(g.get_solution()[1], o.solution()[1]) <= 1e-7
    assert pg.after.est_dual == po.after.est_dual


def test_dual_push_stopped_before_its_first_check_keeps_the_solve_y():
    """push_max_iter below push_min_iters: no check runs, the status is the
    iteration limit and the answer's y is the solve's, on one LP and on every
    LP of a batch; the oracle does the same."""
    lp = lpgen.planted(200, 500, seed=1, zero_frac=0.8, degen_frac=0.0)
    g = pdhg.Solver(lp, eps_rel=1e-8, max_iter=400000, push_max_iter=50)
    o = OracleSolver(lp, eps_rel=1e-8, max_iter=400000, push_max_iter=50)
    g.solve()
    o.solve()
    y0 = g.get_solution()[1]
    pg, po = g.dual_push(5), o.dual_push(5)
    assert pg.status == po.status == pdhg.PDHG_ITER_LIMIT and pg.iters == po.iters == 50
    assert np.isnan(pg.rel_d_push)
    np.testing.assert_array_equal(g.get_solution()[1], y0)
    assert rel_inf(o.solution()[1], y0) <= 1e-8
    lps = _batch_lps()[:3]
    b = pdhg.Batch(lps, eps_rel=1e-8, push_max_iter=50)
    b.solve()
    ys = [b.get_solution(i)[1] for i in range(len(lps))]
    res = b.dual_push([1, 2, 3])
    for i in range(len(lps)):
        assert res[i].status == pdhg.PDHG_ITER_LIMIT and res[i].iters == 50, i
        np.testing.assert_array_equal(b.get_solution(i)[1], ys[i])


def test_dual_push_after_a_learned_corner_push():
    """The learned corner push (fixes from the predictor, undone at checks)
    leaves the handle ready for the dual push: the face is that of its xhat,
    xhat is kept, and the dual test is met at the stop."""
    lp = lpgen.config0(3)
    net = pdhg.Mlp(1)
    s = pdhg.Solver(lp, record_history=1, eps_rel=1e-7)
    assert s.solve().status == pdhg.PDHG_OPTIMAL
    p = s.corner_push_learned(net, 1e-4, 5)
    assert p.status == pdhg.PDHG_PUSH_DONE
    xh = s.get_solution()[0]
    d = s.dual_push(5)
    print(f"[dual push] after the learned push: {d.iters} iterations, est_dual {d.before.est_dual} -> "
          f"{d.after.est_dual}", flush=True)
    assert d.status == pdhg.PDHG_PUSH_DONE and d.rel_d_push <= 1e-7
    x2, y2, _ = s.get_solution()
    np.testing.assert_array_equal(x2, xh)
    at_lo = np.isfinite(lp.l) & (xh - lp.l <= 1e-6)
    at_up = np.isfinite(lp.u) & (lp.u - xh <= 1e-6)
    assert d.n_cols_free == int(np.sum(~at_lo & ~at_up))
    k = s.kkt(x2, y2)
    assert k.rel_d <= 2e-7
