"""Parity at full size, in the launch configuration the benchmark uses (default
parameters: kernels chosen from the mean row length, graph-replayed cycles,
event timing on).  Checked at any size: the setup (scaling, step size), the
first iterates, the float64 KKT of the GPU's answer evaluated by the oracle's
own code, and the push's fixing decisions recounted from that answer.  The
oracle's own full runs of c1, c2 and c5, made once by the scripts under
tests/golden/, pin the iteration, restart, fix and corner counts."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max())) if a.size else 0.0


@pytest.fixture(scope="module")
def c1():
    print("[full] c1 100k x 400k: generate + oracle setup", flush=True)
    lp = lpgen.config1()
    return lp, OracleSolver(lp)


@pytest.fixture(scope="module")
def c2():
    print("[full] c2 7k x 10M: generate + oracle setup", flush=True)
    lp = lpgen.config2()
    return lp, OracleSolver(lp)


def _setup_and_first_iterates(lp, o, iters):
    g = pdhg.Solver(lp, timing=1)
    sg, so = g.get_scaling(), o.scaling()
    assert rel_inf(sg["dr"], so["dr"]) <= 1e-14
    assert rel_inf(sg["dc"], so["dc"]) <= 1e-14
    assert sg["power_steps"] == so["power_steps"]
    assert abs(sg["eta"] - so["eta"]) <= 1e-13 * so["eta"]
    for t in range(1, iters + 1):
        g.iterate(1)
        o.iterate(1)
        xg, yg = g.get_iterate()
        xo, yo = o.iterate_state()
        print(f"[full] {lp.name} iterate {t}: x {rel_inf(xg, xo):.2e} y {rel_inf(yg, yo):.2e}", flush=True)
        assert rel_inf(xg, xo) <= 1e-10 and rel_inf(yg, yo) <= 1e-10
    return g


def _z_of(lp, y):
    """Reduced costs of the original model split by finite bounds (float64)."""
    a = sp.csr_matrix((lp.val, lp.col, lp.row_ptr), shape=(lp.m, lp.n))
    lam = lp.c - a.T @ y
    lo_fin = np.isfinite(lp.l) & (np.abs(lp.l) < 1e20)
    hi_fin = np.isfinite(lp.u) & (np.abs(lp.u) < 1e20)
    zp = np.where(lo_fin & (lam > 0), lam, 0.0)
    zm = np.where(hi_fin & (lam < 0), -lam, 0.0)
    return zp - zm


def test_c1_setup_iterates_solve_and_push(c1):
    lp, o = c1
    _setup_and_first_iterates(lp, o, 3)
    g = pdhg.Solver(lp, timing=1)
    r = g.solve()
    x, y, z = g.get_solution()
    k = o.kkt(x, y)
    print(f"[full] c1 solve: {pdhg.STATUS[r.status]} {r.iters} iterations; GPU KKT {r.rel_p:.3e}/{r.rel_d:.3e}/"
          f"{r.rel_gap:.3e}, oracle's evaluation {k.rel_p:.3e}/{k.rel_d:.3e}/{k.rel_gap:.3e}", flush=True)
    assert r.status == pdhg.PDHG_OPTIMAL
    assert max(k.rel_p, k.rel_d, k.rel_gap) <= 1e-6
    # the relative measures come from sums over 400k terms (objectives near 200
    # whose difference is the gap): equal up to 1e-12 in absolute terms
    for a, b in ((r.rel_p, k.rel_p), (r.rel_d, k.rel_d), (r.rel_gap, k.rel_gap)):
        assert abs(a - b) <= 1e-6 * b + 1e-12
    assert abs(r.pobj - k.pobj) <= 1e-12 * max(1.0, abs(k.pobj))
    # the push's fixing decisions, recounted from the solve's answer
    zr = _z_of(lp, y)
    np.testing.assert_allclose(z, zr, rtol=0, atol=1e-12 * max(1.0, np.abs(zr).max()))
    p = g.corner_push(1)
    assert p.status == pdhg.PDHG_PUSH_DONE and p.after.rel_p <= 1e-6
    assert p.n_fix_upper == int(np.sum(zr > 1e-6)) and p.n_fix_lower == int(np.sum(zr < -1e-6))
    ineq = np.asarray(lp.sense) != ord("=")
    assert p.n_rows_to_eq == int(np.sum(ineq & (np.abs(y) > 1e-6)))
    # the corner counts of the pushed point, evaluated by the oracle
    xp, yp, _ = g.get_solution()
    np.testing.assert_array_equal(yp, y)
    ka = o.kkt(xp, yp)
    print(f"[full] c1 push: {p.iters} iterations; off-bound {p.before.p_off} -> {p.after.p_off} (oracle {ka.p_off}),"
          f" candidates {p.after.candidates} (oracle {ka.candidates}), primal push estimate {p.after.est_primal}",
          flush=True)
    assert (p.after.p_off, p.after.candidates, p.after.est_primal) == (ka.p_off, ka.candidates, ka.est_primal)
    assert abs(p.after.pobj - ka.pobj) <= 1e-12 * max(1.0, abs(ka.pobj))
    # the oracle's own full solve and push of this LP (tests/golden/make_c1_oracle.py)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.json")))
    gs, gp = gold["solve"], gold["push"]
    print(f"[full] c1 vs the oracle's full run: solve {r.iters}/{gs['iters']} iterations, push {p.iters}/{gp['iters']}, "
          f"off-bound after {p.after.p_off}/{gp['p_off_after']}", flush=True)
    assert r.iters == gs["iters"] and r.restarts == gs["restarts"]
    assert abs(r.pobj - gs["pobj"]) <= 1e-9 * abs(gs["pobj"])
    assert (p.n_fix_lower, p.n_fix_upper, p.n_rows_to_eq) == (gp["n_fix_lower"], gp["n_fix_upper"], gp["n_rows_to_eq"])
    assert (p.before.p_off, p.before.candidates) == (gp["p_off_before"], gp["candidates_before"])
    assert p.status == gp["status"] and p.iters == gp["iters"]
    assert (p.after.p_off, p.after.candidates, p.after.est_primal) == \
        (gp["p_off_after"], gp["candidates_after"], gp["est_primal_after"])
    # crossover's order: the dual push from the pushed x, against the oracle's continuation of its run
    d = g.dual_push(1)
    gd = gold["dual_push_after_push"]
    x3, y3, _ = g.get_solution()
    np.testing.assert_array_equal(x3, xp)
    kd = o.kkt(x3, y3)
    print(f"[full] c1 dual push after the push: {d.iters} iterations (oracle {gd['iters']}); est_dual "
          f"{d.before.est_dual} -> {d.after.est_dual} (oracle's run {gd['est_dual_before']} -> {gd['est_dual_after']})",
          flush=True)
    assert d.status == gd["status"] == pdhg.PDHG_PUSH_DONE and d.rel_d_push <= 1e-6
    assert (d.after.d_zero, d.after.est_dual) == (kd.d_zero, kd.est_dual)
    assert (d.n_cols_free, d.n_rows_fixed) == (gd["n_cols_free"], gd["n_rows_fixed"])
    assert (d.before.d_zero, d.before.est_dual) == (gd["d_zero_before"], gd["est_dual_before"])
    assert d.iters == gd["iters"]
    assert (d.after.d_zero, d.after.est_dual) == (gd["d_zero_after"], gd["est_dual_after"])


def test_c5_solve_and_dual_push_against_the_oracle_full_run():
    """The dual push workload (100k x 400k, primal-degenerate optimum): the
    GPU's solve and dual push against the oracle's own full run
    (tests/golden/make_c5_oracle.py), the face's decisions recounted from the
    GPU's solve answer, and the pushed pair evaluated by the oracle's code."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_oracle.json")))
    print("[full] c5 100k x 400k: generate + oracle setup", flush=True)
    lp = lpgen.config5()
    o = OracleSolver(lp)
    g = pdhg.Solver(lp, timing=1)
    r = g.solve()
    x, y, _ = g.get_solution()
    gs, gd = gold["solve"], gold["dual_push"]
    print(f"[full] c5 solve: {pdhg.STATUS[r.status]} {r.iters} iterations (oracle {gs['iters']})", flush=True)
    assert r.status == pdhg.PDHG_OPTIMAL and r.iters == gs["iters"] and r.restarts == gs["restarts"]
    assert abs(r.pobj - gs["pobj"]) <= 1e-9 * abs(gs["pobj"])
    p = g.dual_push(1)
    # the face's decisions, recounted from the solve's answer
    a = sp.csr_matrix((lp.val, lp.col, lp.row_ptr), shape=(lp.m, lp.n))
    ax = a @ x
    sense = np.asarray(lp.sense)
    slack = np.where(sense == ord("<"), lp.b - ax, np.where(sense == ord(">"), ax - lp.b, 0.0))
    at_lo = np.isfinite(lp.l) & (x - lp.l <= 1e-6)
    at_up = np.isfinite(lp.u) & (lp.u - x <= 1e-6)
    assert p.n_cols_free == int(np.sum(~at_lo & ~at_up))
    assert p.n_rows_fixed == int(np.sum((sense != ord("=")) & (slack > 1e-6)))
    assert (p.n_cols_free, p.n_rows_fixed) == (gd["n_cols_free"], gd["n_rows_fixed"])
    x2, y2, _ = g.get_solution()
    np.testing.assert_array_equal(x2, x)
    ka = o.kkt(x2, y2)
    print(f"[full] c5 dual push: {p.iters} iterations (oracle {gd['iters']}); est_dual {p.before.est_dual} -> "
          f"{p.after.est_dual} (oracle's evaluation {ka.est_dual}; oracle's run {gd['est_dual_before']} -> "
          f"{gd['est_dual_after']})", flush=True)
    assert p.status == gd["status"] == pdhg.PDHG_PUSH_DONE and p.rel_d_push <= 1e-6
    assert (p.after.d_zero, p.after.est_dual) == (ka.d_zero, ka.est_dual)
    assert ka.rel_d <= 2e-6
    assert p.before.est_dual == gd["est_dual_before"]
    assert p.iters == gd["iters"]
    assert p.after.est_dual == gd["est_dual_after"]


def test_c2_setup_iterates_and_solve(c2):
    lp, o = c2
    _setup_and_first_iterates(lp, o, 2)
    g = pdhg.Solver(lp, timing=1)
    r = g.solve()
    x, y, _ = g.get_solution()
    k = o.kkt(x, y)
    print(f"[full] c2 solve: {pdhg.STATUS[r.status]} {r.iters} iterations; GPU KKT {r.rel_p:.3e}/{r.rel_d:.3e}/"
          f"{r.rel_gap:.3e}, oracle's evaluation {k.rel_p:.3e}/{k.rel_d:.3e}/{k.rel_gap:.3e}", flush=True)
    assert r.status == pdhg.PDHG_OPTIMAL
    assert max(k.rel_p, k.rel_d, k.rel_gap) <= 1e-6
    assert abs(r.pobj - k.pobj) <= 1e-12 * max(1.0, abs(k.pobj))


def test_c2_solve_and_push_against_the_oracle_full_run(c2):
    """The default workload's path in float64: the GPU's solve and corner push
    (the push on its free columns) against the oracle's own full run on the
    full push model (tests/golden/make_c2_oracle.py): iteration and restart
    counts, fixes, the corner counts after the push; the fixing decisions
    recounted from the GPU's answer and the pushed point's corner counts
    evaluated by the oracle's code."""
    lp, o = c2
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.json")))
    gs, gp = gold["solve"], gold["push"]
    g = pdhg.Solver(lp, timing=1)
    r = g.solve()
    x, y, z = g.get_solution()
    assert r.status == pdhg.PDHG_OPTIMAL == gs["status"]
    assert r.iters == gs["iters"] and r.restarts == gs["restarts"]
    assert abs(r.pobj - gs["pobj"]) <= 1e-9 * abs(gs["pobj"])
    zr = _z_of(lp, y)
    np.testing.assert_allclose(z, zr, rtol=0, atol=1e-12 * max(1.0, np.abs(zr).max()))
    p = g.corner_push(1)
    xp, yp, _ = g.get_solution()
    ka = o.kkt(xp, yp)
    print(f"[full] c2 vs the oracle's full run: solve {r.iters}/{gs['iters']} iterations, push {p.iters}/{gp['iters']}, "
          f"fixes {p.n_fix_lower + p.n_fix_upper}/{gp['n_fix_lower'] + gp['n_fix_upper']}, off-bound after "
          f"{p.after.p_off}/{gp['p_off_after']} (oracle's evaluation of the GPU's point {ka.p_off})", flush=True)
    assert p.n_fix_upper == int(np.sum(zr > 1e-6)) and p.n_fix_lower == int(np.sum(zr < -1e-6))
    assert (p.after.p_off, p.after.candidates, p.after.est_primal) == (ka.p_off, ka.candidates, ka.est_primal)
    assert (p.n_fix_lower, p.n_fix_upper, p.n_rows_to_eq) == (gp["n_fix_lower"], gp["n_fix_upper"], gp["n_rows_to_eq"])
    assert (p.before.p_off, p.before.candidates, p.before.est_primal) == \
        (gp["p_off_before"], gp["candidates_before"], gp["est_primal_before"])
    assert p.status == gp["status"] and p.iters == gp["iters"]
    assert (p.after.p_off, p.after.candidates, p.after.est_primal) == \
        (gp["p_off_after"], gp["candidates_after"], gp["est_primal_after"])
    assert abs(p.after.pobj - gp["pobj_after"]) <= 1e-9 * abs(gp["pobj_after"])


def test_batch_of_256_every_answer_checked_by_the_oracle():
    lps = [lpgen.config3_instance(i) for i in range(256)]
    print("[full] batch of 256 batched-family LPs, float64", flush=True)
    b = pdhg.Batch(lps, timing=1)
    res = b.solve()
    worst = 0.0
    for i in range(256):
        assert res[i].status == pdhg.PDHG_OPTIMAL, (i, pdhg.STATUS[res[i].status])
        x, y, _ = b.get_solution(i)
        k = OracleSolver(lps[i], power_iters=1).kkt(x, y)  # the report needs only the original model
        worst = max(worst, k.rel_p, k.rel_d, k.rel_gap)
        assert max(k.rel_p, k.rel_d, k.rel_gap) <= 1e-6, i
    print(f"[full] batch: all 256 OPTIMAL, worst float64 KKT by the oracle {worst:.3e}", flush=True)


def test_c1_fp32_mixed_reaches_the_original_optimum(c1):
    """FP32-mixed at full size, as the benchmark runs it: the float32-rounded
    c1 matrix has no optimum, and the iteration on float differences from its
    float64 anchors still ends at the float64 tolerance of the original model
    (the oracle's own KKT of the answer), in the float64 path's iteration
    count, and the push stops with the oracle's primal residual of the pushed
    point at the tolerance."""
    lp, o = c1
    g = pdhg.Solver(pdhg.DeviceLP(lp), precision="fp32", timing=1)
    r = g.solve()
    x, y, _ = g.get_solution()
    k = o.kkt(x, y)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.json")))["solve"]
    obj_err = abs(k.pobj - gold["pobj"]) / (1 + abs(gold["pobj"]))
    print(f"[full] c1 fp32: {pdhg.STATUS[r.status]} in {r.iters} iterations (float64 oracle run {gold['iters']}); "
          f"oracle's KKT {k.rel_p:.2e}/{k.rel_d:.2e}/{k.rel_gap:.2e}; objective error {obj_err:.2e}", flush=True)
    assert r.status == pdhg.PDHG_OPTIMAL
    assert max(k.rel_p, k.rel_d, k.rel_gap) <= 1e-6
    assert obj_err <= 1e-5
    assert r.iters <= 2 * gold["iters"]
    p = g.corner_push(1)
    xh = g.get_solution()[0]
    kh = o.kkt(xh, y)
    print(f"[full] c1 fp32 push: {pdhg.STATUS[p.status]} in {p.iters} iterations; oracle's primal residual of the "
          f"pushed x {kh.rel_p:.2e}; primal push estimate {p.before.est_primal} -> {p.after.est_primal}", flush=True)
    assert p.status == pdhg.PDHG_PUSH_DONE and kh.rel_p <= 1e-6
    assert (p.after.p_off, p.after.est_primal) == (kh.p_off, kh.est_primal)


def test_c2_fp32_mixed_against_the_oracle_full_run(c2):
    """The benchmark's default run itself (FP32-mixed, the LP in HBM, the push
    on its free columns) against the oracle's float64 full run: the answer
    meets the tolerance of the original model as the oracle evaluates it, the
    fixes are those the answer's float64 reduced costs call for, and the
    solve, the push and the corner they reach stay within a restart check of
    the oracle's (a float32 run may take another rounding path)."""
    lp, o = c2
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.json")))
    gs, gp = gold["solve"], gold["push"]
    g = pdhg.Solver(pdhg.DeviceLP(lp), precision="fp32", timing=1)
    r = g.solve()
    x, y, _ = g.get_solution()
    k = o.kkt(x, y)
    obj_err = abs(k.pobj - gs["pobj"]) / (1 + abs(gs["pobj"]))
    print(f"[full] c2 fp32: {pdhg.STATUS[r.status]} in {r.iters} iterations (oracle {gs['iters']}); oracle's KKT "
          f"{k.rel_p:.2e}/{k.rel_d:.2e}/{k.rel_gap:.2e}; objective error {obj_err:.2e}", flush=True)
    assert r.status == pdhg.PDHG_OPTIMAL
    assert max(k.rel_p, k.rel_d, k.rel_gap) <= 1e-6
    assert obj_err <= 2e-6  # both answers meet the relative gap test at 1e-6
    assert r.iters <= 1.25 * gs["iters"] + 128
    zr = _z_of(lp, y)
    p = g.corner_push(1)
    xh = g.get_solution()[0]
    kh = o.kkt(xh, y)
    print(f"[full] c2 fp32 push: {pdhg.STATUS[p.status]} in {p.iters} iterations (oracle {gp['iters']}); oracle's "
          f"primal residual of the pushed x {kh.rel_p:.2e}; off-bound {p.after.p_off} (oracle's run "
          f"{gp['p_off_after']}), primal push estimate {p.after.est_primal} (oracle's run {gp['est_primal_after']})",
          flush=True)
    assert p.n_fix_upper == int(np.sum(zr > 1e-6)) and p.n_fix_lower == int(np.sum(zr < -1e-6))
    assert p.status == pdhg.PDHG_PUSH_DONE and kh.rel_p <= 1e-6
    assert (p.after.p_off, p.after.candidates, p.after.est_primal) == (kh.p_off, kh.candidates, kh.est_primal)
    assert p.iters <= 1.25 * gp["iters"] + 128
    assert p.after.est_primal <= 1.25 * gp["est_primal_after"] + 128


def test_batch_of_256_fp32_all_optimal():
    """The 256-LP batched family in FP32-mixed mode: every LP optimal (the
    batch report's float64 KKT of each answer within the tolerance) and
    every push stopped primal feasible."""
    lps = [lpgen.config3_instance(i) for i in range(256)]
    b = pdhg.Batch(lps, precision="fp32", eps_rel=1e-6)
    res = b.solve()
    push = b.corner_push([1 + i for i in range(len(lps))])
    worst = max(max(r.rel_p, r.rel_d, r.rel_gap) for r in res)
    print(f"[full] batch of 256, fp32: {sum(r.status == pdhg.PDHG_OPTIMAL for r in res)} optimal, worst relative KKT "
          f"{worst:.2e}, pushes done {sum(p.status == pdhg.PDHG_PUSH_DONE for p in push)}", flush=True)
    assert all(r.status == pdhg.PDHG_OPTIMAL for r in res)
    assert worst <= 1e-6
    assert all(p.status == pdhg.PDHG_PUSH_DONE and p.after.rel_p <= 1.0000001e-6 for p in push)
    # spot-check a few answers with the oracle's own KKT evaluation
    for i in (0, 97, 255):
        o = OracleSolver(lps[i])
        x, y, _ = b.get_solve_solution(i)
        k = o.kkt(x, y)
        assert max(k.rel_p, k.rel_d, k.rel_gap) <= 1e-6, i
