"""FP32-mixed mode against the FP64 oracle: the error is stated, not bitwise.

The mixed mode streams the matrix, the bounds and two n-vectors in FP32 and
keeps y and every check in float64.  The n-vectors are stored as float
differences from a float64 anchor: x - x_a and xbar - x_a.  With the
matrix's rounding error E = Ahat - fl32(Ahat), the kernels read the anchored
right-hand side bhat - Ahat x_a and the corrected objective chat - E'y_a,
computed in float64 at every anchor (restart or phase start), so the only
errors are E times a difference (x - x_a or y - y_a) and the differences'
own rounding, which shrink as the restart cycle converges.  Every check
evaluates the float64 products fl32(Ahat) v + E v, so a reported OPTIMAL is
an optimum of the original model at the tolerance.
"""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu

EPS = 1e-6


def _rel(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max()))


CASES = [
    ("c0_s0", lambda: lpgen.config0(0)),
    ("c0_s3", lambda: lpgen.config0(3)),
    ("transport_40x100", lambda: lpgen.transportation(40, 100, seed=5)),
    ("free_mixed_40x120", lambda: lpgen.tiny(207, m=40, n=120, with_free=True)),
    # the c1 family: its float32-rounded LP has no optimum (checked with HiGHS)
    ("c1_family_m500_s0", lambda: lpgen.config1(seed=0, m=500, n=2000)),
    ("c1_family_m500_s1", lambda: lpgen.config1(seed=1, m=500, n=2000)),
    ("c1_family_m500_s2", lambda: lpgen.config1(seed=2, m=500, n=2000)),
    # batched-family LPs the uncorrected float32 iteration solved 20-40x slower or not at all
    ("batched_1", lambda: lpgen.config3_instance(1)),
    ("batched_20", lambda: lpgen.config3_instance(20)),
    ("batched_100", lambda: lpgen.config3_instance(100)),
    # the primal-degenerate family: its rows cancel near the optimum, where
    # float32 iterates (not differences) stalled the solve
    ("c5_family_m500", lambda: lpgen.config5(seed=5, m=500, n=2000)),
    ("c5_family_m1000", lambda: lpgen.config5(seed=5, m=1000, n=4000)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fp32_mixed_solves_the_original_lp(name, make):
    """The mixed path reaches the oracle's status at the float64 tolerance of
    the original model, in about as many iterations as float64 (the anchored
    iteration's fixed point is the original LP's; the matrix rounding may move
    a restart by a check), and the push stops with the float64 primal
    residual at the tolerance."""
    print(f"[fp32] {name}", flush=True)
    lp = make()
    g = pdhg.Solver(lp, precision="fp32", eps_rel=EPS, max_iter=200000)
    o = OracleSolver(lp, eps_rel=EPS, max_iter=200000)
    rg, ro = g.solve(), o.solve()
    assert ro.status == 0
    xg, yg, _ = g.get_solution()
    xo, yo, _ = o.solution()
    ko = o.kkt(xg, yg)  # the oracle's own evaluation of the float32 path's answer
    obj_err = abs(rg.pobj - ro.pobj) / (1 + abs(ro.pobj))
    print(f"[fp32] {name}: {pdhg.STATUS[rg.status]} in {rg.iters} iterations (float64 oracle {ro.iters}); "
          f"oracle's KKT of the answer {ko.rel_p:.2e}/{ko.rel_d:.2e}/{ko.rel_gap:.2e}; objective error "
          f"{obj_err:.2e}; |x - x_oracle| {_rel(xg, xo):.2e}, |y - y_oracle| {_rel(yg, yo):.2e}", flush=True)
    assert rg.status == pdhg.PDHG_OPTIMAL, pdhg.STATUS[rg.status]
    assert max(ko.rel_p, ko.rel_d, ko.rel_gap) <= EPS
    assert abs(ko.rel_p - rg.rel_p) <= 1e-12 and abs(ko.rel_gap - rg.rel_gap) <= 1e-12
    assert obj_err <= 2 * EPS  # both answers meet the relative gap test at EPS
    assert rg.iters <= 1.25 * ro.iters + 128
    pg = g.corner_push(5)
    xh = g.get_solution()[0]
    kh = o.kkt(xh, yg)
    print(f"[fp32] {name}: push {pdhg.STATUS[pg.status]} in {pg.iters} iterations, oracle's primal residual of "
          f"the pushed x {kh.rel_p:.2e}, off-bound {pg.before.p_off} -> {pg.after.p_off}", flush=True)
    assert pg.status == pdhg.PDHG_PUSH_DONE
    assert kh.rel_p <= EPS


def test_fp32_first_iterates_track_the_oracle():
    """The first iterates in FP32 stay within a few FP32 ulps (relative to the
    iterate's scale) of the float64 trajectory."""
    lp = lpgen.config0(4)
    g = pdhg.Solver(lp, precision="fp32")
    o = OracleSolver(lp)
    worst = 0.0
    for t in range(1, 21):
        g.iterate(1)
        o.iterate(1)
        xg, yg = g.get_iterate()
        xo, yo = o.iterate_state()
        worst = max(worst, _rel(xg, xo), _rel(yg, yo))
    print(f"[fp32] worst relative deviation over 20 iterates: {worst:.2e}", flush=True)
    assert worst <= 1e-4


@pytest.mark.parametrize("i", [105, 157])
def test_fp32_status_is_backed_by_float64_kkt(i):
    """The status and KKT values the mixed path reports are the float64
    original model's."""
    lp = lpgen.config3_instance(i)
    g = pdhg.Solver(lp, precision="fp32", eps_rel=EPS, max_iter=60000)
    r = g.solve()
    o = OracleSolver(lp, eps_rel=EPS)
    x, y, _ = g.get_solution()
    k = o.kkt(x, y)
    print(f"[fp32] batched-family LP {i}: {pdhg.STATUS[r.status]} after {r.iters} iterations, float64 KKT "
          f"{r.rel_p:.2e}/{r.rel_d:.2e}/{r.rel_gap:.2e} (oracle {k.rel_p:.2e}/{k.rel_d:.2e}/{k.rel_gap:.2e})",
          flush=True)
    assert r.status == pdhg.PDHG_OPTIMAL
    assert max(k.rel_p, k.rel_d, k.rel_gap) <= EPS


def test_fp32_batch_solves_every_lp():
    """The batch engine in the mixed mode (per-LP anchored data): every
    LP optimal at the float64 tolerance, each confirmed by the oracle, and
    every push stopped primal feasible."""
    lps = [lpgen.config3_instance(i, base_seed=48000, m_range=(100, 3000)) for i in range(8)]
    lps.append(lpgen.config1(seed=2, m=500, n=2000))
    b = pdhg.Batch(lps, precision="fp32", eps_rel=EPS, max_iter=200000)
    res = b.solve()
    push = b.corner_push([7 + i for i in range(len(lps))])
    for i, lp in enumerate(lps):
        o = OracleSolver(lp, eps_rel=EPS)
        x, y, _ = b.get_solve_solution(i)
        k = o.kkt(x, y)
        xh = b.get_solution(i)[0]
        kh = o.kkt(xh, y)
        print(f"[fp32] batch LP {i} (m={lp.m}): {pdhg.STATUS[res[i].status]} in {res[i].iters} iterations, oracle's "
              f"KKT {k.rel_p:.2e}/{k.rel_d:.2e}/{k.rel_gap:.2e}; push {pdhg.STATUS[push[i].status]} "
              f"{push[i].iters} iterations, pushed residual {kh.rel_p:.2e}", flush=True)
        assert res[i].status == pdhg.PDHG_OPTIMAL, i
        assert max(k.rel_p, k.rel_d, k.rel_gap) <= EPS, i
        assert push[i].status == pdhg.PDHG_PUSH_DONE and kh.rel_p <= EPS, i
