"""The push gate (section 4.2's selection rule) and the solve-answer hook,
on one LP and per LP in a batch, against the oracle."""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


def test_gate_single_lp_matches_the_oracle():
    lp = lpgen.config0(0)
    ref = OracleSolver(lp, eps_rel=1e-8)
    ref.solve()
    cand = ref.corner_push(3).before.candidates
    print(f"[gate] c0 seed 0: {cand} candidates after the solve", flush=True)
    for gmin, skip in ((cand + 1, True), (cand, False)):
        g = pdhg.Solver(lp, eps_rel=1e-8, push_gate=1, push_gate_rows=0.0, push_gate_min=gmin)
        o = OracleSolver(lp, eps_rel=1e-8, push_gate=1, push_gate_rows=0.0, push_gate_min=gmin)
        g.solve()
        o.solve()
        xs, ys, zs = g.get_solution()
        pg, po = g.corner_push(3), o.corner_push(3)
        assert pg.before.candidates == po.before.candidates == cand
        assert (pg.status == pdhg.PDHG_PUSH_SKIPPED) == skip and pg.status == po.status
        x1, y1, _ = g.get_solution()
        x2, y2, z2 = g.get_solve_solution()
        np.testing.assert_array_equal(x2, xs)
        np.testing.assert_array_equal(y2, ys)
        np.testing.assert_array_equal(z2, zs)
        if skip:
            assert pg.iters == 0 and pg.after.p_off == pg.before.p_off
            np.testing.assert_array_equal(x1, xs)
        else:
            assert pg.iters == po.iters and pg.iters > 0
            assert np.abs(x1 - xs).max() > 0.0  # the pushed point differs from the solve's
        with pytest.raises(pdhg.PdhgError):
            g.corner_push(3)  # one push per handle, skipped or not


def test_gate_per_lp_in_a_batch():
    lps = [lpgen.config3_instance(i, base_seed=5000, m_range=(40, 400)) for i in range(10)]
    seeds = [11 + i for i in range(len(lps))]
    b0 = pdhg.Batch(lps, eps_rel=1e-7, lanes_at=-64, lanes_a=-64)
    b0.solve()
    r0 = b0.corner_push(seeds)
    cands = [r.before.candidates for r in r0]
    thr = int(np.median(cands))
    b = pdhg.Batch(lps, eps_rel=1e-7, lanes_at=-64, lanes_a=-64, push_gate=1, push_gate_rows=0.0, push_gate_min=thr)
    b.solve()
    pre = [b.get_solution(i) for i in range(len(lps))]
    r = b.corner_push(seeds)
    n_skip = sum(c < thr for c in cands)
    print(f"[gate] batch of {len(lps)}: candidates {cands}, threshold {thr}: {n_skip} skipped", flush=True)
    assert 0 < n_skip < len(lps)
    for i, lp in enumerate(lps):
        o = OracleSolver(lp, eps_rel=1e-7, push_gate=1, push_gate_rows=0.0, push_gate_min=thr)
        o.solve()
        po = o.corner_push(seeds[i])
        assert r[i].status == po.status, (i, r[i].status, po.status)
        xs, ys, zs = b.get_solve_solution(i)
        np.testing.assert_array_equal(xs, pre[i][0])
        np.testing.assert_array_equal(zs, pre[i][2])
        x1 = b.get_solution(i)[0]
        if cands[i] < thr:
            assert r[i].status == pdhg.PDHG_PUSH_SKIPPED and r[i].iters == 0
            np.testing.assert_array_equal(x1, xs)
        else:
            # the other LPs being gated out does not change this LP's push
            assert (r[i].status, r[i].iters) == (r0[i].status, r0[i].iters)
            np.testing.assert_array_equal(x1, b0.get_solution(i)[0])
