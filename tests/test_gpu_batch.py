"""Batch engine (many LPs of uneven sizes in one block-diagonal model) vs
the oracle run on each LP alone."""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


def _family(count, seed0, m_range=(40, 400)):
    return [lpgen.config3_instance(i, base_seed=seed0, m_range=m_range) for i in range(count)]


@pytest.mark.parametrize("kern", [0, -1064, -256])
def test_batch_matches_single_oracle_runs_fp64(kern):
    lps = _family(9, 5000)
    lps.append(lpgen.tiny(3, m=3, n=6))          # general bounds and senses
    lps.append(lpgen.transportation(6, 9, seed=4))
    lps.append(lpgen.tiny(207, m=40, n=120, with_free=True))  # free columns
    print(f"[batch] kern={kern}: sizes {[lp.m for lp in lps]}", flush=True)
    bt = pdhg.Batch(lps, eps_rel=1e-7, lanes_at=kern, lanes_a=kern)
    res = bt.solve()
    seeds = [11 + i for i in range(len(lps))]
    push = bt.corner_push(seeds)
    for i, lp in enumerate(lps):
        o = OracleSolver(lp, eps_rel=1e-7)
        ro = o.solve()
        assert res[i].status == ro.status == 0, (i, res[i].status, ro.status)
        assert res[i].iters == ro.iters, (i, res[i].iters, ro.iters)
        assert abs(res[i].pobj - ro.pobj) <= 1e-6 * (1 + abs(ro.pobj)), i
        xg, yg, zg = bt.get_solution(i)
        po = o.corner_push(seeds[i])
        assert (push[i].n_fix_lower, push[i].n_fix_upper, push[i].n_rows_to_eq) == \
            (po.n_fix_lower, po.n_fix_upper, po.n_rows_to_eq), i
        assert push[i].status == po.status, (i, push[i].status, po.status)
        assert push[i].iters == po.iters, (i, push[i].iters, po.iters)
        assert push[i].after.rel_p <= 1.0000001e-7
        assert push[i].before.p_off == po.before.p_off


def test_batch_iterates_equal_single_gpu_solve_with_same_kernels():
    """An LP inside a batch follows the same trajectory as the same LP
    solved alone with the same tiled kernels (the block-diagonal layout does
    not couple LPs)."""
    lps = _family(5, 6100)
    bt = pdhg.Batch(lps, eps_rel=1e-7, lanes_at=-1064, lanes_a=-1064)
    res = bt.solve()
    for i in (0, 3):
        g = pdhg.Solver(lps[i], eps_rel=1e-7, lanes_at=-1064, lanes_a=-1064)
        r = g.solve()
        assert r.iters == res[i].iters and r.status == res[i].status
        xg, yg, _ = g.get_solution()
        xb, yb, _ = bt.get_solution(i)
        np.testing.assert_allclose(xb, xg, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(yb, yg, rtol=1e-9, atol=1e-12)


def test_batch_fp32_mixed_and_report():
    lps = _family(12, 7000, m_range=(100, 2000))
    bt = pdhg.Batch(lps, precision="fp32", eps_rel=1e-6, timing=1, autotune=1)
    res = bt.solve()
    push = bt.corner_push(list(range(len(lps))))
    rep = bt.report()
    ok = sum(r.status == pdhg.PDHG_OPTIMAL for r in res)
    print(f"[batch] fp32: {ok}/{len(lps)} optimal, lockstep solve {rep.solve_lockstep_iters} push "
          f"{rep.push_lockstep_iters}, kernels {rep.lanes_at}/{rep.lanes_a}, primal {rep.primal_ms * 1e3:.1f} us "
          f"dual {rep.dual_ms * 1e3:.1f} us", flush=True)
    assert ok == len(lps)
    for i, lp in enumerate(lps):
        assert max(res[i].rel_p, res[i].rel_d, res[i].rel_gap) <= 2e-5
        opt = float(lp.c @ lp.x_star)
        assert abs(res[i].pobj - opt) <= 1e-4 * (1 + abs(opt))
        assert push[i].status in (pdhg.PDHG_PUSH_DONE, pdhg.PDHG_ITER_LIMIT)


def test_batch_state_errors():
    lps = _family(2, 8000)
    bt = pdhg.Batch(lps)
    with pytest.raises(pdhg.PdhgError):
        bt.corner_push([1, 2])
    with pytest.raises(pdhg.PdhgError):
        pdhg.Batch(lps, lanes_at=8)


def test_batch_from_device_memory_equals_host_create():
    """pdhg_batch_create_device on the same (row-sorted) LPs gives the same
    solves and pushes, bit for bit, as pdhg_batch_create; an LP whose column
    index passes the block's range but not its own n, or whose row pointers
    do not start at 0, is refused by the device checks."""
    import copy

    for prec in ("fp64", "fp32"):
        lps = _family(7, 5200)
        lps.append(lpgen.transportation(6, 9, seed=4))
        a = pdhg.Batch(lps, precision=prec, eps_rel=1e-6)
        db = pdhg.DeviceBatch(lps)
        b = pdhg.Batch(db, precision=prec, eps_rel=1e-6)
        for d in db.dev:
            d.free()  # the library holds its own copy
        ra, rb = a.solve(), b.solve()
        assert [(r.status, r.iters, r.restarts) for r in ra] == [(r.status, r.iters, r.restarts) for r in rb]
        seeds = [3 + i for i in range(len(lps))]
        pa, pb = a.corner_push(seeds), b.corner_push(seeds)
        assert [(r.status, r.iters) for r in pa] == [(r.status, r.iters) for r in pb]
        for i in range(len(lps)):
            for va, vb in zip(a.get_solution(i), b.get_solution(i)):
                np.testing.assert_array_equal(va, vb)
        print(f"[batch] {prec}: device create equals host create on {len(lps)} LPs "
              f"(solve iterations {[r.iters for r in rb]})", flush=True)
    base = _family(3, 5300)
    x = copy.deepcopy(base[1])
    x.col = x.col.copy()
    x.col[x.row_ptr[2]] = x.n  # inside the block (LP 2 follows) but past this LP's columns
    y = copy.deepcopy(base[1])
    y.row_ptr = y.row_ptr.copy()
    y.row_ptr[0] = 1  # row pointers not starting at 0
    for bad, msg in ((x, "column index out of range"), (y, "row_ptr")):
        db = pdhg.DeviceBatch([base[0], bad, base[2]])
        with pytest.raises(pdhg.PdhgError) as e:
            pdhg.Batch(db)
        print(f"[batch] refused: {e.value}", flush=True)
        assert msg in str(e.value)
