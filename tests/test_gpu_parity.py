"""GPU (HIP, gfx950) path vs the CPU oracle, through the C-ABI.

Float64: the first 50 iterates agree to 1e-10 relative (inf-norm, unscaled),
Dr, Dc and eta to 1e-14, the solve reaches the oracle's status, iteration
count and objective, the corner push fixes the same columns and rows, and KKT
reports agree value by value (integer counts exactly).
"""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max())) if a.size else 0.0


def _cases():
    return [
        ("c0_s0", lambda: lpgen.config0(0)),
        ("c0_s7", lambda: lpgen.config0(7)),
        ("ineq_ub_small", lambda: lpgen.config1(seed=3, m=300, n=1200)),
        ("tiny_general_1", lambda: lpgen.tiny(1, m=3, n=6)),
        ("tiny_general_8", lambda: lpgen.tiny(8, m=4, n=9)),
        ("transport_12x30", lambda: lpgen.transportation(12, 30, seed=3)),
        ("ragged_deg_1_9", lambda: lpgen.planted(333, 777, seed=4, deg_range=(1, 9))),
        ("tiny_free_201", lambda: lpgen.tiny(201, m=3, n=7, with_free=True)),
        ("free_mixed_40x120", lambda: lpgen.tiny(207, m=40, n=120, with_free=True)),
        ("hand_free_variable", lambda: lpgen.from_dense([[1.0, -1.0]], [0.0], [1.0, 0.0], [-np.inf, 1.0],
                                                        [np.inf, np.inf], "=")),
    ]


@pytest.mark.parametrize("name,make", _cases(), ids=[c[0] for c in _cases()])
def test_first_50_iterates_fp64(name, make):
    print(f"[gpu] first-50 iterates: {name}", flush=True)
    lp = make()
    g = pdhg.Solver(lp)
    o = OracleSolver(lp)
    sg, so = g.get_scaling(), o.scaling()
    assert rel_inf(sg["dr"], so["dr"]) <= 1e-14
    assert rel_inf(sg["dc"], so["dc"]) <= 1e-14
    assert abs(sg["eta"] - so["eta"]) <= 1e-14 * so["eta"]
    assert abs(sg["omega"] - so["omega"]) <= 1e-13 * so["omega"]
    assert sg["power_steps"] == so["power_steps"]
    for t in range(1, 51):
        g.iterate(1)
        o.iterate(1)
        xg, yg = g.get_iterate()
        xo, yo = o.iterate_state()
        assert rel_inf(xg, xo) <= 1e-10, (t, rel_inf(xg, xo))
        assert rel_inf(yg, yo) <= 1e-10, (t, rel_inf(yg, yo))


@pytest.mark.parametrize("name,make", _cases(), ids=[c[0] for c in _cases()])
def test_solve_and_push_match_oracle_fp64(name, make):
    print(f"[gpu] solve + push: {name}", flush=True)
    lp = make()
    eps = 1e-8 if lp.n <= 2000 else 1e-6
    g = pdhg.Solver(lp, eps_rel=eps, max_iter=400000)
    o = OracleSolver(lp, eps_rel=eps, max_iter=400000)
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status == 0, (rg.status, ro.status)
    assert rg.iters == ro.iters and rg.restarts == ro.restarts
    assert max(rg.rel_p, rg.rel_d, rg.rel_gap) <= eps
    assert abs(rg.pobj - ro.pobj) <= 1e-6 * (1 + abs(ro.pobj))
    xg, yg, zg = g.get_solution()
    xo, yo, zo = o.solution()
    assert rel_inf(xg, xo) <= 1e-8 and rel_inf(yg, yo) <= 1e-8
    # push: same model modification (integer decisions) and same behaviour
    pg, po = g.corner_push(17), o.corner_push(17)
    assert (pg.n_fix_lower, pg.n_fix_upper, pg.n_rows_to_eq) == (po.n_fix_lower, po.n_fix_upper, po.n_rows_to_eq)
    assert pg.status == po.status
    assert pg.before.p_off == po.before.p_off and pg.before.candidates == po.before.candidates
    assert pg.iters == po.iters, (pg.iters, po.iters)
    xg2, yg2, zg2 = g.get_solution()
    xo2, _, _ = o.solution()
    np.testing.assert_array_equal(yg2, yg)
    assert pg.after.rel_p <= eps * 1.0000001 or pg.status != 3
    assert rel_inf(xg2, xo2) <= 1e-7


@pytest.mark.parametrize("seed", [0, 3])
def test_kkt_report_matches_oracle(seed):
    print(f"[gpu] kkt report seed {seed}", flush=True)
    lp = lpgen.config1(seed=seed, m=500, n=2000)
    rng = np.random.default_rng(seed)
    x = np.clip(rng.standard_normal(lp.n), lp.l, lp.u)
    x[rng.random(lp.n) < 0.3] = 0.0
    y = rng.standard_normal(lp.m)
    y[rng.random(lp.m) < 0.2] = 0.0
    g = pdhg.Solver(lp)
    o = OracleSolver(lp)
    kg, ko = g.kkt(x, y).as_dict(), o.kkt(x, y).as_dict()
    for key in kg:
        if key in ("p_off", "d_zero", "candidates", "est_primal", "est_dual"):
            assert kg[key] == ko[key], key
        else:
            assert kg[key] == pytest.approx(ko[key], rel=1e-12, abs=1e-12), key


def test_lane_counts_and_graph_replay_give_the_same_trajectory():
    """Every lanes-per-row choice and the captured-graph replay follow the
    oracle; replay is bitwise equal to eager launches."""
    lp = lpgen.config1(seed=9, m=400, n=1600)
    o = OracleSolver(lp)
    o.iterate(300)
    xo, yo = o.iterate_state()
    ref = None
    for la, lat in [(1, 1), (4, 2), (16, 8), (64, 64), (-32, -64), (-128, -256), (-256, -32), (-1032, -1064), (-1064, -1032), (0, 0)]:
        for graph in (0, 1):
            print(f"[gpu] lanes A={la} At={lat} graph={graph}", flush=True)
            g = pdhg.Solver(lp, lanes_a=la, lanes_at=lat, use_graph=graph)
            g.iterate(300)
            xg, yg = g.get_iterate()
            assert rel_inf(xg, xo) <= 1e-10 and rel_inf(yg, yo) <= 1e-10
            if la == 0:
                if ref is None:
                    ref = (xg, yg)
                else:
                    np.testing.assert_array_equal(xg, ref[0])
                    np.testing.assert_array_equal(yg, ref[1])


def test_autotuned_kernels_follow_the_oracle():
    lp = lpgen.config1(seed=4, m=600, n=2400)
    o = OracleSolver(lp)
    o.iterate(200)
    xo, yo = o.iterate_state()
    g = pdhg.Solver(lp, autotune=1, timing=1)
    g.iterate(200)
    xg, yg = g.get_iterate()
    t = g.get_timing()
    print(f"[gpu] autotune picked primal {t.lanes_at} dual {t.lanes_a}", flush=True)
    assert rel_inf(xg, xo) <= 1e-10 and rel_inf(yg, yo) <= 1e-10


def test_rerun_is_bitwise_deterministic():
    lp = lpgen.config0(5)
    outs = []
    for _ in range(2):
        g = pdhg.Solver(lp, eps_rel=1e-8)
        r = g.solve()
        x, y, _ = g.get_solution()
        outs.append((r.iters, x, y))
    assert outs[0][0] == outs[1][0]
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_edge_cases_empty_rows_columns_and_single_row(prec):
    """Float64: the oracle's iterations and objective.  FP32-mixed: optimal at
    the same tolerance with the oracle's objective (its anchored storage keeps
    float64 accuracy on these LPs)."""
    print(f"[gpu] edge cases {prec}", flush=True)
    a = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    lp = lpgen.from_dense(a, [2.0, 0.0], [1.0, 2.0, -1.0], [0, 0, 0], [np.inf, np.inf, 4.0], "==")
    for make in (lambda: lp, lambda: lpgen.from_dense([[1.0, 1.0, 1.0, 1.0]], [2.0], [0.0, 0.0, 0.0, 1.0],
                                                       [0, 0, 0, 0], [1, 1, 1, 1], "=")):
        q = make()
        g = pdhg.Solver(q, eps_rel=1e-10, precision=prec)
        o = OracleSolver(q, eps_rel=1e-10)
        rg, ro = g.solve(), o.solve()
        print(f"[gpu] edge {q.name} {prec}: {rg.iters} iterations (oracle {ro.iters}), pobj {rg.pobj!r} "
              f"(oracle {ro.pobj!r})", flush=True)
        assert rg.status == ro.status == 0
        if prec == "fp64":
            assert rg.iters == ro.iters
        assert abs(rg.pobj - ro.pobj) <= 1e-8


def test_iteration_limit_and_state_errors():
    lp = lpgen.config0(0)
    g = pdhg.Solver(lp, max_iter=100)
    with pytest.raises(pdhg.PdhgError) as e:
        g.corner_push(1)
    assert e.value.code == -2
    r = g.solve()
    assert r.status == pdhg.PDHG_ITER_LIMIT and r.iters == 100
    o = OracleSolver(lp, max_iter=100)
    ro = o.solve()
    assert r.rel_p == pytest.approx(ro.rel_p, rel=1e-9)
    bad = lpgen.config0(0)
    bad.l = bad.l.copy()
    bad.l[4] = 3.0
    bad.u = bad.u.copy()
    bad.u[4] = 2.0
    with pytest.raises(pdhg.PdhgError) as e:
        pdhg.Solver(bad)
    assert e.value.code == -1


def test_time_limit_status():
    lp = lpgen.config1(seed=2, m=2000, n=8000)
    g = pdhg.Solver(lp, time_limit=1e-9, eps_rel=1e-12)
    r = g.solve()
    assert r.status == pdhg.PDHG_TIME_LIMIT and r.iters >= 64


def test_duplicate_entries_and_unsorted_rows():
    lp = lpgen.config0(2)
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
    g = pdhg.Solver(lp2)
    o = OracleSolver(lp)
    g.iterate(40)
    o.iterate(40)
    xg, yg = g.get_iterate()
    xo, yo = o.iterate_state()
    assert rel_inf(xg, xo) <= 1e-10 and rel_inf(yg, yo) <= 1e-10


def _sell_cases():
    a = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    return [
        ("transport_40x100", lambda: lpgen.transportation(40, 100, seed=5)),
        ("ragged_deg_1_9", lambda: lpgen.planted(333, 777, seed=4, deg_range=(1, 9))),
        ("ineq_ub", lambda: lpgen.config1(seed=3, m=300, n=1200)),
        ("empty_row", lambda: lpgen.from_dense(a, [2.0, 0.0], [1.0, 2.0, -1.0], [0, 0, 0], [np.inf, np.inf, 4.0],
                                                "==")),
    ]


@pytest.mark.parametrize("name,make", _sell_cases(), ids=[c[0] for c in _sell_cases()])
def test_sliced_ellpack_dual_follows_the_oracle(name, make):
    """The sliced ELLPACK dual half (forced) on row counts that are not
    multiples of the slice height, ragged and empty rows: first 50 iterates
    within 1e-10, then the same solve and push as the oracle."""
    print(f"[gpu] sliced ELLPACK dual: {name}", flush=True)
    lp = make()
    g = pdhg.Solver(lp, lanes_a=-3032, eps_rel=1e-8)
    o = OracleSolver(lp, eps_rel=1e-8)
    assert g.get_timing().lanes_a == -3032
    for t in range(1, 51):
        g.iterate(1)
        o.iterate(1)
        xg, yg = g.get_iterate()
        xo, yo = o.iterate_state()
        assert rel_inf(xg, xo) <= 1e-10 and rel_inf(yg, yo) <= 1e-10, t
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status and rg.iters == ro.iters
    assert abs(rg.pobj - ro.pobj) <= 1e-9 * max(1.0, abs(ro.pobj))
    if rg.status == pdhg.PDHG_OPTIMAL:
        pg, po = g.corner_push(7), o.corner_push(7)
        assert (pg.iters, pg.n_fix_lower, pg.n_fix_upper) == (po.iters, po.n_fix_lower, po.n_fix_upper)


def _rows_permuted(lp, order):
    """The same LP with its rows in the given order."""
    order = np.asarray(order)
    lens = np.diff(lp.row_ptr)[order]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([lp.col[lp.row_ptr[r]:lp.row_ptr[r + 1]] for r in order])
    val = np.concatenate([lp.val[lp.row_ptr[r]:lp.row_ptr[r + 1]] for r in order])
    return lpgen.LP(lp.m, lp.n, rp, col, val, lp.b[order], lp.c, lp.l, lp.u, lp.sense[order], name=lp.name + "_perm")


def _alternating_transport():
    """Source and sink rows interleaved in runs of 5: more runs of one kind
    than the dual half has segments."""
    lp = lpgen.transportation(30, 80, seed=2)
    src, snk = list(range(30)), list(range(30, 110))
    order = []
    while src or snk:
        order += src[:5] + snk[:5]
        src, snk = src[5:], snk[5:]
    return _rows_permuted(lp, order)


def _seg_cases():
    a = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    return [
        # sources of 100 contiguous entries (32 lanes), sinks of 40 spread ones (16)
        ("transport_40x100", lambda: lpgen.transportation(40, 100, seed=5)),
        # sinks of 600 spread entries: past 512, 16 lanes; sources of 90 contiguous ones (32)
        ("transport_600x90", lambda: lpgen.transportation(600, 90, seed=8)),
        ("alternating_runs", _alternating_transport),
        ("ragged_deg_1_9", lambda: lpgen.planted(333, 777, seed=4, deg_range=(1, 9))),
        ("empty_row", lambda: lpgen.from_dense(a, [2.0, 0.0], [1.0, 2.0, -1.0], [0, 0, 0], [np.inf, np.inf, 4.0],
                                                "==")),
    ]


@pytest.mark.parametrize("name,make", _seg_cases(), ids=[c[0] for c in _seg_cases()])
def test_row_segment_dual_follows_the_oracle(name, make):
    """The dual half on row segments (forced), each run of contiguous or
    spread-out rows with its own lane-group width: first 50 iterates within
    1e-10, then the oracle's solve and push, the push on the free columns
    planning segments of its own rows."""
    print(f"[gpu] row-segment dual: {name}", flush=True)
    lp = make()
    g = pdhg.Solver(lp, lanes_a=-4000, eps_rel=1e-8)
    o = OracleSolver(lp, eps_rel=1e-8)
    assert g.get_timing().lanes_a == -4000
    for t in range(1, 51):
        g.iterate(1)
        o.iterate(1)
        xg, yg = g.get_iterate()
        xo, yo = o.iterate_state()
        assert rel_inf(xg, xo) <= 1e-10 and rel_inf(yg, yo) <= 1e-10, t
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status and rg.iters == ro.iters
    assert abs(rg.pobj - ro.pobj) <= 1e-9 * max(1.0, abs(ro.pobj))
    if rg.status == pdhg.PDHG_OPTIMAL:
        pg, po = g.corner_push(7), o.corner_push(7)
        assert (pg.iters, pg.n_fix_lower, pg.n_fix_upper) == (po.iters, po.n_fix_lower, po.n_fix_upper)
        assert rel_inf(g.get_solution()[0], o.solution()[0]) <= 1e-8


def test_row_segments_are_the_default_for_long_rows_and_one_segment_equals_its_lane_kernel():
    """Rows of more than 48 entries get the row-segment dual by default.  With
    more runs than segments the rows form one segment of 32 lanes, whose
    iterates equal the 32-lane kernel's bit for bit."""
    lp = lpgen.transportation(40, 100, seed=5)
    assert pdhg.Solver(lp).get_timing().lanes_a == -4000
    lp = _alternating_transport()
    out = []
    for la in (-4000, 32):
        for graph in (0, 1):
            g = pdhg.Solver(lp, lanes_a=la, use_graph=graph)
            r = g.solve()
            out.append((r.iters, g.get_iterate()))
    for it, (x, y) in out[1:]:
        assert it == out[0][0]
        np.testing.assert_array_equal(x, out[0][1][0])
        np.testing.assert_array_equal(y, out[0][1][1])


@pytest.mark.parametrize("name,make,prec", [
    ("transport_60x150", lambda: lpgen.transportation(60, 150, seed=7), "fp64"),
    ("transport_60x150_fp32", lambda: lpgen.transportation(60, 150, seed=7), "fp32"),
    ("multicommodity", lambda: lpgen.multicommodity(300, 2400, 4, seed=11, walks=40, max_len=8), "fp64"),
])
def test_uniform_column_kernel_equals_the_tiles(name, make, prec):
    """Columns of 2 (transportation) or 3 (multicommodity) entries: the
    library's choice, the one-thread-per-column kernel without row pointers,
    gives the 256-row tiles' iterates bit for bit, through the solve and the
    push on the free columns (whose model is uniform too)."""
    lp = make()
    out = []
    for lanes_at in (0, -256):
        g = pdhg.Solver(lp, precision=prec, lanes_at=lanes_at, eps_rel=1e-7)
        assert g.get_timing().lanes_at == -256
        r = g.solve()
        p = g.corner_push(3)
        out.append((r.iters, p.iters, g.get_solution()[0], g.get_iterate()))
    print(f"[uniform] {name}: solve {out[0][0]} / {out[1][0]}, push {out[0][1]} / {out[1][1]}", flush=True)
    assert out[0][:2] == out[1][:2]
    np.testing.assert_array_equal(out[0][2], out[1][2])
    np.testing.assert_array_equal(out[0][3][0], out[1][3][0])
    np.testing.assert_array_equal(out[0][3][1], out[1][3][1])
