"""Learned warm start of the corner push: features, learned fixes, the undo
rule, and the end-to-end pipeline on small LPs of the batched family."""
import numpy as np
import pytest

from oracle import OracleSolver, push_uniform
from paper_2511_13894_amd import learned, lpgen, pdhg

pytestmark = pytest.mark.gpu


def test_features_match_a_host_computation():
    """Features 0, 2, 3 and 12-15 recomputed on the host from the solve's
    scaled quantities and the published splitmix64 draw agree with the
    device features."""
    lp = lpgen.config0(2)
    s = pdhg.Solver(lp, record_history=1, eps_rel=1e-8)
    s.solve()
    seed = 77
    f = s.features(seed)
    assert f.shape == (lp.n, 16) and np.all(np.isfinite(f))
    sc = s.get_scaling()
    x, _, _ = s.get_solution()
    dc = sc["dc"]
    xs = x / dc
    cs = np.abs(lp.c * dc)
    a = lp.dense() * sc["dr"][:, None] * dc[None, :]
    cn = np.linalg.norm(a, axis=0)
    lo, hi = lp.l / dc, lp.u / dc
    flo, fhi = np.isfinite(lo), np.isfinite(hi)
    pc = dc * np.array([push_uniform(seed, j) for j in range(lp.n)])
    dl = np.where(flo, xs - np.where(flo, lo, 0), -1.0)
    du = np.where(fhi, np.where(fhi, hi, 0) - xs, -1.0)
    both = flo & fhi & (hi > lo)
    rel = np.where(both, (xs - np.where(both, lo, 0)) / np.where(both, hi - lo, 1), -1.0)

    def nrm(v):
        sc_ = np.sqrt(np.mean(v * v))
        sc_ = sc_ if sc_ > 0 else 1.0
        return np.sign(v) * np.log1p(np.abs(v) / sc_)

    for q, v in ((0, xs), (2, cs), (3, cn), (12, pc), (13, dl), (14, du), (15, rel)):
        np.testing.assert_allclose(f[:, q], nrm(v), atol=2e-6, err_msg=f"feature {q}")
    # trend features exist once restarts happened
    assert np.abs(f[:, 4:12]).sum() > 0


def test_learned_push_fixes_undoes_and_stays_feasible():
    """With theta tiny every free column is fixed at its nearer bound; the
    undo rule releases the wrong ones at push checks, and the push still ends
    primal feasible at the tolerance with the solve's y and z."""
    lp = lpgen.config0(3)
    net = pdhg.Mlp(1)
    s = pdhg.Solver(lp, record_history=1, eps_rel=1e-7)
    r = s.solve()
    x0, y0, z0 = s.get_solution()
    p = s.corner_push_learned(net, 1e-4, 5)
    print(f"[learned] tiny theta: fixed {p.n_learned_fix}, undone {p.n_learned_undo}, status "
          f"{pdhg.STATUS[p.status]}, push iters {p.iters}, off-bound {p.before.p_off} -> {p.after.p_off}", flush=True)
    free = int(np.sum(np.abs(z0) <= 1e-6))
    assert 0 < p.n_learned_fix <= free
    assert p.n_learned_undo > 0
    assert p.status == pdhg.PDHG_PUSH_DONE
    assert p.after.rel_p <= 1.0000001e-7
    x1, y1, z1 = s.get_solution()
    np.testing.assert_array_equal(y1, y0)
    assert np.all(x1 >= lp.l - 1e-9)
    # same fixing decisions as the oracle for the plain part
    o = OracleSolver(lp, eps_rel=1e-7)
    o.solve()
    po = o.corner_push(5)
    assert (p.n_fix_lower, p.n_fix_upper) == (po.n_fix_lower, po.n_fix_upper)


def test_pipeline_trains_and_compares():
    lps = [lpgen.config3_instance(i, base_seed=45000, m_range=(60, 200)) for i in range(16)]
    f, y = learned.build_dataset(lps[:12], list(range(12)))
    assert f.shape[0] == y.shape[0] > 0
    net = pdhg.Mlp(2)
    rep = net.train(f, y, epochs=10, batch=1024, lr=2e-3, seed=1)
    z = net.forward(f)
    acc = float(np.mean((z > 0) == (y > 0.5)))
    print(f"[learned] small pipeline: {f.shape[0]} free columns, positives {y.mean():.3f}, loss "
          f"{rep.loss_first:.3f} -> {rep.loss_last:.3f}, train accuracy {acc:.3f}", flush=True)
    assert rep.loss_last < rep.loss_first
    rows = learned.theta_table(net, f, y)
    assert len(rows) == len(learned.THETAS)
    for lp in lps[12:]:
        a = learned.time_to_corner(lp, 3)
        b = learned.time_to_corner(lp, 3, net=net, theta=0.9)
        assert a is not None and b is not None
        assert b["push_status"] in ("PUSH_DONE", "ITER_LIMIT")
        if b["push_status"] == "PUSH_DONE":
            assert b["rel_p_after"] <= 1.0000001e-6


def test_batch_features_and_learned_push_match_single_lp_runs():
    """Inside a batch (same kernels), an LP's features equal those of the LP
    solved alone, and the learned push fixes the same columns; every push
    still ends primal feasible."""
    lps = [lpgen.config3_instance(i, base_seed=46000, m_range=(60, 200)) for i in range(4)]
    seeds = [11 + i for i in range(4)]
    kw = dict(record_history=1, eps_rel=1e-7, lanes_at=-1064, lanes_a=-1064)
    b = pdhg.Batch(lps, **kw)
    b.solve()
    fb = b.features(seeds)
    net = pdhg.Mlp(4)
    push = b.corner_push_learned(net, 1e-4, seeds)
    for i in (0, 2):
        g = pdhg.Solver(lps[i], **kw)
        g.solve()
        fg = g.features(seeds[i])
        np.testing.assert_allclose(fb[i], fg, rtol=0, atol=2e-6)
        p = g.corner_push_learned(net, 1e-4, seeds[i])
        print(f"[learned] batch LP {i}: fixes {push[i].n_learned_fix} (alone {p.n_learned_fix}), undone "
              f"{push[i].n_learned_undo} (alone {p.n_learned_undo}), push iters {push[i].iters} (alone {p.iters})",
              flush=True)
        assert push[i].n_learned_fix == p.n_learned_fix > 0
    for i, p in enumerate(push):
        assert p.status == pdhg.PDHG_PUSH_DONE, (i, pdhg.STATUS[p.status])
        assert p.after.rel_p <= 1.0000001e-7


def test_learned_push_on_free_columns_equals_the_full_push():
    """push_compact drops only the plain rule's fixes in the learned push:
    learned fixes stay, so the undo rule frees the same columns and the push
    follows the full model's, single and batched."""
    lp = lpgen.config0(3)
    net = pdhg.Mlp(1)
    out = {}
    for compact in (0, 1):
        s = pdhg.Solver(lp, record_history=1, eps_rel=1e-7, push_compact=compact)
        s.solve()
        p = s.corner_push_learned(net, 1e-4, 5)
        out[compact] = (p, s.get_solution()[0])
    (p0, x0), (p1, x1) = out[0], out[1]
    print(f"[learned] compact push: fixed {p1.n_learned_fix}/{p0.n_learned_fix}, undone {p1.n_learned_undo}/"
          f"{p0.n_learned_undo}, iterations {p1.iters}/{p0.iters}", flush=True)
    assert (p1.n_learned_fix, p1.n_learned_undo, p1.status, p1.iters) == \
        (p0.n_learned_fix, p0.n_learned_undo, p0.status, p0.iters)
    assert np.abs(x1 - x0).max() <= 1e-8 * max(1.0, np.abs(x0).max())
    lps = [lpgen.config3_instance(i, base_seed=5000, m_range=(40, 300)) for i in range(6)]
    res = {}
    for compact in (0, 1):
        b = pdhg.Batch(lps, record_history=1, eps_rel=1e-7, push_compact=compact)
        b.solve()
        r = b.corner_push_learned(net, 1e-4, [5 + i for i in range(len(lps))])
        res[compact] = (r, [b.get_solution(i)[0] for i in range(len(lps))])
    for i in range(len(lps)):
        a, c = res[0][0][i], res[1][0][i]
        assert (c.n_learned_fix, c.n_learned_undo, c.status, c.iters) == \
            (a.n_learned_fix, a.n_learned_undo, a.status, a.iters), i
        xa, xc = res[0][1][i], res[1][1][i]
        assert np.abs(xc - xa).max() <= 1e-8 * max(1.0, np.abs(xa).max()), i


def _feature_bound(fo, so):
    """Per-element bound on |GPU - oracle| for the normalised features of an
    FP64 solve.  The device rounds each raw value v to float32 before the
    map t = sign(v) ln(1 + |v|/s) (|dt| <= |dv| / (s + |v|)) and stores the
    restart history in float32, so a trend feature v = h - base carries the
    rounding of h = v + base (base = x_j for 4..7, z_j for 8..11); the
    result is rounded to float32 once more.  Both sides also carry their
    float64 trajectories, which agree to about 1e-12 relative after
    thousands of iterations (different summation order): 1e-10 of the x or
    objective scale covers that in every x- or z-derived feature.  Raw values
    come back from the oracle's own features and scales."""
    u = 2.0 ** -24
    v = np.sign(fo) * so[None, :] * np.expm1(np.abs(fo))
    dv = u * np.abs(v)
    base = np.zeros_like(v)
    base[:, 4:8] = np.abs(v[:, 0:1])
    base[:, 8:12] = np.abs(v[:, 1:2])
    dv = dv + u * (np.abs(v) + base)
    xs = max(1.0, np.abs(v[:, 0]).max())
    cs = max(1.0, np.abs(v[:, 2]).max())
    traj = np.zeros(16)
    traj[[0, 4, 5, 6, 7, 13, 14, 15]] = 1e-10 * xs
    traj[[1, 8, 9, 10, 11]] = 1e-10 * cs
    dv = dv + traj[None, :]
    return 4.0 * (dv / (so[None, :] + np.abs(v)) + u * np.abs(fo)) + 1e-12


LEARNED_CASES = [
    ("c0_s3", lambda: lpgen.config0(3)),
    ("ineq_ub_300x1200", lambda: lpgen.config1(seed=3, m=300, n=1200)),
    ("ragged_deg_1_9", lambda: lpgen.planted(333, 777, seed=4, deg_range=(1, 9), upper_frac=0.3)),
    ("tiny_general_8", lambda: lpgen.tiny(8, m=4, n=9)),
]


@pytest.mark.parametrize("name,make", LEARNED_CASES, ids=[c[0] for c in LEARNED_CASES])
def test_features_follow_the_oracle(name, make):
    """All 16 features, the restart trends included, equal the oracle's
    (computed in float64 from its own restart history) within the float32
    storage bound of the device."""
    print(f"[learned] features vs oracle: {name}", flush=True)
    lp = make()
    g = pdhg.Solver(lp, record_history=1, eps_rel=1e-7)
    o = OracleSolver(lp, record_history=1, eps_rel=1e-7)
    rg, ro = g.solve(), o.solve()
    assert (rg.iters, rg.restarts) == (ro.iters, ro.restarts)
    fg = g.features(21).astype(np.float64)
    fo, so = o.features(21, with_scale=True)
    bound = _feature_bound(fo, so)
    err = np.abs(fg - fo)
    worst = np.unravel_index(np.argmax(err / bound), err.shape)
    print(f"[learned] {name}: {ro.restarts} restarts, max |gpu - oracle| {err.max():.2e}, worst ratio to bound "
          f"{(err / bound).max():.3f} at column {worst[0]} feature {worst[1]}", flush=True)
    assert np.all(err <= bound), (worst, fg[worst], fo[worst], bound[worst])
    if ro.restarts > 0:
        assert np.abs(fo[:, 4]).max() > 0  # the trend features are exercised


@pytest.mark.parametrize("compact", [1, 0])
@pytest.mark.parametrize("theta", [0.5, 0.9])
@pytest.mark.parametrize("name,make", LEARNED_CASES, ids=[c[0] for c in LEARNED_CASES])
def test_learned_push_from_logits_follows_the_oracle(name, make, theta, compact):
    """The learned warm start from the same seeded logits on both sides:
    the same plain and learned fixes, the same undos at the push checks, the
    same push iterations and status, and the same pushed point."""
    print(f"[learned] logits push vs oracle: {name} theta {theta} compact {compact}", flush=True)
    lp = make()
    logits = np.random.default_rng(1234).normal(0.0, 2.0, lp.n).astype(np.float32)
    g = pdhg.Solver(lp, eps_rel=1e-7, push_compact=compact)
    o = OracleSolver(lp, eps_rel=1e-7)
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status == 0 and rg.iters == ro.iters
    pg = g.corner_push_logits(logits, theta, 5)
    po = o.corner_push_learned(logits, theta, 5)
    got = (pg.n_fix_lower, pg.n_fix_upper, pg.n_rows_to_eq, pg.n_learned_fix, pg.n_learned_undo, pg.status, pg.iters)
    want = (po.n_fix_lower, po.n_fix_upper, po.n_rows_to_eq, po.n_learned_fix, po.n_learned_undo, po.status, po.iters)
    print(f"[learned] {name}: (lower, upper, rows, learned fixes, undone, status, iterations) gpu {got} / oracle {want}",
          flush=True)
    assert got == want
    assert (pg.after.p_off, pg.after.candidates) == (po.after.p_off, po.after.candidates)
    xg, yg, _ = g.get_solution()
    xo, yo, _ = o.solution()
    assert np.abs(xg - xo).max() <= 1e-7 * max(1.0, np.abs(xo).max())
    np.testing.assert_array_equal(yg, g.get_solve_solution()[1])


def test_batch_learned_push_from_logits_follows_the_oracle():
    """The batch engine's learned push from caller logits: every LP's fixes,
    undos, push iterations and pushed point equal the oracle's on that LP."""
    lps = [lpgen.config3_instance(i, base_seed=47000, m_range=(60, 300)) for i in range(5)]
    seeds = [31 + i for i in range(len(lps))]
    logits = np.random.default_rng(99).normal(0.0, 2.0, sum(lp.n for lp in lps)).astype(np.float32)
    b = pdhg.Batch(lps, eps_rel=1e-7)
    b.solve()
    res = b.corner_push_logits(logits, 0.6, seeds)
    off = 0
    for i, lp in enumerate(lps):
        lg = logits[off: off + lp.n]
        off += lp.n
        o = OracleSolver(lp, eps_rel=1e-7)
        o.solve()
        po = o.corner_push_learned(lg, 0.6, seeds[i])
        pg = res[i]
        got = (pg.n_fix_lower, pg.n_fix_upper, pg.n_learned_fix, pg.n_learned_undo, pg.status, pg.iters)
        want = (po.n_fix_lower, po.n_fix_upper, po.n_learned_fix, po.n_learned_undo, po.status, po.iters)
        print(f"[learned] batch LP {i} (m={lp.m}): gpu {got} / oracle {want}", flush=True)
        assert got == want, i
        xg = b.get_solution(i)[0]
        xo = o.solution()[0]
        assert np.abs(xg - xo).max() <= 1e-7 * max(1.0, np.abs(xo).max()), i


@pytest.mark.parametrize("compact", [1, 0])
@pytest.mark.parametrize("name,make", LEARNED_CASES[:3], ids=[c[0] for c in LEARNED_CASES[:3]])
def test_learned_push_fp32_mixed(name, make, compact):
    """The learned warm start in the mixed mode, where a learned fix sets the
    float64 anchor (the stored difference 0): the push ends primal feasible on
    the original model as the oracle evaluates it, and the learned fixes and
    undos stay within a few columns of the float64 oracle's from the same
    logits (the float32 solve's answer moves reduced costs near eps_abs)."""
    print(f"[learned] fp32 logits push: {name} compact {compact}", flush=True)
    lp = make()
    logits = np.random.default_rng(1234).normal(0.0, 2.0, lp.n).astype(np.float32)
    g = pdhg.Solver(lp, eps_rel=1e-6, precision="fp32", push_compact=compact)
    o = OracleSolver(lp, eps_rel=1e-6)
    rg, ro = g.solve(), o.solve()
    assert rg.status == ro.status == 0
    y_solve = g.get_solution()[1]
    pg = g.corner_push_logits(logits, 0.6, 5)
    po = o.corner_push_learned(logits, 0.6, 5)
    xg = g.get_solution()[0]
    k = o.kkt(xg, y_solve)
    print(f"[learned] {name} fp32: status {pdhg.STATUS[pg.status]} in {pg.iters} iterations (oracle {po.iters}); "
          f"learned fixes {pg.n_learned_fix} (oracle {po.n_learned_fix}), undone {pg.n_learned_undo} "
          f"(oracle {po.n_learned_undo}); oracle's primal residual of the pushed x {k.rel_p:.2e}", flush=True)
    assert pg.status == pdhg.PDHG_PUSH_DONE
    assert k.rel_p <= 1e-6
    assert pg.n_learned_fix > 0
    assert abs(pg.n_learned_fix - po.n_learned_fix) <= max(2, po.n_learned_fix // 50)
    assert abs(pg.n_learned_undo - po.n_learned_undo) <= max(2, po.n_learned_undo // 20)
