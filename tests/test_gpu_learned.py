"""Learned warm start of the corner push: features, learned fixes, the undo
rule, and the end-to-end pipeline on small LPs of the batched family."""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import learned, lpgen, pdhg

pytestmark = pytest.mark.gpu


def test_features_match_a_host_computation():
    """x, |c| and column norms (features 0, 2, 3) recomputed on the host from
    the solve's scaled quantities agree with the device features."""
    lp = lpgen.config0(2)
    s = pdhg.Solver(lp, record_history=1, eps_rel=1e-8)
    s.solve()
    f = s.features()
    assert f.shape == (lp.n, 16) and np.all(np.isfinite(f))
    assert np.all(f[:, 12:] == 0)
    # host side: unscaled solution -> scaled values via the scaling vectors
    sc = s.get_scaling()
    x, _, _ = s.get_solution()
    xs = x / sc["dc"]
    cs = np.abs(lp.c * sc["dc"])
    a = lp.dense() * sc["dr"][:, None] * sc["dc"][None, :]
    cn = np.linalg.norm(a, axis=0)

    def nrm(v):
        sc_ = np.sqrt(np.mean(v * v))
        sc_ = sc_ if sc_ > 0 else 1.0
        return np.sign(v) * np.log1p(np.abs(v) / sc_)

    np.testing.assert_allclose(f[:, 0], nrm(xs), atol=2e-6)
    np.testing.assert_allclose(f[:, 2], nrm(cs), atol=2e-6)
    np.testing.assert_allclose(f[:, 3], nrm(cn), atol=2e-6)
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
    f, y, free = learned.build_dataset(lps[:12], list(range(12)))
    assert f.shape[0] == y.shape[0] == free.shape[0] > 0
    net = pdhg.Mlp(2)
    rep = net.train(f, y, epochs=10, batch=1024, lr=2e-3, seed=1)
    z = net.forward(f)
    acc = float(np.mean((z > 0) == (y > 0.5)))
    print(f"[learned] small pipeline: {f.shape[0]} columns, positives {y.mean():.3f}, loss {rep.loss_first:.3f} -> "
          f"{rep.loss_last:.3f}, train accuracy {acc:.3f}", flush=True)
    assert rep.loss_last < rep.loss_first
    for lp in lps[12:]:
        a = learned.time_to_corner(lp, 3)
        b = learned.time_to_corner(lp, 3, net=net, theta=0.9)
        assert a is not None and b is not None
        assert b["push_status"] in ("PUSH_DONE", "ITER_LIMIT")
        assert b["rel_p_after"] <= 1.0000001e-6 or b["push_status"] != "PUSH_DONE"
