"""A small push objective (push_obj_scale < 1; section 5 discusses objective
terms near the dual tolerance): the GPU push on the scaled random objective
follows the oracle's."""
import numpy as np
import pytest

from oracle import OracleSolver
from paper_2511_13894_amd import lpgen, pdhg

pytestmark = pytest.mark.gpu


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max())) if a.size else 0.0


@pytest.mark.parametrize("scale", [1e-2, 1e-4, 1e-6])
@pytest.mark.parametrize("name,make", [("c0_s0", lambda: lpgen.config0(0)),
                                       ("ineq_ub_small", lambda: lpgen.config1(seed=3, m=300, n=1200))],
                         ids=["c0_s0", "ineq_ub_small"])
def test_small_push_objective_follows_the_oracle(name, make, scale):
    lp = make()
    g = pdhg.Solver(lp, eps_rel=1e-8, max_iter=400000, push_obj_scale=scale)
    o = OracleSolver(lp, eps_rel=1e-8, max_iter=400000, push_obj_scale=scale)
    g.solve()
    o.solve()
    pg, po = g.corner_push(17), o.corner_push(17)
    print(f"[scale] {name} scale {scale:g}: push {pg.iters} (oracle {po.iters}) iterations, "
          f"primal push estimate {pg.before.est_primal} -> {pg.after.est_primal} (oracle {po.after.est_primal})",
          flush=True)
    assert (pg.n_fix_lower, pg.n_fix_upper, pg.n_rows_to_eq) == (po.n_fix_lower, po.n_fix_upper, po.n_rows_to_eq)
    assert pg.status == po.status and pg.iters == po.iters
    assert rel_inf(g.get_solution()[0], o.solution()[0]) <= 1e-7
    assert (pg.after.p_off, pg.after.est_primal) == (po.after.p_off, po.after.est_primal)
