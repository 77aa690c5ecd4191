"""Write c1_oracle.json: the oracle's full solve and corner push of the
100k x 400k power-law LP (seed 1, push seed 1), the workload the benchmark
runs, then the dual corner push from the pushed x on the same handle
(crossover's order, push seed 1).  Only the oracle and the seeded input
generator are used; a full run takes a few minutes on a multi-core host.

    python tests/golden/make_c1_oracle.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import OracleSolver  # noqa: E402
from paper_2511_13894_amd import lpgen  # noqa: E402


def main():
    lp = lpgen.config1()
    t0 = time.time()
    o = OracleSolver(lp, eps_rel=1e-6)
    r = o.solve()
    t1 = time.time()
    p = o.corner_push(1)
    t2 = time.time()
    d = o.dual_push(1)
    t3 = time.time()
    out = {
        "about": "oracle (oracle/pdhg_oracle.c, float64) on lpgen.config1(): m=100000, n=400000, seed 1; "
                 "solve to 1e-6 relative KKT, then corner push with seed 1 (Algorithm 1)",
        "solve": {"status": r.status, "iters": r.iters, "restarts": r.restarts, "pobj": r.pobj,
                  "rel_p": r.rel_p, "rel_d": r.rel_d, "rel_gap": r.rel_gap, "seconds": round(t1 - t0, 1)},
        "push": {"status": p.status, "iters": p.iters, "n_fix_lower": p.n_fix_lower, "n_fix_upper": p.n_fix_upper,
                 "n_rows_to_eq": p.n_rows_to_eq,
                 "p_off_before": p.before.p_off, "p_off_after": p.after.p_off,
                 "candidates_before": p.before.candidates, "candidates_after": p.after.candidates,
                 "est_primal_before": p.before.est_primal, "est_primal_after": p.after.est_primal,
                 "pobj_after": p.after.pobj, "seconds": round(t2 - t1, 1)},
        "dual_push_after_push": {"status": d.status, "iters": d.iters, "restarts": d.restarts,
                                 "n_cols_free": d.n_cols_free, "n_rows_fixed": d.n_rows_fixed,
                                 "rel_d_push": d.rel_d_push, "d_zero_before": d.before.d_zero,
                                 "d_zero_after": d.after.d_zero, "est_dual_before": d.before.est_dual,
                                 "est_dual_after": d.after.est_dual, "seconds": round(t3 - t2, 1)},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
