"""Write c2_oracle.json: the oracle's full solve and corner push of the
2,000 x 5,000 transportation LP (n = 10M arcs, seed 2, push seed 1), the
benchmark's default workload.  Only the oracle and the seeded input
generator are used; the push runs on the full model (every fixed column
kept with equal bounds), about an hour on an 8-core host.

    python tests/golden/make_c2_oracle.py
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
    lp = lpgen.config2()
    t0 = time.time()
    o = OracleSolver(lp, eps_rel=1e-6)
    r = o.solve()
    t1 = time.time()
    print(f"solve: status {r.status}, {r.iters} iterations, {t1 - t0:.0f} s", flush=True)
    p = o.corner_push(1)
    t2 = time.time()
    out = {
        "about": "oracle (oracle/pdhg_oracle.c, float64) on lpgen.config2(): transportation 2000 x 5000, "
                 "m=7000, n=10000000, seed 2; solve to 1e-6 relative KKT, then corner push with seed 1 "
                 "(Algorithm 1) on the full model",
        "solve": {"status": r.status, "iters": r.iters, "restarts": r.restarts, "pobj": r.pobj,
                  "rel_p": r.rel_p, "rel_d": r.rel_d, "rel_gap": r.rel_gap, "seconds": round(t1 - t0, 1)},
        "push": {"status": p.status, "iters": p.iters, "n_fix_lower": p.n_fix_lower, "n_fix_upper": p.n_fix_upper,
                 "n_rows_to_eq": p.n_rows_to_eq,
                 "p_off_before": p.before.p_off, "p_off_after": p.after.p_off,
                 "candidates_before": p.before.candidates, "candidates_after": p.after.candidates,
                 "est_primal_before": p.before.est_primal, "est_primal_after": p.after.est_primal,
                 "pobj_after": p.after.pobj, "seconds": round(t2 - t1, 1)},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
