"""Write c5_oracle.json: the oracle's full solve and dual corner push of the
100k x 400k primal-degenerate LP (lpgen.config5(), seed 5, push seed 1), the
workload of the dual push benchmark.  Only the oracle and the seeded input
generator are used; a full run takes several minutes on a multi-core host.

    python tests/golden/make_c5_oracle.py
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
    lp = lpgen.config5()
    t0 = time.time()
    o = OracleSolver(lp, eps_rel=1e-6)
    r = o.solve()
    t1 = time.time()
    print(f"solve: status {r.status}, {r.iters} iterations, {t1 - t0:.0f} s", flush=True)
    p = o.dual_push(1)
    t2 = time.time()
    out = {
        "about": "oracle (oracle/pdhg_oracle.c, float64) on lpgen.config5(): m=100000, n=400000, seed 5; "
                 "solve to 1e-6 relative KKT, then the dual corner push with seed 1",
        "solve": {"status": r.status, "iters": r.iters, "restarts": r.restarts, "pobj": r.pobj,
                  "rel_p": r.rel_p, "rel_d": r.rel_d, "rel_gap": r.rel_gap, "seconds": round(t1 - t0, 1)},
        "dual_push": {"status": p.status, "iters": p.iters, "restarts": p.restarts,
                      "n_cols_free": p.n_cols_free, "n_rows_fixed": p.n_rows_fixed,
                      "rel_d_push": p.rel_d_push,
                      "d_zero_before": p.before.d_zero, "d_zero_after": p.after.d_zero,
                      "est_dual_before": p.before.est_dual, "est_dual_after": p.after.est_dual,
                      "dobj_after": p.after.dobj, "seconds": round(t2 - t1, 1)},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
