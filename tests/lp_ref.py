"""Independent reference solvers used to pin the oracle (test helpers only).

* ``vertex_enumeration``: brute force over every choice of n linearly
  independent active constraints of a tiny general-form LP; exact optimum up
  to linear-solve rounding.
* ``highs``: scipy's HiGHS ``linprog`` on the same general form.
* ``knapsack_greedy``: closed form of the continuous knapsack.
None of them shares code with the oracle or with the GPU library.
"""
from __future__ import annotations

import itertools

import numpy as np


def _constraints(lp, a=None):
    """Rows of G x (op) h as a list of (g, h, kind) with kind in {'eq', 'le'}."""
    a = lp.dense() if a is None else a
    cons = []
    for i in range(lp.m):
        s = chr(lp.sense[i])
        if s == "=":
            cons.append((a[i], lp.b[i], "eq"))
        elif s == "<":
            cons.append((a[i], lp.b[i], "le"))
        else:
            cons.append((-a[i], -lp.b[i], "le"))
    for j in range(lp.n):
        e = np.zeros(lp.n)
        e[j] = 1.0
        if np.isfinite(lp.l[j]):
            cons.append((-e, -lp.l[j], "le"))
        if np.isfinite(lp.u[j]):
            cons.append((e, lp.u[j], "le"))
    return cons


def vertices(lp, c=None, tol=1e-9, l=None, u=None, sense=None):
    """All vertices of the feasible set {x : rows, l <= x <= u} of a tiny LP."""
    import copy

    lp2 = copy.copy(lp)
    if l is not None:
        lp2.l = np.asarray(l, dtype=float)
    if u is not None:
        lp2.u = np.asarray(u, dtype=float)
    if sense is not None:
        lp2.sense = np.frombuffer(bytes(sense), dtype=np.uint8).copy()
    cons = _constraints(lp2)
    eqs = [q for q in cons if q[2] == "eq"]
    les = [q for q in cons if q[2] == "le"]
    n = lp.n
    k = n - len(eqs)
    out = []
    if k < 0:
        return out
    for pick in itertools.combinations(range(len(les)), k):
        rows = eqs + [les[p] for p in pick]
        g = np.array([r[0] for r in rows]).reshape(len(rows), n)
        h = np.array([r[1] for r in rows])
        if np.linalg.matrix_rank(g) < n:
            continue
        x = np.linalg.solve(g, h)
        ok = all(abs(r[0] @ x - r[1]) <= tol * (1 + abs(r[1])) for r in eqs) and all(
            r[0] @ x - r[1] <= tol * (1 + abs(r[1])) for r in les)
        if ok:
            out.append(x)
    return out


def vertex_enumeration(lp, c=None, **kw):
    """(optimal objective, minimiser) of min c'x over the vertices."""
    c = lp.c if c is None else c
    vs = vertices(lp, **kw)
    if not vs:
        return None, None
    objs = np.array([c @ v for v in vs])
    i = int(np.argmin(objs))
    return float(objs[i]), vs[i]


def highs(lp, c=None, l=None, u=None, sense=None):
    """Optimal objective and x from scipy's HiGHS on the general form."""
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix

    c = lp.c if c is None else c
    l = lp.l if l is None else l
    u = lp.u if u is None else u
    sense = lp.sense if sense is None else np.frombuffer(bytes(sense), dtype=np.uint8)
    a = csr_matrix((lp.val, lp.col, lp.row_ptr), shape=(lp.m, lp.n))
    eq = sense == ord("=")
    le = sense == ord("<")
    ge = sense == ord(">")
    a_ub = None
    b_ub = None
    if le.any() or ge.any():
        from scipy.sparse import vstack

        a_ub = vstack([a[le], -a[ge]]).tocsr()
        b_ub = np.concatenate([lp.b[le], -lp.b[ge]])
    bounds = np.column_stack([np.where(np.isfinite(l), l, -np.inf), np.where(np.isfinite(u), u, np.inf)])
    res = linprog(c, A_ub=a_ub, b_ub=b_ub, A_eq=a[eq] if eq.any() else None, b_eq=lp.b[eq] if eq.any() else None,
                  bounds=[(lo if np.isfinite(lo) else None, hi if np.isfinite(hi) else None) for lo, hi in bounds],
                  method="highs")
    if res.status != 0:
        return None, None
    return float(res.fun), res.x


def knapsack_greedy(a, b, c, u):
    """min c'x s.t. a'x = b, 0 <= x <= u, with a > 0, c arbitrary: fill by c_j / a_j.

    Items with c_j < 0 are profitable per unit of capacity in ratio order; an
    equality forces the capacity to be used completely, so fill by ascending
    c_j / a_j until b is met."""
    order = np.argsort(c / a, kind="stable")
    x = np.zeros_like(c)
    left = b
    for j in order:
        take = min(u[j], left / a[j])
        x[j] = take
        left -= take * a[j]
        if left <= 0:
            break
    return float(c @ x), x
