"""Seeded synthetic LP generators.

These build the inputs that both the GPU library and the CPU reference consume.
The module holds no part of the solver's arithmetic: it only draws random
structure and plants a known optimal primal/dual pair (x*, y*, z*) so that the
resulting LP has a certified optimum (primal feasible, dual feasible and
complementary, which is the optimality statement of the paper's section 2).

Every generator returns an :class:`LP` with the matrix in row-compressed form
(int64 row pointers, int32 column indices, float64 values), float64 b, c, l, u
(infinite bounds as +-inf) and one sense byte per row: ``=``, ``<`` (a_i'x <= b_i)
or ``>`` (a_i'x >= b_i).

Draw order for the planted family (``planted``), from ``numpy.random.default_rng(seed)``:
  1. column degrees (fixed, uniform integer, or power law),
  2. row indices of every column (uniform, distinct within a column),
  3. matrix values N(0, 1),
  4. the zero set of x* (a permutation; the first round(zero_frac*n) columns),
  5. x* on the support, U(0, 1],
  6. the dual-degenerate subset of the zero set (a permutation of it),
  7. z* on the other zeros, U(0, 1],
  8. y* ~ N(0, 1) on equality rows,
  9. (inequality rows) tight subset, their y* and the slack of loose rows,
 10. (upper bounds) the bounded subset and u ~ U(1, 10).
U(0, 1] is drawn as 1 - U[0, 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class LP:
    m: int
    n: int
    row_ptr: np.ndarray  # int64, m+1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz
    b: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    sense: np.ndarray  # uint8 codes of b'=', b'<', b'>'
    x_star: Optional[np.ndarray] = None
    y_star: Optional[np.ndarray] = None
    z_star: Optional[np.ndarray] = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        np.add.at(a, (rows, self.col), self.val)
        return a

    def sense_str(self) -> str:
        return bytes(self.sense).decode()


def _csr_from_coo(m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Row-compressed arrays from coordinates; rows sorted, columns ascending within a row."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), vals.astype(np.float64)


def _distinct_rows(rng: np.random.Generator, m: int, deg: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Row index of every entry; entries of a column hold distinct rows."""
    n = deg.size
    cols = np.repeat(np.arange(n, dtype=np.int64), deg)
    rows = rng.integers(0, m, size=cols.size)
    while True:
        key = cols * m + rows
        order = np.argsort(key, kind="stable")
        dup = np.zeros(key.size, dtype=bool)
        dup[order[1:]] = key[order[1:]] == key[order[:-1]]
        nd = int(dup.sum())
        if nd == 0:
            return rows, cols
        rows[dup] = rng.integers(0, m, size=nd)


def _uniform_open0(rng, size):
    return 1.0 - rng.random(size)  # U(0, 1]


def power_law_degrees(rng: np.random.Generator, n: int, dmin: int, dmax: int, alpha: float) -> np.ndarray:
    """Column degrees with P(d) proportional to d^-alpha on dmin..dmax."""
    d = np.arange(dmin, dmax + 1, dtype=np.float64)
    p = d ** (-alpha)
    p /= p.sum()
    return rng.choice(np.arange(dmin, dmax + 1), size=n, p=p).astype(np.int64)


def planted(
    m: int,
    n: int,
    seed: int,
    deg=5,
    zero_frac: float = 0.4,
    degen_frac: float = 0.1,
    ineq_frac: float = 0.0,
    upper_frac: float = 0.0,
    deg_range: Optional[tuple] = None,
    power_law: Optional[tuple] = None,
    name: str = "",
) -> LP:
    """Random sparse LP with a planted degenerate optimum.

    ``deg`` entries per column at distinct uniformly random rows with N(0,1)
    values (or degrees uniform on ``deg_range`` / power law ``(dmin, dmax,
    alpha)``).  x* >= 0 has round(zero_frac*n) zeros; round(degen_frac*#zeros)
    of them are dual degenerate (z*_j = 0), so the optimal face is not a vertex.
    The last round(ineq_frac*m) rows are '<' rows with implicit slacks;
    round(upper_frac*n) columns get an upper bound U(1, 10) that is inactive
    at x* (x* <= 1).  b = A x* + s*, c = A'y* + z*.
    """
    rng = np.random.default_rng(seed)
    if power_law is not None:
        degs = power_law_degrees(rng, n, *power_law)
    elif deg_range is not None:
        degs = rng.integers(deg_range[0], deg_range[1] + 1, size=n).astype(np.int64)
    else:
        degs = np.full(n, int(deg), dtype=np.int64)
    degs = np.minimum(degs, m)
    rows, cols = _distinct_rows(rng, m, degs)
    vals = rng.standard_normal(rows.size)
    row_ptr, ci, va = _csr_from_coo(m, rows, cols, vals)

    nz = int(round(zero_frac * n))
    perm = rng.permutation(n)
    zeros, support = perm[:nz], perm[nz:]
    x = np.zeros(n)
    x[support] = _uniform_open0(rng, support.size)
    nd = int(round(degen_frac * nz))
    zperm = rng.permutation(zeros)
    degen, strict = zperm[:nd], zperm[nd:]
    z = np.zeros(n)
    z[strict] = _uniform_open0(rng, strict.size)

    n_ineq = int(round(ineq_frac * m))
    n_eq = m - n_ineq
    sense = np.full(m, ord("="), dtype=np.uint8)
    sense[n_eq:] = ord("<")
    y = np.zeros(m)
    y[:n_eq] = rng.standard_normal(n_eq)
    slack = np.zeros(m)
    if n_ineq:
        ineq = np.arange(n_eq, m)
        tight_mask = rng.random(n_ineq) < 0.4
        tight, loose = ineq[tight_mask], ineq[~tight_mask]
        active = rng.random(tight.size) < 0.85
        y[tight[active]] = -_uniform_open0(rng, int(active.sum()))
        slack[loose] = _uniform_open0(rng, loose.size)

    l = np.zeros(n)
    u = np.full(n, np.inf)
    nu = int(round(upper_frac * n))
    if nu:
        bounded = rng.permutation(n)[:nu]
        u[bounded] = rng.uniform(1.0, 10.0, size=nu)

    # b = A x* + s*, c = A'y* + z*  (plain products, float64)
    rr = np.repeat(np.arange(m), np.diff(row_ptr))
    ax = np.zeros(m)
    np.add.at(ax, rr, va * x[ci])
    aty = np.zeros(n)
    np.add.at(aty, ci, va * y[rr])
    b = ax + slack
    c = aty + z
    return LP(m, n, row_ptr, ci, va, b, c, l, u, sense, x, y, z, name=name or f"planted_m{m}_n{n}_s{seed}")


def config0(seed: int = 0) -> LP:
    """Single random sparse LP, m=200, n=500, 5 nnz per column, 40% zeros, 10% degenerate."""
    return planted(200, 500, seed, deg=5, zero_frac=0.4, degen_frac=0.1, name=f"c0_s{seed}")


def config1(seed: int = 1, m: int = 100_000, n: int = 400_000) -> LP:
    """m=100k, n=400k, power-law column degree 1..200 (alpha 1.75, mean ~6, nnz ~2.4M),
    half the rows '<' with implicit slacks, 30% of columns with u ~ U(1,10), 15% degenerate."""
    return planted(m, n, seed, zero_frac=0.4, degen_frac=0.15, ineq_frac=0.5, upper_frac=0.3,
                   power_law=(1, 200, 1.75), name=f"c1_s{seed}_m{m}_n{n}")


def config5(seed: int = 5, m: int = 100_000, n: int = 400_000) -> LP:
    """The c1 structure with a primal-degenerate planted optimum (dual push workload):
    85% of columns at zero and no dual-degenerate zeros, so about 0.15 n columns and
    0.3 m slacks sit off their bounds against m rows and the dual optimal face has
    dimension of order m - 0.15 n - 0.3 m."""
    return planted(m, n, seed, zero_frac=0.85, degen_frac=0.0, ineq_frac=0.5, upper_frac=0.3,
                   power_law=(1, 200, 1.75), name=f"c5_s{seed}_m{m}_n{n}")


def config3_instance(i: int, base_seed: int = 3000, m_range=(500, 20_000)) -> LP:
    """Instance i of the batched family: m log-uniform, n = round(2.5 m), degree U{4..8}."""
    seed = base_seed + i
    rng = np.random.default_rng(seed)
    m = int(round(math.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1])))))
    n = int(round(2.5 * m))
    return planted(m, n, seed + 1_000_000, deg_range=(4, 8), zero_frac=0.4, degen_frac=0.1,
                   name=f"c3_i{i}_m{m}")


def transportation(n_src: int = 2000, n_snk: int = 5000, seed: int = 2) -> LP:
    """Balanced transportation LP; arcs source-major (j = s*n_snk + t).

    Demands d_t ~ U{1..100}; supplies split sum(d) over sources by weights
    U{1..100} with largest remainders so that supply and demand balance
    exactly; integer costs U{1..20}.  Rows: sources first, then sinks, all
    equalities; x >= 0.  Every column has two unit entries.
    """
    rng = np.random.default_rng(seed)
    demand = rng.integers(1, 101, size=n_snk).astype(np.float64)
    w = rng.integers(1, 101, size=n_src).astype(np.float64)
    total = int(demand.sum())
    share = w / w.sum() * total
    supply = np.floor(share)
    rem = total - int(supply.sum())
    order = np.argsort(-(share - supply), kind="stable")
    supply[order[:rem]] += 1.0
    cost = rng.integers(1, 21, size=n_src * n_snk).astype(np.float64)
    m = n_src + n_snk
    n = n_src * n_snk
    # source rows: contiguous arcs; sink rows: stride n_snk
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:n_src + 1] = np.arange(1, n_src + 1, dtype=np.int64) * n_snk
    row_ptr[n_src + 1:] = n + np.arange(1, n_snk + 1, dtype=np.int64) * n_src
    col = np.empty(2 * n, dtype=np.int32)
    col[:n] = np.arange(n, dtype=np.int32)
    col[n:] = (np.arange(n_src, dtype=np.int64)[None, :] * n_snk
               + np.arange(n_snk, dtype=np.int64)[:, None]).reshape(-1).astype(np.int32)
    val = np.ones(2 * n)
    b = np.concatenate([supply, demand])
    return LP(m, n, row_ptr, col, val, b, cost, np.zeros(n), np.full(n, np.inf),
              np.full(m, ord("="), dtype=np.uint8), name=f"transport_{n_src}x{n_snk}_s{seed}")


def config2(seed: int = 2) -> LP:
    return transportation(2000, 5000, seed)


def tiny(seed: int, m: int = 3, n: int = 6, with_ineq: bool = True, with_bounds: bool = True,
         with_free: bool = False) -> LP:
    """Small feasible, bounded LP for brute-force checks.

    Bounds: each column gets a finite lower bound, a finite upper bound or
    both, and with ``with_free`` also neither (a free column); rows get random
    senses.  A primal point x0 inside the box fixes b (so the LP is feasible)
    and a sign-consistent dual pair (y0, z0) fixes c (so it is dual feasible,
    hence bounded); a free column has z0 = 0."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    a[rng.random((m, n)) < 0.3] = 0.0
    kind = rng.integers(0, 4 if with_free else 3, size=n) if with_bounds else np.zeros(n, dtype=np.int64)
    l = np.where((kind == 1) | (kind == 3), -np.inf, np.round(rng.uniform(-2, 0, size=n), 1))
    u = np.where((kind == 0) | (kind == 3), np.inf, np.round(rng.uniform(1, 3, size=n), 1))
    if not with_bounds:
        l = np.zeros(n)
    x0 = np.where(np.isfinite(l), l, np.where(np.isfinite(u), u - 1.0, -0.5)) + rng.uniform(0, 1, size=n)
    x0 = np.minimum(x0, np.where(np.isfinite(u), u, np.inf))
    sense = np.full(m, ord("="), dtype=np.uint8)
    if with_ineq:
        sense = np.array([ord("="), ord("<"), ord(">")], dtype=np.uint8)[rng.integers(0, 3, size=m)]
    ax = a @ x0
    slack = rng.uniform(0, 1, size=m)
    b = np.where(sense == ord("<"), ax + slack, np.where(sense == ord(">"), ax - slack, ax))
    y0 = rng.standard_normal(m)
    y0 = np.where(sense == ord("<"), -np.abs(y0), np.where(sense == ord(">"), np.abs(y0), y0))
    z0 = rng.uniform(-1, 1, size=n)
    z0 = np.where(np.isinf(u), np.abs(z0), np.where(np.isinf(l), -np.abs(z0), z0))
    z0 = np.where(np.isinf(l) & np.isinf(u), 0.0, z0)
    c = a.T @ y0 + z0
    rows, cols = np.nonzero(a)
    row_ptr, ci, va = _csr_from_coo(m, rows, cols, a[rows, cols])
    return LP(m, n, row_ptr, ci, va, b, c, l, u, sense, name=f"tiny_s{seed}")


def from_dense(a, b, c, l=None, u=None, sense=None, name="dense") -> LP:
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    rows, cols = np.nonzero(a)
    row_ptr, ci, va = _csr_from_coo(m, rows, cols, a[rows, cols])
    l = np.zeros(n) if l is None else np.asarray(l, dtype=np.float64)
    u = np.full(n, np.inf) if u is None else np.asarray(u, dtype=np.float64)
    if sense is None:
        s = np.full(m, ord("="), dtype=np.uint8)
    else:
        s = np.frombuffer(sense.encode() if isinstance(sense, str) else bytes(sense), dtype=np.uint8).copy()
    return LP(m, n, row_ptr, ci, va, np.asarray(b, dtype=np.float64), np.asarray(c, dtype=np.float64), l, u, s,
              name=name)


def multicommodity(n_nodes: int = 50_000, n_arcs: int = 400_000, n_comm: int = 8, seed: int = 4100,
                   walks: int = 500, max_len: int = 20) -> LP:
    """Multicommodity flow LP with shared arc capacities.

    Graph: a Hamiltonian cycle over a random node order plus random extra
    arcs (no self-loops, no duplicates) up to n_arcs.  Per commodity, flow is
    planted on `walks` random walks (length <= max_len along out-arcs,
    amounts U(1,5)); b_k is the node balance of the planted flow.  Arc
    capacities U(10,100), scaled down where needed so that the planted total
    load is at most 0.8 of capacity (the LP is feasible); costs U(1,50) per
    arc, shared by all commodities.  Variables x[a, k] >= 0, column index
    k * n_arcs + a.  Rows: node balance (node v, commodity k) at
    k * n_nodes + v ('='), then arc capacity (a) at n_comm * n_nodes + a ('<').
    """
    rng = np.random.default_rng(seed)
    order = rng.permutation(n_nodes)
    tail = list(order)
    head = list(np.roll(order, -1))
    seen = set(zip(tail, head))
    need = n_arcs - n_nodes
    while need > 0:
        t = rng.integers(0, n_nodes, size=2 * need)
        h = rng.integers(0, n_nodes, size=2 * need)
        for a, b2 in zip(t.tolist(), h.tolist()):
            if a != b2 and (a, b2) not in seen:
                seen.add((a, b2))
                tail.append(a)
                head.append(b2)
                need -= 1
                if need == 0:
                    break
    tail = np.array(tail, dtype=np.int64)
    head = np.array(head, dtype=np.int64)
    # out-arc lists for the walks
    order_out = np.argsort(tail, kind="stable")
    start = np.searchsorted(tail[order_out], np.arange(n_nodes + 1))
    flow = np.zeros((n_comm, n_arcs))
    for k in range(n_comm):
        src = rng.integers(0, n_nodes, size=walks)
        lens = rng.integers(1, max_len + 1, size=walks)
        amt = rng.uniform(1.0, 5.0, size=walks)
        for w in range(walks):
            v = src[w]
            for _ in range(lens[w]):
                deg = start[v + 1] - start[v]
                a = order_out[start[v] + rng.integers(0, deg)]
                flow[k, a] += amt[w]
                v = head[a]
    cap = rng.uniform(10.0, 100.0, size=n_arcs)
    load = flow.sum(axis=0)
    cap = np.maximum(cap, load / 0.8)
    cost = rng.uniform(1.0, 50.0, size=n_arcs)
    m = n_comm * n_nodes + n_arcs
    n = n_comm * n_arcs
    cols = np.arange(n, dtype=np.int64)
    k_of = cols // n_arcs
    a_of = cols % n_arcs
    rows = np.concatenate([k_of * n_nodes + tail[a_of], k_of * n_nodes + head[a_of], n_comm * n_nodes + a_of])
    vals = np.concatenate([np.ones(n), -np.ones(n), np.ones(n)])
    cc = np.concatenate([cols, cols, cols])
    row_ptr, ci, va = _csr_from_coo(m, rows, cc, vals)
    bal = np.zeros((n_comm, n_nodes))
    for k in range(n_comm):
        np.add.at(bal[k], tail, flow[k])
        np.subtract.at(bal[k], head, flow[k])
    b = np.concatenate([bal.reshape(-1), cap])
    sense = np.concatenate([np.full(n_comm * n_nodes, ord("="), dtype=np.uint8), np.full(n_arcs, ord("<"), dtype=np.uint8)])
    c = np.tile(cost, n_comm)
    return LP(m, n, row_ptr, ci, va, b, c, np.zeros(n), np.full(n, np.inf), sense,
              x_star=flow.reshape(-1), name=f"mcf_{n_nodes}n_{n_arcs}a_{n_comm}k_s{seed}")


def config4(seed: int = 4100) -> LP:
    """Evaluation LP of the learned part: 50k nodes, 400k arcs, 8 commodities."""
    return multicommodity(50_000, 400_000, 8, seed)
