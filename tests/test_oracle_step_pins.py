"""Pins of the oracle's iteration, restart rule, primal weight and scaling
against values worked out by hand (tests/golden/halpern_hand.json,
tests/golden/scaling_hand.json) and against the rules as the oracle's loop
applies them.

Each pin is chosen so that a plausible slip fails it: a Halpern weight of
1/(k+1) instead of 1/(k+2), a dropped reflection (gamma = 0), swapped step
sizes tau and sigma, no extrapolation x_bar = x+, Dr used the wrong way round,
Ruiz norms taken from a half-updated matrix, a wrong pass count, a swapped
dx/dy in the weight update, or the primal weight on the dual residual.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import OracleSolver, kkt_weighted, restart_decision, weight_update
from paper_2511_13894_amd import lpgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lp(d, name):
    inf = np.inf
    l = [(-inf if v is None else v) for v in d["l"]]
    u = [(inf if v is None else v) for v in d["u"]]
    return lpgen.from_dense(d["A"], d["b"], d["c"], l, u, d["sense"], name=name)


HALPERN = json.load(open(os.path.join(GOLDEN, "halpern_hand.json")))
SCALING = json.load(open(os.path.join(GOLDEN, "scaling_hand.json")))


@pytest.mark.parametrize("case", HALPERN["cases"], ids=lambda c: c["name"])
def test_first_two_iterates_match_the_hand_derivation(case):
    """Scaling, step size, primal weight and the first two (reflected
    Halpern) PDHG iterates of a 1 x 2 LP, against the hand derivation."""
    lp = _lp(HALPERN["lp"], case["name"])
    o = OracleSolver(lp, eps_rel=1e-30, **case["params"])
    sc = o.scaling()
    np.testing.assert_allclose(sc["dr"], HALPERN["dr"], rtol=1e-15)
    np.testing.assert_allclose(sc["dc"], HALPERN["dc"], rtol=1e-15)
    assert sc["eta"] == pytest.approx(HALPERN["eta"], rel=1e-14)
    assert sc["omega"] == pytest.approx(HALPERN["omega"], rel=1e-14)
    for it in case["iterates"]:
        o.iterate(1)
        x, y = o.iterate_state()
        np.testing.assert_allclose(x, it["x"], rtol=1e-13, atol=1e-15, err_msg=f"x at t={it['t']}")
        np.testing.assert_allclose(y, it["y"], rtol=1e-13, atol=1e-15, err_msg=f"y at t={it['t']}")


def test_scaling_closed_form_after_ten_ruiz_passes_and_pock_chambolle():
    """Dr, Dc, the scaled matrix and eta of [4, 1] in closed form."""
    lp = _lp(SCALING["lp"], "ruiz_4_1")
    o = OracleSolver(lp, eps_rel=1e-30)
    sc = o.scaling()
    np.testing.assert_allclose(sc["dr"], SCALING["dr"], rtol=1e-14)
    np.testing.assert_allclose(sc["dc"], SCALING["dc"], rtol=1e-14)
    _, _, v = o.ahat()
    np.testing.assert_allclose(v, SCALING["ahat"], rtol=1e-14)
    assert sc["eta"] == pytest.approx(SCALING["eta"], rel=1e-13)


def test_nine_passes_would_not_match():
    """The closed form separates the pass count: 9 passes give 2^(-1/256)."""
    lp = _lp(SCALING["lp"], "ruiz_4_1")
    o = OracleSolver(lp, eps_rel=1e-30, ruiz_iters=9)
    a9 = 2 ** (-1 / 256)
    want = 2 ** (-1 / 512) / math.sqrt(1 + a9)
    _, _, v = o.ahat()
    assert v[1] == pytest.approx(want, rel=1e-14)
    assert abs(v[1] - SCALING["ahat"][1]) > 1e-4


# --------------------------------------------------------- restart rule ----
def test_weighted_kkt_weights_primal_up_and_dual_down():
    # omega = 2: 4 * 1 + 4 / 4 + 9 = 14
    assert kkt_weighted(2.0, 1.0, 4.0, 9.0) == pytest.approx(math.sqrt(14.0), rel=1e-15)
    # omega = 1/2: 1/4 * 4 + 1 / (1/4) + 0 = 1 + 4
    assert kkt_weighted(0.5, 4.0, 1.0, 0.0) == pytest.approx(math.sqrt(5.0), rel=1e-15)


@pytest.mark.parametrize("kc,ka,kprev,k,t,want,why", [
    (0.19, 1.0, 0.10, 1, 100, True, "sufficient decay: 0.19 <= 0.2"),
    (0.20, 1.0, 0.10, 1, 100, True, "sufficient decay at equality"),
    (0.50, 1.0, 0.40, 1, 100, True, "necessary decay (0.5 <= 0.8) and no progress since the last check (0.5 > 0.4)"),
    (0.50, 1.0, 0.60, 1, 100, False, "necessary decay but still progressing (0.5 < 0.6)"),
    (0.85, 1.0, 0.10, 1, 100, False, "no decay, short inner run"),
    (0.85, 1.0, 0.10, 36, 100, True, "artificial: 36 >= 0.36 * 100"),
    (0.85, 1.0, 0.10, 35, 100, False, "artificial not yet: 35 < 36"),
    (0.90, 1.0, 0.95, 64, 64, True, "the first check of a phase always restarts (k = t)"),
])
def test_restart_rule_cases(kc, ka, kprev, k, t, want, why):
    assert restart_decision(kc, ka, kprev, k, t) is want, why


def test_restart_rule_follows_its_parameters():
    # still progressing (0.29 < 0.5), so only the sufficient rule can restart
    assert restart_decision(0.29, 1.0, 0.5, 1, 100, restart_suff=0.3) is True
    assert restart_decision(0.29, 1.0, 0.5, 1, 100, restart_suff=0.2) is False
    assert restart_decision(0.7, 1.0, 0.5, 1, 100, restart_nec=0.6) is False
    assert restart_decision(0.85, 1.0, 0.1, 10, 100, restart_art=0.1) is True


def test_primal_weight_update_closed_form():
    # dy/dx = 4 from omega = 1 with smoothing 1/2: exp(ln 4 / 2) = 2
    assert weight_update(1.0, 1.0, 4.0) == pytest.approx(2.0, rel=1e-15)
    # the swap dx <-> dy would give 1/2
    assert weight_update(1.0, 4.0, 1.0) == pytest.approx(0.5, rel=1e-15)
    # omega = 9, dy/dx = 1: sqrt(9 * 1) = 3
    assert weight_update(9.0, 2.0, 2.0) == pytest.approx(3.0, rel=1e-15)
    # smoothing 0 keeps omega, smoothing 1 takes dy/dx
    assert weight_update(5.0, 1.0, 3.0, pw_smooth=0.0) == pytest.approx(5.0, rel=1e-15)
    assert weight_update(5.0, 1.0, 3.0, pw_smooth=1.0) == pytest.approx(3.0, rel=1e-15)
    # a move below 1e-10 keeps omega
    assert weight_update(5.0, 1e-11, 3.0) == 5.0
    assert weight_update(5.0, 3.0, 0.0) == 5.0


def test_first_check_restarts_and_sets_the_weight_from_the_anchor_moves():
    """At t = 64 the artificial rule (k = t) restarts; the anchor was the
    start (x0, 0), so the new weight is sqrt(omega0 * ||y+ - 0|| / ||x+ - x0||)
    on the scaled candidate, which becomes the iterate and the anchor."""
    lp = lpgen.config0(1)
    o = OracleSolver(lp, eps_rel=1e-30)
    w0 = o.scaling()["omega"]
    lh, uh, _, _ = o.model_scaled()
    x0 = np.clip(np.zeros(lp.n), lh, uh)
    r = o.iterate(64)
    assert r.restarts == 1
    xs, ys = o.iterate_state(scaled=True)
    dx = np.linalg.norm(xs - x0)
    dy = np.linalg.norm(ys)
    assert o.scaling()["omega"] == pytest.approx(math.sqrt(w0 * dy / dx), rel=1e-13)
    assert o.scaling()["omega"] != pytest.approx(math.sqrt(w0 * dx / dy), rel=1e-3)


def test_restart_resets_the_halpern_counter():
    """After the restart at t = 64 the anchor is the candidate and k = 0.
    With gamma = 1 and x = x_anchor the next Halpern average is
    (1/2)(2 T(x) - x) + x/2 = T(x): the iterate at t = 65 is one plain PDHG
    step from the restart point (a counter left at 64 would weigh it 65/66,
    a stale anchor would pull it back towards the start)."""
    lp = lpgen.config0(1)
    a = OracleSolver(lp, eps_rel=1e-30)
    a.iterate(64)
    xs, ys = a.iterate_state(scaled=True)
    w = a.scaling()["omega"]
    a.iterate(1)
    x65, y65 = a.iterate_state()
    # one plain PDHG step from (xs, ys) with the same eta and omega, by hand
    sc = a.scaling()
    rp, ci, v = a.ahat()
    m, n = lp.m, lp.n
    A = np.zeros((m, n))
    for i in range(m):
        A[i, ci[rp[i]:rp[i + 1]]] += v[rp[i]:rp[i + 1]]
    lh, uh, ch, sense = a.model_scaled()
    bh = a.rhs_scaled()
    tau, sig = sc["eta"] / w, sc["eta"] * w
    xp = np.clip(xs - tau * (ch - A.T @ ys), lh, uh)
    yp = ys + sig * (bh - A @ (2 * xp - xs))
    yp = np.where(np.frombuffer(sense, dtype=np.uint8) == ord("<"), np.minimum(yp, 0), yp)
    yp = np.where(np.frombuffer(sense, dtype=np.uint8) == ord(">"), np.maximum(yp, 0), yp)
    np.testing.assert_allclose(x65, sc["dc"] * xp, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(y65, sc["dr"] * yp, rtol=1e-11, atol=1e-13)
