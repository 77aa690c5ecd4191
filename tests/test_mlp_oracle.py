"""Pins of the CPU reference fix predictor: analytic gradients against
finite differences (with the rounding points switched off, where the loss is
smooth), closed forms on tiny cases, and a loss that falls under Adam."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def _no_round(monkeypatch):
    monkeypatch.setattr(M, "bf16", lambda a: np.asarray(a, dtype=np.float64))


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert M.bf16(-2.5) == -2.5
    # 3e38 = 1.7632.. * 2^127; the 7-bit mantissa step is 2^-7: 225.69 steps -> 226
    assert M.bf16(3.0e38) == (226.0 / 128.0) * 2.0 ** 127


def test_gradients_match_finite_differences(monkeypatch):
    _no_round(monkeypatch)
    rng = np.random.default_rng(0)
    p = M.init_params(3)
    p = {k: v + 0.05 * rng.standard_normal(v.shape) for k, v in p.items()}  # nonzero biases
    f = rng.standard_normal((40, M.NF))
    f[:, 12:] = 0.0
    y = (rng.random(40) < 0.3).astype(float)
    pw = 2.5
    loss, g, _ = M.loss_and_grad(p, f, y, pw)
    h = 1e-6
    for key in ("w1", "b1", "w2", "b2", "w3", "b3"):
        idx = [tuple(rng.integers(0, s) for s in p[key].shape) for _ in range(6)]
        for ix in idx:
            if key == "w1" and ix[1] >= 12:
                continue
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[key][ix] += h
            pm[key][ix] -= h
            lp, _, _ = M.loss_and_grad(pp, f, y, pw)
            lm, _, _ = M.loss_and_grad(pm, f, y, pw)
            fd = (lp - lm) / (2 * h)
            assert g[key][ix] == pytest.approx(fd, rel=1e-5, abs=1e-9), (key, ix)


def test_zero_network_closed_form(monkeypatch):
    """All weights zero: logit = b3 for every sample; dL/db3 is the mean of
    s(b3)(pw y + 1 - y) - pw y; every weight gradient vanishes."""
    _no_round(monkeypatch)
    p = {k: np.zeros_like(v) for k, v in M.init_params(0).items()}
    p["b3"][0] = 0.3
    y = np.array([1.0, 0.0, 0.0, 1.0])
    f = np.ones((4, M.NF))
    pw = 3.0
    loss, g, z = M.loss_and_grad(p, f, y, pw)
    s = 1 / (1 + np.exp(-0.3))
    np.testing.assert_allclose(z, 0.3)
    assert g["b3"][0] == pytest.approx(np.mean(s * (pw * y + 1 - y) - pw * y))
    assert loss == pytest.approx(np.mean(-pw * y * np.log(s) - (1 - y) * np.log(1 - s)))
    for k in ("w1", "w2", "w3", "b1", "b2"):
        assert np.all(g[k] == 0)


def test_flat_roundtrip_and_size():
    p = M.init_params(5)
    v = M.flat(p)
    assert v.size == M.N_PARAMS == 5313
    q = M.unflat(v)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])
    assert np.all(p["w1"][:, 12:] == 0)


def test_adam_lowers_the_loss_on_a_separable_problem():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((512, M.NF))
    f[:, 12:] = 0
    y = (f[:, 0] + 0.5 * f[:, 3] > 0).astype(float)
    p = M.init_params(7)
    st = {}
    l0, _, _ = M.loss_and_grad(p, f, y, 1.0)
    for _ in range(150):
        _, g, _ = M.loss_and_grad(p, f, y, 1.0)
        p = M.adam_step(p, g, st, lr=3e-3)
    l1, _, z = M.loss_and_grad(p, f, y, 1.0)
    assert l1 < 0.5 * l0
    assert np.mean((z > 0) == (y > 0)) > 0.9


def _one_param(v):
    return {"w": np.array([v], dtype=np.float64)}


def test_adam_first_step_is_lr_times_the_gradient_sign():
    """Adam (Kingma and Ba 2015) with bias correction: after one step
    m_hat = g and v_hat = g^2, so the move is lr g / (|g| + eps), which is
    lr sign(g) when |g| >> eps.  Without the correction the move would be
    lr * 0.1 g / (sqrt(0.001) |g|) = 3.16 lr."""
    st = {}
    p = M.adam_step(_one_param(0.5), {"w": np.array([2.0])}, st, lr=1e-3)
    assert p["w"][0] == pytest.approx(np.float32(0.5 - 1e-3 * 2.0 / (2.0 + 1e-8)), rel=0, abs=1e-9)
    st = {}
    p = M.adam_step(_one_param(0.5), {"w": np.array([-3e-4])}, st, lr=1e-3)
    assert p["w"][0] == pytest.approx(np.float32(0.5 + 1e-3 * 3e-4 / (3e-4 + 1e-8)), rel=0, abs=1e-9)


def test_adam_second_step_closed_form():
    """Step 2: m = 0.9 (0.1 g1) + 0.1 g2, v = 0.999 (0.001 g1^2) + 0.001 g2^2,
    m_hat = m / (1 - 0.9^2) = m / 0.19, v_hat = v / (1 - 0.999^2) = v / 0.001999.
    g2 = g1 = g: m_hat = g, v_hat = g^2, move lr sign(g) again.
    g2 = -g1: m = -0.01 g1, m_hat = -g1 / 19, v_hat = g1^2, move -lr/19 sign(g1)."""
    lr, g = 1e-3, 0.25
    st = {}
    p = M.adam_step(_one_param(1.0), {"w": np.array([g])}, st, lr=lr)
    p = M.adam_step(p, {"w": np.array([g])}, st, lr=lr)
    p1 = np.float32(1.0 - lr * g / (g + 1e-8))
    assert p["w"][0] == pytest.approx(np.float32(p1 - lr * g / (g + 1e-8)), rel=0, abs=2e-9)
    st = {}
    p = M.adam_step(_one_param(1.0), {"w": np.array([g])}, st, lr=lr)
    p = M.adam_step(p, {"w": np.array([-g])}, st, lr=lr)
    m_hat = -g / 19.0
    v_hat = g * g
    assert p["w"][0] == pytest.approx(np.float32(p1 - lr * m_hat / (np.sqrt(v_hat) + 1e-8)), rel=0, abs=2e-9)
    assert st["t"] == 2
