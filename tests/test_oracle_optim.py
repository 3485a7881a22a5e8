"""Pins of oracle.optim (CPU only), and the host-only schedule of the C-ABI."""
import math

import numpy as np
import pytest

from oracle import optim as oo


def test_adam_first_step_and_constant_gradient():
    """With bias correction, m_hat = g and v_hat = g^2 exactly while the gradient is
    constant, so every step moves theta by eta g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    g = rng.standard_normal(1000) * np.exp(rng.uniform(-5, 5, 1000))
    th = np.zeros(1000, np.float32)
    m = np.zeros(1000)
    v = np.zeros(1000)
    lr, eps = 1e-3, 1e-8
    ref = np.zeros(1000)
    for t in range(1, 6):
        th, m, v = oo.adam_step(th, g, m, v, t, lr, eps=eps)
        ref -= lr * g / (np.abs(g) + eps)
        assert np.allclose(th, ref, rtol=1e-5, atol=0)


def test_adam_moments():
    """After two steps: m = (1-b1)(b1 g1 + g2), v = (1-b2)(b2 g1^2 + g2^2)."""
    g1, g2 = np.array([0.5, -2.0]), np.array([1.5, 3.0])
    b1, b2 = 0.9, 0.999
    _, m, v = oo.adam_step(np.zeros(2, np.float32), g1, np.zeros(2), np.zeros(2), 1, 0.1)
    _, m, v = oo.adam_step(np.zeros(2, np.float32), g2, m, v, 2, 0.1)
    assert np.allclose(m, (1 - b1) * (b1 * g1 + g2), rtol=1e-15)
    assert np.allclose(v, (1 - b2) * (b2 * g1 ** 2 + g2 ** 2), rtol=1e-15)


def test_sgd_on_a_quadratic():
    """f = a theta^2 / 2: theta_k = (1 - eta a)^k theta_0."""
    a, lr = 3.0, 0.05
    th = np.array([1.0, -2.0], np.float32)
    th0 = th.astype(np.float64)
    for k in range(1, 30):
        th = oo.sgd_step(th, a * th.astype(np.float64), lr)
        assert np.allclose(th, (1 - lr * a) ** k * th0, rtol=1e-5)


def test_schedule_values():
    """eta0 before the switch, eta0 (1 + alpha) at it, (1/2 + alpha) eta0 halfway,
    alpha eta0 at the end of the decay and after it."""
    e, s, d, a = 0.0061, 30000, 40000, 0.001
    assert oo.lr_schedule(0, e, s, d, a) == e and oo.lr_schedule(s - 1, e, s, d, a) == e
    assert math.isclose(oo.lr_schedule(s, e, s, d, a), e * (1 + a), rel_tol=1e-15)
    assert math.isclose(oo.lr_schedule(s + d // 2, e, s, d, a), e * (0.5 + a), rel_tol=1e-12)
    assert math.isclose(oo.lr_schedule(s + d, e, s, d, a), a * e, rel_tol=1e-9)
    assert math.isclose(oo.lr_schedule(s + 3 * d, e, s, d, a), a * e, rel_tol=1e-9)
    vals = [oo.lr_schedule(k, e, s, d, a) for k in range(s, s + d + 1, 1000)]
    assert all(x >= y for x, y in zip(vals, vals[1:]))


@pytest.mark.parametrize("step", [0, 29999, 30000, 41234, 50000, 70000, 150000])
def test_library_schedule_matches_oracle(step):
    """tdo_lr_schedule is host code: it runs without a GPU."""
    from paper_2502_20723_amd import tdo
    got = tdo.lr_schedule(step, 0.0061, 30000, 40000, 0.001)
    assert got == pytest.approx(oo.lr_schedule(step, 0.0061, 30000, 40000, 0.001), rel=1e-15, abs=0)
