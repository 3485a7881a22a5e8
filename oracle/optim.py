"""Oracle: first-order parameter updates and the learning-rate schedule
(test infrastructure only).

App. C, optimisation procedure: the parameters move by a first-order update,
theta <- theta - eta grad, by SGD or by Adam, with eta from the schedule of the
learning-rate scheduling paragraph.

* SGD: theta - eta g.
* Adam as published (Kingma and Ba, ICLR 2015, Algorithm 1): first and second
  moment estimates with decay rates b1, b2, bias-corrected by 1 - b^t at step
  t = 1, 2, ..., and the step eta m_hat / (sqrt(v_hat) + eps).  Moments in FP64;
  FP32 parameters are updated in FP64 and rounded once.
* Schedule: eta0 before i_switch; afterwards eta0 (1 + cos(pi x)) / 2 + alpha
  eta0 with x = (step - i_switch) / i_decay.  Reading: x is clamped to 1, so the
  rate stays at alpha eta0 after the decay period (the printed formula would
  rise again as the cosine passes pi).

Parity: pinned in tests/test_oracle_optim.py by closed forms: Adam's first step
and its steps under a constant gradient are eta g / (|g| + eps); SGD on
f = a theta^2 / 2 gives theta_k = (1 - eta a)^k theta_0; the schedule's values
at the switch, the end of the decay and the midpoint.
"""
from __future__ import annotations

import math

import numpy as np


def sgd_step(theta, grad, lr):
    theta = np.asarray(theta, np.float32)
    return (theta.astype(np.float64) - lr * np.asarray(grad, np.float64)).astype(np.float32)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step; returns (theta', m', v').  t counts from 1."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * (g * g)
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    th = np.asarray(theta, np.float32).astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return th.astype(np.float32), m, v


def lr_schedule(step, eta0, i_switch, i_decay, alpha):
    if step < i_switch:
        return eta0
    x = min(1.0, (step - i_switch) / i_decay) if i_decay > 0 else 1.0
    return eta0 * (1.0 + math.cos(math.pi * x)) / 2.0 + alpha * eta0
