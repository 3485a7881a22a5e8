"""Oracle: stochastic reconfiguration (test infrastructure only).

App. C, metric tensor in stochastic reconfiguration and the hybrid update: the
preconditioned direction x = (S + lambda I)^-1 grad, with the metric
S_ij = <dO_i^* dO_j> over the samples, dO = O - <O>, and the log-derivatives
O_i(x) = d log rho(x) / d theta_i.

Readings:
* The parameters are real, so the metric is the real part of the Hermitian
  form: S = Re sum_b w_b conj(dO_b) dO_b^T.
* Expectations over the samples use their weights normalised to sum 1 (the
  same weights as the cost); equal weights when none are given.
* The solve is exact here (dense, FP64); the GPU path uses conjugate gradients
  with a caller-chosen iteration count.

Parity: pinned in tests/test_oracle_sr.py: the Jacobian against central finite
differences of log rho; S symmetric positive semi-definite; the row of the
head's real bias vanishes (that bias adds the same constant to every log rho,
so its centred derivative is zero); one sample gives S = 0 and x = grad/lambda;
the real-part form equals the real/imaginary split.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ansatz


def jacobian(theta, arch, cfg, n):
    """O(x_b) as float64 [B, 2, P]: real and imaginary parts of d log rho / d theta."""
    th = torch.as_tensor(np.asarray(theta, np.float64)).clone().requires_grad_(True)
    cfg = np.asarray(cfg, np.uint64).reshape(-1, 2)
    out = np.zeros((cfg.shape[0], 2, th.numel()))
    for b in range(cfg.shape[0]):
        lr = ansatz.log_rho(th, arch, cfg[b:b + 1], n)[0]
        gr, = torch.autograd.grad(lr.real, th, retain_graph=True)
        gi, = torch.autograd.grad(lr.imag, th)
        out[b, 0], out[b, 1] = gr.numpy(), gi.numpy()
    return out


def metric(jac, weights=None):
    """S = Re sum_b w_b conj(dO_b) dO_b^T with dO = O - sum_b w_b O_b."""
    O = jac[:, 0] + 1j * jac[:, 1]
    w = np.ones(O.shape[0]) if weights is None else np.asarray(weights, np.float64)
    w = w / w.sum()
    dO = O - (w[:, None] * O).sum(axis=0)
    return np.real((w[:, None] * dO.conj()).T @ dO)


def sr_direction(jac, grad, lam, weights=None):
    S = metric(jac, weights)
    return np.linalg.solve(S + lam * np.eye(S.shape[0]), np.asarray(grad, np.float64))
