"""Oracle: local Lindbladian, cost and gradient in FP64 (test infrastructure only).

Definitions followed (App. C, "Optimization Procedure"):

* local estimator  L(x) = sum_{x'} Lhat(x; x') rho(x') / rho(x), evaluated as
  sum_s c_s exp(log rho(y_s) - log rho(x)) over the nonzero entries of row x;
* cost (Eq. lossnetk)  Cost = ||Lhat rho||^2 / ||rho||^2 = E_{x ~ |rho|^2} |L(x)|^2,
  estimated on a sample set as F = sum_b w_b |L(x_b)|^2 / sum_b w_b
  (w_b = 1 for Monte Carlo samples; w_x = |rho(x)|^2 under full enumeration);
* gradient.  The paper's printed gradient line is garbled; the reading used
  here is the gradient, at fixed samples, of the self-normalised estimator
      F_IS(theta) = sum_b r_b |L(x_b)|^2 / sum_b r_b,
      r_b = w_b |rho_theta(x_b)|^2 / |rho_theta0(x_b)|^2,
  evaluated at theta = theta0 ("mode B").  Its value is
      2 Re sum_b w_b conj(L_b) sum_s c_s e^{lr(y_s)-lr(x_b)} O(y_s) - 2 F sum_b w_b Re O(x_b)
  (normalised by sum w), O = d log rho / d theta, and under full enumeration
  with w_x = |rho(x)|^2 it equals d Cost / d theta exactly.  "Mode A" is the
  gradient of sum_b w_b |L_b|^2 / sum w with the weights held fixed.
  Both are obtained here by reverse-mode differentiation (torch.autograd) of
  those scalar definitions; nothing is hand-derived.

A row x with rho(x) = 0 (log rho = -inf) gets L(x) = 0: it has probability 0
and is never sampled.

Parity: pinned in tests/test_oracle_vmc.py by the matrix form of Eq. lossnetk
under full enumeration (dense Lhat from Kronecker products), L = 0 on the
exact steady state (dense null vector, N = 4) and on the V = 0 product state
at large N, the g = 0 dark state, and FP64 central finite differences of
F_IS, of the fixed-weight mean, and of the exact cost.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ansatz, lindblad


def local_lindbladian(coef_rows, lr_x, lr_rows):
    """L(x_b) = sum_s c_s exp(lr(y_s) - lr(x_b)) for each row b.

    coef_rows: list of complex arrays/tensors [k_b]; lr_x: complex [B];
    lr_rows: list of complex [k_b] (log rho at the connected configurations).
    Works on torch tensors (differentiable) or numpy arrays.
    """
    out = []
    for b, (c, lr_y) in enumerate(zip(coef_rows, lr_rows)):
        lx = lr_x[b]
        if torch.is_tensor(lx):
            if torch.isneginf(lx.real) or len(c) == 0:
                out.append(torch.zeros((), dtype=torch.complex128))
                continue
            c = torch.as_tensor(np.asarray(c), dtype=torch.complex128)
            out.append((c * torch.exp(lr_y - lx)).sum())
        else:
            if np.isneginf(np.real(lx)) or len(c) == 0:
                out.append(0j)
                continue
            out.append(np.sum(np.asarray(c) * np.exp(np.asarray(lr_y) - lx)))
    if out and torch.is_tensor(out[0]):
        return torch.stack(out)
    return np.asarray(out, dtype=np.complex128)


def _rows_and_eval_list(model, cfg):
    rows = lindblad.connected(model, cfg)
    return rows


def _chunks(rows, max_configs):
    """Split sample indices into chunks holding at most ~max_configs evaluations."""
    cur, tot = [], 0
    for b, (conn, _) in enumerate(rows):
        k = 1 + len(conn)
        if cur and tot + k > max_configs:
            yield cur
            cur, tot = [], 0
        cur.append(b)
        tot += k
    if cur:
        yield cur


def _chunk_terms(theta, arch, model, cfg, rows, idx):
    """log rho at x_b and at every connected y of the rows in idx, and L."""
    n = model.n
    xs = cfg[idx]
    ys = [rows[b][0] for b in idx]
    allc = np.concatenate([xs] + [y for y in ys if len(y)], axis=0) if any(len(y) for y in ys) else xs
    lr = ansatz.log_rho(theta, arch, allc, n)
    lr_x = lr[:len(idx)]
    off = len(idx)
    lr_rows = []
    for y in ys:
        lr_rows.append(lr[off:off + len(y)])
        off += len(y)
    L = local_lindbladian([rows[b][1] for b in idx], lr_x, lr_rows)
    return lr_x, L


def loss(theta, arch, model, cfg, weights=None, max_configs=20000):
    """Monte Carlo (or weighted) cost F and L(x_b); no gradient.

    Returns (F, L [B] complex128, log rho(x_b) [B] complex128).
    """
    cfg = np.asarray(cfg, dtype=np.uint64).reshape(-1, 2)
    B = cfg.shape[0]
    w = np.full(B, 1.0) if weights is None else np.asarray(weights, dtype=np.float64)
    rows = lindblad.connected(model, cfg)
    L = np.zeros(B, np.complex128)
    lrx = np.zeros(B, np.complex128)
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    with torch.no_grad():
        for idx in _chunks(rows, max_configs):
            lr_x, Lc = _chunk_terms(th, arch, model, cfg, rows, idx)
            L[idx] = Lc.numpy()
            lrx[idx] = lr_x.numpy()
    F = float(np.sum(w * np.abs(L) ** 2) / np.sum(w))
    return F, L, lrx


def loss_grad(theta, arch, model, cfg, weights=None, mode="B", max_configs=20000):
    """Cost F and its gradient (float64 [P]) at fixed samples cfg [B, 2].

    mode "B": gradient of the self-normalised reweighted estimator F_IS
    (equals d Cost/d theta under full enumeration); mode "A": gradient of the
    fixed-weight mean.  See the module docstring.
    """
    cfg = np.asarray(cfg, dtype=np.uint64).reshape(-1, 2)
    B = cfg.shape[0]
    w_np = np.full(B, 1.0) if weights is None else np.asarray(weights, dtype=np.float64)
    W = float(np.sum(w_np))
    F, L, _ = loss(theta, arch, model, cfg, w_np, max_configs)
    rows = lindblad.connected(model, cfg)
    th0 = np.asarray(theta, dtype=np.float64)
    grad = np.zeros(th0.size, np.float64)
    for idx in _chunks(rows, max_configs):
        th = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
        lr_x, Lc = _chunk_terms(th, arch, model, cfg, rows, idx)
        w = torch.as_tensor(w_np[idx])
        if mode == "B":
            finite = torch.isfinite(lr_x.real)
            lrx_safe = torch.where(finite, lr_x.real, torch.zeros_like(lr_x.real))
            r = w * torch.exp(2.0 * (lrx_safe - lrx_safe.detach()))
            r = torch.where(finite, r, torch.zeros_like(r))
            obj = torch.sum(r * (Lc.abs() ** 2) - F * r) / W
        elif mode == "A":
            obj = torch.sum(w * Lc.abs() ** 2) / W
        else:
            raise ValueError(mode)
        (g,) = torch.autograd.grad(obj, th, allow_unused=True)
        if g is not None:
            grad += g.numpy()
    return F, grad, L


def log_rho_vjp(theta, arch, cfg, n, seed):
    """sum_b seed_re[b] d Re log rho(x_b)/d theta + seed_im[b] d Im log rho(x_b)/d theta."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
    lr = ansatz.log_rho(th, arch, cfg, n)
    seed = torch.as_tensor(np.asarray(seed, dtype=np.float64)).reshape(-1, 2)
    obj = torch.sum(seed[:, 0] * lr.real + seed[:, 1] * lr.imag)
    (g,) = torch.autograd.grad(obj, th)
    return g.numpy()


def all_configs(n: int) -> np.ndarray:
    """Every doubled configuration (alpha, beta), alpha-major; uint64 [4^n, 2]."""
    k = np.arange(1 << n, dtype=np.uint64)
    a = np.repeat(k, 1 << n)
    b = np.tile(k, 1 << n)
    return np.stack([a, b], axis=1)


def exact_weights(theta, arch, n) -> tuple[np.ndarray, np.ndarray]:
    """Full-enumeration configurations and weights |rho(x)|^2 / sum |rho|^2."""
    cfg = all_configs(n)
    with torch.no_grad():
        lr = ansatz.log_rho(torch.as_tensor(np.asarray(theta, np.float64)), arch, cfg, n).numpy()
    re = np.real(lr)
    w = np.exp(2.0 * (re - np.max(re)))
    return cfg, w / w.sum()
