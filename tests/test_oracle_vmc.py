"""Pins of oracle.vmc (CPU only).

* Eq. lossnetk: under full enumeration the estimator equals the matrix form
  ||Lhat rho||^2 / ||rho||^2 with Lhat built from Kronecker products.
* Gradients against FP64 central finite differences of three scalar
  definitions: the reweighted estimator F_IS (mode B), the fixed-weight mean
  (mode A), and the exact cost (mode B under full enumeration).
* The vector-Jacobian product of log rho against finite differences.
"""
import math

import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from tests import dense_ref as dr
from tests.test_oracle_ansatz import stress_params

SMALL = oa.Arch(d=8, heads=2, layers=1, mlp=16)


def exact_cost_dense(theta, arch, n, dense):
    """||Lhat rho||^2 / ||rho||^2 from the dense generator and all amplitudes."""
    cfg = vmc.all_configs(n)
    with torch.no_grad():
        lr = oa.log_rho(torch.as_tensor(theta), arch, cfg, n).numpy()
    idx = np.array([dr.doubled_index(a, b, n) for a, b in cfg])
    rho = np.zeros(cfg.shape[0], np.complex128)
    rho[idx] = np.exp(lr - np.max(lr.real))
    r = dense @ rho
    return float(np.vdot(r, r).real / np.vdot(rho, rho).real)


@pytest.mark.parametrize("kind,kw", [(0, dict(V=2.0, g=1.0)), (1, dict(Jx=0.9, Jy=1.0, Jz=1.1))])
def test_enumerated_estimator_equals_matrix_cost(kind, kw):
    n = 4
    arch = oa.Arch(d=16, heads=2, layers=1, mlp=64)
    th = stress_params(arch, 21)
    cfg, w = vmc.exact_weights(th, arch, n)
    F, _, _ = vmc.loss(th, arch, ol.Model(kind=kind, n=n, **kw), cfg, w)
    ref = exact_cost_dense(th, arch, n, dr.lindbladian(kind, n, **kw))
    assert abs(F - ref) < 1e-11 * ref


def test_loss_zero_iff_steady_and_nonnegative():
    """Loss >= 0; the analytic V = 0 product steady state (fed as log rho) gives 0."""
    n = 6
    g = 0.8
    model = ol.Model(kind=0, n=n, V=0.0, g=g)
    cfg = vmc.all_configs(n)[::7]
    rows = ol.connected(model, cfg)
    r1 = np.array([[g * g, -1j * g], [1j * g, 1 + g * g]]) / (1 + 2 * g * g)

    def lr_of(c):
        a = ((c[:, 0:1] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(int)
        b = ((c[:, 1:2] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(int)
        return np.log(r1[a, b]).sum(axis=1)

    L = vmc.local_lindbladian([c for _, c in rows], lr_of(cfg), [lr_of(c) for c, _ in rows])
    assert np.max(np.abs(L)) < 1e-12
    arch = SMALL
    F, _, _ = vmc.loss(stress_params(arch, 3), arch, model, cfg)
    assert F > 0


def fd_grad(fun, th, idx, h=1e-6):
    out = []
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        out.append((fun(tp) - fun(tm)) / (2 * h))
    return np.array(out)


def f_is(th, th0, arch, model, cfg, w):
    """F_IS(theta) = sum r |L|^2 / sum r, r = w |rho_th(x)|^2 / |rho_th0(x)|^2."""
    _, L, lrx = vmc.loss(th, arch, model, cfg, w)
    _, _, lrx0 = vmc.loss(th0, arch, model, cfg, w)
    r = w * np.exp(2 * (lrx.real - lrx0.real))
    return float(np.sum(r * np.abs(L) ** 2) / np.sum(r))


@pytest.mark.parametrize("kind,kw", [(0, dict(V=2.0, g=1.0)), (1, dict(Jx=0.9, Jy=1.0, Jz=1.1))])
def test_grad_mode_b_matches_fd_of_reweighted_estimator(kind, kw):
    n = 5
    arch = SMALL
    model = ol.Model(kind=kind, n=n, **kw)
    th0 = stress_params(arch, 31)
    rng = np.random.default_rng(32)
    cfg = rng.integers(0, 1 << n, size=(24, 2), dtype=np.uint64)
    w = rng.uniform(0.5, 1.5, size=24)
    _, g, _ = vmc.loss_grad(th0, arch, model, cfg, w, mode="B")
    idx = rng.choice(th0.size, 16, replace=False)
    fd = fd_grad(lambda t: f_is(t, th0, arch, model, cfg, w), th0, idx)
    assert np.linalg.norm(g[idx] - fd) < 1e-7 * np.linalg.norm(fd)


def test_grad_mode_a_matches_fd_of_fixed_weight_mean():
    n = 5
    arch = SMALL
    model = ol.Model(kind=0, n=n, V=2.0, g=1.0)
    th0 = stress_params(arch, 41)
    rng = np.random.default_rng(42)
    cfg = rng.integers(0, 1 << n, size=(24, 2), dtype=np.uint64)
    _, g, _ = vmc.loss_grad(th0, arch, model, cfg, None, mode="A")
    idx = rng.choice(th0.size, 16, replace=False)
    fd = fd_grad(lambda t: vmc.loss(t, arch, model, cfg)[0], th0, idx)
    assert np.linalg.norm(g[idx] - fd) < 1e-7 * np.linalg.norm(fd)


def test_grad_mode_b_enumerated_is_gradient_of_exact_cost():
    """Under full enumeration, mode B is d Cost / d theta (Eq. lossnetk)."""
    n = 3
    arch = SMALL
    kw = dict(V=2.0, g=1.0)
    model = ol.Model(kind=0, n=n, **kw)
    dense = dr.lindbladian(0, n, **kw)
    th0 = stress_params(arch, 51)
    cfg, w = vmc.exact_weights(th0, arch, n)
    F, g, _ = vmc.loss_grad(th0, arch, model, cfg, w, mode="B")
    assert abs(F - exact_cost_dense(th0, arch, n, dense)) < 1e-11 * F
    rng = np.random.default_rng(52)
    idx = rng.choice(th0.size, 16, replace=False)
    fd = fd_grad(lambda t: exact_cost_dense(t, arch, n, dense), th0, idx)
    assert np.linalg.norm(g[idx] - fd) < 1e-7 * np.linalg.norm(fd)


def test_log_rho_vjp_matches_fd():
    n = 6
    arch = SMALL
    th0 = stress_params(arch, 61)
    rng = np.random.default_rng(62)
    cfg = rng.integers(0, 1 << n, size=(10, 2), dtype=np.uint64)
    seed = rng.standard_normal((10, 2))
    g = vmc.log_rho_vjp(th0, arch, cfg, n, seed)

    def obj(t):
        with torch.no_grad():
            lr = oa.log_rho(torch.as_tensor(t), arch, cfg, n).numpy()
        return float(np.sum(seed[:, 0] * lr.real + seed[:, 1] * lr.imag))

    idx = rng.choice(th0.size, 16, replace=False)
    fd = fd_grad(obj, th0, idx)
    assert np.linalg.norm(g[idx] - fd) < 1e-7 * np.linalg.norm(fd)
