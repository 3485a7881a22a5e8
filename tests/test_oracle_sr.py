"""Pins of oracle.sr (CPU only)."""
import numpy as np
import torch

from oracle import ansatz as oa
from oracle import sr as osr
from tests.test_oracle_ansatz import rand_cfg, stress_params

ARCH = oa.Arch(d=8, heads=2, layers=1, mlp=16)
N = 4


def test_jacobian_matches_central_differences():
    th = stress_params(ARCH, 3)
    cfg = rand_cfg(N, 3, 4)
    J = osr.jacobian(th, ARCH, cfg, N)
    rng = np.random.default_rng(0)
    for k in rng.choice(th.size, 12, replace=False):
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        with torch.no_grad():
            d = (oa.log_rho(tp, ARCH, cfg, N) - oa.log_rho(tm, ARCH, cfg, N)).numpy() / (2 * h)
        assert np.allclose(J[:, 0, k], d.real, atol=1e-7, rtol=1e-6)
        assert np.allclose(J[:, 1, k], d.imag, atol=1e-7, rtol=1e-6)


def test_metric_properties():
    th = stress_params(ARCH, 5)
    cfg = rand_cfg(N, 10, 6)
    w = np.random.default_rng(1).uniform(0.5, 2.0, 10)
    J = osr.jacobian(th, ARCH, cfg, N)
    S = osr.metric(J, w)
    assert np.allclose(S, S.T, atol=1e-14)
    assert np.linalg.eigvalsh(S).min() > -1e-12
    # the real head bias shifts every log rho by the same constant
    k = oa.num_params(ARCH) - 2
    assert np.allclose(J[:, 0, k], 1.0, atol=1e-12) and np.allclose(J[:, 1, k], 0.0, atol=1e-12)
    assert np.max(np.abs(S[k])) < 1e-13
    # Re(conj(a) b) = a_r b_r + a_i b_i: the split form
    wn = w / w.sum()
    dR = J[:, 0] - (wn[:, None] * J[:, 0]).sum(0)
    dI = J[:, 1] - (wn[:, None] * J[:, 1]).sum(0)
    S2 = (wn[:, None] * dR).T @ dR + (wn[:, None] * dI).T @ dI
    assert np.allclose(S, S2, atol=1e-13)


def test_one_sample_gives_plain_gradient():
    th = stress_params(ARCH, 7)
    J = osr.jacobian(th, ARCH, rand_cfg(N, 1, 8), N)
    g = np.random.default_rng(2).standard_normal(th.size)
    assert np.allclose(osr.sr_direction(J, g, 0.3), g / 0.3, rtol=1e-14)
