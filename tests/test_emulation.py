"""CPU checks of the tolerance helpers in tests/bf16_emulation.py."""
import numpy as np

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from paper_2502_20723_amd import synth
import pytest

from tests.bf16_emulation import kink_free_configs, kink_margins, kink_sensitivity


def _case():
    wl = synth.workload("ising_n4")
    arch, model = oa.Arch(**wl["arch"]), ol.Model(**dict(wl["model"], n=4))
    params = synth.params(wl["arch"], 5, "mid").astype(np.float64)
    cfg = synth.configs(4, 6, 7)
    w = np.random.default_rng(8).uniform(0.5, 1.5, 6)
    _, g, _ = vmc.loss_grad(params, arch, model, cfg, w, mode="B")
    return params, arch, model, cfg, w, g


def test_kink_sensitivity_zero_band_is_the_oracle():
    """With an empty band the replaced feed-forward function is the oracle's own:
    the gradient is unchanged bit for bit, and the oracle's function is restored."""
    params, arch, model, cfg, w, g = _case()
    orig = oa.mlp
    assert kink_sensitivity(params, arch, model, cfg, w, "B", g, kappa=0.0) == 0.0
    assert oa.mlp is orig


def test_kink_sensitivity_full_band_moves_the_gradient():
    """With every unit in the band all ReLU branches switch, which changes the gradient."""
    params, arch, model, cfg, w, g = _case()
    assert kink_sensitivity(params, arch, model, cfg, w, "B", g, kappa=2.0) > 1e-2


def test_kink_margins_bounds_and_a_planted_kink():
    """|u| <= |b1| + sum |x W1| puts every margin in [0, 1]; a hidden unit with zero weights
    and bias sits on the kink in every row (margin 0), so no sample is kink-free; the
    oracle's feed-forward function is restored afterwards."""
    params, arch, model, cfg, w, g = _case()
    orig = oa.mlp
    m = kink_margins(params, arch, model, cfg)
    assert oa.mlp is orig
    assert np.all((m > 0) & (m <= 1))
    p = oa.unflatten(__import__("torch").as_tensor(params.copy()), arch)
    p["l0_w1"][:, 3] = 0.0
    p["l0_b1"][3] = 0.0
    planted = np.concatenate([v.reshape(-1).numpy() for v in p.values()])
    assert np.all(kink_margins(planted, arch, model, cfg) == 0)
    with pytest.raises(AssertionError):
        kink_free_configs(planted, arch, model, 2, 9)


def test_vjp_emulation_fp32_is_the_oracle_and_bf16_is_not():
    """The emulated VJP in FP32 agrees with the FP64 oracle's VJP to FP32 rounding, so the
    emulation differentiates the same network with the same seed convention; in BF16 it
    moves by the BF16 rounding (between 1e-4 and 0.2, pointing the oracle's way)."""
    from tests.bf16_emulation import log_rho_vjp_emulated
    wl = synth.workload("ising_n8")
    arch = oa.Arch(**wl["arch"])
    params = synth.params(wl["arch"], 3, "mid").astype(np.float64)
    cfg = synth.configs(8, 5, 9)
    seed = np.random.default_rng(4).standard_normal((5, 2))
    ref = vmc.log_rho_vjp(params, arch, cfg, 8, seed)
    r32 = log_rho_vjp_emulated(params, arch, cfg, 8, seed, "fp32")
    r16 = log_rho_vjp_emulated(params, arch, cfg, 8, seed, "bf16")
    e32 = np.linalg.norm(r32 - ref) / np.linalg.norm(ref)
    e16 = np.linalg.norm(r16 - ref) / np.linalg.norm(ref)
    assert e32 < 1e-5
    assert 1e-4 < e16 < 0.2
    assert np.dot(r16, ref) / (np.linalg.norm(r16) * np.linalg.norm(ref)) > 0.99
