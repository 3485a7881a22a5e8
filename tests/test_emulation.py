"""CPU checks of the tolerance helpers in tests/bf16_emulation.py."""
import numpy as np

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from paper_2502_20723_amd import synth
from tests.bf16_emulation import kink_sensitivity


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
