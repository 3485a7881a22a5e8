"""The torch.autograd.Function wrappers of the binding: LogRho's backward is the
library's vector-Jacobian product, checked against the oracle's VJP; LossGrad's
backward is the library's gradient estimator times the upstream scalar."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from paper_2502_20723_amd import synth, tdo
from tests.bf16_emulation import kink_free_configs
from tests.parity import log_rho_err, rel_l2

pytestmark = pytest.mark.gpu


def test_log_rho_function_forward_and_backward(gpu):
    arch = synth.WORKLOADS["ising_n8"]["arch"]
    n, B = 8, 50
    params = synth.params(arch, 81, "mid")
    cfg = synth.configs(n, B, 82)
    seed = np.random.default_rng(83).standard_normal((B, 2))
    p = torch.from_numpy(params).cuda().requires_grad_(True)
    out = tdo.LogRho.apply(p, arch, n, torch.from_numpy(cfg).cuda(), "fp32")
    (out * torch.from_numpy(seed).float().cuda()).sum().backward()
    ref = oa.log_rho(params.astype(np.float64), oa.Arch(**arch), cfg, n).numpy()
    g_ref = vmc.log_rho_vjp(params.astype(np.float64), oa.Arch(**arch), cfg, n, seed.astype(np.float32).astype(np.float64))
    ferr = log_rho_err(out.detach().cpu().numpy(), ref)
    gerr = rel_l2(p.grad.cpu().numpy(), g_ref)
    print(f"LogRho: forward err {ferr:.3e}, backward rel L2 {gerr:.3e}")
    assert p.grad.dtype == torch.float32
    assert ferr < 1e-5 and gerr < 1e-3


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_loss_grad_function_scales_by_the_upstream_scalar(gpu, prec):
    """BF16 width-64 kernels are deterministic, so the wrapper's gradient is 3x the
    direct call's bit for bit; in FP32 (LDS atomics in the generic kernels) to 1e-6."""
    arch = synth.WORKLOADS["ising_n32"]["arch"]
    model = dict(synth.workload("ising_n32")["model"], n=8)
    A, M = oa.Arch(**arch), ol.Model(**model)
    params = synth.params(arch, 84, "mid")
    cfg = kink_free_configs(params, A, M, 20, 85)
    p = torch.from_numpy(params).cuda().requires_grad_(True)
    c = torch.from_numpy(cfg).cuda()
    loss = tdo.LossGrad.apply(p, arch, model, c, None, prec, "B")
    (3.0 * loss).backward()
    _, g_direct, _ = tdo.default_ctx().loss_grad(arch, p.detach(), model, c, None, prec, "B")
    F, g, _ = vmc.loss_grad(params.astype(np.float64), A, M, cfg, None, mode="B")
    lerr = abs(float(loss.detach()) - F) / F
    want = (3.0 * g_direct).float()
    print(f"LossGrad {prec}: loss err {lerr:.3e}, wrapper vs 3 x direct max diff "
          f"{float((p.grad - want).abs().max()):.3e}, vs 3 x oracle rel L2 {rel_l2(p.grad.cpu().numpy(), 3 * g):.3e}")
    assert lerr < {"fp32": 1e-5, "bf16": 2e-2}[prec]
    if prec == "bf16":
        assert torch.equal(p.grad, want)
    else:
        assert rel_l2(p.grad.cpu().numpy(), want.cpu().numpy()) < 1e-6
        assert rel_l2(p.grad.cpu().numpy(), 3 * g) < 1e-3
