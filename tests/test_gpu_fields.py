"""GPU parity of the loss and gradient of the dissipative XYZ chain with fields
(Heisenberg section: H = sum_i sum_k J_k s^k_i s^k_{i+1} + B_k s^k_i), at the
couplings the paper uses there (J = (1.4, 2.0, 1.0), B_x = -1, B_z = 0.1, jumps
sigma^- at gamma = 1), through tdo_loss_grad against the FP64 oracle: sampled
rows at n = 5, and the exact cost and its gradient over all 4^4 configurations at
n = 4 (Eq. loss with |rho|^2 weights; mode B then equals d Cost / d theta)."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from paper_2502_20723_amd import synth
from tests.bf16_emulation import kink_free_configs
from tests.parity import rel_l2
from tests.test_gpu_backward import GTOL, LTOL, assert_grad

pytestmark = pytest.mark.gpu

FIELDS = dict(kind=1, Jx=1.4, Jy=2.0, Jz=1.0, Bx=-1.0, By=0.0, Bz=0.1, gamma=1.0)


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("mode", ["B", "A"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("arch_name,B", [("ising_n4", 40), ("xyz_n16", 24)])
def test_loss_grad_with_fields(gpu, arch_name, B, prec, mode):
    n = 5
    arch = synth.WORKLOADS[arch_name]["arch"]
    model = dict(FIELDS, n=n)
    A, M = oa.Arch(**arch), ol.Model(**model)
    params = synth.params(arch, 61, "mid")
    cfg = kink_free_configs(params, A, M, B, 62)
    w = np.random.default_rng(63).uniform(0.5, 1.5, B)
    ctx = gpu.Ctx(0)
    loss, grad, L = ctx.loss_grad(arch, cuda(params), model, cuda(cfg), cuda(w), prec, mode, want_lloc=True)
    F, g, Lr = vmc.loss_grad(params.astype(np.float64), A, M, cfg, w, mode=mode)
    lerr = abs(float(loss.cpu()[0]) - F) / abs(F)
    Lg = L.cpu().numpy()
    Lerr = float(np.max(np.abs(Lg[:, 0] + 1j * Lg[:, 1] - Lr)) / max(1.0, np.max(np.abs(Lr))))
    gerr = rel_l2(grad.cpu().numpy(), g)
    print(f"fields {arch_name} n={n} B={B} {prec} mode {mode}: loss {lerr:.3e} L {Lerr:.3e} grad {gerr:.3e}")
    assert lerr < LTOL[prec] and Lerr < LTOL[prec] * 10
    assert_grad(prec, grad.cpu().numpy(), params, arch, model, cfg, w, mode, g)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_exact_cost_and_gradient_with_fields_n4(gpu, prec):
    """All 256 configurations at n = 4 with weights |rho|^2 / sum |rho|^2: the loss is the
    exact cost and the mode-B gradient its exact gradient (both from the oracle)."""
    n = 4
    arch = synth.WORKLOADS["ising_n4"]["arch"]
    model = dict(FIELDS, n=n)
    A, M = oa.Arch(**arch), ol.Model(**model)
    params = synth.params(arch, 64, "stress")
    cfg, p = vmc.exact_weights(params.astype(np.float64), A, n)
    F, g, _ = vmc.loss_grad(params.astype(np.float64), A, M, cfg, p, mode="B")
    ctx = gpu.Ctx(0)
    loss, grad, _ = ctx.loss_grad(arch, cuda(params), model, cuda(cfg), cuda(p), prec, "B")
    lerr = abs(float(loss.cpu()[0]) - F) / abs(F)
    gerr = rel_l2(grad.cpu().numpy(), g)
    print(f"fields n=4 exact cost {F:.6e} {prec}: rel err {lerr:.3e}, gradient rel L2 {gerr:.3e}")
    assert lerr < LTOL[prec]
    assert_grad(prec, grad.cpu().numpy(), params, arch, model, cfg, p, "B", g)
