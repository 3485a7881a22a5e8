"""GPU parity of the parameter updates (tdo_sgd_step, tdo_adam_step) through the
C-ABI against oracle.optim, and a short training loop: exact-enumeration Adam on
the N = 4 Ising chain, whose cost must fall as the oracle's does.

The update kernels form every operation in FP64 in the order of the
definition, without fused multiply-adds, so the moments are bit-identical to the
oracle's and the FP32 parameters agree to one unit in the last place (the FP64
square root is the only operation not pinned to IEEE rounding here)."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import optim as oo
from oracle import vmc
from paper_2502_20723_amd import synth

pytestmark = pytest.mark.gpu


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def ulps(a, b):
    a, b = np.asarray(a, np.float32), np.asarray(b, np.float32)
    return np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))


@pytest.mark.parametrize("P", [1, 257, 4099, 206597])
def test_adam_and_sgd_match_oracle(gpu, P):
    rng = np.random.default_rng(P)
    th = (rng.standard_normal(P) * 0.1).astype(np.float32)
    m, v = np.zeros(P), np.zeros(P)
    pt, mt, vt = cuda(th), cuda(m), cuda(v)
    for t in range(1, 5):
        g = rng.standard_normal(P) * np.exp(rng.uniform(-8, 3, P))
        gpu.adam_step(pt, cuda(g), mt, vt, t, 3e-3)
        th, m, v = oo.adam_step(th, g, m, v, t, 3e-3)
        assert np.array_equal(mt.cpu().numpy(), m) and np.array_equal(vt.cpu().numpy(), v)
        d = ulps(pt.cpu().numpy(), th)
        assert d.max() <= 1 and (d == 0).mean() > 0.999, (t, d.max(), (d == 0).mean())
    g = rng.standard_normal(P)
    gpu.sgd_step(pt, cuda(g), 0.01)
    th = oo.sgd_step(th, g, 0.01)
    assert np.array_equal(pt.cpu().numpy(), th)


def test_invalid_updates(gpu):
    p = torch.zeros(4, dtype=torch.float32, device="cuda")
    g = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.TdoError):
        gpu.adam_step(p, g, g.clone(), g.clone(), 0, 1e-3)            # t counts from 1
    with pytest.raises(gpu.TdoError):
        gpu.adam_step(p, g, g.clone(), g.clone(), 1, 1e-3, beta1=1.0)
    gpu.sgd_step(torch.zeros(0, dtype=torch.float32, device="cuda"),
                 torch.zeros(0, dtype=torch.float64, device="cuda"), 0.1)   # P = 0: nothing to do


def test_training_loop_exact_enumeration_n4(gpu):
    """Adam on the exact cost of the N = 4 Ising chain (all 256 configurations
    weighted by |rho|^2 from tdo_log_rho, gradient from tdo_loss_grad, update by
    tdo_adam_step): after the first step the parameters equal the oracle's
    wherever the gradient is clear of its FP32 error, and after 60 steps the
    exact cost has fallen more than tenfold (the oracle's run: 5.25 to 0.14 in
    50 steps)."""
    wl = synth.workload("ising_n4")
    arch, model, n = wl["arch"], wl["model"], wl["model"]["n"]
    A, M = oa.Arch(**arch), ol.Model(**model)
    th0 = synth.params(arch, wl["seed"], "init")
    cfg = vmc.all_configs(n)
    ctx = gpu.Ctx(0)
    pt, ct = cuda(th0), cuda(cfg)
    mt = torch.zeros(th0.size, dtype=torch.float64, device="cuda")
    vt = torch.zeros_like(mt)
    costs = []
    for t in range(1, 61):
        lr = ctx.log_rho(arch, pt, n, ct, "fp32").double()
        w = torch.exp(2.0 * (lr[:, 0] - lr[:, 0].max()))
        w = (w / w.sum()).contiguous()
        loss, grad, _ = ctx.loss_grad(arch, pt, model, ct, w, "fp32", "B")
        costs.append(float(loss.cpu()[0]))
        if t == 1:
            g1 = grad.cpu().numpy()
        gpu.adam_step(pt, grad, mt, vt, t, 1e-2)
        if t == 1:
            c0, p0 = vmc.exact_weights(th0.astype(np.float64), A, n)
            F0, g0, _ = vmc.loss_grad(th0.astype(np.float64), A, M, c0, p0, mode="B")
            th1, _, _ = oo.adam_step(th0, g0, np.zeros(th0.size), np.zeros(th0.size), 1, 1e-2)
            clear = np.abs(g0) > 1e-3 * np.abs(g0).max()
            got = pt.cpu().numpy()
            print(f"step 1: cost GPU {costs[0]:.6e} oracle {F0:.6e}; gradient rel L2 "
                  f"{np.linalg.norm(g1 - g0) / np.linalg.norm(g0):.2e}; {clear.sum()} of {th0.size} clear")
            assert abs(costs[0] - F0) < 1e-5 * F0
            assert np.max(np.abs(got[clear] - th1[clear])) < 1e-6
    print("exact cost every 10 steps: " + ", ".join(f"{c:.4g}" for c in costs[::10]) + f", last {costs[-1]:.4g}")
    assert costs[-1] < 0.1 * costs[0]
