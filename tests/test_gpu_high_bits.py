"""Bits of a configuration at positions >= n are ignored (through the C-ABI):
connected rows, log rho, the loss and its gradient, and the sampler's log rho are
those of the configuration with the bits cleared."""
import numpy as np
import pytest
import torch

from paper_2502_20723_amd import synth

pytestmark = pytest.mark.gpu


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def with_high_bits(cfg, n, seed):
    rng = np.random.default_rng(seed)
    junk = rng.integers(0, 2**63, size=cfg.shape, dtype=np.uint64) << np.uint64(1)
    mask = np.uint64((1 << n) - 1) if n < 64 else np.uint64(2**64 - 1)
    return cfg | (junk & ~mask)


@pytest.mark.parametrize("name,n,B", [("ising_n8", 8, 64), ("xyz_n16", 16, 48), ("ising_n32", 27, 24)])
def test_high_bits_ignored(gpu, name, n, B):
    wl = synth.workload(name)
    arch, model = wl["arch"], dict(wl["model"], n=n)
    params = cuda(synth.params(arch, 21, "mid"))
    clean = synth.configs(n, B, 22)
    dirty = with_high_bits(clean, n, 23)
    assert not np.array_equal(clean, dirty)
    ctx = gpu.Ctx(0)
    c0, m0, k0 = ctx.connected(model, cuda(clean))
    c1, m1, k1 = ctx.connected(model, cuda(dirty))
    assert torch.equal(k0, k1) and torch.equal(m0, m1) and torch.equal(c0, c1)
    for prec in ("fp32", "bf16"):
        assert torch.equal(ctx.log_rho(arch, params, n, cuda(clean), prec), ctx.log_rho(arch, params, n, cuda(dirty), prec))
        l0, g0, L0 = ctx.loss_grad(arch, params, model, cuda(clean), None, prec, "B", want_lloc=True)
        l1, g1, L1 = ctx.loss_grad(arch, params, model, cuda(dirty), None, prec, "B", want_lloc=True)
        torch.cuda.synchronize()
        assert float(l0[0]) == float(l1[0])
        assert torch.equal(L0, L1)
        # the FP32 kernels and those for width 32 add weight gradients with LDS atomics (order varies)
        tol = 0.0 if prec == "bf16" and n <= 32 and arch["d"] == 64 else 1e-5
        nh = 2 * arch["d"] + 2
        scale = float(g0.abs().max())
        assert float((g0[:-nh] - g1[:-nh]).abs().max()) <= tol * scale
        assert float((g0[-nh:] - g1[-nh:]).abs().max()) <= tol * scale
