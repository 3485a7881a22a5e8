"""Workspace chunking (through the C-ABI): with a workspace budget just above
what one sample (or chain) needs, every entry point processes its batch in many
chunks; the results must equal those of a single chunk.  Also the error path
when the budget cannot hold one sample."""
import numpy as np
import pytest
import torch

from paper_2502_20723_amd import synth
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu

MIB = 1 << 20


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def smallest_ctx(gpu, call, budgets=(2, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256)):
    """The context with the smallest budget (MiB) for which `call` succeeds; smaller
    budgets must fail with an out-of-memory status, never with wrong results."""
    for mb in budgets:
        ctx = gpu.Ctx(0, mb * MIB)
        try:
            out = call(ctx)
            torch.cuda.synchronize()
            return ctx, out, mb
        except gpu.TdoError as e:
            assert e.code == -2, e  # TDO_ENOMEM
            ctx.close()
    pytest.fail("no budget fits one sample")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name,n,B", [("ising_n8", 8, 300), ("xyz_n16", 16, 120)])
def test_loss_grad_chunked(gpu, name, n, B, prec):
    wl = synth.workload(name)
    arch, model = wl["arch"], dict(wl["model"], n=n)
    params = cuda(synth.params(arch, 5, "mid"))
    cfg = cuda(synth.configs(n, B, 6))
    w = cuda(np.random.default_rng(7).uniform(0.5, 1.5, B))
    big = gpu.Ctx(0)
    l0, g0, L0 = big.loss_grad(arch, params, model, cfg, w, prec, "B", want_lloc=True)
    small, (l1, g1, L1), mb = smallest_ctx(gpu, lambda c: c.loss_grad(arch, params, model, cfg, w, prec, "B", want_lloc=True))
    print(f"{name} {prec}: smallest budget {mb} MiB")
    assert mb < 256
    assert abs(float(l1[0]) - float(l0[0])) <= 1e-9 * abs(float(l0[0]))
    assert torch.equal(L1, L0)
    # the chunks' weight gradients are summed in FP32 in a different grouping
    err = rel_l2(g1.cpu().numpy(), g0.cpu().numpy())
    print(f"  gradient rel L2 difference {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_log_rho_and_vjp_chunked(gpu, prec):
    wl = synth.workload("xyz_n16")
    arch, n = wl["arch"], 16
    params = cuda(synth.params(arch, 8, "mid"))
    B = 5000
    cfg = cuda(synth.configs(n, B, 9))
    seed = cuda(np.random.default_rng(10).standard_normal((B, 2)).astype(np.float32))
    big = gpu.Ctx(0)
    lr0 = big.log_rho(arch, params, n, cfg, prec)
    v0 = big.log_rho_vjp(arch, params, n, cfg, seed, prec)
    _, lr1, mb1 = smallest_ctx(gpu, lambda c: c.log_rho(arch, params, n, cfg, prec))
    _, v1, mb2 = smallest_ctx(gpu, lambda c: c.log_rho_vjp(arch, params, n, cfg, seed, prec))
    print(f"{prec}: log_rho budget {mb1} MiB, vjp budget {mb2} MiB")
    assert torch.equal(lr1, lr0)
    err = rel_l2(v1.cpu().numpy(), v0.cpu().numpy())
    print(f"  vjp rel L2 difference {err:.2e}")
    assert err < 1e-4


def test_sampler_chunked(gpu):
    """Chains are independent: a budget that splits them into chunks gives the same chains."""
    arch = synth.WORKLOADS["ising_n4"]["arch"]
    n, C = 6, 3000
    params = cuda(synth.params(arch, 11, "stress"))
    st0 = synth.configs(n, C, 12)
    big = gpu.Ctx(0)
    s_big = cuda(st0)
    lr_big = big.log_rho(arch, params, n, s_big)
    out0, _ = big.sample(arch, params, n, s_big, lr_big, 5, 0, 2, 0.5)

    def run(c):
        s = cuda(st0)
        lr = c.log_rho(arch, params, n, s)
        return c.sample(arch, params, n, s, lr, 5, 0, 2, 0.5)[0]

    _, out1, mb = smallest_ctx(gpu, run, budgets=(1, 2, 3, 4, 6, 8, 16, 32))
    print(f"sampler budget {mb} MiB")
    assert torch.equal(out1, out0)
