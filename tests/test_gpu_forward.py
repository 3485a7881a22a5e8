"""GPU parity of log rho (tdo_log_rho through the C-ABI) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from paper_2502_20723_amd import synth
from tests.bf16_emulation import log_rho_bf16
from tests.parity import log_rho_err

pytestmark = pytest.mark.gpu

ARCH = {k: synth.WORKLOADS[k]["arch"] for k in synth.WORKLOADS}
# Stated tolerances for the workloads' init and the well-conditioned mid scale;
# at the ill-conditioned stress scale the FP32 tolerance is derived from the
# FP32 CPU evaluation of the oracle (6e-6 at N = 32, x16 margin for a
# different summation order).  BF16 at the stress scale: within the stated 2e-2,
# or, where BF16 rounding itself is further off (the BF16 emulation of the same
# inputs, error e against FP64), within 0.5 e of the emulated log rho and, while
# 1.5 e < 0.5, within 1.5 e of the oracle.
TOL = {("init", "fp32"): 1e-5, ("init", "bf16"): 2e-2, ("mid", "fp32"): 1e-5, ("mid", "bf16"): 2e-2,
       ("stress", "fp32"): 1e-4, ("stress", "bf16"): None}

CASES = [  # (arch name, n, B)
    ("ising_n4", 4, 256), ("ising_n4", 3, 37), ("ising_n8", 8, 1000), ("ising_n8", 5, 333),
    ("xyz_n16", 16, 600), ("xyz_n16", 7, 129), ("ising_n32", 32, 300), ("ising_n32", 29, 65),
    ("batched_uneven", 40, 200), ("batched_uneven", 33, 31), ("batched_uneven", 64, 20), ("batched_uneven", 24, 77),
    # spanning passes at the other widths: the benchmark network (8-wide heads), width 32, width 16
    ("ising_n32", 40, 40), ("ising_n8", 45, 50), ("ising_n4", 36, 40),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("scale", ["init", "mid", "stress"])
@pytest.mark.parametrize("name,n,B", CASES)
def test_log_rho_parity(gpu, name, n, B, scale, prec):
    arch = ARCH[name]
    params = synth.params(arch, 17 + n, scale)
    cfg = synth.configs(n, B, 23 + n)
    cfg[0] = cfg[0, ::-1]
    if B > 2:
        cfg[1, 1] = cfg[1, 0]  # a diagonal configuration
    ctx = gpu.Ctx(0)
    got = ctx.log_rho(arch, torch.from_numpy(params).cuda(), n, torch.from_numpy(cfg).cuda(), prec).cpu().numpy()
    ref = oa.log_rho(params.astype(np.float64), oa.Arch(**arch), cfg, n).numpy()
    err = log_rho_err(got, ref)
    print(f"{name} n={n} B={B} {scale} {prec}: err {err:.3e}")
    tol = TOL[(scale, prec)]
    if tol is not None:
        assert err < tol
        return
    emu_lr = log_rho_bf16(params, oa.Arch(**arch), cfg, n)
    emu, dist = log_rho_err(emu_lr, ref), log_rho_err(got, emu_lr)
    print(f"  bf16 emulation err {emu:.3e}, GPU distance to the emulation {dist:.3e}")
    if err >= 2e-2:
        assert dist < 0.5 * emu
        if 1.5 * emu < 0.5:
            assert err < 1.5 * emu


def test_log_rho_empty_batch(gpu):
    arch = ARCH["ising_n8"]
    ctx = gpu.Ctx(0)
    out = ctx.log_rho(arch, torch.from_numpy(synth.params(arch, 1)).cuda(), 8,
                      torch.zeros((0, 2), dtype=torch.uint64).cuda())
    assert out.shape == (0, 2)
