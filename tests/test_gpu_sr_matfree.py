"""GPU parity of the Jacobian-vector product of log rho (tdo_log_rho_jvp) and of the
matrix-free stochastic reconfiguration (tdo_sr_solve_matfree), through the C-ABI,
against the oracle: J p from the oracle's Jacobian (pinned by finite differences in
tests/test_oracle_sr.py) and the SR direction (S + lambda I)^-1 g from its metric,
dense at small n and, at the benchmark shape where the P x P metric does not fit,
through the Woodbury identity on the rows that carry weight:
(A^T A + lambda I)^-1 g = (g - A^T (A A^T + lambda I)^-1 A g) / lambda, A the rows
sqrt(w_b) dO_b (real and imaginary parts)."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import sr as osr
from paper_2502_20723_amd import synth
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu

ARCH = {k: synth.WORKLOADS[k]["arch"] for k in synth.WORKLOADS}


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def woodbury_direction(J, g, lam, w):
    """(S + lam I)^-1 g, S = Re sum_b w_b conj(dO_b) dO_b^T (w normalised), from J [B, 2, P]."""
    wn = np.asarray(w, np.float64) / np.sum(w)
    keep = wn > 0
    J, wn = J[keep], wn[keep]
    dO = J - (wn[:, None, None] * J).sum(axis=0)
    A = (np.sqrt(wn)[:, None, None] * dO).reshape(-1, J.shape[2])       # rows: Re and Im parts
    Ag = A @ g
    return (g - A.T @ np.linalg.solve(A @ A.T + lam * np.eye(A.shape[0]), Ag)) / lam


@pytest.mark.parametrize("name,n,B", [("ising_n4", 4, 33), ("ising_n8", 8, 40), ("xyz_n16", 16, 20),
                                      ("ising_n32", 32, 12), ("batched_uneven", 40, 6), ("batched_uneven", 64, 3),
                                      ("ising_n8", 5, 17)])
def test_jvp_matches_oracle_jacobian(gpu, name, n, B):
    arch = ARCH[name]
    params = synth.params(arch, 101 + n, "mid")
    cfg = synth.configs(n, B, 102 + n)
    tan = np.random.default_rng(103 + n).standard_normal(params.size) * 0.1
    J = osr.jacobian(params.astype(np.float64), oa.Arch(**arch), cfg, n)
    ref = J[:, 0] @ tan + 1j * (J[:, 1] @ tan)
    ctx = gpu.Ctx(0)
    got = ctx.log_rho_jvp(arch, cuda(params), n, cuda(cfg), cuda(tan)).cpu().numpy()
    err = float(np.linalg.norm(got[:, 0] + 1j * got[:, 1] - ref) / np.linalg.norm(ref))
    print(f"jvp {name} n={n} B={B}: rel L2 {err:.3e}")
    assert err < 1e-3


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-3), ("bf16", 2e-2)])
def test_matfree_sr_matches_dense_direction(gpu, prec, tol):
    """n = 4, the smallest network (P = 3794), 24 weighted samples: 60 CG iterations
    (S has rank at most 48) against the oracle's dense solve; in BF16 the reverse-mode
    product carries BF16 rounding, so the BF16 bar of 2e-2 applies."""
    arch, n, B, lam = ARCH["ising_n4"], 4, 24, 0.1
    params = synth.params(arch, 111, "mid")
    cfg = synth.configs(n, B, 112)
    w = np.random.default_rng(113).uniform(0.5, 1.5, B)
    g = np.random.default_rng(114).standard_normal(params.size)
    J = osr.jacobian(params.astype(np.float64), oa.Arch(**arch), cfg, n)
    ref = osr.sr_direction(J, g, lam, w)
    assert rel_l2(woodbury_direction(J, g, lam, w), ref) < 1e-10   # the two reference forms agree
    ctx = gpu.Ctx(0)
    x, info = ctx.sr_solve_matfree(arch, cuda(params), n, cuda(cfg), cuda(g), lam, 60, cuda(w), prec)
    err = rel_l2(x.cpu().numpy(), ref)
    print(f"matrix-free SR {prec}: rel L2 {err:.3e}, CG residual {float(info[0]):.2e}")
    assert err < tol


def test_matfree_sr_full_size_weighted_rows(gpu):
    """The benchmark's launch configuration: n = 32, the benchmark network, B = 65536
    samples through the forward- and reverse-mode passes; weights vanish except on 8 rows,
    so the direction is that of those rows (rank 16), against the oracle's Jacobian of
    the 8 rows through the Woodbury identity."""
    wl = synth.workload("ising_n32")
    arch, n, B, lam = wl["arch"], 32, wl["B"], 0.1
    params = synth.params(arch, wl["seed"], "mid")
    cfg = synth.configs(n, B, 3000)
    pick = np.sort(np.random.default_rng(115).choice(B, 8, replace=False))
    w = np.zeros(B)
    w[pick] = np.random.default_rng(116).uniform(0.5, 1.5, 8)
    g = np.random.default_rng(117).standard_normal(params.size)
    J = osr.jacobian(params.astype(np.float64), oa.Arch(**arch), cfg[pick], n)
    ref = woodbury_direction(J, g, lam, w[pick])
    ctx = gpu.Ctx(0, 64 << 30)
    x, info = ctx.sr_solve_matfree(arch, cuda(params), n, cuda(cfg), cuda(g), lam, 30, cuda(w), "fp32")
    err = rel_l2(x.cpu().numpy(), ref)
    print(f"matrix-free SR at B = {B}: rel L2 {err:.3e}, CG residual {float(info[0]):.2e}")
    assert err < 1e-3
