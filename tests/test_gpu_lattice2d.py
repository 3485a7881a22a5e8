"""GPU parity of the 2D dissipative Ising model (an M x C periodic lattice,
sites row-major) through the C-ABI: connected indices bit-exact against
oracle.lindblad, the loss, L_loc and gradient against the FP64 oracle, and the
exact cost of the 2 x 3 lattice over all 4^6 configurations.  Tolerances as
for the chains: 1e-5 (FP32) and 2e-2 (BF16) relative on the loss, 1e-3 on the
FP32 gradient (with the ReLU-kink sensitivity as a floor)."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from paper_2502_20723_amd import synth
from tests.parity import rel_l2
from tests.test_gpu_backward import GTOL, LTOL, grad_tol

pytestmark = pytest.mark.gpu


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("M,C", [(2, 2), (2, 3), (3, 2), (3, 3), (4, 4), (2, 16), (16, 2), (4, 8), (3, 7),
                                 (8, 8), (2, 32), (5, 1)])
@pytest.mark.parametrize("V,g,gamma", [(2.0, 1.0, 1.0), (0.73, 1.61, 0.8), (2.0, 0.0, 1.0)])
def test_connected_bit_exact_2d(gpu, M, C, V, g, gamma):
    n = M * C
    m = dict(kind=0, n=n, rows=M, V=V, g=g, gamma=gamma)
    cfg = vmc.all_configs(n) if n <= 4 else synth.configs(n, 400, 200 + n)
    if n > 4:
        ones = np.uint64((1 << n) - 1) if n < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
        cfg[0] = (ones, ones)
        cfg[1] = (ones, ones ^ np.uint64(1))
        cfg[2] = (0, 0)
    ctx = gpu.Ctx(0)
    conn, mel, ncon = ctx.connected(m, cuda(cfg))
    conn, mel, ncon = conn.cpu().numpy(), mel.cpu().numpy(), ncon.cpu().numpy()
    rows = ol.connected(ol.Model(**m), cfg)
    for b in range(cfg.shape[0]):
        rc, rv = rows[b]
        k = ncon[b]
        assert k == len(rc), (b, k, len(rc))
        got = conn[b, :k]
        order = np.lexsort((got[:, 1], got[:, 0]))
        assert np.array_equal(got[order], rc), b
        gv = mel[b, :k, 0][order] + 1j * mel[b, :k, 1][order]
        assert np.max(np.abs(gv - rv) / np.maximum(np.abs(rv), 1e-30)) < 2e-7, b


def test_invalid_lattices(gpu):
    ctx = gpu.Ctx(0)
    cfg = cuda(synth.configs(6, 4, 1))
    for m in (dict(kind=0, n=6, rows=4, V=1.0, g=1.0), dict(kind=1, n=6, rows=2, Jx=1.0, Jy=1.0, Jz=1.0),
              dict(kind=0, n=6, rows=-1, V=1.0, g=1.0)):
        with pytest.raises(gpu.TdoError):
            ctx.connected(m, cfg)


@pytest.mark.parametrize("mode", ["B", "A"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name,B,scale", [("ising2d_2x3", 48, "stress"), ("ising2d_4x8", 12, "mid")])
def test_loss_grad_2d(gpu, name, B, scale, prec, mode):
    wl = synth.workload(name)
    arch, model, n = wl["arch"], wl["model"], wl["model"]["n"]
    params = synth.params(arch, 51 + n, scale)
    cfg = synth.configs(n, B, 53 + n)
    w = np.random.default_rng(n).uniform(0.5, 1.5, B)
    ctx = gpu.Ctx(0)
    loss, grad, L = ctx.loss_grad(arch, cuda(params), model, cuda(cfg), cuda(w), prec, mode, want_lloc=True)
    F, g, Lr = vmc.loss_grad(params.astype(np.float64), oa.Arch(**arch), ol.Model(**model), cfg, w, mode=mode)
    lerr = abs(float(loss.cpu()[0]) - F) / abs(F)
    gerr = rel_l2(grad.cpu().numpy(), g)
    Lg = L.cpu().numpy()
    Lerr = np.max(np.abs(Lg[:, 0] + 1j * Lg[:, 1] - Lr)) / max(1.0, np.max(np.abs(Lr)))
    print(f"2D {name} B={B} {scale} {prec} mode {mode}: loss {lerr:.3e} grad {gerr:.3e} L {Lerr:.3e}")
    assert lerr < LTOL[prec]
    assert Lerr < LTOL[prec] * 10
    if gerr >= GTOL[prec]:
        assert gerr < grad_tol(prec, params, arch, model, cfg, w, mode, g)


def test_exact_cost_2x3(gpu):
    """All 4^6 configurations of the 2 x 3 lattice with weights |rho|^2: the GPU's
    loss is the exact cost sum |rho|^2 |L|^2 / sum |rho|^2 (FP32)."""
    wl = synth.workload("ising2d_2x3")
    arch, model, n = wl["arch"], wl["model"], wl["model"]["n"]
    params = synth.params(arch, wl["seed"], "stress")
    cfg, p = vmc.exact_weights(params.astype(np.float64), oa.Arch(**arch), n)
    F = vmc.loss(params.astype(np.float64), oa.Arch(**arch), ol.Model(**model), cfg, p)[0]
    ctx = gpu.Ctx(0)
    loss, _, _ = ctx.loss_grad(arch, cuda(params), model, cuda(cfg), cuda(p), "fp32", "B")
    err = abs(float(loss.cpu()[0]) - F) / abs(F)
    print(f"2 x 3 exact cost {F:.6e}, GPU rel err {err:.3e}")
    assert err < 1e-5
