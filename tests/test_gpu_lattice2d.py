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
from tests.test_gpu_backward import GTOL, LTOL, assert_grad

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
    assert_grad(prec, grad.cpu().numpy(), params, arch, model, cfg, w, mode, g)


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


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_mixes_lattices_and_chains(gpu, prec):
    """tdo_loss_grad_batched over lattice and chain problems (eager, recorded and
    replayed) equals separate tdo_loss_grad calls, and a lattice problem's loss
    equals the oracle's."""
    from tests.test_gpu_batched import REPEAT_TOL
    arch = synth.WORKLOADS["batched_uneven"]["arch"]
    models = [dict(kind=0, n=16, rows=2, V=1.3, g=0.9, gamma=1.0), dict(kind=0, n=12, V=0.8, g=1.2, gamma=1.0),
              dict(kind=0, n=16, rows=4, V=2.0, g=1.0, gamma=1.0), dict(kind=1, n=10, Jx=0.9, Jy=1.1, Jz=1.2, gamma=1.0),
              dict(kind=0, n=15, rows=3, V=0.7, g=1.4, gamma=0.9)]
    params = [synth.params(arch, 300 + i, "mid") for i in range(len(models))]
    cfgs = [synth.configs(m["n"], 48, 310 + i) for i, m in enumerate(models)]
    ctx = gpu.Ctx(0)
    pt, ct = [cuda(p) for p in params], [cuda(c) for c in cfgs]
    ref = [ctx.loss_grad(arch, pt[i], models[i], ct[i], None, prec, "B") for i in range(len(models))]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out = (torch.empty(len(models), dtype=torch.float64, device="cuda"),
               [torch.empty(synth.num_params(arch), dtype=torch.float64, device="cuda") for _ in models])
        for call in range(3):  # eager, recorded, replayed (same output buffers)
            loss, grads = ctx.loss_grad_batched(arch, pt, models, ct, None, prec, "B", out=out)
            s.synchronize()
            for i in range(len(models)):
                assert abs(float(loss[i]) - float(ref[i][0][0])) <= 1e-12 * abs(float(ref[i][0][0])), (call, i)
                assert rel_l2(grads[i].cpu().numpy(), ref[i][1].cpu().numpy()) <= REPEAT_TOL[prec], (call, i)
    torch.cuda.synchronize()
    F = vmc.loss(params[2].astype(np.float64), oa.Arch(**arch), ol.Model(**models[2]), cfgs[2])[0]
    err = abs(float(ref[2][0][0]) - F) / abs(F)
    print(f"batched lattice {prec}: 4 x 4 loss rel err {err:.3e}")
    assert err < LTOL[prec]
