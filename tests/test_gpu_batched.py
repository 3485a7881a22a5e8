"""GPU parity of tdo_loss_grad_batched (through the C-ABI): uneven problems of the
batched workload (chain lengths 8..40, half Ising, half XYZ, each with its own
parameters) against the FP64 oracle, the single-problem entry point, and the
recorded-graph replays."""
import numpy as np
import pytest
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc
from paper_2502_20723_amd import synth
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["batched_uneven"]
ARCH = WL["arch"]


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def problems(count, B, seed, scale="mid"):
    models = synth.uneven_problems(count, seed)
    params = [synth.params(ARCH, seed + 7 * i, scale) for i in range(count)]
    cfgs = [synth.configs(m["n"], B, seed + 11 * i) for i, m in enumerate(models)]
    return models, params, cfgs


def test_matches_oracle_per_problem(gpu):
    """Six problems (with chain lengths on both sides of 32), B = 16 each, FP32, mode B."""
    models, params, cfgs = problems(64, 16, WL["seed"])
    pick = [0, 1, 2, 3]
    pick += [i for i, m in enumerate(models) if m["n"] > 32][:2]
    models = [models[i] for i in pick]
    params = [params[i] for i in pick]
    cfgs = [cfgs[i] for i in pick]
    assert any(m["n"] > 32 for m in models) and any(m["n"] <= 32 for m in models)
    ctx = gpu.Ctx(0)
    loss, grads = ctx.loss_grad_batched(ARCH, [cuda(p) for p in params], models, [cuda(c) for c in cfgs], None, "fp32", "B")
    loss = loss.cpu().numpy()
    for i, m in enumerate(models):
        F, g, _ = vmc.loss_grad(params[i].astype(np.float64), oa.Arch(**ARCH), ol.Model(**m), cfgs[i], None, mode="B")
        lerr = abs(loss[i] - F) / abs(F)
        gerr = rel_l2(grads[i].cpu().numpy(), g)
        print(f"problem {pick[i]} kind={m['kind']} n={m['n']}: loss {lerr:.2e} grad {gerr:.2e}")
        assert lerr < 1e-5
        assert gerr < 1e-3


# Run-to-run agreement of the gradient: the FP32 kernels add weight gradients into
# LDS with FP32 atomics whose order varies from run to run; the BF16 kernels of
# width 64 have no atomics (bit-identical).
REPEAT_TOL = {"fp32": 1e-5, "bf16": 0.0}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_equals_single_problem_calls_and_replays(gpu, prec):
    """The batched call (eager, then recorded, then replayed) gives the results of
    separate tdo_loss_grad calls on the same context, which use the tile shapes the
    first batched call tuned; a replay reads the current contents of its inputs."""
    models, params, cfgs = problems(8, 64, 77)
    ctx = gpu.Ctx(0)
    pt = [cuda(p) for p in params]
    ct = [cuda(c) for c in cfgs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out = (torch.empty(8, dtype=torch.float64, device="cuda"),
               [torch.empty(synth.num_params(ARCH), dtype=torch.float64, device="cuda") for _ in range(8)])
        ctx.loss_grad_batched(ARCH, pt, models, ct, None, prec, "B", out=out)  # tunes the shapes
        ref = [ctx.loss_grad(ARCH, pt[i], models[i], ct[i], None, prec, "B") for i in range(8)]
        s.synchronize()
        for call in range(3):  # eager, recorded, replayed
            loss, grads = ctx.loss_grad_batched(ARCH, pt, models, ct, None, prec, "B", out=out)
            s.synchronize()
            for i in range(8):
                assert abs(float(loss[i]) - float(ref[i][0][0])) <= 1e-12 * abs(float(ref[i][0][0])), (call, i)
                assert rel_l2(grads[i].cpu().numpy(), ref[i][1].cpu().numpy()) <= REPEAT_TOL[prec], (call, i)
        # change the parameters of problem 3 in place: the replay must see them
        pt[3].mul_(0.5)
        loss, grads = ctx.loss_grad_batched(ARCH, pt, models, ct, None, prec, "B", out=out)
        s.synchronize()
    torch.cuda.synchronize()
    l3, g3, _ = ctx.loss_grad(ARCH, pt[3], models[3], ct[3], None, prec, "B")
    torch.cuda.synchronize()
    assert abs(float(loss[3]) - float(l3[0])) <= 1e-12 * abs(float(l3[0]))
    assert rel_l2(grads[3].cpu().numpy(), g3.cpu().numpy()) <= REPEAT_TOL[prec]


def test_full_size_workload_sampled(gpu):
    """All 64 problems with B = 2048 each (the batched workload, BF16): the loss of
    4 problems restricted by the weights to 2 sampled rows each is checked against
    the oracle on those rows; every loss and gradient is finite."""
    models, params, cfgs = problems(64, WL["B"], WL["seed"], "init")
    rng = np.random.default_rng(5)
    checked = [0, 1, 2, 3]
    weights = []
    rows = {}
    for i in range(64):
        w = np.ones(WL["B"])
        if i in checked:
            r = np.sort(rng.choice(WL["B"], 2, replace=False))
            w[:] = 0.0
            w[r] = 1.0
            rows[i] = r
        weights.append(cuda(w))
    ctx = gpu.Ctx(0)
    loss, grads = ctx.loss_grad_batched(ARCH, [cuda(p) for p in params], models, [cuda(c) for c in cfgs], weights,
                                        "bf16", "B")
    loss = loss.cpu().numpy()
    assert np.all(np.isfinite(loss))
    assert all(bool(torch.isfinite(g).all()) for g in grads)
    for i in checked:
        F, _, _ = vmc.loss(params[i].astype(np.float64), oa.Arch(**ARCH), ol.Model(**models[i]), cfgs[i][rows[i]])
        err = abs(loss[i] - F) / abs(F)
        print(f"problem {i} n={models[i]['n']}: bf16 loss rel err {err:.2e}")
        assert err < 2e-2


def test_validation_before_launch(gpu):
    models, params, cfgs = problems(3, 8, 5)
    models[2] = dict(models[2], n=2)  # invalid chain length
    ctx = gpu.Ctx(0)
    with pytest.raises(gpu.TdoError):
        ctx.loss_grad_batched(ARCH, [cuda(p) for p in params], models, [cuda(c) for c in cfgs])
    loss, grads = ctx.loss_grad_batched(ARCH, [], [], [])
    assert loss.shape == (0,) and grads == []


def test_autotune_cache_file(gpu, tmp_path, monkeypatch):
    """TDO_AUTOTUNE_CACHE: the first context's batched call tunes the tile shapes and
    writes them to the file (one entry per distinct shape); a second context reads them,
    so its results equal the first context's bit for bit (BF16)."""
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("TDO_AUTOTUNE_CACHE", str(path))
    models, params, cfgs = problems(6, 64, 78)
    pt = [cuda(p) for p in params]
    ct = [cuda(c) for c in cfgs]
    ctx1 = gpu.Ctx(0)
    l1, g1 = ctx1.loss_grad_batched(ARCH, pt, models, ct, None, "bf16", "B")
    torch.cuda.synchronize()
    doc = json.loads(path.read_text())
    shapes = {(m["n"]) for m in models}
    print(f"cache: {len(doc['entries'])} entries for {len(shapes)} chain lengths: "
          + "; ".join(f"{e['shape']}: fwd {e['fwd_waves']} waves x {e['fwd_wg_per_cu']}/CU, mlp {e['mlp_waves']} waves"
                      for e in doc["entries"]))
    assert len(doc["entries"]) == len(shapes)
    for e in doc["entries"]:
        assert e["fwd_waves"] in (4, 8) and e["mlp_waves"] in (4, 8) and e["fwd_wg_per_cu"] in (1, 2)
    ctx2 = gpu.Ctx(0)
    ref = [ctx2.loss_grad(ARCH, pt[i], models[i], ct[i], None, "bf16", "B") for i in range(6)]
    torch.cuda.synchronize()
    for i in range(6):
        assert float(ref[i][0][0]) == float(l1[i])
        assert torch.equal(ref[i][1], g1[i])


def test_autotune_entry_point(gpu, tmp_path, monkeypatch):
    """tdo_autotune on one problem returns shapes from the candidate sets, adds the shape to
    the cache file, and later calls of that shape give the oracle's loss."""
    import json
    path = tmp_path / "tune1.json"
    monkeypatch.setenv("TDO_AUTOTUNE_CACHE", str(path))
    models, params, cfgs = problems(1, 48, 79)
    ctx = gpu.Ctx(0)
    shapes = ctx.autotune(ARCH, cuda(params[0]), models[0], cuda(cfgs[0]), "bf16", "B")
    print(f"tuned shapes n={models[0]['n']}: {shapes}")
    assert shapes[0] in (4, 8) and shapes[1] in (1, 2) and shapes[2] in (4, 8)
    assert len(json.loads(path.read_text())["entries"]) == 1
    loss, _, _ = ctx.loss_grad(ARCH, cuda(params[0]), models[0], cuda(cfgs[0]), None, "bf16", "B")
    F = vmc.loss(params[0].astype(np.float64), oa.Arch(**ARCH), ol.Model(**models[0]), cfgs[0])[0]
    assert abs(float(loss[0]) - F) / F < 2e-2
