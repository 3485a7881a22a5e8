"""CPU emulations of the GPU path's rounding, used only to derive tolerances
where the stated ones cannot hold for the arithmetic itself.

* ``bf16``: the same network as oracle.ansatz evaluated in FP64, with every
  matrix-product operand rounded to BF16 as the BF16 MFMA path does
  (activations entering QKV, q scaled by log2(e)/sqrt(dh), k, P.V, W_O and
  the MLP, and the weights).
  Differentiated by autograd, the casts also round the gradients flowing back
  through those operands to BF16, which is what the BF16 backward does.
* ``fp32``: the same network evaluated entirely in FP32 (torch on the CPU).

The error of an emulation against the FP64 oracle is the error that precision
incurs by itself; a GPU result is required to stay within a small factor of
it.  It is not a reference for parity (the FP64 oracle is).

``kink_sensitivity`` measures a second effect of rounding on the gradient:
the feed-forward ReLU decides a unit's branch from the sign of its
pre-activation, and for a pre-activation within rounding distance of zero that
sign is decided by summation order.  ``kink_margins`` gives, per sample, the
smallest relative distance of any pre-activation of its evaluated
configurations from zero, so that tests can assert the stated FP32 gradient
bar on samples that have no unit in that band.
"""
import math

import numpy as np
import torch

from oracle import ansatz as oa
from oracle import lindblad as ol
from oracle import vmc

KINK_KAPPA = 2.0 ** -23  # two FP32 rounding steps


def _r16(t):
    return t.to(torch.bfloat16).to(torch.float64)


def _ident(t):
    return t


def _z(p, arch, bl, br, R):
    x = oa.embed(p, 1 - 2 * bl, 1 - 2 * br)
    for l in range(arch.layers):
        B, N, d = x.shape
        H = arch.heads
        dh = d // H
        xr = R(x)
        q = (xr @ R(p[f"l{l}_wq"])).reshape(B, N, H, dh).transpose(1, 2)
        k = (xr @ R(p[f"l{l}_wk"])).reshape(B, N, H, dh).transpose(1, 2)
        v = (xr @ R(p[f"l{l}_wv"])).reshape(B, N, H, dh).transpose(1, 2)
        # the kernels fold the softmax scale log2(e)/sqrt(dh) into q before rounding it
        c = math.log2(math.e) / math.sqrt(dh)
        s = (R(q * c) @ R(k).transpose(-1, -2)) / math.log2(math.e)
        e = torch.exp(s - s.max(-1, keepdim=True).values)
        o = (R(e) @ R(v)) / e.sum(-1, keepdim=True)
        x = x + R(o.transpose(1, 2).reshape(B, N, d)) @ R(p[f"l{l}_wo"])
        u = torch.clamp(R(x) @ R(p[f"l{l}_w1"]) + p[f"l{l}_b1"], min=0)
        x = x + R(u) @ R(p[f"l{l}_w2"]) + p[f"l{l}_b2"]
    h = x.mean(1)
    f = h @ p["head_w"] + p["head_b"]
    return torch.complex(f[:, 0], f[:, 1])


def _setup(prec):
    if prec == "bf16":
        return torch.float64, _r16
    if prec == "fp32":
        return torch.float32, _ident
    raise ValueError(prec)


def _log_rho(th, arch, cfg, n, prec):
    dt, R = _setup(prec)
    p = oa.unflatten(th, arch)
    a, b = oa.unpack_bits(cfg, n)
    a, b = a.to(dt), b.to(dt)
    return oa.symmetrise(_z(p, arch, a, b, R), _z(p, arch, b, a, R))


def log_rho_emulated(theta, arch, cfg, n, prec):
    dt, _ = _setup(prec)
    th = torch.as_tensor(np.asarray(theta)).to(dt)
    with torch.no_grad():
        return _log_rho(th, arch, cfg, n, prec).to(torch.complex128).numpy()


def log_rho_bf16(theta, arch, cfg, n):
    return log_rho_emulated(theta, arch, cfg, n, "bf16")


def log_rho_vjp_emulated(theta, arch, cfg, n, seed, prec):
    """sum_b seed[b, 0] d Re log rho_b + seed[b, 1] d Im log rho_b, with the network
    evaluated and differentiated at the emulated precision."""
    dt, _ = _setup(prec)
    th = torch.tensor(np.asarray(theta), dtype=dt, requires_grad=True)
    lr = _log_rho(th, arch, np.asarray(cfg, dtype=np.uint64).reshape(-1, 2), n, prec)
    s = torch.as_tensor(np.asarray(seed)).to(dt)
    (g,) = torch.autograd.grad((s[:, 0] * lr.real + s[:, 1] * lr.imag).sum(), th)
    return g.double().numpy()


def loss_grad_emulated(theta, arch, model, cfg, weights, mode, prec):
    """(F, grad) of the cost at fixed samples (modes "A"/"B" as in oracle.vmc),
    with the network evaluated and differentiated at the emulated precision."""
    dt, _ = _setup(prec)
    cdt = torch.complex64 if dt == torch.float32 else torch.complex128
    cfg = np.asarray(cfg, dtype=np.uint64).reshape(-1, 2)
    rows = ol.connected(model, cfg)
    th = torch.tensor(np.asarray(theta), dtype=dt, requires_grad=True)
    B = len(cfg)
    allc = np.concatenate([cfg] + [r[0] for r in rows if len(r[0])], 0)
    lr = _log_rho(th, arch, allc, model.n, prec)
    lrx, off, Ls = lr[:B], B, []
    for b in range(B):
        k = len(rows[b][0])
        c = torch.as_tensor(rows[b][1]).to(cdt)
        Ls.append((c * torch.exp(lr[off:off + k] - lrx[b])).sum())
        off += k
    L = torch.stack(Ls)
    w = torch.as_tensor(np.ones(B) if weights is None else np.asarray(weights), dtype=dt)
    W = w.sum()
    F = ((w * L.abs() ** 2).sum() / W).detach()
    if mode == "A":
        obj = (w * L.abs() ** 2).sum() / W
    else:
        r = w * torch.exp(2 * (lrx.real - lrx.real.detach()))
        obj = (r * L.abs() ** 2 - F * r).sum() / W
    (g,) = torch.autograd.grad(obj, th)
    return float(F), g.double().numpy()


def kink_sensitivity(params, A, M, cfg, w, mode, g_ref, kappa=KINK_KAPPA):
    """Relative change of the FP64 gradient when the ReLU of every feed-forward unit
    whose pre-activation u lies within kappa (|b1| + sum |x W1|) of zero takes the
    other branch (the oracle's feed-forward function is replaced for one call)."""
    orig = oa.mlp

    def mlp_flipped(x, w1, b1, w2, b2):
        u = x @ w1 + b1
        near = u.detach().abs() < kappa * (x.abs() @ w1.abs() + b1.abs()).detach()
        h = torch.where(near, torch.where(u > 0, torch.zeros_like(u), u), torch.clamp(u, min=0.0))
        return h @ w2 + b2

    oa.mlp = mlp_flipped
    try:
        _, gk, _ = vmc.loss_grad(params.astype(np.float64), A, M, cfg, w, mode=mode)
    finally:
        oa.mlp = orig
    return float(np.linalg.norm(gk - g_ref) / max(np.linalg.norm(g_ref), 1e-300))


def kink_margins(params, A, M, cfg):
    """Per sample b: min over the layers, the sites, the hidden units and the evaluated
    configurations of the row (the sample and its connected configurations) of
    |u| / (|b1| + sum |x W1|), u the feed-forward pre-activation, in FP64."""
    cfg = np.asarray(cfg, dtype=np.uint64).reshape(-1, 2)
    rows = ol.connected(M, cfg)
    rec = []
    orig = oa.mlp

    def mlp_rec(x, w1, b1, w2, b2):
        u = x @ w1 + b1
        scale = x.abs() @ w1.abs() + b1.abs()
        # a unit whose summands all vanish sits on the kink itself: margin 0
        r = torch.where(scale > 0, u.abs() / torch.where(scale > 0, scale, torch.ones_like(scale)), torch.zeros_like(u))
        rec.append(r.amin(dim=(1, 2)))
        return orig(x, w1, b1, w2, b2)

    th = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out = np.empty(len(cfg))
    oa.mlp = mlp_rec
    try:
        with torch.no_grad():
            for b in range(len(cfg)):
                rec.clear()
                oa.log_rho(th, A, np.concatenate([cfg[b:b + 1], rows[b][0]], 0), M.n)
                out[b] = min(float(r.min()) for r in rec)
    finally:
        oa.mlp = orig
    return out


def kink_free_configs(params, A, M, B, seed, kappa=KINK_KAPPA, pool=8):
    """B samples (uniform bits, PCG64 seed) whose rows have no feed-forward pre-activation
    within kappa of zero relative to its summands: the first B such among pool * B draws."""
    rng = np.random.default_rng(seed)
    cand = rng.integers(0, 1 << M.n, size=(pool * B, 2), dtype=np.uint64)
    keep = cand[kink_margins(params, A, M, cand) > kappa][:B]
    assert len(keep) == B, f"only {len(keep)} of {pool * B} candidate samples are outside the kink band"
    return keep
