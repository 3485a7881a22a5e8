"""CPU emulation of BF16 GEMM-operand rounding, used only to derive the BF16
tolerance at the ill-conditioned stress scale.

It evaluates the same network as oracle.ansatz in FP64, but rounds every
matrix-product operand to BF16 as the BF16 MFMA path does (activations entering
QKV, scores, P.V, W_O and the MLP, and the weights).  The error of this
emulation against the FP64 oracle is the error the BF16 arithmetic itself
incurs; the GPU's BF16 result is required to stay within a small factor of it.
It is not a reference for parity (the FP64 oracle is).
"""
import math

import numpy as np
import torch

from oracle import ansatz as oa


def _r(t):
    return t.to(torch.bfloat16).to(torch.float64)


def _z(theta, arch, bl, br):
    p = oa.unflatten(theta, arch)
    x = oa.embed(p, 1 - 2 * bl, 1 - 2 * br)
    for l in range(arch.layers):
        B, N, d = x.shape
        H = arch.heads
        dh = d // H
        xr = _r(x)
        q = (xr @ _r(p[f"l{l}_wq"])).reshape(B, N, H, dh).transpose(1, 2)
        k = (xr @ _r(p[f"l{l}_wk"])).reshape(B, N, H, dh).transpose(1, 2)
        v = (xr @ _r(p[f"l{l}_wv"])).reshape(B, N, H, dh).transpose(1, 2)
        s = (_r(q) @ _r(k).transpose(-1, -2)) / math.sqrt(dh)
        e = torch.exp(s - s.max(-1, keepdim=True).values)
        o = (_r(e) @ _r(v)) / e.sum(-1, keepdim=True)
        x = x + _r(o.transpose(1, 2).reshape(B, N, d)) @ _r(p[f"l{l}_wo"])
        u = torch.clamp(_r(x) @ _r(p[f"l{l}_w1"]) + p[f"l{l}_b1"], min=0)
        x = x + _r(u) @ _r(p[f"l{l}_w2"]) + p[f"l{l}_b2"]
    h = x.mean(1)
    f = h @ p["head_w"] + p["head_b"]
    return torch.complex(f[:, 0], f[:, 1])


def log_rho_bf16(theta, arch, cfg, n):
    a, b = oa.unpack_bits(cfg, n)
    th = torch.as_tensor(np.asarray(theta, np.float64))
    with torch.no_grad():
        return oa.symmetrise(_z(th, arch, a, b), _z(th, arch, b, a)).numpy()
