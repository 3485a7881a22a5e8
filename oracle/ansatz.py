"""Oracle: the transformer density operator log rho(alpha, beta) in FP64
(test infrastructure only).

Architecture (main text "Transformer density operator ansatz"; App. B):

1. input stacking: the two spin rows alpha, beta of a configuration become a
   two-channel sequence of length N, spin values s = 1 - 2*bit (App. B,
   "Feature Embedding");
2. two circularly padded convolutions with a 2x1 kernel over sites, each
   followed by the activation (Eq. circ-conv and the second convolution "in
   the same manner");
3. per layer: multi-head self-attention with W^Q, W^K, W^V split by head,
   softmax(Q K^T / sqrt(C2/h)) V, concatenation, W^O and a residual
   (Eq. attn-head-appendix and the X' equation); then a residual MLP
   sub-layer x + max(0, x W1 + b1) W2 + b2 (the workloads give an MLP width;
   the paper's block omits the feed-forward sub-layer, so it follows the
   position-wise feed-forward network of the transformer the paper builds on,
   Vaswani et al., with its ReLU);
4. mean pooling over sites (Eq. global-pool-final), a dense head to two
   outputs [F0, F1], z = F0 + i F1;
5. Hermitian symmetrisation log rho = log(exp z(alpha,beta) + conj exp z(beta,alpha))
   (Eq. log_sum_exp_conjugate).

Readings where the paper is silent (listed with reasons in the design notes):
convolution activation = exact GELU u * Phi(u); MLP activation = ReLU; conv taps (i, i+1 mod N) with channels
(alpha, beta); C1 = C2 = d; no bias on the attention projections; attention
scale 1/sqrt(d/h); principal branch of the complex log.

Parameters are one flat real vector, row-major, x @ W convention, in the order
returned by ``param_layout``.

Parity: unpinned by printed values (the paper prints no weights or outputs).
Pinned by invariants, closed forms and independent re-derivations in
tests/test_oracle_ansatz.py: cyclic-shift invariance, Hermiticity, the closed
form of the symmetrisation when the head weights vanish, n-independence of log
rho at uniform configurations (the 1/N mean pooling), the convolution against
torch's own circular conv2d, the attention block against
torch.nn.MultiheadAttention, the MLP against torch.nn.Linear/ReLU, the whole
network against a second assembly from torch.nn modules (which fixes the
composition: residual attention, then residual feed-forward, mean over sites,
head), and parameter-layout independence of N.  Sum pooling, a dropped
feed-forward residual and a swapped sub-layer order are planted there and
each fails a pin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch


@dataclass(frozen=True)
class Arch:
    """Network shape: width d, heads, layers, MLP width mlp, conv-1 filters c1."""

    d: int
    heads: int
    layers: int
    mlp: int
    c1: int = 0  # 0 means c1 = d

    @property
    def C1(self) -> int:
        return self.c1 if self.c1 > 0 else self.d


def param_layout(arch: Arch):
    """Ordered (name, shape) list of the flat parameter vector."""
    d, m, C1 = arch.d, arch.mlp, arch.C1
    lay = [("conv1_w", (2, 2, C1)), ("conv1_b", (C1,)),
           ("conv2_w", (2, C1, d)), ("conv2_b", (d,))]
    for l in range(arch.layers):
        lay += [(f"l{l}_wq", (d, d)), (f"l{l}_wk", (d, d)), (f"l{l}_wv", (d, d)),
                (f"l{l}_wo", (d, d)), (f"l{l}_w1", (d, m)), (f"l{l}_b1", (m,)),
                (f"l{l}_w2", (m, d)), (f"l{l}_b2", (d,))]
    lay += [("head_w", (d, 2)), ("head_b", (2,))]
    return lay


def num_params(arch: Arch) -> int:
    return int(sum(np.prod(s) for _, s in param_layout(arch)))


def unflatten(theta: torch.Tensor, arch: Arch) -> dict:
    out, off = {}, 0
    for name, shape in param_layout(arch):
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    assert off == theta.numel(), (off, theta.numel())
    return out


def gelu(u: torch.Tensor) -> torch.Tensor:
    """Exact GELU: u * Phi(u) with Phi the standard normal CDF."""
    return u * 0.5 * (1.0 + torch.erf(u / math.sqrt(2.0)))


def unpack_bits(cfg, n: int) -> tuple[torch.Tensor, torch.Tensor]:
    """uint64 [B, 2] (alpha, beta) -> two float64 bit tensors [B, n]."""
    cfg = np.asarray(cfg, dtype=np.uint64).reshape(-1, 2)
    sh = np.arange(n, dtype=np.uint64)
    a = ((cfg[:, 0:1] >> sh) & np.uint64(1)).astype(np.float64)
    b = ((cfg[:, 1:2] >> sh) & np.uint64(1)).astype(np.float64)
    return torch.from_numpy(a), torch.from_numpy(b)


def embed(p: dict, sa: torch.Tensor, sb: torch.Tensor) -> torch.Tensor:
    """Two circular 2x1 convolutions with activation (Eq. circ-conv).

    sa, sb: spins [B, N] of the two channels.  Tap 0 reads site i, tap 1 reads
    site i+1 (mod N).  Returns X [B, N, d].
    """
    x_in = torch.stack([sa, sb], dim=-1)                       # [B, N, 2]
    x_nb = torch.roll(x_in, shifts=-1, dims=1)                 # site i+1
    e = gelu(p["conv1_b"] + x_in @ p["conv1_w"][0] + x_nb @ p["conv1_w"][1])
    e_nb = torch.roll(e, shifts=-1, dims=1)
    return gelu(p["conv2_b"] + e @ p["conv2_w"][0] + e_nb @ p["conv2_w"][1])


def attention(x: torch.Tensor, wq, wk, wv, wo, heads: int) -> torch.Tensor:
    """Multi-head self-attention with residual (Eq. attn-head-appendix, X')."""
    B, N, d = x.shape
    dh = d // heads
    q = (x @ wq).reshape(B, N, heads, dh).transpose(1, 2)      # [B, h, N, dh]
    k = (x @ wk).reshape(B, N, heads, dh).transpose(1, 2)
    v = (x @ wv).reshape(B, N, heads, dh).transpose(1, 2)
    s = (q @ k.transpose(-1, -2)) / math.sqrt(dh)              # [B, h, N, N]
    a = torch.softmax(s, dim=-1) @ v                           # [B, h, N, dh]
    cat = a.transpose(1, 2).reshape(B, N, d)
    return x + cat @ wo


def mlp(x: torch.Tensor, w1, b1, w2, b2) -> torch.Tensor:
    """Position-wise feed-forward sub-layer max(0, x W1 + b1) W2 + b2 (no residual)."""
    return torch.clamp(x @ w1 + b1, min=0.0) @ w2 + b2


def z_out(theta: torch.Tensor, arch: Arch, bits_l: torch.Tensor, bits_r: torch.Tensor) -> torch.Tensor:
    """Complex network output z for the channel order (bits_l, bits_r)."""
    p = unflatten(theta, arch)
    x = embed(p, 1.0 - 2.0 * bits_l, 1.0 - 2.0 * bits_r)
    for l in range(arch.layers):
        x = attention(x, p[f"l{l}_wq"], p[f"l{l}_wk"], p[f"l{l}_wv"], p[f"l{l}_wo"], arch.heads)
        x = x + mlp(x, p[f"l{l}_w1"], p[f"l{l}_b1"], p[f"l{l}_w2"], p[f"l{l}_b2"])
    h = x.mean(dim=1)                                          # Eq. global-pool-final
    f = h @ p["head_w"] + p["head_b"]
    return torch.complex(f[:, 0], f[:, 1])


def symmetrise(z1: torch.Tensor, z2: torch.Tensor) -> torch.Tensor:
    """log(exp(z1) + conj(exp(z2))) on the principal branch
    (Eq. log_sum_exp_conjugate), computed after shifting by the larger real part."""
    m = torch.maximum(z1.real, z2.real)
    s = torch.exp(z1 - m) + torch.exp(torch.conj(z2) - m)
    return torch.complex(m + torch.log(torch.abs(s)), torch.angle(s))


def log_rho(theta, arch: Arch, cfg, n: int) -> torch.Tensor:
    """log rho(alpha, beta) for uint64 configurations cfg [B, 2]; complex128 [B].

    theta: float64 tensor of num_params(arch) values (may require grad).
    """
    theta = torch.as_tensor(theta, dtype=torch.float64)
    a, b = unpack_bits(cfg, n)
    return symmetrise(z_out(theta, arch, a, b), z_out(theta, arch, b, a))
