"""Pins of oracle.ansatz (CPU only).

The paper prints no weights and no network outputs, so the forward is pinned
by (i) the symmetries the paper designs in (translation invariance from the
pooling, Hermiticity from the symmetrisation), (ii) closed forms: of the
symmetrisation, and of the mean pooling at uniform configurations (log rho
independent of n), (iii) independent library routines for each stage:
torch's circular conv2d for the embedding, torch.nn.MultiheadAttention for
the attention block, torch.nn.Linear/ReLU for the feed-forward sub-layer, and
(iv) the whole network assembled a second time from torch.nn modules, which
fixes how the stages compose.  A transposed operand, a wrong tap, a dropped
residual, a swapped sub-layer order, a sum instead of a mean over sites or a
wrong softmax scale fails one of these; the composition mistakes are planted
in test_planted_composition_mistakes_fail_a_pin.
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn

from oracle import ansatz as oa

ARCHS = {
    "c1": oa.Arch(d=16, heads=2, layers=1, mlp=64),
    "c2": oa.Arch(d=32, heads=4, layers=2, mlp=128),
    "c3": oa.Arch(d=64, heads=4, layers=2, mlp=256),
    "c4": oa.Arch(d=64, heads=8, layers=4, mlp=256),
    "c5": oa.Arch(d=64, heads=4, layers=3, mlp=256),
}


def stress_params(arch, seed=0):
    """Weights of O(1/sqrt(fan_in)) so that log rho varies by O(1) across configs."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in oa.param_layout(arch):
        fan_in = shape[0] * (shape[1] if name in ("conv1_w", "conv2_w") else 1) if len(shape) > 1 else 4
        out.append(rng.standard_normal(int(np.prod(shape))) / math.sqrt(fan_in))
    return np.concatenate(out)


def rand_cfg(n, B, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << n, size=(B, 2), dtype=np.uint64)


def test_param_counts():
    """P = 5 C1 + 2 C1 d + d + L (4 d^2 + 2 d m + m + d) + 2 d + 2 with C1 = d."""
    expect = {"c1": 3794, "c2": 27202, "c3": 107650, "c4": 206594, "c5": 157122}
    for k, a in ARCHS.items():
        d, m, L, C1 = a.d, a.mlp, a.layers, a.C1
        assert oa.num_params(a) == 5 * C1 + 2 * C1 * d + d + L * (4 * d * d + 2 * d * m + m + d) + 2 * d + 2
        assert oa.num_params(a) == expect[k]


def test_gelu_is_exact_erf_form():
    u = torch.linspace(-6, 6, 1001, dtype=torch.float64)
    assert torch.max(torch.abs(oa.gelu(u) - Fnn.gelu(u, approximate="none"))) < 1e-15


@pytest.mark.parametrize("n", [4, 7, 16])
def test_cyclic_shift_invariance(n):
    """Mean pooling over sites makes log rho invariant under a simultaneous
    cyclic shift of alpha and beta (App. B, global mean pooling)."""
    arch = ARCHS["c3"]
    th = stress_params(arch, 1)
    cfg = rand_cfg(n, 64, 2)
    mask = np.uint64((1 << n) - 1)
    for sh in (1, 3):
        rot = ((cfg << np.uint64(sh)) | (cfg >> np.uint64(n - sh))) & mask
        a = oa.log_rho(th, arch, cfg, n)
        b = oa.log_rho(th, arch, rot, n)
        dz = a - b
        assert torch.max(torch.abs(dz.real)) < 1e-12
        assert torch.max(torch.abs(torch.remainder(dz.imag + math.pi, 2 * math.pi) - math.pi)) < 1e-12


def test_hermiticity():
    """Eq. log_sum_exp_conjugate makes rho(beta, alpha) = conj rho(alpha, beta)."""
    arch = ARCHS["c2"]
    n = 8
    th = stress_params(arch, 3)
    cfg = rand_cfg(n, 128, 4)
    a = oa.log_rho(th, arch, cfg, n)
    b = oa.log_rho(th, arch, cfg[:, ::-1].copy(), n)
    assert torch.max(torch.abs(a.real - b.real)) < 1e-12
    dz = a.imag + b.imag
    assert torch.max(torch.abs(torch.remainder(dz + math.pi, 2 * math.pi) - math.pi)) < 1e-12


def test_symmetrisation_closed_form():
    """With head weights zero, z = b0 + i b1 for every configuration, so
    log rho = log(2 Re e^z) = b0 + log 2 + log cos b1 (cos b1 > 0)."""
    arch = ARCHS["c1"]
    th = stress_params(arch, 5)
    P = oa.num_params(arch)
    th[P - 2 - 2 * arch.d:P - 2] = 0.0
    th[P - 2:] = [0.3, 0.7]
    cfg = rand_cfg(4, 32, 6)
    lr = oa.log_rho(th, arch, cfg, 4)
    assert torch.max(torch.abs(lr.real - (0.3 + math.log(2) + math.log(math.cos(0.7))))) < 1e-14
    assert torch.max(torch.abs(lr.imag)) < 1e-14
    th[P - 1] = 2.0   # cos < 0: principal branch gives Im = pi
    lr = oa.log_rho(th, arch, cfg, 4)
    assert torch.max(torch.abs(lr.real - (0.3 + math.log(2) + math.log(-math.cos(2.0))))) < 1e-14
    assert torch.max(torch.abs(lr.imag - math.pi)) < 1e-14


def test_embedding_against_torch_circular_conv2d():
    """Eq. circ-conv read as a 2x1 kernel over (sites x dummy) with the (alpha,
    beta) channels as input channels and circular padding after the last site."""
    arch = ARCHS["c2"]
    n, B = 8, 16
    th = torch.as_tensor(stress_params(arch, 7))
    p = oa.unflatten(th, arch)
    a, b = oa.unpack_bits(rand_cfg(n, B, 8), n)
    sa, sb = 1 - 2 * a, 1 - 2 * b
    mine = oa.embed(p, sa, sb)
    x = torch.stack([sa, sb], dim=1).unsqueeze(-1)                   # [B, 2, N, 1]
    w1 = p["conv1_w"].permute(2, 1, 0).unsqueeze(-1)                 # [C1, 2, 2 taps, 1]
    e = Fnn.gelu(Fnn.conv2d(Fnn.pad(x, (0, 0, 0, 1), mode="circular"), w1, p["conv1_b"]))
    w2 = p["conv2_w"].permute(2, 1, 0).unsqueeze(-1)                 # [d, C1, 2, 1]
    y = Fnn.gelu(Fnn.conv2d(Fnn.pad(e, (0, 0, 0, 1), mode="circular"), w2, p["conv2_b"]))
    ref = y.squeeze(-1).transpose(1, 2)                              # [B, N, d]
    assert torch.max(torch.abs(mine - ref)) < 1e-13


def test_embedding_window_is_three_sites():
    """Two width-2 convolutions see sites i, i+1, i+2: x_i is unchanged when
    any other site flips."""
    arch = ARCHS["c2"]
    n = 8
    th = torch.as_tensor(stress_params(arch, 9))
    p = oa.unflatten(th, arch)
    a, b = oa.unpack_bits(rand_cfg(n, 4, 10), n)
    x0 = oa.embed(p, 1 - 2 * a, 1 - 2 * b)
    for j in range(n):
        a2 = a.clone()
        a2[:, j] = 1 - a2[:, j]
        x1 = oa.embed(p, 1 - 2 * a2, 1 - 2 * b)
        changed = torch.any(torch.abs(x1 - x0) > 0, dim=(0, 2))
        expect = torch.zeros(n, dtype=torch.bool)
        for i in ((j - 2) % n, (j - 1) % n, j):
            expect[i] = True
        assert torch.equal(changed, expect), j


@pytest.mark.parametrize("heads", [1, 4, 8])
def test_attention_against_multihead_attention(heads):
    """Eq. attn-head-appendix + X' residual against torch.nn.MultiheadAttention."""
    d, n, B = 64, 12, 5
    g = torch.Generator().manual_seed(heads)
    x = torch.randn(B, n, d, dtype=torch.float64, generator=g)
    wq, wk, wv, wo = (torch.randn(d, d, dtype=torch.float64, generator=g) / 8 for _ in range(4))
    mine = oa.attention(x, wq, wk, wv, wo, heads)
    mha = torch.nn.MultiheadAttention(d, heads, bias=False, batch_first=True, dtype=torch.float64)
    with torch.no_grad():
        mha.in_proj_weight.copy_(torch.cat([wq.T, wk.T, wv.T], dim=0))
        mha.out_proj.weight.copy_(wo.T)
        ref, _ = mha(x, x, x, need_weights=False)
    assert torch.max(torch.abs(mine - (x + ref))) < 1e-12


def test_layout_independent_of_n():
    """The same parameter vector evaluates any chain length (App. B: pooling
    removes the N dependence of the head)."""
    arch = ARCHS["c5"]
    th = stress_params(arch, 11)
    for n in (3, 8, 40):
        lr = oa.log_rho(th, arch, rand_cfg(n, 4, n), n)
        assert torch.all(torch.isfinite(lr.real))


def test_mlp_against_torch_linear_relu():
    """The residual MLP sub-layer equals Linear -> ReLU -> Linear of torch.nn."""
    d, m = 32, 128
    g = torch.Generator().manual_seed(5)
    x = torch.randn(7, 9, d, dtype=torch.float64, generator=g)
    w1, w2 = torch.randn(d, m, dtype=torch.float64, generator=g), torch.randn(m, d, dtype=torch.float64, generator=g)
    b1, b2 = torch.randn(m, dtype=torch.float64, generator=g), torch.randn(d, dtype=torch.float64, generator=g)
    net = torch.nn.Sequential(torch.nn.Linear(d, m), torch.nn.ReLU(), torch.nn.Linear(m, d)).double()
    with torch.no_grad():
        net[0].weight.copy_(w1.T); net[0].bias.copy_(b1)
        net[2].weight.copy_(w2.T); net[2].bias.copy_(b2)
        ref = net(x)
    assert torch.max(torch.abs(oa.mlp(x, w1, b1, w2, b2) - ref)) < 1e-12


# ---------------------------------------------------------------- composition of the stages
# The stage pins above (convolution, attention, feed-forward) do not fix how z_out chains
# them: residual attention sub-layer, then residual feed-forward sub-layer, per layer
# (App. B, the X' equation and the transformer block it extends), the 1/N mean over sites
# (Eq. global-pool-final) and the head.  Two pins do: a closed form of the pooling, and the
# network assembled a second time from torch.nn modules.  Each takes the z function under
# test, so the planted-mistake test below can hand it a wrong composition.

def _uniform_cfg(a_bit, b_bit, n):
    """Every site in the same doubled state (alpha_i, beta_i) = (a_bit, b_bit)."""
    full = (1 << n) - 1
    return np.array([[full if a_bit else 0, full if b_bit else 0]], dtype=np.uint64)


def _uniform_spread(zfn, arch, th):
    """Largest spread over n in {3, 8, 40} of log rho at a uniform configuration.  Every
    site then has the same window code, so every row of x is the same vector through
    every layer (identical keys give uniform attention weights, and a convex mix of
    identical rows is that row) and the 1/N mean of the pooling returns it whatever n is:
    log rho does not depend on n.  A sum over sites would scale z by n."""
    th = torch.as_tensor(th)
    worst = 0.0
    for ab in ((0, 0), (0, 1), (1, 0), (1, 1)):
        vals = []
        for n in (3, 8, 40):
            cfg = _uniform_cfg(ab[0], ab[1], n)
            a, b = oa.unpack_bits(cfg, n)
            vals.append(oa.symmetrise(zfn(th, arch, a, b), zfn(th, arch, b, a))[0])
        for v in vals[1:]:
            worst = max(worst, abs(complex(v) - complex(vals[0])))
    return worst


class _TorchNet(torch.nn.Module):
    """The network assembled from torch.nn modules only: Conv2d over (sites x 1) with the
    (alpha, beta) spins as two input channels and one circular pad after the last site,
    GELU, a second such convolution and GELU (Eq. circ-conv); per layer
    MultiheadAttention without biases plus residual, then Linear-ReLU-Linear plus
    residual; the mean over sites (Eq. global-pool-final) and a Linear head to (F0, F1)."""

    def __init__(self, arch, p):
        super().__init__()
        d, C1, L = arch.d, arch.C1, arch.layers
        f64 = dict(dtype=torch.float64)
        self.pad = torch.nn.CircularPad2d((0, 0, 0, 1))
        self.conv1 = torch.nn.Conv2d(2, C1, kernel_size=(2, 1), **f64)
        self.conv2 = torch.nn.Conv2d(C1, d, kernel_size=(2, 1), **f64)
        self.act = torch.nn.GELU()
        self.att = torch.nn.ModuleList(torch.nn.MultiheadAttention(d, arch.heads, bias=False, batch_first=True, **f64)
                                       for _ in range(L))
        self.ffn = torch.nn.ModuleList(torch.nn.Sequential(torch.nn.Linear(d, arch.mlp, **f64), torch.nn.ReLU(),
                                                           torch.nn.Linear(arch.mlp, d, **f64)) for _ in range(L))
        self.head = torch.nn.Linear(d, 2, **f64)
        with torch.no_grad():
            # flat layout: conv W[tap][in-channel][out]; Conv2d wants [out][in][tap][1]
            self.conv1.weight.copy_(p["conv1_w"].permute(2, 1, 0).unsqueeze(-1))
            self.conv1.bias.copy_(p["conv1_b"])
            self.conv2.weight.copy_(p["conv2_w"].permute(2, 1, 0).unsqueeze(-1))
            self.conv2.bias.copy_(p["conv2_b"])
            for l in range(L):   # x @ W convention in the flat vector; torch.nn stores W^T
                self.att[l].in_proj_weight.copy_(torch.cat([p[f"l{l}_wq"].T, p[f"l{l}_wk"].T, p[f"l{l}_wv"].T]))
                self.att[l].out_proj.weight.copy_(p[f"l{l}_wo"].T)
                self.ffn[l][0].weight.copy_(p[f"l{l}_w1"].T)
                self.ffn[l][0].bias.copy_(p[f"l{l}_b1"])
                self.ffn[l][2].weight.copy_(p[f"l{l}_w2"].T)
                self.ffn[l][2].bias.copy_(p[f"l{l}_b2"])
            self.head.weight.copy_(p["head_w"].T)
            self.head.bias.copy_(p["head_b"])

    def forward(self, sa, sb):
        img = torch.stack([sa, sb], dim=1).unsqueeze(-1)          # [B, 2 channels, N sites, 1]
        e = self.act(self.conv1(self.pad(img)))
        x = self.act(self.conv2(self.pad(e))).squeeze(-1).transpose(1, 2)   # [B, N, d]
        for att, ffn in zip(self.att, self.ffn):
            x = x + att(x, x, x, need_weights=False)[0]
            x = x + ffn(x)
        f = self.head(x.mean(dim=1))
        return torch.complex(f[:, 0], f[:, 1])


def _torch_nn_gap(zfn, arch, th, n, B, seed):
    """Largest |z - z_torch.nn| over B random configurations, both channel orders."""
    net = _TorchNet(arch, oa.unflatten(torch.as_tensor(th), arch))
    a, b = oa.unpack_bits(rand_cfg(n, B, seed), n)
    worst = 0.0
    with torch.no_grad():
        for bl, br in ((a, b), (b, a)):
            ref = net(1 - 2 * bl, 1 - 2 * br)
            worst = max(worst, float(torch.max(torch.abs(zfn(torch.as_tensor(th), arch, bl, br) - ref))))
    return worst


# the workloads' smallest and benchmark networks, with their chain lengths
COMPOSITION_CASES = [("c1", 4, 64), ("c4", 32, 16)]


@pytest.mark.parametrize("key", ["c1", "c5"])
def test_uniform_configurations_do_not_depend_on_n(key):
    arch = ARCHS[key]
    assert _uniform_spread(oa.z_out, arch, stress_params(arch, 21)) < 1e-12


@pytest.mark.parametrize("key,n,B", COMPOSITION_CASES)
def test_network_against_torch_nn_assembly(key, n, B):
    arch = ARCHS[key]
    th = stress_params(arch, 23)
    assert _torch_nn_gap(oa.z_out, arch, th, n, B, 24) < 1e-11


def _z_planted(mistake):
    """z_out with one composition mistake planted: the oracle's own stage functions
    chained in a wrong way."""

    def z(theta, arch, bl, br):
        p = oa.unflatten(theta, arch)
        x = oa.embed(p, 1.0 - 2.0 * bl, 1.0 - 2.0 * br)
        for l in range(arch.layers):
            att = lambda u: oa.attention(u, p[f"l{l}_wq"], p[f"l{l}_wk"], p[f"l{l}_wv"], p[f"l{l}_wo"], arch.heads)
            ffn = lambda u: oa.mlp(u, p[f"l{l}_w1"], p[f"l{l}_b1"], p[f"l{l}_w2"], p[f"l{l}_b2"])
            if mistake == "ffn_first":
                x = att(x + ffn(x))
            elif mistake == "no_ffn_residual":
                x = ffn(att(x))
            else:
                x = att(x)
                x = x + ffn(x)
        h = x.sum(dim=1) if mistake == "sum_pool" else x.mean(dim=1)
        f = h @ p["head_w"] + p["head_b"]
        return torch.complex(f[:, 0], f[:, 1])

    return z


def test_planted_composition_mistakes_fail_a_pin():
    """Sum pooling, a dropped feed-forward residual and the feed-forward sub-layer before
    attention each fail at least one of the two composition pins, while the harness with
    no mistake reproduces the oracle."""
    for key, n, B in COMPOSITION_CASES:
        arch, th = ARCHS[key], stress_params(ARCHS[key], 23)
        assert _torch_nn_gap(_z_planted(None), arch, th, n, B, 24) < 1e-11
    for mistake in ("sum_pool", "no_ffn_residual", "ffn_first"):
        caught = []
        for key, n, B in COMPOSITION_CASES:
            arch = ARCHS[key]
            th = stress_params(arch, 23)
            caught.append(_torch_nn_gap(_z_planted(mistake), arch, th, n, B, 24) > 1e-6)
            caught.append(_uniform_spread(_z_planted(mistake), arch, stress_params(arch, 21)) > 1e-6)
        assert any(caught), mistake
