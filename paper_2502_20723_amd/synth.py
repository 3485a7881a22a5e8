"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the method: it only draws parameters,
configurations and model couplings from numpy PCG64 generators.  The paper
trains on configurations sampled from |rho|^2 of analytic spin-chain models;
there is no dataset, so every workload here is synthetic by construction.

Recipe
------
* parameters: N(0, 0.02) per entry ("init" scale, the workloads' own
  initialisation; log rho is then nearly constant across configurations),
  N(0, 1/fan_in) ("stress" scale: log rho varies by O(1), and the network is
  ill-conditioned: rounding the weights alone to BF16 moves log rho by ~3%),
  or 0.7/sqrt(fan_in) ("mid" scale: well-conditioned, log rho varies by a few
  percent); drawn in FP64 and rounded to FP32; both the GPU path and the
  oracle receive the rounded values;
* configurations: i.i.d. uniform bits for alpha and beta (bits above n are 0);
  at the "init" scale |rho|^2 is nearly flat, so this is what the sampler
  produces there;
* couplings of the batched workload: N uniform in [8, 40], half Ising, half
  XYZ, couplings uniform in [0.5, 1.5], gamma = 1, no fields.
"""
from __future__ import annotations

import numpy as np

ISING, XYZ = 0, 1

ARCH_FIELDS = ("d", "heads", "layers", "mlp")


def arch(d, heads, layers, mlp):
    return dict(d=d, heads=heads, layers=layers, mlp=mlp)


# Named workloads (sizes of the paper's models; arch widths per the runs measured).
WORKLOADS = {
    "ising_n4": dict(model=dict(kind=ISING, n=4, V=2.0, g=1.0, gamma=1.0),
                     arch=arch(16, 2, 1, 64), B=1024, seed=1000),
    "ising_n8": dict(model=dict(kind=ISING, n=8, V=2.0, g=1.0, gamma=1.0),
                     arch=arch(32, 4, 2, 128), B=4096, seed=1001),
    "xyz_n16": dict(model=dict(kind=XYZ, n=16, Jx=0.9, Jy=1.0, Jz=1.1, gamma=1.0),
                    arch=arch(64, 4, 2, 256), B=16384, seed=1002),
    "ising_n32": dict(model=dict(kind=ISING, n=32, V=2.0, g=None, gamma=1.0),
                      arch=arch(64, 8, 4, 256), B=65536, seed=1003),
    "batched_uneven": dict(model=None, arch=arch(64, 4, 3, 256), B=2048, seed=1004, problems=64),
    # 2D dissipative Ising: the paper's 2 x 3 lattice (V = 2 gamma) with the small
    # network, and a 4 x 8 lattice (n = 32) with the benchmark network
    "ising2d_2x3": dict(model=dict(kind=ISING, n=6, rows=2, V=2.0, g=1.0, gamma=1.0),
                        arch=arch(16, 2, 1, 64), B=1024, seed=1005),
    "ising2d_4x8": dict(model=dict(kind=ISING, n=32, rows=4, V=2.0, g=1.0, gamma=1.0),
                        arch=arch(64, 8, 4, 256), B=65536, seed=1006),
}


def workload(name: str) -> dict:
    """A copy of the named workload with its random couplings drawn."""
    w = {k: (dict(v) if isinstance(v, dict) else v) for k, v in WORKLOADS[name].items()}
    if name == "ising_n32":
        rng = np.random.default_rng(w["seed"] + 500)
        w["model"]["g"] = float(rng.uniform(0.5, 2.0))
    return w


def num_params(a: dict) -> int:
    d, m, L = a["d"], a["mlp"], a["layers"]
    C1 = a.get("c1", 0) or d
    return 5 * C1 + 2 * C1 * d + d + L * (4 * d * d + 2 * d * m + m + d) + 2 * d + 2


def _fan_ins(a: dict):
    d, m, L = a["d"], a["mlp"], a["layers"]
    C1 = a.get("c1", 0) or d
    out = [(4 * C1, 4), (C1, 4), (2 * C1 * d, 2 * C1), (d, 4)]
    for _ in range(L):
        out += [(d * d, d)] * 4 + [(d * m, d), (m, 4), (m * d, m), (d, 4)]
    out += [(2 * d, d), (2, 4)]
    return out


def params(a: dict, seed: int, scale: str = "init") -> np.ndarray:
    """Flat FP32 parameter vector for architecture a (layout of the ansatz)."""
    rng = np.random.default_rng(seed)
    if scale == "init":
        x = rng.standard_normal(num_params(a)) * 0.02
    elif scale in ("stress", "mid"):
        x = np.concatenate([rng.standard_normal(k) / np.sqrt(f) for k, f in _fan_ins(a)])
        if scale == "mid":
            x *= 0.7
    else:
        raise ValueError(scale)
    return x.astype(np.float32)


def configs(n: int, B: int, seed: int) -> np.ndarray:
    """uint64 [B, 2]: alpha and beta with i.i.d. uniform bits 0..n-1."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << n, size=(B, 2), dtype=np.uint64)


def uneven_problems(count: int, seed: int):
    """Model couplings of the batched workload: list of model dicts."""
    out = []
    for c in range(count):
        rng = np.random.default_rng(seed + 1000 + c)
        n = int(rng.integers(8, 41))
        if c % 2 == 0:
            V, g = rng.uniform(0.5, 1.5, size=2)
            out.append(dict(kind=ISING, n=n, V=float(V), g=float(g), gamma=1.0))
        else:
            Jx, Jy, Jz = rng.uniform(0.5, 1.5, size=3)
            out.append(dict(kind=XYZ, n=n, Jx=float(Jx), Jy=float(Jy), Jz=float(Jz), gamma=1.0))
    return out
