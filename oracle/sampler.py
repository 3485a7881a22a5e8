"""Oracle: Metropolis-Hastings chains on P(x) ~ |rho(x)|^2 (test infrastructure only).

App. C, "Efficient Sampling Strategy": propose a local update of one degree
of freedom of the doubled configuration, accept with probability
min(1, P(x')/P(x)) (the proposal is symmetric), else keep x.

Proposal kernel (reading; the paper names only a local single-DOF move):
with probability p_pair flip alpha_i and beta_i together at a uniform site i,
otherwise flip one uniform bit among the 2N bits (bits 0..N-1 are alpha,
N..2N-1 are beta).  Both moves are their own inverse and uniform, so the
kernel is symmetric.  The pair move keeps parity(alpha) - parity(beta), which
the single move alone cannot leave unchanged in one step; the XYZ steady state
vanishes on configurations with parity(alpha) != parity(beta).

Random numbers: proposal t of chain c uses one Philox4x32-10 block with
counter (t mod 2^32, t >> 32, c, 0) and key (seed mod 2^32, seed >> 32),
output words r0, r1, r2:
  pair move      iff r0 < floor(p_pair * 2^32)
  pair site      i = (r1 * N) >> 32
  single bit     j = (r1 * 2N) >> 32
  accept         iff (r2 + 0.5) * 2^-32 < exp(2 Re(log rho(x') - log rho(x))).
One sweep is 2N proposals; a sample is recorded after each sweep.

Parity: pinned in tests/test_oracle_philox_sampler.py by a chi-square test of the
visit frequencies against the exactly enumerated |rho|^2 at N = 3, and by the
pure random walk (every move accepted) when log rho is constant.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ansatz
from .philox import philox4x32_10


def proposal(cfg, n, t, chain, seed, p_pair):
    """Proposed configurations and acceptance uniforms for proposal index t.

    cfg: uint64 [C, 2]; chain: int array [C]; t: int (same for all chains).
    Returns (cfg' [C, 2] uint64, u [C] float64).
    """
    C = cfg.shape[0]
    t = int(t)
    r0, r1, r2, _ = philox4x32_10(
        (np.full(C, t & 0xFFFFFFFF), np.full(C, t >> 32), chain, np.zeros(C)),
        (seed & 0xFFFFFFFF, seed >> 32))
    thr = min(int(np.floor(p_pair * 2.0 ** 32)), 1 << 32)
    r0 = r0.astype(np.uint64)
    r1 = r1.astype(np.uint64)
    pair = r0 < np.uint64(thr) if thr < (1 << 32) else np.ones(C, bool)
    site_pair = (r1 * np.uint64(n)) >> np.uint64(32)
    bit_single = (r1 * np.uint64(2 * n)) >> np.uint64(32)
    a = cfg[:, 0].copy()
    b = cfg[:, 1].copy()
    one = np.uint64(1)
    fa = np.where(pair, one << site_pair, np.where(bit_single < n, one << (bit_single % np.uint64(n)), 0)).astype(np.uint64)
    fb = np.where(pair, one << site_pair, np.where(bit_single >= n, one << (bit_single % np.uint64(n)), 0)).astype(np.uint64)
    new = np.stack([a ^ fa, b ^ fb], axis=1)
    u = (r2.astype(np.float64) + 0.5) * 2.0 ** -32
    return new, u


def metropolis(theta, arch, n, state, state_lr, seed, counter, sweeps, p_pair=0.5):
    """Run C chains for `sweeps` sweeps of 2N proposals.

    state: uint64 [C, 2]; state_lr: complex [C] log rho of the states.
    Returns (samples [sweeps, C, 2], state, state_lr, counter').
    """
    state = np.asarray(state, dtype=np.uint64).copy()
    lr = np.asarray(state_lr, dtype=np.complex128).copy()
    C = state.shape[0]
    chain = np.arange(C)
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    out = np.zeros((sweeps, C, 2), dtype=np.uint64)
    t = int(counter)
    for s in range(sweeps):
        for _ in range(2 * n):
            prop, u = proposal(state, n, t, chain, seed, p_pair)
            with torch.no_grad():
                lr_p = ansatz.log_rho(th, arch, prop, n).numpy()
            with np.errstate(over="ignore", invalid="ignore"):
                ratio = np.exp(2.0 * (np.real(lr_p) - np.real(lr)))
            acc = u < ratio
            state[acc] = prop[acc]
            lr[acc] = lr_p[acc]
            t += 1
        out[s] = state
    return out, state, lr, t
