"""Oracle: mixed-state observables of the ansatz (test infrastructure only).

Supplementary section on mixed-state observables, and the evaluation of local
observables in App. C: the expectation value of an operator A is
    <A> = Tr(rho A) / Tr rho = sum_alpha P(alpha) A~(alpha),
with the diagonal distribution P(alpha) = rho(alpha, alpha) / Tr rho and the
local estimator
    A~(alpha) = sum_beta rho(alpha, beta) / rho(alpha, alpha) <beta|A|alpha>.
The operators are the single-site Pauli operators sigma^k_i, k in {x, y, z},
and their site averages (1/N) sum_i sigma^k_i, the magnetisation components of
the Heisenberg section.  Samples alpha ~ P come from a Metropolis chain over
the diagonal (App. C, sampling strategy, applied to the diagonal).

Readings:
* Basis: bit 0 of a site is spin up, the first basis vector of the 2x2 Pauli
  matrices; sigma^y = [[0, -i], [i, 0]] in that basis.  <beta|sigma^k_i|alpha>
  is taken from the explicit matrices: sigma^k[beta_i, alpha_i] times
  delta(beta_j, alpha_j) for every other site j.
* The ansatz is Hermitian, so rho(alpha, alpha) = 2 Re exp z is real, but it is
  not forced to be positive.  P is taken proportional to |rho(alpha, alpha)|,
  and the sign s(alpha) of rho(alpha, alpha) is carried as a weight:
  <A> = E[s A~] / E[s] under P ~ |rho(alpha, alpha)|.  This is the paper's
  estimator whenever every diagonal entry is positive.
* A configuration with rho(alpha, alpha) = 0 has P = 0 and is never visited by
  the chain; for it A~ is defined with rho(alpha, beta)/rho(alpha, alpha) read
  as 1 for beta = alpha and 0 otherwise.
* Purity: Tr(rho^2) / (Tr rho)^2 (Ising section).  With alpha, beta drawn
  independently from P, and rho(beta, alpha) = conj rho(alpha, beta),
      Tr rho^2 / (Tr rho)^2 = E[|rho(alpha,beta)|^2 / (|rho(alpha,alpha)| |rho(beta,beta)|)] / E[s]^2.
* Diagonal Metropolis chain: a proposal flips one uniform site of alpha (both
  halves of the doubled configuration (alpha, alpha)); it is accepted iff
  u < |rho(alpha', alpha')| / |rho(alpha, alpha)| = exp(Re log rho' - Re log rho).
  One sweep is N proposals; a sample is recorded after each sweep.  Proposal t
  of chain c uses one Philox4x32-10 block with counter (t mod 2^32, t >> 32, c,
  1) and key (seed mod 2^32, seed >> 32): site i = (r1 N) >> 32 and
  u = (r2 + 0.5) 2^-32.  Counter word 3 = 1 keeps this stream apart from the
  doubled-space chain's, which uses word 3 = 0.

Parity: pinned in tests/test_oracle_observables.py against Kronecker-product
traces Tr(rho sigma^k_i)/Tr rho of dense density matrices (the ansatz's own, a
dense steady state of the Ising Lindbladian, product states with a known Bloch
vector, the dark state), the closed-form purity of product states and of the
maximally mixed state, and chi-square and random-walk checks of the chain.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ansatz
from .philox import philox4x32_10

PAULI = {
    "x": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}
KINDS = ("x", "y", "z")


def ansatz_log_rho(theta, arch, n):
    """log rho(alpha, beta) of the ansatz as a function of uint64 [B, 2] configurations."""
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64))

    def f(cfg):
        with torch.no_grad():
            return ansatz.log_rho(th, arch, np.asarray(cfg, np.uint64).reshape(-1, 2), n).numpy()

    return f


def _ratio(lr_ab, lr_aa, same):
    """rho(alpha, beta) / rho(alpha, alpha) from the logs; zero-diagonal reading above."""
    zero = ~np.isfinite(lr_aa.real) & (lr_aa.real < 0)
    with np.errstate(over="ignore", invalid="ignore"):
        r = np.exp(lr_ab - np.where(zero, 0.0, lr_aa))
    r = np.where(np.isfinite(lr_ab.real), r, 0.0)
    return np.where(zero, np.where(same, 1.0, 0.0), r)


def local_estimators(log_rho, alpha, n):
    """A~(alpha) for A = sigma^k_i: complex [S, n, 3] (k = x, y, z).

    alpha: uint64 [S].  Only beta that differ from alpha at site i or nowhere
    have <beta|sigma^k_i|alpha> != 0; both are summed for every k, with the
    element read from the Pauli matrix.
    """
    alpha = np.asarray(alpha, dtype=np.uint64).reshape(-1)
    S = alpha.shape[0]
    lr_aa = log_rho(np.stack([alpha, alpha], axis=1))
    out = np.zeros((S, n, 3), np.complex128)
    one = np.uint64(1)
    for i in range(n):
        a_i = ((alpha >> np.uint64(i)) & one).astype(np.int64)
        for b_i in (0, 1):
            beta = (alpha & ~(one << np.uint64(i))) | (np.uint64(b_i) << np.uint64(i))
            same = beta == alpha
            lr_ab = np.where(same, lr_aa, log_rho(np.stack([alpha, beta], axis=1)))
            r = _ratio(lr_ab, lr_aa, same)
            for k, name in enumerate(KINDS):
                out[:, i, k] += PAULI[name][b_i, a_i] * r
    return out


def diagonal_sign(lr_aa):
    """s(alpha) = sign of the real diagonal rho(alpha, alpha) (0 where it vanishes)."""
    lr_aa = np.asarray(lr_aa, np.complex128)
    with np.errstate(under="ignore", invalid="ignore"):
        v = np.exp(lr_aa - lr_aa.real)          # unit phase: +1 or -1 up to rounding
    s = np.sign(np.real(v))
    return np.where(np.isfinite(lr_aa.real), s, 0.0)


def sampled_expectation(lr_aa, est):
    """Estimate of <sigma^k> (site average) from samples alpha ~ |rho(alpha, alpha)|:
    sum s A~ / sum s, complex [3]; and the mean sign."""
    s = diagonal_sign(lr_aa)
    avg = est.mean(axis=1)                      # (1/N) sum_i
    return (s[:, None] * avg).sum(axis=0) / s.sum(), s.mean()


def enumerated_expectation(log_rho, n):
    """sum_alpha rho(alpha, alpha) A~(alpha) / sum_alpha rho(alpha, alpha) over all 2^n alpha:
    complex [n, 3] for sigma^k_i."""
    alpha = np.arange(1 << n, dtype=np.uint64)
    lr_aa = log_rho(np.stack([alpha, alpha], axis=1))
    m = np.max(lr_aa.real[np.isfinite(lr_aa.real)])
    with np.errstate(under="ignore"):
        d = np.real(np.exp(lr_aa - m))          # rho(alpha, alpha), scaled
    d = np.where(np.isfinite(lr_aa.real), d, 0.0)
    est = local_estimators(log_rho, alpha, n)
    return np.einsum("a,aik->ik", d, est) / d.sum()


def purity_terms(lr_ab, lr_aa, lr_bb):
    """|rho(alpha,beta)|^2 / (|rho(alpha,alpha)| |rho(beta,beta)|) for independent pairs."""
    with np.errstate(over="ignore", invalid="ignore"):
        return np.exp(2.0 * np.real(lr_ab) - np.real(lr_aa) - np.real(lr_bb))


def sampled_purity(lr_ab, lr_aa, lr_bb):
    """E[purity term] / E[s]^2 over pairs of independent diagonal samples."""
    s = np.concatenate([diagonal_sign(lr_aa), diagonal_sign(lr_bb)])
    return purity_terms(lr_ab, lr_aa, lr_bb).mean() / s.mean() ** 2


def enumerated_purity(log_rho, n):
    """Tr(rho^2) / (Tr rho)^2 = sum |rho(alpha,beta)|^2 / (sum rho(alpha,alpha))^2 over all 4^n."""
    k = np.arange(1 << n, dtype=np.uint64)
    cfg = np.stack([np.repeat(k, 1 << n), np.tile(k, 1 << n)], axis=1)
    lr = log_rho(cfg)
    m = np.max(lr.real[np.isfinite(lr.real)])
    with np.errstate(under="ignore"):
        rho = np.exp(lr - m).reshape(1 << n, 1 << n)
    rho = np.where(np.isfinite(rho), rho, 0.0)
    return float(np.sum(np.abs(rho) ** 2) / np.real(np.trace(rho)) ** 2)


def diag_proposal(alpha, n, t, chain, seed):
    """Proposed alpha' (one site flipped) and acceptance uniforms for proposal index t.

    alpha: uint64 [C]; chain: int array [C].
    """
    C = alpha.shape[0]
    t = int(t)
    _, r1, r2, _ = philox4x32_10(
        (np.full(C, t & 0xFFFFFFFF), np.full(C, t >> 32), chain, np.ones(C)),
        (seed & 0xFFFFFFFF, seed >> 32))
    site = (r1.astype(np.uint64) * np.uint64(n)) >> np.uint64(32)
    u = (r2.astype(np.float64) + 0.5) * 2.0 ** -32
    return np.asarray(alpha, np.uint64) ^ (np.uint64(1) << site), u


def diag_metropolis(log_rho, n, state, state_lr, seed, counter, sweeps):
    """Run C chains on P(alpha) ~ |rho(alpha, alpha)| for `sweeps` sweeps of n proposals.

    state: uint64 [C]; state_lr: complex [C], log rho(alpha, alpha) of the states.
    Returns (samples [sweeps, C], state, state_lr, counter').
    """
    state = np.asarray(state, dtype=np.uint64).reshape(-1).copy()
    lr = np.asarray(state_lr, dtype=np.complex128).reshape(-1).copy()
    C = state.shape[0]
    chain = np.arange(C)
    out = np.zeros((sweeps, C), dtype=np.uint64)
    t = int(counter)
    for s in range(sweeps):
        for _ in range(n):
            prop, u = diag_proposal(state, n, t, chain, seed)
            lr_p = log_rho(np.stack([prop, prop], axis=1))
            with np.errstate(over="ignore", invalid="ignore"):
                ratio = np.exp(np.real(lr_p) - np.real(lr))
            acc = u < ratio
            state[acc] = prop[acc]
            lr[acc] = lr_p[acc]
            t += 1
        out[s] = state
    return out, state, lr, t
