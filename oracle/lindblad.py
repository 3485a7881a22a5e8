"""Oracle: rows of the vectorised Lindbladian (test infrastructure only).

What is computed
----------------
For a configuration x = (alpha, beta) of the doubled space, the nonzero
entries of row x of the vectorised GKSL generator

    Lhat = -i (H (x) 1 - 1 (x) H^T)
           + sum_j gamma_j [ L_j (x) L_j^* - 1/2 (L_j^dag L_j (x) 1) - 1/2 (1 (x) L_j^T L_j^*) ]

(Eq. VecLin of the main text; restated in App. A, where A rho B maps to
(A (x) B^T)|rho>> and |rho>> = sum rho_{ab} |a>|b>).  The row is built
directly from the local operator matrices of each Hamiltonian term and each
jump operator: a term acting on sites S contributes, for every local
configuration a' of S, an entry at the column obtained by overwriting the bits
of alpha (or beta, or both) on S.  Entries landing on the same column are
summed with an exactly rounded sum; an entry is dropped iff that sum is zero,
i.e. iff its exact value is zero.

Conventions (fixed by the paper's own closed forms)
--------------------------------------------------
* bit 0 is spin up (sigma^z = +1), bit 1 is spin down; sigma^- = |1><0|.  This
  is the reading under which the g = 0 dark state |1...1><1...1| is steady
  (Ising section: sigma^-|1> = 0) and the single-qubit steady state has
  rho_11 = (1+g^2)/(1+2g^2) (Ising section, single-qubit closed form).
* site i of a configuration is bit i of the packed integer; bonds are periodic,
  (i, i+1 mod N).
* 2D Ising (the 2D dissipative Ising paragraph of the results, and its 2 x 2
  companion in the supplement): an M x C periodic square lattice (M = rows > 1)
  with n = M C sites numbered row-major, site (r, c) = bit r C + c.  The sum
  over nearest-neighbour pairs <ij> runs over distinct unordered pairs, each
  once: a ring of length 2 has one bond, a ring of length 1 none, so the 2 x 2
  lattice has the 4 bonds the paper counts.  Only the Ising model is defined on
  the lattice.
* a two-site local matrix kron(A, B) on sites (i, j) is indexed by
  2*bit_i + bit_j.
* Hamiltonians, read literally with Pauli matrices:
  Ising  H = (V/4) sum_i sz_i sz_{i+1} + (g/2) sum_i sx_i     (Ising section)
  XYZ    H = sum_i sum_k (J_k sk_i sk_{i+1} + B_k sk_i)        (Heisenberg section)
  jumps  L_i = sigma^-_i with uniform rate gamma (both sections).

Parity: pinned.  tests/test_oracle_lindblad.py checks these rows entry by entry
against a dense generator assembled from global Kronecker products (a separate
construction), checks trace preservation (GKSL property iii), Hermiticity
preservation, the single-qubit closed form as the null vector at N = 1, the
dark state at g = 0, the exact product steady state at V = 0, and the
nonzero-count histogram at N = 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ISING = 0
XYZ = 1

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
SMINUS = np.array([[0, 0], [1, 0]], dtype=np.complex128)  # <1|s-|0> = 1


@dataclass
class Model:
    """A dissipative spin chain: kind ISING or XYZ, n sites, couplings."""

    kind: int
    n: int
    V: float = 0.0
    g: float = 0.0
    Jx: float = 0.0
    Jy: float = 0.0
    Jz: float = 0.0
    Bx: float = 0.0
    By: float = 0.0
    Bz: float = 0.0
    gamma: float = 1.0
    rows: int = 1
    extra: dict = field(default_factory=dict)


def bonds(model: Model):
    """The bond list: (i, i+1 mod n) for a chain (rows <= 1); for an M x C
    lattice the distinct nearest-neighbour pairs of the periodic square lattice."""
    n, M = model.n, max(1, int(model.rows))
    if M == 1:
        return [(i, (i + 1) % n) for i in range(n)]
    if n % M:
        raise ValueError(f"n={n} is not a multiple of rows={M}")
    C = n // M
    out = []
    for r in range(M):
        for c in range(C):
            i = r * C + c
            for j in (r * C + (c + 1) % C, ((r + 1) % M) * C + c):
                if j != i and (min(i, j), max(i, j)) not in out:
                    out.append((min(i, j), max(i, j)))
    return out


def operator_terms(model: Model):
    """Local Hamiltonian terms and jump operators of the model.

    Returns (ham, jumps): ham is a list of (sites, matrix) with matrix of size
    2^len(sites); jumps is a list of (site, matrix, rate).
    Ising section: H = (V/4) sum sz sz + (g/2) sum sx, L_i = sigma^-_i, the
    sum over the bonds of the chain or of the 2D lattice.
    Heisenberg section: H = sum_i sum_k J_k sk_i sk_{i+1} + B_k sk_i.
    """
    n = model.n
    ham = []
    if model.kind == ISING:
        bond = (model.V / 4.0) * np.kron(SZ, SZ)
        site = (model.g / 2.0) * SX
    elif model.kind == XYZ:
        bond = model.Jx * np.kron(SX, SX) + model.Jy * np.kron(SY, SY) + model.Jz * np.kron(SZ, SZ)
        site = model.Bx * SX + model.By * SY + model.Bz * SZ
    else:
        raise ValueError(f"unknown model kind {model.kind}")
    if model.rows > 1 and model.kind != ISING:
        raise ValueError("only the Ising model is defined on a 2D lattice")
    if np.any(bond != 0):
        if n < 2:
            raise ValueError("a bond term needs n >= 2")
        for b in bonds(model):
            ham.append((b, bond))
    if np.any(site != 0):
        for i in range(n):
            ham.append(((i,), site))
    jumps = [(i, SMINUS, model.gamma) for i in range(n)] if model.gamma != 0 else []
    return ham, jumps


def _local_index(cfg: np.ndarray, sites) -> np.ndarray:
    k = len(sites)
    idx = np.zeros(cfg.shape, dtype=np.int64)
    for t, s in enumerate(sites):
        idx |= ((cfg >> np.uint64(s)) & np.uint64(1)).astype(np.int64) << (k - 1 - t)
    return idx


def _overwrite(cfg: np.ndarray, sites, local: int) -> np.ndarray:
    k = len(sites)
    out = cfg.copy()
    for t, s in enumerate(sites):
        bit = np.uint64((local >> (k - 1 - t)) & 1)
        out = (out & ~np.uint64(1 << s)) | (bit << np.uint64(s))
    return out


def lindblad_rows(model: Model, alpha, beta):
    """Nonzero entries of rows (alpha_b, beta_b) of Lhat (Eq. VecLin).

    alpha, beta: integer arrays of shape [B] (bit i = site i).
    Returns (row_ptr [B+1], conn [M, 2] uint64, coef [M] complex128), the
    entries of each row sorted by (alpha', beta').
    """
    alpha = np.asarray(alpha, dtype=np.uint64).reshape(-1)
    beta = np.asarray(beta, dtype=np.uint64).reshape(-1)
    B = alpha.shape[0]
    rows_l, a_l, b_l, v_l = [], [], [], []
    rid = np.arange(B, dtype=np.int64)

    def emit(mask, a_new, b_new, val):
        rows_l.append(rid[mask])
        a_l.append(a_new[mask])
        b_l.append(b_new[mask])
        v_l.append(val[mask])

    ham, jumps = operator_terms(model)
    for sites, h in ham:
        ia = _local_index(alpha, sites)
        ib = _local_index(beta, sites)
        for loc in range(h.shape[0]):
            # -i (h (x) 1): column (alpha with sites <- loc, beta), value h[alpha_S, loc]
            v = -1j * h[ia, loc]
            emit(v != 0, _overwrite(alpha, sites, loc), beta, v)
            # +i (1 (x) h^T): column (alpha, beta with sites <- loc), value h^T[beta_S, loc]
            v = 1j * h.T[ib, loc]
            emit(v != 0, alpha, _overwrite(beta, sites, loc), v)
    for s, L, rate in jumps:
        sites = (s,)
        ia = _local_index(alpha, sites)
        ib = _local_index(beta, sites)
        LdL = L.conj().T @ L
        LtLc = L.T @ L.conj()
        for la in range(2):
            # gamma L (x) L^*: column (alpha_S <- la, beta_S <- lb)
            for lb in range(2):
                v = rate * L[ia, la] * np.conj(L[ib, lb])
                emit(v != 0, _overwrite(alpha, sites, la), _overwrite(beta, sites, lb), v)
            # -gamma/2 (L^dag L (x) 1)
            v = -0.5 * rate * LdL[ia, la]
            emit(v != 0, _overwrite(alpha, sites, la), beta, v)
            # -gamma/2 (1 (x) L^T L^*)
            v = -0.5 * rate * LtLc[ib, la]
            emit(v != 0, alpha, _overwrite(beta, sites, la), v)

    if rows_l:
        rows = np.concatenate(rows_l)
        ca = np.concatenate(a_l)
        cb = np.concatenate(b_l)
        vals = np.concatenate(v_l).astype(np.complex128)
    else:
        rows = np.zeros(0, np.int64)
        ca = cb = np.zeros(0, np.uint64)
        vals = np.zeros(0, np.complex128)
    order = np.lexsort((cb, ca, rows))
    rows, ca, cb, vals = rows[order], ca[order], cb[order], vals[order]
    # sum entries that land on the same column of the same row
    if rows.size:
        new = np.ones(rows.size, dtype=bool)
        new[1:] = (rows[1:] != rows[:-1]) | (ca[1:] != ca[:-1]) | (cb[1:] != cb[:-1])
        starts = np.flatnonzero(new)
        ends = np.append(starts[1:], rows.size)
        summed = vals[starts].copy()
        # exactly rounded sums (math.fsum) so that an entry is dropped iff its
        # exact sum vanishes, whatever the order the terms were emitted in
        for g in np.flatnonzero(ends - starts > 1):
            seg = vals[starts[g]:ends[g]]
            summed[g] = complex(math.fsum(seg.real), math.fsum(seg.imag))
        rows, ca, cb = rows[starts], ca[starts], cb[starts]
        keep = summed != 0
        rows, ca, cb, summed = rows[keep], ca[keep], cb[keep], summed[keep]
    else:
        summed = vals
    counts = np.bincount(rows, minlength=B)
    row_ptr = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    conn = np.stack([ca, cb], axis=1).astype(np.uint64)
    return row_ptr, conn, summed


def connected(model: Model, cfg):
    """Connected configurations of each row, cfg uint64 [B, 2] (alpha, beta).

    Returns a list of (conn [k, 2] uint64, coef [k] complex128), one per row,
    sorted by (alpha', beta').
    """
    cfg = np.asarray(cfg, dtype=np.uint64).reshape(-1, 2)
    ptr, conn, coef = lindblad_rows(model, cfg[:, 0], cfg[:, 1])
    return [(conn[ptr[b]:ptr[b + 1]], coef[ptr[b]:ptr[b + 1]]) for b in range(cfg.shape[0])]
