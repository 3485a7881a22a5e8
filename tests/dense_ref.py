"""Dense vectorised Lindbladian from global Kronecker products (tests only).

A second construction of Eq. VecLin, independent of oracle.lindblad: the
Hamiltonian and jump operators are embedded in the full 2^N space with
numpy.kron and combined as
    Lhat = -i (H (x) 1 - 1 (x) H^T) + sum_j g_j (L_j (x) L_j^* - 1/2 L_j^dag L_j (x) 1 - 1/2 1 (x) L_j^T L_j^*).
Kronecker factor 0 is site 0, so the kron index of a configuration is its
bit-reversed integer; helpers below convert between the two.
"""
from functools import reduce

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
LOWER = np.array([[0, 0], [1, 0]], dtype=np.complex128)


def site_op(ops: dict, n: int) -> np.ndarray:
    """Tensor product over n sites with ops[site] at the given sites, identity elsewhere."""
    return reduce(np.kron, [ops.get(i, I2) for i in range(n)])


def torus_neighbours(M, C):
    """Nearest-neighbour pairs of an M x C periodic square lattice, sites row-major,
    as a set of unordered pairs: the four lattice neighbours of each site, with the
    pairs that coincide (rings of length 2) or are self-pairs (length 1) counted once
    or not at all."""
    out = set()
    for r in range(M):
        for c in range(C):
            for dr_, dc in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                j = ((r + dr_) % M) * C + (c + dc) % C
                i = r * C + c
                if i != j:
                    out.add(frozenset((i, j)))
    return sorted(tuple(sorted(p)) for p in out)


def hamiltonian(kind, n, V=0.0, g=0.0, Jx=0.0, Jy=0.0, Jz=0.0, Bx=0.0, By=0.0, Bz=0.0, lattice=None):
    D = 1 << n
    H = np.zeros((D, D), np.complex128)
    if lattice is not None:                      # 2D Ising on an M x C torus
        assert kind == 0
        for i, j in torus_neighbours(*lattice):
            H += (V / 4) * site_op({i: PZ, j: PZ}, n)
        for i in range(n):
            H += (g / 2) * site_op({i: PX}, n)
        return H
    for i in range(n):
        j = (i + 1) % n
        if kind == 0:
            if n > 1 and V != 0:
                H += (V / 4) * site_op({i: PZ, j: PZ}, n) if i != j else 0
            H += (g / 2) * site_op({i: PX}, n)
        else:
            for J, P in ((Jx, PX), (Jy, PY), (Jz, PZ)):
                if J != 0 and n > 1:
                    H += J * site_op({i: P, j: P}, n)
            for Bk, P in ((Bx, PX), (By, PY), (Bz, PZ)):
                H += Bk * site_op({i: P}, n)
    return H


def lindbladian(kind, n, gamma=1.0, **kw) -> np.ndarray:
    H = hamiltonian(kind, n, **kw)
    D = 1 << n
    Id = np.eye(D, dtype=np.complex128)
    L = -1j * (np.kron(H, Id) - np.kron(Id, H.T))
    for i in range(n):
        Lj = site_op({i: LOWER}, n)
        L += gamma * (np.kron(Lj, Lj.conj()) - 0.5 * np.kron(Lj.conj().T @ Lj, Id)
                      - 0.5 * np.kron(Id, Lj.T @ Lj.conj()))
    return L


def kron_index(cfg_int, n):
    """Configuration integer (bit i = site i) -> kron index (site 0 most significant)."""
    out = 0
    for i in range(n):
        out |= ((int(cfg_int) >> i) & 1) << (n - 1 - i)
    return out


def doubled_index(alpha, beta, n):
    return (kron_index(alpha, n) << n) | kron_index(beta, n)


def null_vector(L):
    """Right null vector of Lhat via SVD, normalised to unit trace-like phase."""
    _, s, vh = np.linalg.svd(L)
    v = vh[-1].conj()
    return v, s
