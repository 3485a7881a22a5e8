"""Pins of the 2D Ising rows of oracle.lindblad (CPU only).

The M x C lattice's rows are checked entry by entry against the dense Lhat
assembled with Kronecker products over the torus neighbour pairs
(tests/dense_ref.py), their diagonal against the dense Hamiltonian's at sizes
where Lhat itself is too large, and the bond counts against the paper's (four
bonds on the 2 x 2 lattice) and the coordination of the square lattice."""
from functools import reduce

import numpy as np
import pytest

from oracle import lindblad as ol
from oracle import vmc
from tests import dense_ref as dr
from tests.test_oracle_lindblad import rows_as_dense

LATTICES = [(2, 2), (2, 3), (3, 2)]


@pytest.mark.parametrize("M,C,want", [(2, 2, 4), (2, 3, 9), (3, 2, 9), (3, 3, 18), (4, 4, 32), (2, 16, 48),
                                      (4, 8, 64), (8, 8, 128), (3, 1, 3)])
def test_bond_counts(M, C, want):
    """2 x 2 has the paper's 4 bonds; with both sides >= 3 every site has 4
    neighbours (2n bonds); a side of 2 gives one bond per ring."""
    b = ol.bonds(ol.Model(kind=0, n=M * C, rows=M))
    assert len(b) == len(set(b)) == want
    assert sorted(b) == dr.torus_neighbours(M, C)


@pytest.mark.parametrize("M,C", LATTICES)
@pytest.mark.parametrize("V,g,gamma", [(2.0, 1.0, 1.0), (0.73, 1.61, 0.8)])
def test_rows_equal_kronecker_lindbladian_2d(M, C, V, g, gamma):
    n = M * C
    model = ol.Model(kind=0, n=n, V=V, g=g, gamma=gamma, rows=M)
    dense = dr.lindbladian(0, n, gamma=gamma, V=V, g=g, lattice=(M, C))
    mine = rows_as_dense(model)
    assert np.max(np.abs(mine - dense)) < 1e-14
    assert np.array_equal(np.abs(dense) > 1e-14, mine != 0)


@pytest.mark.parametrize("M,C", [(3, 3), (3, 4), (4, 3), (2, 5)])
def test_diagonal_equals_dense_hamiltonian(M, C):
    """Row (alpha, beta) has diagonal -i (E(alpha) - E(beta)) - (gamma/2)(#down...)
    with E the diagonal of H; E is taken from Kronecker products of the diagonal
    of sigma^z over the torus pairs."""
    n, V, g, gamma = M * C, 1.3, 0.7, 1.0
    zdiag = np.array([1.0, -1.0])
    E = np.zeros(1 << n)
    for i, j in dr.torus_neighbours(M, C):
        E += (V / 4) * reduce(np.kron, [zdiag if s in (i, j) else np.ones(2) for s in range(n)])
    rng = np.random.default_rng(M * 10 + C)
    cfg = rng.integers(0, 1 << n, size=(300, 2), dtype=np.uint64)
    model = ol.Model(kind=0, n=n, V=V, g=g, gamma=gamma, rows=M)
    rows = ol.connected(model, cfg)
    for (a, b), (conn, coef) in zip(cfg, rows):
        ka, kb = dr.kron_index(int(a), n), dr.kron_index(int(b), n)
        down = bin(int(a)).count("1") + bin(int(b)).count("1")
        want = -1j * (E[ka] - E[kb]) - 0.5 * gamma * (2 * n - down)
        hit = [c for (a2, b2), c in zip(conn, coef) if a2 == a and b2 == b]
        assert (hit[0] if hit else 0.0) == pytest.approx(want, abs=1e-13)
        assert len(conn) == len(hit) + 2 * n + sum(1 for i in range(n) if (int(a) >> i) & (int(b) >> i) & 1)


@pytest.mark.slow
def test_null_vector_2x3():
    """The dense steady state of the 2 x 3 lattice (V = 2, g = 1) is annihilated by the rows."""
    M, C = 2, 3
    n = M * C
    dense = dr.lindbladian(0, n, V=2.0, g=1.0, lattice=(M, C))
    v, s = dr.null_vector(dense)
    assert s[-1] < 1e-10 * s[0]
    cfg = vmc.all_configs(n)
    idx = np.array([dr.doubled_index(a, b, n) for a, b in cfg])
    rho = v[idx]
    ptr, conn, coef = ol.lindblad_rows(ol.Model(kind=0, n=n, V=2.0, g=1.0, rows=M), cfg[:, 0], cfg[:, 1])
    code = conn[:, 0].astype(np.int64) * (1 << n) + conn[:, 1].astype(np.int64)
    acc = np.add.reduceat(coef * rho[code], ptr[:-1])
    assert np.max(np.abs(acc)) < 1e-10 * np.max(np.abs(rho))


def test_xyz_lattice_rejected():
    with pytest.raises(ValueError):
        ol.operator_terms(ol.Model(kind=1, n=4, Jx=1.0, Jy=1.0, Jz=1.0, rows=2))
