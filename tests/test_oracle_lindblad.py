"""Pins of oracle.lindblad (CPU only).

Each check is tied to something other than the oracle's own formula: the
dense Kronecker construction of Eq. VecLin, the GKSL axioms, and the closed
forms the paper prints in the Ising section.
"""
import numpy as np
import pytest

from oracle import lindblad as ol
from oracle import vmc
from tests import dense_ref as dr

MODELS = [
    ("ising", dict(kind=0, V=2.0, g=1.0), dict(V=2.0, g=1.0)),
    ("ising_rand", dict(kind=0, V=0.73, g=1.61, gamma=0.8), dict(V=0.73, g=1.61)),
    ("xyz", dict(kind=1, Jx=0.9, Jy=1.0, Jz=1.1), dict(Jx=0.9, Jy=1.0, Jz=1.1)),
    ("xyz_fields", dict(kind=1, Jx=1.4, Jy=2.0, Jz=1.0, Bx=-1.0, By=0.7, Bz=0.1),
     dict(Jx=1.4, Jy=2.0, Jz=1.0, Bx=-1.0, By=0.7, Bz=0.1)),
]


def rows_as_dense(model: ol.Model) -> np.ndarray:
    n = model.n
    cfg = vmc.all_configs(n)
    ptr, conn, coef = ol.lindblad_rows(model, cfg[:, 0], cfg[:, 1])
    D = 1 << (2 * n)
    M = np.zeros((D, D), np.complex128)
    for b in range(cfg.shape[0]):
        r = dr.doubled_index(cfg[b, 0], cfg[b, 1], n)
        for k in range(ptr[b], ptr[b + 1]):
            M[r, dr.doubled_index(conn[k, 0], conn[k, 1], n)] += coef[k]
    return M


@pytest.mark.parametrize("name,okw,dkw", MODELS, ids=[m[0] for m in MODELS])
@pytest.mark.parametrize("n", [3, 4])
def test_rows_equal_kronecker_lindbladian(name, okw, dkw, n):
    """Every row equals the dense Lhat of Eq. VecLin built with numpy.kron."""
    gamma = okw.get("gamma", 1.0)
    model = ol.Model(n=n, **okw)
    dense = dr.lindbladian(okw["kind"], n, gamma=gamma, **dkw)
    mine = rows_as_dense(model)
    assert np.max(np.abs(mine - dense)) < 1e-14
    # zero dropping: no stored entry is zero, and every nonzero of dense is stored
    assert np.array_equal(np.abs(dense) > 1e-14, mine != 0)


@pytest.mark.parametrize("name,okw,dkw", MODELS, ids=[m[0] for m in MODELS])
def test_trace_preservation(name, okw, dkw):
    """GKSL property (iii): sum_alpha Lhat[(alpha,alpha), y] = 0 for every column y."""
    n = 3
    M = rows_as_dense(ol.Model(n=n, **okw))
    diag_rows = [dr.doubled_index(a, a, n) for a in range(1 << n)]
    assert np.max(np.abs(M[diag_rows].sum(axis=0))) < 1e-13


@pytest.mark.parametrize("name,okw,dkw", MODELS, ids=[m[0] for m in MODELS])
def test_hermiticity_preservation(name, okw, dkw):
    """c[(a,b) -> (a',b')] = conj c[(b,a) -> (b',a')]: Lhat maps Hermitian rho to Hermitian."""
    n = 4
    model = ol.Model(n=n, **okw)
    cfg = vmc.all_configs(n)
    rows = ol.connected(model, cfg)
    table = {}
    for b in range(cfg.shape[0]):
        for (a2, b2), c in zip(rows[b][0], rows[b][1]):
            table[(int(cfg[b, 0]), int(cfg[b, 1]), int(a2), int(b2))] = c
    for (a, b, a2, b2), c in table.items():
        assert abs(table[(b, a, b2, a2)] - np.conj(c)) < 1e-14


@pytest.mark.parametrize("g", [1.0, 4.0, 0.37])
def test_single_qubit_closed_form(g):
    """Ising section: for H = (g/2) sx, L = s-, gamma = 1 the steady state is
    [[g^2, -ig], [ig, 1+g^2]] / (1+2g^2); it must be the null vector of the rows at N = 1."""
    M = rows_as_dense(ol.Model(kind=0, n=1, V=0.0, g=g))
    v, s = dr.null_vector(M)
    assert s[-1] < 1e-12 * s[0]
    rho = v.reshape(2, 2)
    rho = rho / np.trace(rho)
    expect = np.array([[g * g, -1j * g], [1j * g, 1 + g * g]]) / (1 + 2 * g * g)
    assert np.max(np.abs(rho - expect)) < 1e-12


def rho1(g):
    return np.array([[g * g, -1j * g], [1j * g, 1 + g * g]]) / (1 + 2 * g * g)


def product_log_rho(cfg, n, g):
    r = rho1(g)
    a = ((cfg[:, 0:1] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(int)
    b = ((cfg[:, 1:2] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(int)
    return np.log(r[a, b]).sum(axis=1)


@pytest.mark.parametrize("n", [4, 32, 40])
def test_product_state_is_steady_at_V0(n):
    """Ising section: with V = 0 the chain decouples and rho_ss = (x) rho^(1); L(x) = 0 on it."""
    g = 1.3
    model = ol.Model(kind=0, n=n, V=0.0, g=g)
    rng = np.random.default_rng(7)
    cfg = vmc.all_configs(n) if n == 4 else rng.integers(0, 1 << n, size=(200, 2), dtype=np.uint64)
    rows = ol.connected(model, cfg)
    lr_x = product_log_rho(cfg, n, g)
    lr_rows = [product_log_rho(c, n, g) if len(c) else np.zeros(0) for c, _ in rows]
    L = vmc.local_lindbladian([c for _, c in rows], lr_x, lr_rows)
    scale = np.array([np.sum(np.abs(c)) for _, c in rows])
    assert np.max(np.abs(L) / scale) < 1e-12


def test_dark_state_at_g0():
    """Ising section: at g = 0, |1..1><1..1| is steady.  No row other than the
    all-down one reaches the all-down configuration, and that row's diagonal is 0."""
    n = 4
    ones = (1 << n) - 1
    model = ol.Model(kind=0, n=n, V=2.0, g=0.0)
    cfg = vmc.all_configs(n)
    rows = ol.connected(model, cfg)
    for b in range(cfg.shape[0]):
        for (a2, b2), c in zip(rows[b][0], rows[b][1]):
            assert not (int(a2) == ones and int(b2) == ones), (cfg[b], c)


def test_exact_steady_state_null_vector():
    """Lhat rho_ss = 0: the dense null vector at N = 4 gives L(x) ~ 0 through the rows."""
    n = 4
    dense = dr.lindbladian(0, n, V=2.0, g=1.0)
    v, s = dr.null_vector(dense)
    assert s[-1] < 1e-12 * s[0]
    cfg = vmc.all_configs(n)
    idx = np.array([dr.doubled_index(a, b, n) for a, b in cfg])
    rho = v[idx]
    model = ol.Model(kind=0, n=n, V=2.0, g=1.0)
    rows = ol.connected(model, cfg)
    lookup = {(int(a), int(b)): rho[k] for k, (a, b) in enumerate(cfg)}
    worst = 0.0
    for b in range(cfg.shape[0]):
        acc = sum(c * lookup[(int(a2), int(b2))] for (a2, b2), c in zip(*rows[b]))
        worst = max(worst, abs(acc))
    assert worst < 1e-12 * np.max(np.abs(rho))


@pytest.mark.parametrize("okw", [dict(kind=0, V=2.0, g=1.0), dict(kind=1, Jx=0.9, Jy=1.0, Jz=1.1)])
def test_nonzero_count_histogram_n4(okw):
    """Per row: diagonal (absent only for all-down), 2N one-sided moves, one
    dissipator move per site where alpha_i = beta_i = 1: mean 1 + 2N + N/4 - 1/4^N."""
    n = 4
    cfg = vmc.all_configs(n)
    ptr, _, _ = ol.lindblad_rows(ol.Model(n=n, **okw), cfg[:, 0], cfg[:, 1])
    k = np.diff(ptr)
    assert k.min() == 9 and k.max() == 12
    assert abs(k.mean() - (1 + 2 * n + n / 4 - 1 / 4 ** n)) < 1e-15
