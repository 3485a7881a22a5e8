"""Pins of oracle.observables (CPU only).

The estimator sum_alpha rho(alpha,alpha) A~(alpha) / sum rho(alpha,alpha) is
checked against Tr(rho A) / Tr rho computed a second way, as a dense trace with
Kronecker-product Pauli operators (tests/dense_ref.py), for the ansatz's own
density matrix and for the exact Ising steady state; against the Bloch vector
of product states (Tr(rho_1 sigma^k) = r_k, the 2x2 matrix written out from
(1 + r.sigma)/2); and against the dark state.  The purity is checked against
its closed forms, and the diagonal chain against exact enumeration."""
import numpy as np
import pytest
from scipy import stats

from oracle import ansatz as oa
from oracle import observables as ob
from tests import dense_ref as dr
from tests.test_oracle_ansatz import stress_params

ARCH = oa.Arch(d=8, heads=2, layers=1, mlp=16)


def bloch_rho1(r):
    """(1 + r.sigma)/2 written out entry by entry (bit 0 = spin up = row 0)."""
    rx, ry, rz = r
    return 0.5 * np.array([[1 + rz, rx - 1j * ry], [rx + 1j * ry, 1 - rz]], dtype=np.complex128)


def product_log_rho(rhos):
    """log rho(alpha, beta) = sum_i log rho_i(alpha_i, beta_i) for a product state."""
    n = len(rhos)

    def f(cfg):
        cfg = np.asarray(cfg, np.uint64).reshape(-1, 2)
        out = np.zeros(cfg.shape[0], np.complex128)
        for i, r1 in enumerate(rhos):
            a = ((cfg[:, 0] >> np.uint64(i)) & np.uint64(1)).astype(np.int64)
            b = ((cfg[:, 1] >> np.uint64(i)) & np.uint64(1)).astype(np.int64)
            with np.errstate(divide="ignore"):
                out += np.log(r1[a, b].astype(np.complex128))
        return out

    assert n >= 1
    return f


def matrix_log_rho(rho, n):
    """log rho(alpha, beta) read from a dense matrix in Kronecker index order."""
    kidx = np.array([dr.kron_index(k, n) for k in range(1 << n)])

    def f(cfg):
        cfg = np.asarray(cfg, np.uint64).reshape(-1, 2)
        v = rho[kidx[cfg[:, 0].astype(np.int64)], kidx[cfg[:, 1].astype(np.int64)]]
        with np.errstate(divide="ignore"):
            return np.log(v.astype(np.complex128))

    return f


def dense_rho(log_rho, n):
    """The dense matrix rho[kron(alpha), kron(beta)] = exp log rho(alpha, beta)."""
    k = np.arange(1 << n, dtype=np.uint64)
    cfg = np.stack([np.repeat(k, 1 << n), np.tile(k, 1 << n)], axis=1)
    lr = log_rho(cfg)
    rho = np.zeros((1 << n, 1 << n), np.complex128)
    for (a, b), v in zip(cfg, lr):
        rho[dr.kron_index(int(a), n), dr.kron_index(int(b), n)] = np.exp(v)
    return rho


def kron_expectations(rho, n):
    """Tr(rho sigma^k_i) / Tr rho from Kronecker-product operators: [n, 3]."""
    out = np.zeros((n, 3), np.complex128)
    for i in range(n):
        for k, P in enumerate((dr.PX, dr.PY, dr.PZ)):
            out[i, k] = np.trace(rho @ dr.site_op({i: P}, n)) / np.trace(rho)
    return out


RS = [(0.3, -0.5, 0.4), (-0.6, 0.2, -0.1), (0.0, 0.7, 0.5)]


def test_product_state_bloch_vector():
    """<sigma^k_i> of (x)_i (1 + r_i.sigma)/2 is r_i,k, site by site."""
    f = product_log_rho([bloch_rho1(r) for r in RS])
    got = ob.enumerated_expectation(f, len(RS))
    assert np.allclose(got, np.array(RS), atol=1e-12), got


def test_product_state_purity_closed_form():
    """Tr rho^2 of a product of qubits is prod (1 + |r_i|^2) / 2."""
    f = product_log_rho([bloch_rho1(r) for r in RS])
    want = np.prod([(1 + np.dot(r, r)) / 2 for r in RS])
    assert abs(ob.enumerated_purity(f, len(RS)) - want) < 1e-12


def test_dark_state():
    """|1...1><1...1| (every site down): sigma^z = -1, sigma^x = sigma^y = 0, purity 1;
    the zero-diagonal reading gives A~ = s_i for sigma^z elsewhere."""
    n = 4
    full = (1 << n) - 1

    def f(cfg):
        cfg = np.asarray(cfg, np.uint64).reshape(-1, 2)
        hit = (cfg[:, 0] == full) & (cfg[:, 1] == full)
        return np.where(hit, 0.0, -np.inf).astype(np.complex128)

    got = ob.enumerated_expectation(f, n)
    assert np.allclose(got, np.array([[0, 0, -1]] * n), atol=0)
    assert ob.enumerated_purity(f, n) == 1.0
    est = ob.local_estimators(f, np.array([0b0101], np.uint64), n)[0]
    assert np.array_equal(est[:, 2], np.array([-1, 1, -1, 1]))
    assert np.all(est[:, :2] == 0)


def test_maximally_mixed_state():
    """I / 2^n: every <sigma^k_i> = 0, purity 2^-n."""
    n = 3

    def f(cfg):
        cfg = np.asarray(cfg, np.uint64).reshape(-1, 2)
        return np.where(cfg[:, 0] == cfg[:, 1], 0.0, -np.inf).astype(np.complex128)

    assert np.allclose(ob.enumerated_expectation(f, n), 0, atol=0)
    assert abs(ob.enumerated_purity(f, n) - 2.0 ** -n) < 1e-15


@pytest.mark.parametrize("seed", [3, 11])
def test_ansatz_matches_kronecker_trace(seed):
    """The ansatz's density matrix at n = 3: the estimator sum equals the dense trace."""
    n = 3
    f = ob.ansatz_log_rho(stress_params(ARCH, seed), ARCH, n)
    rho = dense_rho(f, n)
    assert np.allclose(rho, rho.conj().T, atol=1e-12)          # Hermitian ansatz
    want = kron_expectations(rho, n)
    got = ob.enumerated_expectation(f, n)
    assert np.allclose(got, want, rtol=0, atol=1e-11), (got, want)
    assert np.allclose(want.imag, 0, atol=1e-12)               # Hermitian rho, Hermitian sigma
    pur = np.real(np.trace(rho @ rho) / np.trace(rho) ** 2)
    assert abs(ob.enumerated_purity(f, n) - pur) < 1e-12


def test_ising_steady_state_observables_and_purity():
    """Exact steady state of the dissipative Ising chain (n = 4, V = 2, g = 1), from
    the null vector of the dense Lindbladian: estimator sums equal Kronecker traces,
    translation invariance makes every site alike, and the decay leaves sigma^z < 0."""
    n = 4
    L = dr.lindbladian(0, n, gamma=1.0, V=2.0, g=1.0)
    v, s = dr.null_vector(L)
    assert s[-1] < 1e-10 * s[0]
    rho = v.reshape(1 << n, 1 << n)
    rho = rho / np.trace(rho)
    f = matrix_log_rho(rho, n)
    want = kron_expectations(rho, n)
    got = ob.enumerated_expectation(f, n)
    assert np.allclose(got, want, atol=1e-10)
    assert np.allclose(got, got[0:1], atol=1e-10)
    assert np.allclose(got.imag, 0, atol=1e-10) and got[0, 2].real < 0
    pur = np.real(np.trace(rho @ rho))
    assert abs(ob.enumerated_purity(f, n) - pur) < 1e-10


def test_single_qubit_steady_state_closed_form():
    """n = 1 (no coupling), drive g, decay gamma = 1, H = (g/2) sigma^x, L = sigma^-
    (to spin down).  The Bloch equations dx/dt = -x/2, dy/dt = -g z - y/2,
    dz/dt = g y - (z + 1) have the fixed point (0, 2g/(1 + 2g^2), -1/(1 + 2g^2))."""
    g = 0.8
    L = dr.lindbladian(0, 1, gamma=1.0, V=0.0, g=g)
    v, _ = dr.null_vector(L)
    rho1 = v.reshape(2, 2) / np.trace(v.reshape(2, 2))
    got = ob.enumerated_expectation(matrix_log_rho(rho1, 1), 1)[0]
    want = np.array([0.0, 2 * g / (1 + 2 * g * g), -1 / (1 + 2 * g * g)])
    assert np.allclose(got, want, atol=1e-12), got


def test_sampled_estimators_converge():
    """i.i.d. samples from |rho(alpha,alpha)| (a negative diagonal included) give
    E[s A~]/E[s] -> the enumerated value and the pair estimator -> the purity."""
    n = 3
    th = stress_params(ARCH, 5)
    f = ob.ansatz_log_rho(th, ARCH, n)
    alpha = np.arange(1 << n, dtype=np.uint64)
    lr = f(np.stack([alpha, alpha], axis=1))
    p = np.exp(lr.real - lr.real.max())
    p /= p.sum()
    rng = np.random.default_rng(0)
    S = 200000
    a = rng.choice(1 << n, size=S, p=p).astype(np.uint64)
    b = rng.choice(1 << n, size=S, p=p).astype(np.uint64)
    est = ob.local_estimators(f, alpha, n)[a.astype(np.int64)]
    mean, _ = ob.sampled_expectation(lr[a.astype(np.int64)], est)
    want = ob.enumerated_expectation(f, n).mean(axis=0)
    assert np.allclose(mean, want, atol=2e-2), (mean, want)
    pur = ob.sampled_purity(f(np.stack([a, b], axis=1)), lr[a.astype(np.int64)], lr[b.astype(np.int64)])
    assert abs(pur - ob.enumerated_purity(f, n)) < 2e-2 * ob.enumerated_purity(f, n)


def test_diag_random_walk_when_log_rho_constant():
    """Zero weights: log rho(alpha, alpha) = log 2 everywhere, every proposal is
    accepted, and each one flips exactly the site the proposal stream names."""
    n, C = 5, 16
    th = np.zeros(oa.num_params(ARCH))
    f = ob.ansatz_log_rho(th, ARCH, n)
    st = np.arange(C, dtype=np.uint64)
    lr = f(np.stack([st, st], axis=1))
    samples, _, _, ctr = ob.diag_metropolis(f, n, st, lr, seed=77, counter=5, sweeps=3)
    assert ctr == 5 + 3 * n
    cur = st.copy()
    for t in range(5, 5 + 3 * n):
        nxt, u = ob.diag_proposal(cur, n, t, np.arange(C), 77)
        d = nxt ^ cur
        assert all(bin(int(x)).count("1") == 1 for x in d)
        assert np.all((u > 0) & (u < 1))
        cur = nxt
        if (t - 5 + 1) % n == 0:
            assert np.array_equal(samples[(t - 5 + 1) // n - 1], cur)


@pytest.mark.slow
def test_diag_chain_chi_square():
    """Visit frequencies of many diagonal chains match |rho(alpha,alpha)| / sum, enumerated."""
    n = 4
    th = stress_params(ARCH, 13) * 1.5
    f = ob.ansatz_log_rho(th, ARCH, n)
    alpha = np.arange(1 << n, dtype=np.uint64)
    lr = f(np.stack([alpha, alpha], axis=1))
    p = np.exp(lr.real - lr.real.max())
    p /= p.sum()
    C = 1024
    st = np.random.default_rng(1).integers(0, 1 << n, size=C, dtype=np.uint64)
    slr = f(np.stack([st, st], axis=1))
    _, st, slr, ctr = ob.diag_metropolis(f, n, st, slr, seed=4, counter=0, sweeps=10)
    samples, _, _, _ = ob.diag_metropolis(f, n, st, slr, seed=4, counter=ctr, sweeps=30)
    counts = np.bincount(samples.reshape(-1).astype(np.int64), minlength=1 << n)
    expect = p * counts.sum()
    keep = expect > 5
    chi2 = np.sum((counts[keep] - expect[keep]) ** 2 / expect[keep])
    assert stats.chi2.sf(chi2 / 2.0, keep.sum() - 1) > 1e-4, (chi2, counts, expect)


def test_sign_weighted_estimators_with_negative_diagonal():
    """A Hermitian, non-positive rho (one negative diagonal entry): i.i.d. samples
    from |rho(alpha,alpha)| with the sign as weight recover the dense traces
    Tr(rho sigma^k)/Tr rho and Tr(rho^2)/(Tr rho)^2."""
    n = 2
    rng = np.random.default_rng(8)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    rho = 0.3 * (A + A.conj().T)
    np.fill_diagonal(rho, [1.0, -0.4, 0.8, 0.6])
    f = matrix_log_rho(rho, n)
    alpha = np.arange(1 << n, dtype=np.uint64)
    lr = f(np.stack([alpha, alpha], axis=1))
    assert np.sum(ob.diagonal_sign(lr) < 0) == 1
    p = np.exp(lr.real)
    p /= p.sum()
    S = 400000
    a = rng.choice(1 << n, size=S, p=p)
    b = rng.choice(1 << n, size=S, p=p)
    est = ob.local_estimators(f, alpha, n)[a]
    mean, msign = ob.sampled_expectation(lr[a], est)
    want = kron_expectations(rho, n).mean(axis=0)
    assert np.allclose(mean, want, atol=1.5e-2), (mean, want)
    assert abs(msign - np.real(np.trace(rho)) / np.sum(np.abs(np.diag(rho)))) < 1e-2
    pur = ob.sampled_purity(f(np.stack([alpha[a], alpha[b]], axis=1)), lr[a], lr[b])
    want_p = np.real(np.trace(rho @ rho)) / np.real(np.trace(rho)) ** 2
    assert abs(pur - want_p) < 3e-2 * want_p, (pur, want_p)
