"""Pins of oracle.philox and oracle.sampler (CPU only)."""
import numpy as np
import pytest
import torch
from scipy import stats

from oracle import ansatz as oa
from oracle import sampler as osm
from oracle import vmc
from oracle.philox import philox4x32_10
from tests.test_oracle_ansatz import stress_params

# Published known-answer vectors for Philox4x32-10 (Salmon et al., SC'11,
# distributed with the Random123 library): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = tuple(int(x) for x in philox4x32_10(ctr, key))
    assert got == out


def test_random_walk_when_log_rho_constant():
    """Zero weights make log rho constant, so every proposal is accepted: the
    chain is the pure proposal walk, and each move flips exactly one alpha bit,
    one beta bit, or the same site of both."""
    arch = oa.Arch(d=8, heads=2, layers=1, mlp=16)
    n, C = 5, 16
    th = np.zeros(oa.num_params(arch))
    st = np.zeros((C, 2), np.uint64)
    lr = oa.log_rho(th, arch, st, n).numpy()
    samples, _, _, ctr = osm.metropolis(th, arch, n, st, lr, seed=123, counter=0, sweeps=2)
    assert ctr == 2 * 2 * n
    prev = st
    cur = st.copy()
    for t in range(2 * 2 * n):
        nxt, _ = osm.proposal(cur, n, t, np.arange(C), 123, 0.5)
        da = nxt[:, 0] ^ cur[:, 0]
        db = nxt[:, 1] ^ cur[:, 1]
        pa = np.array([bin(int(v)).count("1") for v in da])
        pb = np.array([bin(int(v)).count("1") for v in db])
        assert np.all(pa + pb >= 1) and np.all(pa <= 1) and np.all(pb <= 1)
        assert np.all((pa + pb == 1) | (da == db))
        cur = nxt
        if (t + 1) % (2 * n) == 0:
            assert np.array_equal(samples[(t + 1) // (2 * n) - 1], cur)


@pytest.mark.slow
def test_chi_square_against_exact_distribution():
    """Visit frequencies of many chains match |rho|^2 / sum |rho|^2 enumerated exactly."""
    arch = oa.Arch(d=8, heads=2, layers=1, mlp=16)
    n = 3
    th = stress_params(arch, 71) * 1.5   # |rho|^2 spans ~6 decades over the 64 states
    cfg_all, p = vmc.exact_weights(th, arch, n)
    C = 512
    rng = np.random.default_rng(72)
    st = rng.integers(0, 1 << n, size=(C, 2), dtype=np.uint64)
    lr = oa.log_rho(th, arch, st, n).numpy()
    _, st, lr, ctr = osm.metropolis(th, arch, n, st, lr, seed=9, counter=0, sweeps=20)   # burn-in
    samples, _, _, _ = osm.metropolis(th, arch, n, st, lr, seed=9, counter=ctr, sweeps=40)
    code = (samples[..., 0].astype(np.int64) << n) | samples[..., 1].astype(np.int64)
    counts = np.bincount(code.reshape(-1), minlength=1 << (2 * n))
    idx = (cfg_all[:, 0].astype(np.int64) << n) | cfg_all[:, 1].astype(np.int64)
    expect = np.zeros(1 << (2 * n))
    expect[idx] = p
    expect *= counts.sum()
    keep = expect > 5
    # samples 1 sweep apart are correlated: use a generous threshold
    chi2 = np.sum((counts[keep] - expect[keep]) ** 2 / expect[keep])
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2 / 2.0, dof) > 1e-4, (chi2, dof)
