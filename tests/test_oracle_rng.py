"""Pins of the oracle's random numbers: Philox4x32-10 (Salmon et al., SC'11)
and the Box-Muller transform that the paper's exchange step names.  The
published known-answer vectors are not available here; Philox is pinned by
the properties a keyed bijection with full diffusion must have, and by the
rocRAND library's own Philox4x32-10 stream on the GPU (tests/test_gpu_rng.py)."""
import numpy as np
import pytest
from scipy import stats


def _outputs(O, n, key=(7, 11), base=(0, 0, 0, 0)):
    out = np.empty((n, 4), np.uint32)
    for i in range(n):
        out[i] = O.philox((base[0] + i, base[1], base[2], base[3]), key)
    return out


def test_u01_range_and_resolution(oracle_lib):
    O = oracle_lib
    assert O.u01(0, 0) == 0.0
    assert O.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert O.u01(0, 0x80000000) == 0.5
    assert O.u01(0x800, 0) == 2.0 ** -53
    assert O.u01(0x7FF, 0) == 0.0  # the low 11 bits are dropped


def test_philox_bit_balance_and_uniqueness(oracle_lib):
    w = _outputs(oracle_lib, 1 << 14)
    bits = ((w[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(len(w), -1)
    frac = bits.mean(axis=0)
    sigma = 0.5 / np.sqrt(len(w))
    assert np.abs(frac - 0.5).max() < 5 * sigma
    assert len({tuple(r) for r in w}) == len(w)
    # consecutive counters are uncorrelated
    u = w[:, 0].astype(np.float64) / 2 ** 32
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / np.sqrt(len(u))
    # uniform in distribution
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_philox_avalanche(oracle_lib):
    """Flipping any single counter or key bit flips about half the 128 output
    bits (full diffusion after ten rounds)."""
    O = oracle_lib
    rng = np.random.default_rng(1)
    flips = []
    for _ in range(24):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        ref = O.philox(ctr, key)
        for word in range(6):
            for b in range(0, 32, 3):
                c2, k2 = ctr.copy(), key.copy()
                if word < 4:
                    c2[word] ^= np.uint32(1 << b)
                else:
                    k2[word - 4] ^= np.uint32(1 << b)
                out = O.philox(c2, k2)
                flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(out, ref)))
    flips = np.array(flips)
    assert abs(flips.mean() - 64) < 1.0
    assert flips.min() > 30


def test_philox_key_matters(oracle_lib):
    a = _outputs(oracle_lib, 64, key=(1, 0))
    b = _outputs(oracle_lib, 64, key=(1, 1))
    assert not np.any(np.all(a == b, axis=1))


def test_box_muller_normal(oracle_lib):
    rng = np.random.default_rng(2)
    u = rng.random((20000, 2))
    z = np.array([oracle_lib.box_muller(a, b) for a, b in u])
    for k in range(2):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-3
        assert abs(z[:, k].mean()) < 5 / np.sqrt(len(z))
        assert abs(z[:, k].var() - 1) < 5 * np.sqrt(2 / len(z))
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5 / np.sqrt(len(z))
    # the transform is exact at the landmarks: u0 = 0 gives radius 0 and
    # (u0, u1) = (1 - e^{-1/2}, 0) gives (1, 0)
    assert oracle_lib.box_muller(0.0, 0.3) == (0.0, 0.0)
    z0, z1 = oracle_lib.box_muller(1 - np.exp(-0.5), 0.0)
    assert abs(z0 - 1) < 1e-15 and z1 == 0.0
    z0, z1 = oracle_lib.box_muller(1 - np.exp(-0.5), 0.25)
    assert abs(z0) < 1e-15 and abs(z1 - 1) < 1e-15
