"""Pins of the oracle's start-block generator (oracle/rng.py): the published
known-answer vectors of Philox-4x32-10, the closed-form extremes of the
53-bit uniform map, and the distribution of the Box-Muller block."""
import numpy as np
import pytest
from scipy import stats

from oracle import rng

# Known-answer vectors published with the Random123 library for
# Philox-4x32-10: (counter, key) -> output words.
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT, ids=["zeros", "ones", "pi"])
def test_philox_known_answers(ctr, key, out):
    assert [int(w) for w in rng.philox4x32_10(ctr, key)] == list(out)


def test_philox_vectorised_equals_scalar():
    """A batch of counters gives what each counter gives alone."""
    r = np.random.default_rng(1)
    ctr = r.integers(0, 2 ** 32, size=(17, 4), dtype=np.uint64)
    batch = rng.philox4x32_10(ctr, (0x12345678, 0x9abcdef0))
    for c, b in zip(ctr, batch):
        assert np.array_equal(rng.philox4x32_10(c, (0x12345678, 0x9abcdef0)), b)


def test_uniform_map_extremes():
    """All-zero words map to 2^-54, all-one words to 1 - 2^-54: strictly
    inside (0, 1), so ln u1 is finite; consecutive codes are 2^-53 apart."""
    assert rng.uniform53(0, 0) == 2.0 ** -54
    assert rng.uniform53(0xffffffff, 0xffffffff) == 1.0 - 2.0 ** -54
    assert rng.uniform53(0, 1 << 6) - rng.uniform53(0, 0) == 2.0 ** -53
    assert rng.uniform53(1 << 5, 0) - rng.uniform53(0, 0) == 2.0 ** -27


def test_start_block_is_standard_normal():
    X = rng.start_block(20000, 5, 203, False)
    assert X.shape == (20000, 5) and X.dtype == np.float64
    for j in range(5):
        assert stats.kstest(X[:, j], "norm").pvalue > 1e-3
    assert abs(X.mean()) < 5 / np.sqrt(X.size)
    assert abs(X.var() - 1.0) < 5 * np.sqrt(2.0 / X.size)
    C = np.corrcoef(X.T)
    assert np.abs(C - np.eye(5)).max() < 5 / np.sqrt(20000)


def test_complex_start_block_parts():
    """Complex entries: real and imaginary parts N(0, 1/2), uncorrelated;
    |z|^2 is exponential with mean 1."""
    Z = rng.start_block(20000, 3, 7, True)
    assert Z.dtype == np.complex128
    for part in (Z.real, Z.imag):
        assert stats.kstest(part.ravel(), "norm", args=(0.0, np.sqrt(0.5))).pvalue > 1e-3
    assert abs(np.corrcoef(Z.real.ravel(), Z.imag.ravel())[0, 1]) < 5 / np.sqrt(Z.size)
    assert stats.kstest((np.abs(Z) ** 2).ravel(), "expon").pvalue > 1e-3


def test_start_block_seeds_and_columns():
    """The seed's high word enters the key; columns and seeds give
    different streams; rows of a shorter block are a prefix of a longer one."""
    a = rng.start_block(64, 4, 5, False)
    b = rng.start_block(64, 4, 5 + (1 << 32), False)
    c = rng.start_block(100, 4, 5, False)
    assert not np.array_equal(a, b)
    assert np.array_equal(a, c[:64])
    assert len({tuple(a[:, j]) for j in range(4)}) == 4
