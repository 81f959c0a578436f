"""Pin the oracle's Philox4x64-10 to an independent implementation: numpy's
``Philox`` bit generator (same published algorithm, Salmon et al. SC'11).

numpy increments its 256-bit counter before producing each 4-word block, so
the first block of ``Philox(counter=c)`` is the oracle's block at counter c+1.
"""
import numpy as np
import pytest


def _numpy_block(key, ctr_prev):
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array(ctr_prev, dtype=np.uint64))
    return g.random_raw(4).astype(np.uint64)


def _inc(ctr):
    c = [int(v) for v in ctr]
    for k in range(4):
        c[k] = (c[k] + 1) & ((1 << 64) - 1)
        if c[k] != 0:
            break
    return c


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((5, 7), (0, 0, 0, 0)),
    ((2024, 3), (17, 311, 4095, 1)),
    ((0xFFFFFFFFFFFFFFFF, 0x123456789ABCDEF0), (2**64 - 2, 2**63, 12345, 2)),
    ((99, 0), (999, 1999, 54871, 0)),
])
def test_philox_matches_numpy(oracle_mod, key, ctr):
    want = _numpy_block(key, ctr)
    got = oracle_mod.philox(key, _inc(ctr))
    assert np.array_equal(got, want)


def test_philox_counter_carry(oracle_mod):
    # counter word 0 wraps into word 1
    key = (11, 13)
    prev = (2**64 - 1, 5, 0, 0)
    want = _numpy_block(key, prev)
    got = oracle_mod.philox(key, (0, 6, 0, 0))
    assert np.array_equal(got, want)


def test_philox_stream(oracle_mod):
    key = (31337, 1)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array([0, 0, 0, 0], dtype=np.uint64))
    raw = g.random_raw(4 * 64).astype(np.uint64).reshape(64, 4)
    for b in range(64):
        assert np.array_equal(oracle_mod.philox(key, (b + 1, 0, 0, 0)), raw[b])
