"""Pins of the counter-based generator and its transforms.

The width-generic Philox of philox_ref.py is checked against numpy's
independent Philox-4x64-10; its 4x32 instance and the published known
answers then pin the oracle's own C Philox4x32-10."""
import os

import numpy as np
import pytest

from philox_ref import counter_for, philox4, u01
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123, 456), (7, 8, 9, 10)),
                                     ((2**64 - 1, 5), (2**63, 1, 2, 3))])
def test_reference_philox4x64_matches_numpy(key, ctr):
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = [int(x) for x in g.random_raw(8)]
    # numpy increments the counter before producing a block
    exp = []
    c = list(ctr)
    for _ in range(2):
        c[0] = (c[0] + 1) % 2**64
        exp += philox4(c, key, width=64)
    assert raw == exp


def _kats():
    out = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        a, b, c = line.split("|")
        out.append(([int(t, 16) for t in a.split()], [int(t, 16) for t in b.split()],
                    [int(t, 16) for t in c.split()]))
    return out


def test_known_answers_reference_and_oracle():
    for ctr, key, exp in _kats():
        assert philox4(ctr, key, width=32) == exp
        assert oracle.philox(ctr, key).tolist() == exp


def test_oracle_philox_random_counters():
    rng = np.random.default_rng(1)
    for _ in range(500):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64).tolist()
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64).tolist()
        assert oracle.philox(ctr, key).tolist() == philox4(ctr, key, width=32)


def test_u01_range_and_exactness():
    assert u01(0, 0) == 0.5 * 2.0**-52
    assert u01(0xFFFFFFFF, 0xFFFFFFFF) == (2.0**52 - 0.5) * 2.0**-52
    assert 0.0 < u01(0, 0) < u01(0xFFFFFFFF, 0xFFFFFFFF) < 1.0
    # mean and variance of many draws
    ws = [philox4(counter_for(i, 3, 5, 0), [0, 0]) for i in range(20000)]
    u = np.array([u01(w[0], w[1]) for w in ws] + [u01(w[2], w[3]) for w in ws])
    n = len(u)
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 4 * np.sqrt(1 / 180 / n)


def test_counter_layout():
    c = counter_for(0x12345678, 9, 5, (3 << 24) | 0xABCDEF)
    assert c == [0x12345678, 9, (5 << 24) | 0xABCDEF, 3]
