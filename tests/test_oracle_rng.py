"""Pins for the oracle's counter-based generator and bounded draws."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")


def test_philox_known_answers(ox):
    kat = json.load(open(GOLDEN))
    for v in kat["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        out = [int(h, 16) for h in v["out"]]
        assert list(ox.philox4x32_10(ctr, key)) == out


def test_philox_avalanche(ox):
    # flipping one counter bit flips about half of the 128 output bits
    rng = np.random.default_rng(1)
    flips = []
    for _ in range(200):
        ctr = rng.integers(0, 2**32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2**32, 2, dtype=np.uint64).astype(np.uint32)
        bit = int(rng.integers(0, 128))
        c2 = ctr.copy()
        c2[bit // 32] ^= np.uint32(1 << (bit % 32))
        a, b = ox.philox4x32_10(ctr, key), ox.philox4x32_10(c2, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert 60 < np.mean(flips) < 68


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 7, 8, 36, 100, 289, 2**31 + 11])
def test_uniform_is_floor_of_scaled_word(ox, n):
    for word in [0, 1, 2**31, 2**32 - 1, 123456789, 0xDEADBEEF]:
        assert ox.uniform(word, n) == (word * n) >> 32
        assert 0 <= ox.uniform(word, n) < n


def test_policy_actions_uniform_and_keyed(ox):
    counts = np.zeros(7)
    seen = {}
    for ep in range(40):
        for t in range(100):
            a = ox.policy_action(7, 3, ep, t)
            counts[a] += 1
            seen[(ep, t)] = a
    # chi-square with 6 degrees of freedom, 0.1 % critical value 22.46
    exp = counts.sum() / 7
    assert ((counts - exp) ** 2 / exp).sum() < 22.46
    # deterministic in (seed, id, episode, t); other ids give other streams
    assert all(ox.policy_action(7, 3, ep, t) == a for (ep, t), a in list(seen.items())[:50])
    other = [ox.policy_action(7, 4, 0, t) for t in range(100)]
    assert other != [seen[(0, t)] for t in range(100)]
