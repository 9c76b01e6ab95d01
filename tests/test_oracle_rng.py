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
    calls = range(4000)
    acts = [ox.policy_action(7, 3, c) for c in calls]
    counts = np.bincount(acts, minlength=7)
    # chi-square with 6 degrees of freedom, 0.1 % critical value 22.46
    exp = counts.sum() / 7
    assert ((counts - exp) ** 2 / exp).sum() < 22.46
    # the action is lane (call % 4) of the block (call / 4) of the stream
    for c in (0, 1, 5, 4003, 2**32 + 6):
        blk = ox.philox4x32_10([3, (c // 4) & 0xFFFFFFFF, (c // 4) >> 32, 1], [7, 0])
        assert ox.policy_action(7, 3, c) == (int(blk[c % 4]) * 7) >> 32
    # other ids and seeds give other streams
    assert [ox.policy_action(7, 4, c) for c in range(100)] != acts[:100]
    assert [ox.policy_action(8, 3, c) for c in range(100)] != acts[:100]


def test_policy_rollout_uses_call_index(ox):
    from paper_2407_19396_amd import workloads as wl
    t = wl.uniform_table(3, 0, 8, seed=21)
    b = ox.Batch(t.family, t.side, t.max_steps, t.seed, t.rng_id)
    s = ox.State.empty(b)
    ox.reset(b, s)
    assert (s.calls == 0).all()
    s.calls[:] = 5                    # a state can carry any call count
    out = ox.rollout(b, s, 9)
    assert (s.calls == 14).all()
    for k in range(9):
        for i in range(3):
            if out.flags[k, i] & 4:
                assert out.action[k, i] == 0xFF
            else:
                assert out.action[k, i] == ox.policy_action(21, i, 5 + k)
