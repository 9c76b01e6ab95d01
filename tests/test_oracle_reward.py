"""Pins for the goal reward r = 1 - 0.9 * (t / T) in fp32 (Sec. 3.2.1,
Eq. (1), with t counted after the step; Table 'rewards', on_goal_reached)."""
from fractions import Fraction

import numpy as np
import pytest

import gridtools as gt

ULP_1 = 2.0 ** -23  # ulp of fp32 numbers in [1, 2); results lie in [0.1, 1)


@pytest.mark.parametrize("T", [1, 2, 3, 7, 64, 100, 144, 196, 256, 361, 640, 1024, 2560, 4096])
def test_reward_is_the_exact_rational_within_fp32_error(ox, T):
    """Three rounded fp32 operations stay within a few ulp of the exact
    value 1 - 9t/(10T); a dropped or shifted term misses it by far more."""
    for t in range(1, T + 1):
        r = ox.goal_reward(t, T)
        exact = 1 - Fraction(9, 10) * Fraction(t, T)
        assert abs(Fraction(r) - exact) <= 3 * ULP_1, (t, T, r, float(exact))
        assert 0.1 - 1e-6 <= r <= 1.0


def test_reward_special_values(ox):
    # t = T: 1 - fl(0.9); t/T = 1/2 is exact, 0.9 * 0.5 is exact
    assert ox.goal_reward(100, 100) == float(np.float32(1) - np.float32(0.9))
    assert ox.goal_reward(50, 100) == float(np.float32(1) - np.float32(0.45))
    assert ox.goal_reward(3, 3) == ox.goal_reward(640, 640)
    assert ox.goal_reward(5, 100, reward_mode=1) == 1.0


def test_reward_uses_post_step_counter(ox):
    """Reaching the goal on the first step of an episode pays 1 - 0.9/T."""
    pic = """
# # # # #
# . . . #
# . > G #
# . . . #
# # # # #
"""
    for T in (10, 100):
        b, s = gt.one_env(ox, pic, T=T)
        out = ox.step(b, s, [2])
        exact = 1 - Fraction(9, 10) * Fraction(1, T)
        assert abs(Fraction(float(out.reward[0, 0])) - exact) <= 3 * ULP_1
        assert out.reward[0, 0] == np.float32(ox.goal_reward(1, T))


# T of every workload family: Empty, lava, Dynamic-Obstacles and GoToDoor
# use 4 S^2, DoorKey 10 S^2, FourRooms 100, KeyCorridor 30 s^2 (rooms of s)
WORKLOAD_T = sorted({100, 256, 640} | {4 * S * S for S in range(4, 33)} |
                    {10 * S * S for S in range(5, 33)} | {30 * s * s for s in range(3, 12)})


def three_op(t, T):
    """numpy's IEEE single precision, one rounding per operation:
    1 - 0.9 * (t / T)."""
    q = np.float32(t) / np.float32(T)
    return np.float32(1) - np.float32(0.9) * q


def fused(t, T):
    """1 - 0.9 q with the multiply-add rounded once (what FMA contraction
    would compute); the exact value fits a double here."""
    q = np.float32(np.float32(t) / np.float32(T))
    return np.float32(1.0 - np.float64(np.float32(0.9)) * np.float64(q))


def double_09(t, T):
    """0.9 taken as a double constant: p = (float)(0.9 * (double)q)."""
    q = np.float32(np.float32(t) / np.float32(T))
    return np.float32(1) - np.float32(0.9 * np.float64(q))


def test_reward_bits_equal_numpy_three_op_for_every_workload_T(ox):
    """Bit equality with numpy's float32 evaluation, one rounding per
    operation, for every 1 <= t <= T of every workload's T (Eq. (1) read
    as 1 - 0.9 (t / T) in fp32)."""
    lib = ox.lib()
    for T in WORKLOAD_T:
        t = np.arange(1, T + 1)
        want = three_op(t.astype(np.float32), T).view(np.uint32)
        got = np.array([lib.ox_goal_reward(int(i), T, 0) for i in t], dtype=np.float32).view(np.uint32)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (T, t[bad[:5]], got[bad[:5]], want[bad[:5]])


def test_reward_pin_tells_rounding_orders_apart():
    """The pin above has power: a contracted multiply-add, or 0.9 as a
    double, each disagree with the three-op bits on many (t, T) pairs of
    the same set (both stay within the 3-ulp bound of the first test)."""
    for variant in (fused, double_09):
        differ = 0
        for T in WORKLOAD_T:
            t = np.arange(1, T + 1).astype(np.float32)
            a = three_op(t, T).view(np.uint32)
            b = np.array([variant(x, T) for x in t], dtype=np.float32).view(np.uint32)
            differ += int(np.count_nonzero(a != b))
        assert differ > 100, (variant.__name__, differ)
