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
