"""Pins for the oracle's Dynamic-Obstacles family (Table 'envs', reward R3;
Fig. 1): layouts, the obstacle transition (each ball in list order to a
uniformly drawn free cell of the 8 around it, never the agent's), the
three-action space, and the -1 ending for walking into a ball or a wall
(checked before the balls move)."""
import itertools

import numpy as np
import pytest

import gridtools as gt
from test_oracle_layouts import check_border, chi2_ok

DYNOBS = 6
FORWARD = 2


def dyn_env(ox, picture, obst=None, t=0, T=100, seed=0, calls=0, n=None, reward_mode=0):
    g, *_ = gt.parse(picture)
    n = int((g[:, :, 0] == gt.BALL).sum()) if n is None else n
    return gt.one_env(ox, picture, t=t, T=T, family=DYNOBS, seed=seed, param=n, obst=obst,
                      calls=calls, reward_mode=reward_mode)


def balls(grid):
    return {(int(x), int(y)) for y, x in np.argwhere(grid[:, :, 0] == gt.BALL)}


def obst_list(s, i=0):
    ob = s.obst[16 * i:16 * i + 16]
    return [(int(ob[2 * b]), int(ob[2 * b + 1])) for b in range(8) if ob[2 * b] != 0xFF]


def test_side_limits(ox):
    assert ox.side_ok(DYNOBS, 5, 2) and ox.side_ok(DYNOBS, 16, 8)
    assert not ox.side_ok(DYNOBS, 5, 0) and not ox.side_ok(DYNOBS, 16, 9)
    assert not ox.side_ok(DYNOBS, 4, 1)
    assert ox.side_ok(DYNOBS, 5, 7) and not ox.side_ok(DYNOBS, 5, 8)   # 9 interior cells


@pytest.mark.parametrize("side,n", [(5, 2), (6, 3), (8, 4), (16, 8), (5, 7)])
def test_layouts(ox, side, n):
    first = {}
    for i in range(6000 if side <= 8 else 1500):
        g, x, y, d, ob = ox.layout(DYNOBS, side, 7, i, 0, n, with_obst=True)
        check_border(g)
        assert (x, y, d) == (1, 1, 0)
        assert tuple(g[side - 2, side - 2]) == (8, 1, 0)
        bs = balls(g)
        assert len(bs) == n and (1, 1) not in bs
        assert (g[g[:, :, 0] == gt.BALL] == (6, 2, 0)).all()
        lst = [(int(ob[2 * b]), int(ob[2 * b + 1])) for b in range(n)]
        assert set(lst) == bs and (ob[2 * n:] == 0xFF).all()
        inner = g[1:-1, 1:-1, 0]
        assert ((inner == gt.EMPTY) | (inner == gt.BALL)).sum() == (side - 2) ** 2 - 1
        first[lst[0]] = first.get(lst[0], 0) + 1
    # ball 0 is uniform over the interior minus the agent's and the goal's cells
    assert len(first) == (side - 2) ** 2 - 2
    if side <= 8:
        assert chi2_ok(list(first.values()))[0]


def test_other_families_list_no_obstacles(ox):
    for fam, side, p in [(0, 8, 0), (1, 8, 0), (2, 19, 0), (3, 7, 0), (4, 9, 2), (5, 8, 1)]:
        *_, ob = ox.layout(fam, side, 3, 4, 0, p, with_obst=True)
        assert (ob == 0xFF).all()


POCKET = """
# # # # # # #
# # # # # # #
# # o . # # #
# # # # # # #
# > . . . . #
# . . . . G #
# # # # # # #
"""


def test_ball_with_one_free_neighbour_moves_there(ox):
    for seed in range(20):
        b, s = dyn_env(ox, POCKET, seed=seed)
        ox.step(b, s, [0])
        g = gt.grid_of(s, 7)
        assert balls(g) == {(3, 2)} and obst_list(s) == [(3, 2)]
        assert tuple(g[2, 2]) == (1, 0, 0)


SEALED = """
# # # # # #
# # # # # #
# # o # # #
# # # # # #
# > . . G #
# # # # # #
"""


def test_ball_with_no_free_neighbour_stays(ox):
    b, s = dyn_env(ox, SEALED, seed=3)
    for _ in range(5):
        ox.step(b, s, [1])
    assert balls(gt.grid_of(s, 6)) == {(2, 2)} and obst_list(s) == [(2, 2)]


NEXT_TO_AGENT = """
# # # # # #
# # # # # #
# # o # # #
# # > # # #
# # . . G #
# # # # # #
"""


def test_ball_never_moves_onto_the_agent(ox):
    # the ball's free neighbours: the agent's cell (excluded) only
    for seed in range(20):
        b, s = dyn_env(ox, NEXT_TO_AGENT, seed=seed)
        ox.step(b, s, [0])
        assert balls(gt.grid_of(s, 6)) == {(2, 2)}


COMPETE = """
# # # # # # #
# # # # # # #
# # o . o # #
# # # # # # #
# > . . . . #
# . . . . G #
# # # # # # #
"""


@pytest.mark.parametrize("order", [[(2, 2), (4, 2)], [(4, 2), (2, 2)]])
def test_balls_move_in_list_order(ox, order):
    # both balls' only free neighbour is (3, 2): the first in the list takes it
    b, s = dyn_env(ox, COMPETE, obst=order, seed=5)
    ox.step(b, s, [0])
    g = gt.grid_of(s, 7)
    moved, stayed = order
    assert balls(g) == {(3, 2), stayed}
    assert obst_list(s) == [(3, 2), stayed]


OPEN = """
# # # # # # #
# . . . . . #
# . . . . . #
# . . o . . #
# . . . . . #
# > . . . G #
# # # # # # #
"""


def test_move_is_uniform_over_the_eight_neighbours(ox):
    counts = {}
    for call in range(16000):
        b, s = dyn_env(ox, OPEN, seed=11, calls=call)
        ox.step(b, s, [1])
        (dest,) = obst_list(s)
        counts[dest] = counts.get(dest, 0) + 1
    assert set(counts) == {(3 + dx, 3 + dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)} - {(3, 3)}
    assert chi2_ok(list(counts.values()))[0]


WALL_AHEAD = """
# # # # # #
# . . . > #
# . . . . #
# . . . o #
# . . . G #
# # # # # #
"""


@pytest.mark.parametrize("reward_mode", [0, 1])
def test_forward_into_a_wall_ends_with_minus_one(ox, reward_mode):
    b, s = dyn_env(ox, WALL_AHEAD, seed=2, reward_mode=reward_mode)
    out = ox.step(b, s, [FORWARD])
    assert (s.x[0], s.y[0]) == (4, 1)
    assert out.flags[0, 0] == 1 and out.reward[0, 0] == np.float32(-1)


BALL_AHEAD_PINNED = """
# # # # # # #
# # # # # # #
# > o # # # #
# # # # # # #
# . . . . . #
# . . . . G #
# # # # # # #
"""


def test_forward_into_a_pinned_ball_ends_with_minus_one(ox):
    b, s = dyn_env(ox, BALL_AHEAD_PINNED, seed=1)
    out = ox.step(b, s, [FORWARD])
    assert (s.x[0], s.y[0]) == (1, 2)
    assert balls(gt.grid_of(s, 7)) == {(2, 2)}
    assert out.flags[0, 0] == 1 and out.reward[0, 0] == np.float32(-1)


BALL_AHEAD_LEAVES = """
# # # # # # #
# # # . # # #
# > o # # # #
# # # # # # #
# . . . . . #
# . . . . G #
# # # # # # #
"""


def test_ball_ahead_that_moves_away_still_ends_with_minus_one(ox):
    # the cell ahead is checked before the balls move: the ball leaves to (3, 1),
    # the agent walks into the freed cell and the episode still ends with -1
    b, s = dyn_env(ox, BALL_AHEAD_LEAVES, seed=1)
    out = ox.step(b, s, [FORWARD])
    assert balls(gt.grid_of(s, 7)) == {(3, 1)}
    assert (s.x[0], s.y[0]) == (2, 2)
    assert out.flags[0, 0] == 1 and out.reward[0, 0] == np.float32(-1)


BALL_ARRIVES = """
# # # # # # #
# # o # # # #
# > . # # # #
# # # # # # #
# . . . . . #
# . . . . G #
# # # # # # #
"""


def test_ball_arriving_ahead_blocks_without_penalty(ox):
    # the cell ahead was empty when checked; the ball then moves into it
    b, s = dyn_env(ox, BALL_ARRIVES, seed=4)
    out = ox.step(b, s, [FORWARD])
    assert balls(gt.grid_of(s, 7)) == {(2, 2)}
    assert (s.x[0], s.y[0]) == (1, 2)
    assert out.flags[0, 0] == 0 and out.reward[0, 0] == 0


@pytest.mark.parametrize("action", [3, 4, 5, 6, 9])
def test_other_actions_turn_left(ox, action):
    b, s = dyn_env(ox, SEALED, seed=3)
    out = ox.step(b, s, [action])
    assert s.dir[0] == 3 and out.action[0, 0] == 0 and out.flags[0, 0] == 0


GOAL_AHEAD = """
# # # # # #
# # # # # #
# # o # # #
# # # # # #
# . . > G #
# # # # # #
"""


def test_goal_reached(ox):
    b, s = dyn_env(ox, GOAL_AHEAD, seed=3, t=9, T=100)
    out = ox.step(b, s, [FORWARD])
    assert (s.x[0], s.y[0]) == (4, 4) and out.flags[0, 0] == 1
    assert out.reward[0, 0] == ox.goal_reward(10, 100)


def test_reset_restores_the_obstacle_list(ox):
    b, s = dyn_env(ox, WALL_AHEAD, seed=8)
    out = ox.rollout(b, s, 2, np.array([[FORWARD], [0]], np.uint8))
    assert out.flags[:, 0].tolist() == [1, 4]
    g1, x1, y1, d1, ob1 = ox.layout(DYNOBS, 6, 8, 0, 1, 1, with_obst=True)
    np.testing.assert_array_equal(gt.grid_of(s, 6), g1)
    np.testing.assert_array_equal(s.obst[:16], ob1)


def test_brute_force_invariants(ox):
    """All 3^6 sequences of the three actions from 5x5 starts with 2 balls:
    the list always matches the grid, balls stay on free interior cells
    (never the agent's, the goal's, a wall), the agent never shares a cell
    with a ball, and the episode ends exactly on the goal (+) or after a
    forward step whose cell ahead held a ball or wall (-1)."""
    seqs = np.array(list(itertools.product(range(3), repeat=6)), np.uint8)
    n = len(seqs)
    for seed in range(3):
        fam = np.full(n, DYNOBS, np.uint8)
        b = ox.Batch(fam, np.full(n, 5, np.uint8), np.full(n, 100, np.int32),
                     np.full(n, seed, np.uint64), np.arange(n, dtype=np.uint32) % 7, 0,
                     np.full(n, 2, np.uint8))
        s = ox.State.empty(b)
        ox.reset(b, s)
        alive = np.ones(n, bool)
        for k in range(6):
            grids0 = s.grid.reshape(n, 5, 5, 3).copy()
            x0, y0, d0 = s.x.copy(), s.y.copy(), s.dir.copy()
            out = ox.rollout(b, s, 1, seqs[:, k:k + 1].T.copy(), with_obs=False)
            grids = s.grid.reshape(n, 5, 5, 3)
            live = alive & ((out.flags[0] & 4) == 0)
            for i in np.nonzero(live)[0][::37]:
                g = grids[i]
                bs = balls(g)
                assert len(bs) == 2 and set(obst_list(s, i)) == bs
                assert (int(s.x[i]), int(s.y[i])) not in bs and (3, 3) not in bs
                assert g[0, 0, 0] == gt.WALL
                fx = x0[i] + [1, 0, -1, 0][d0[i]]
                fy = y0[i] + [0, 1, 0, -1][d0[i]]
                ahead = grids0[i][fy, fx, 0]
                blocked = seqs[i, k] == FORWARD and ahead not in (gt.EMPTY, gt.GOAL)
                on_goal = g[s.y[i], s.x[i], 0] == gt.GOAL
                term = bool(out.flags[0, i] & 1)
                assert term == (blocked or on_goal)
                if blocked:
                    assert out.reward[0, i] == np.float32(-1)
                elif on_goal:
                    assert out.reward[0, i] > 0
                else:
                    assert out.reward[0, i] == 0
            alive &= (out.flags[0] & 1) == 0


def test_malformed_list_entries_do_not_move(ox):
    """An obstacle list holding fewer balls than the family parameter (a
    malformed state): entries off the interior are left alone and no cell
    outside the grid is touched."""
    b, s = dyn_env(ox, POCKET, obst=[(2, 2)], n=3, seed=4)
    s.obst[2:6] = [0xFF, 0xFF, 0, 9]          # (255, 255) and (0, 9): off the interior
    before = s.obst.copy()
    grid_before = s.grid.copy()
    ox.step(b, s, [0])
    g = gt.grid_of(s, 7)
    assert balls(g) == {(3, 2)}
    np.testing.assert_array_equal(s.obst[2:6], before[2:6])
    changed = np.nonzero(s.grid != grid_before)[0] // 3
    assert set(changed.tolist()) == {2 * 7 + 2, 2 * 7 + 3}
