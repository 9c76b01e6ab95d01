"""Pins for the oracle's KeyCorridor family (Table 'envs': KeyCorridorS3R1
.. S6R3, reward R1): the room lattice, the hallway, the locked room with
the goal, the key of the locked door's colour, the doors that connect every
room, reachability, and uniformity of every placement."""
from collections import deque

import numpy as np
import pytest

from test_oracle_layouts import chi2_ok

KEYCORRIDOR = 8
WALL, EMPTY, DOOR, KEY, GOAL = 2, 1, 4, 5, 8


def test_side_limits(ox):
    for S in (7, 10, 13, 16, 31):
        for R in (1, 2, 3):
            assert ox.side_ok(KEYCORRIDOR, S, R)
    assert not ox.side_ok(KEYCORRIDOR, 8, 1) and not ox.side_ok(KEYCORRIDOR, 4, 1)
    assert not ox.side_ok(KEYCORRIDOR, 7, 0) and not ox.side_ok(KEYCORRIDOR, 7, 4)
    assert not ox.side_ok(KEYCORRIDOR, 34, 1)


def reach(g, start, passable):
    S = g.shape[0]
    seen = {start}
    todo = deque([start])
    while todo:
        x, y = todo.popleft()
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            nx, ny = x + dx, y + dy
            if 0 <= nx < S and 0 <= ny < S and (nx, ny) not in seen and passable(g[ny, nx]):
                seen.add((nx, ny))
                todo.append((nx, ny))
    return seen


def check_layout(g, x, y, d, S, R):
    """Structure of one layout; returns (locked row, key row, goal, key, agent
    cell offsets, locked door offset)."""
    t = g[:, :, 0]
    s = (S + 2) // 3
    st = s - 1
    H = R * st + 1
    assert (g[H:] == (WALL, 5, 0)).all()
    for yy in range(H):
        for xx in range(S):
            lattice = xx % st == 0 or yy % st == 0
            v = tuple(g[yy, xx])
            if not lattice:
                assert v in ((EMPTY, 0, 0), (GOAL, 1, 0)) or v[0] == KEY, (xx, yy, v)
                continue
            if v == (WALL, 5, 0):
                continue
            corner = xx % st == 0 and yy % st == 0
            border = xx in (0, S - 1) or yy in (0, H - 1)
            assert not corner and not border, (xx, yy, v)
            hallway = yy % st == 0 and st < xx < 2 * st
            if hallway:
                assert v == (EMPTY, 0, 0)
            else:
                assert v[0] == DOOR and v[2] in (1, 2) and v[1] <= 5, (xx, yy, v)
    # the hallway walls are all open
    for j in range(1, R):
        assert (t[j * st, st + 1:2 * st] == EMPTY).all()
    doors = np.argwhere(t == DOOR)
    locked = [(int(xx), int(yy)) for yy, xx in doors if g[yy, xx, 2] == 2]
    assert len(locked) == 1
    lx, ly = locked[0]
    assert lx == 2 * st
    rl = (ly - 1) // st
    colour = int(g[ly, lx, 1])
    # at most one door per wall between two rooms
    walls = set()
    for yy, xx in doors:
        key = (int(xx) // st, int(yy) // st, int(xx) % st == 0)
        assert key not in walls
        walls.add(key)
    # the goal alone in the locked room, whose only door is the locked one
    goals = np.argwhere(t == GOAL)
    assert len(goals) == 1
    gy, gx = (int(v) for v in goals[0])
    assert 2 * st < gx < 3 * st and rl * st < gy < (rl + 1) * st
    for yy, xx in doors:
        on_room = (xx in (2 * st, 3 * st) and rl * st < yy < (rl + 1) * st) or \
                  (yy in (rl * st, (rl + 1) * st) and 2 * st < xx < 3 * st)
        assert not on_room or (int(xx), int(yy)) == (lx, ly)
    # one key, of the locked door's colour, in a left-column room
    keys = np.argwhere(t == KEY)
    assert len(keys) == 1
    ky, kx = (int(v) for v in keys[0])
    assert tuple(g[ky, kx]) == (KEY, colour, 0)
    assert 0 < kx < st
    rk = (ky - 1) // st
    # the agent in the hallway room of row R // 2
    ra = R // 2
    assert st < x < 2 * st and ra * st < y < (ra + 1) * st and t[y, x] == EMPTY
    # every room reachable through doors of any state; the key without the locked door
    every = reach(g, (x, y), lambda c: c[0] != WALL)
    for j in range(R):
        for i in range(3):
            assert (i * st + 1, j * st + 1) in every
    no_lock = reach(g, (x, y), lambda c: c[0] != WALL and not (c[0] == DOOR and c[2] == 2))
    assert (kx, ky) in no_lock and (gx, gy) not in no_lock
    return rl, rk, (gx - 2 * st - 1, gy - rl * st - 1), (kx - 1, ky - rk * st - 1), \
        (x - st - 1, y - ra * st - 1), ly - rl * st - 1, colour


@pytest.mark.parametrize("S,R", [(7, 1), (7, 2), (7, 3), (10, 3), (13, 3), (16, 3)])
def test_layout_structure_and_uniformity(ox, S, R):
    n = 6000
    s = (S + 2) // 3
    inner = s - 2
    stats = [[] for _ in range(8)]
    for i in range(n):
        g, x, y, d = ox.layout(KEYCORRIDOR, S, 13, i, 0, R)
        rl, rk, goal, key, agent, lpos, colour = check_layout(g, x, y, d, S, R)
        for k, v in enumerate((rl, rk, goal[1] * inner + goal[0], key[1] * inner + key[0],
                               agent[1] * inner + agent[0], lpos, colour, d)):
            stats[k].append(v)
    sizes = [R, R, inner * inner, inner * inner, inner * inner, inner, 6, 4]
    for v, k in zip(stats, sizes):
        assert chi2_ok(np.bincount(v, minlength=k))[0]


def test_episodes_draw_new_layouts(ox):
    a = ox.layout(KEYCORRIDOR, 10, 5, 3, 0, 3)[0]
    b = ox.layout(KEYCORRIDOR, 10, 5, 3, 1, 3)[0]
    assert not np.array_equal(a, b)


def test_reaching_the_goal_through_the_locked_door(ox):
    """KeyCorridorS3R1: pick up the key, open the locked door, reach the goal
    (reward R1)."""
    import gridtools as gt
    pic = """
# # # # # # #
# Kr Dg1 < Dr2 G #
# # # # # # #
# # # # # # #
# # # # # # #
# # # # # # #
# # # # # # #
"""
    b, s = gt.one_env(ox, pic, family=KEYCORRIDOR, param=1, T=270)
    acts = [5, 2,             # open the green door, step onto it: the key is ahead
            3,                # pick up the red key
            0, 0, 2,          # turn around, step back to (3, 1)
            5, 2, 2]          # unlock the red door, step onto it, then onto the goal
    out = ox.rollout(b, s, len(acts), np.array(acts, np.uint8).reshape(-1, 1))
    assert s.carry[0] == gt.carry_of(5, 0)
    assert out.flags[-1, 0] == 1 and out.reward[-1, 0] == np.float32(1) - np.float32(0.9) * (
        np.float32(9) / np.float32(270))
    assert (out.flags[:-1, 0] == 0).all()
