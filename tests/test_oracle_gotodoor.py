"""Pins for the oracle's GoToDoor family (Table 'envs': GoToDoor-5x5/6x6/8x8;
Tables 'rewards' and 'terminations': on_door_done, the done action in front
of the door whose colour the mission names): the structure of every
generated layout, uniformity of every random choice, and hand-worked
transitions (done at the right door, at a wrong door, at a wall; toggling;
the mission output across an autoreset)."""
import itertools

import numpy as np
import pytest

import gridtools as gt
from test_oracle_layouts import chi2_ok

GOTODOOR = 7
DONE, TOGGLE, FORWARD = 6, 5, 2


def layouts(ox, side, n, seed=9):
    return [ox.layout(GOTODOOR, side, seed, i, 0, 0, with_obst=True) for i in range(n)]


def room_of(g):
    """Width and height of the walled room in the top-left corner: the room's
    interior is the set of non-wall cells, a rectangle from (1, 1)."""
    t = g[:, :, 0]
    free = np.argwhere((t != 2) & (t != 4))
    return int(free[:, 1].max()) + 2, int(free[:, 0].max()) + 2


def test_side_limits(ox):
    assert ox.side_ok(GOTODOOR, 5) and ox.side_ok(GOTODOOR, 32)
    assert not ox.side_ok(GOTODOOR, 4) and not ox.side_ok(GOTODOOR, 33)


@pytest.mark.parametrize("side", [5, 6, 8, 11])
def test_layout_structure_and_uniformity(ox, side):
    n = 12000 if side <= 8 else 8000
    widths, heights, cols0, subsets, targets, dirs = [], [], [], [], [], []
    pos = [[] for _ in range(4)]
    cells = []
    for g, x, y, d, ob in layouts(ox, side, n):
        # the outer ring: walls, and the doors of the room's top and left walls
        for edge in (g[0], g[-1], g[:, 0], g[:, -1]):
            assert ((edge == (2, 5, 0)).all(axis=1) | ((edge[:, 0] == 4) & (edge[:, 2] == 1))).all()
        t = g[:, :, 0]
        w, h = room_of(g)
        assert 5 <= w <= side and 5 <= h <= side
        # the room: interior empty (the agent stands on an empty cell), walls
        # around it, every cell outside it wall
        inner = g[1:h - 1, 1:w - 1]
        assert (inner == (1, 0, 0)).all()
        outside = np.ones((side, side), bool)
        outside[1:h - 1, 1:w - 1] = False
        doors = np.argwhere(t == 4)
        assert len(doors) == 4
        door_cells = {(int(xx), int(yy)) for yy, xx in doors}
        for yy, xx in np.argwhere(outside):
            if (xx, yy) not in door_cells:
                assert tuple(g[yy, xx]) == (2, 5, 0)
        # one closed door per room wall, off the corners: top, right, bottom, left
        want = [lambda xx, yy: yy == 0 and 1 <= xx <= w - 2,
                lambda xx, yy: xx == w - 1 and 1 <= yy <= h - 2,
                lambda xx, yy: yy == h - 1 and 1 <= xx <= w - 2,
                lambda xx, yy: xx == 0 and 1 <= yy <= h - 2]
        colours = []
        for i, ok in enumerate(want):
            hit = [c for c in door_cells if ok(*c)]
            assert len(hit) == 1, (i, door_cells, w, h)
            xx, yy = hit[0]
            assert g[yy, xx, 2] == 1                     # closed
            colours.append(int(g[yy, xx, 1]))
            pos[i].append((xx - 1) if i % 2 == 0 else (yy - 1))
        assert len(set(colours)) == 4 and max(colours) <= 5
        assert ob[0] in colours and (ob[1:] == 0xFF).all()
        assert 1 <= x <= w - 2 and 1 <= y <= h - 2
        assert not (t == 8).any()                        # no goal square
        widths.append(w - 5)
        heights.append(h - 5)
        cols0.append(colours[0])
        subsets.append(tuple(sorted(colours)))
        targets.append(colours.index(int(ob[0])))
        dirs.append(d)
        if w == 5 and h == 5:
            cells.append((y - 1) * 3 + (x - 1))
    assert chi2_ok(np.bincount(widths, minlength=side - 4))[0]
    assert chi2_ok(np.bincount(heights, minlength=side - 4))[0]
    assert chi2_ok(np.bincount(cols0, minlength=6))[0]
    all_subsets = list(itertools.combinations(range(6), 4))
    assert chi2_ok([subsets.count(c) for c in all_subsets])[0]
    assert chi2_ok(np.bincount(targets, minlength=4))[0]
    assert chi2_ok(np.bincount(dirs, minlength=4))[0]
    assert chi2_ok(np.bincount(cells, minlength=9))[0]
    # door positions, uniform along each wall given the room's size: pool
    # the layouts whose room is the full grid
    for i in range(4):
        full = [p for p, w, h in zip(pos[i], widths, heights) if w == side - 5 and h == side - 5]
        assert chi2_ok(np.bincount(full, minlength=side - 2))[0]


# a 5 x 5 room filling the grid: green door ahead of (2, 1), red door west of
# (1, 2), blue door east of (3, 2), yellow door south of (2, 3); the agent at
# (2, 2) faces north
ROOM = """
# # Dg1 # #
# . . . #
Dr1 . ^ . Db1
# . . . #
# # Dy1 # #
"""
# the agent at (1, 1) facing north, at the top wall
AT_WALL = ROOM.replace("# . . . #\nDr1 . ^", "# ^ . . #\nDr1 . .", 1)
RED, GREEN, BLUE, YELLOW = 0, 1, 2, 4


def one(ox, picture, mission, t=0, T=100, reward_mode=0, carry=gt.EMPTY):
    b, s = gt.one_env(ox, picture, carry=carry, t=t, T=T, family=GOTODOOR, reward_mode=reward_mode)
    s.obst[:] = 0xFF
    s.obst[0] = mission
    return b, s


@pytest.mark.parametrize("reward_mode", [0, 1])
@pytest.mark.parametrize("action", [DONE, 7, 255])
def test_done_facing_the_mission_door(ox, reward_mode, action):
    b, s = one(ox, ROOM, GREEN, t=9, T=100, reward_mode=reward_mode)
    b2, s2 = one(ox, ROOM, GREEN, t=9, T=100, reward_mode=reward_mode)
    out = ox.step(b, s, [DONE])
    # (2, 1) is empty, so the door two cells ahead is not "in front": no success
    assert out.flags[0, 0] == 0 and out.reward[0, 0] == 0
    # step forward, then done with the green door directly ahead
    out = ox.rollout(b2, s2, 2, np.array([[FORWARD], [action]], np.uint8))
    assert (s2.x[0], s2.y[0]) == (2, 1)
    assert out.flags[1, 0] == 1
    expect = np.float32(1.0) if reward_mode else np.float32(1) - np.float32(0.9) * (np.float32(11) / np.float32(100))
    assert out.reward[1, 0] == expect
    assert out.action[1, 0] == action
    assert (out.mission[:, 0] == GREEN).all()
    assert s2.done_prev[0] == 1


def test_done_at_a_wrong_door_or_a_wall(ox):
    for mission in (RED, BLUE, YELLOW):
        b, s = one(ox, ROOM, mission)
        out = ox.rollout(b, s, 2, np.array([[FORWARD], [DONE]], np.uint8))
        assert out.flags[1, 0] == 0 and out.reward[1, 0] == 0 and s.done_prev[0] == 0
    for mission in range(6):
        b, s = one(ox, AT_WALL, mission)
        assert (s.x[0], s.y[0]) == (1, 1)
        out = ox.step(b, s, [DONE])
        assert out.flags[0, 0] == 0 and out.reward[0, 0] == 0


def test_done_at_the_side_doors(ox):
    # (2, 2) facing west: (1, 2) empty, then the red door at (0, 2)
    for mission, ok in ((RED, True), (BLUE, False)):
        b, s = one(ox, ROOM.replace("^", "<"), mission)
        out = ox.rollout(b, s, 2, np.array([[FORWARD], [DONE]], np.uint8))
        assert (out.flags[1, 0] == 1) == ok and (out.reward[1, 0] > 0) == ok


def test_toggle_ends_the_episode_without_reward(ox):
    b, s = one(ox, ROOM, GREEN)
    out = ox.rollout(b, s, 2, np.array([[FORWARD], [TOGGLE]], np.uint8))
    assert out.flags[1, 0] == 1 and out.reward[1, 0] == 0
    assert tuple(gt.grid_of(s, 5)[0, 2]) == (4, GREEN, 0)        # the door opened
    # toggling at nothing ends it too
    b, s = one(ox, ROOM, GREEN)
    out = ox.step(b, s, [TOGGLE])
    assert out.flags[0, 0] == 1 and out.reward[0, 0] == 0


def test_closed_doors_block(ox):
    b, s = one(ox, ROOM, GREEN)
    ox.rollout(b, s, 3, np.array([[FORWARD], [FORWARD], [FORWARD]], np.uint8))
    assert (s.x[0], s.y[0]) == (2, 1)


def test_success_at_the_last_step_sets_both_flags(ox):
    b, s = one(ox, ROOM, GREEN, t=98, T=100)
    out = ox.rollout(b, s, 2, np.array([[FORWARD], [DONE]], np.uint8))
    assert out.flags[1, 0] == 3 and out.reward[1, 0] == np.float32(1) - np.float32(0.9) * np.float32(1.0)


def test_mission_output_follows_autoreset(ox):
    from paper_2407_19396_amd import workloads as wl
    t = wl.uniform_table(64, GOTODOOR, 6, seed=4)
    b = ox.Batch(t.family, t.side, t.max_steps, t.seed, t.rng_id)
    s = ox.State.empty(b)
    first = ox.reset(b, s)
    np.testing.assert_array_equal(first.mission[0], s.obst.reshape(64, 16)[:, 0])
    out = ox.rollout(b, s, 400)
    np.testing.assert_array_equal(out.mission[-1], s.obst.reshape(64, 16)[:, 0])
    # constant within an episode, redrawn at a reset
    m = np.concatenate([first.mission, out.mission])
    fl = np.concatenate([first.flags, out.flags])
    for i in range(64):
        for k in range(1, m.shape[0]):
            if not fl[k, i] & 4:
                assert m[k, i] == m[k - 1, i]
    assert (m <= 5).all()
    assert (fl & 4).sum() > 64        # some episodes ended and reset
    # the other families report no mission
    t2 = wl.uniform_table(8, 0, 6, seed=4)
    b2 = ox.Batch(t2.family, t2.side, t2.max_steps, t2.seed, t2.rng_id)
    s2 = ox.State.empty(b2)
    assert (ox.reset(b2, s2).mission == 0xFF).all()
