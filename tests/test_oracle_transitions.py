"""Hand-worked transitions of the oracle: every action against every kind
of front cell and hand state (intervention system, Table 'systems';
entities Wall, Key, Door, Goal of Table 'entities'; App. A)."""
import numpy as np
import pytest

import gridtools as gt

ROOM = """
# # # # # #
# . . . . #
# . {A} {F} . #
# . . . . #
# . . . G #
# # # # # #
"""


def room(front: str, agent: str = ">"):
    return ROOM.replace("{A}", agent).replace("{F}", front)


def run(ox, picture, action, carry=gt.EMPTY, t=0, T=100):
    b, s = gt.one_env(ox, picture, carry=carry, t=t, T=T)
    out = ox.step(b, s, [action])
    S = int(round((s.grid.size // 3) ** 0.5))
    return s, out, gt.grid_of(s, S)


@pytest.mark.parametrize("d", range(4))
def test_turns(ox, d):
    agent = {0: ">", 1: "v", 2: "<", 3: "^"}[d]
    s, out, _ = run(ox, room(".", agent), 0)
    assert s.dir[0] == (d + 3) % 4 and (s.x[0], s.y[0]) == (2, 2)
    s, out, _ = run(ox, room(".", agent), 1)
    assert s.dir[0] == (d + 1) % 4 and (s.x[0], s.y[0]) == (2, 2)
    assert out.flags[0, 0] == 0 and out.reward[0, 0] == 0 and s.t[0] == 1


@pytest.mark.parametrize("front,moves", [(".", True), ("#", False), ("Kr", False),
                                          ("Dr0", True), ("Dr1", False), ("Dr2", False),
                                          ("G", True)])
def test_forward_into(ox, front, moves):
    s, out, g = run(ox, room(front), 2)
    assert (s.x[0], s.y[0]) == ((3, 2) if moves else (2, 2))
    assert s.t[0] == 1
    term = front == "G"
    assert out.flags[0, 0] == (1 if term else 0)
    assert (out.reward[0, 0] != 0) == term
    # the grid is unchanged by forward moves
    g0, *_ = gt.parse(room(front))
    np.testing.assert_array_equal(g, g0)


def test_forward_heading_vectors(ox):
    pic = """
# # # # #
# . . . #
# . > . #
# . . . #
# # # # #
"""
    for d, dest in [(0, (3, 2)), (1, (2, 3)), (2, (1, 2)), (3, (2, 1))]:
        b, s = gt.one_env(ox, pic)
        s.dir[0] = d
        ox.step(b, s, [2])
        assert (s.x[0], s.y[0]) == dest


def test_pickup_key(ox):
    s, out, g = run(ox, room("Kb"), 3)
    assert s.carry[0] == gt.carry_of(5, 2)
    assert tuple(g[2, 3]) == (1, 0, 0)
    assert tuple(out.obs[0, 0, 6, 3]) == (5, 2, 0)   # the view shows the carried key


@pytest.mark.parametrize("front", [".", "#", "Dr0", "Dr2", "G"])
def test_pickup_nothing_pickable(ox, front):
    s, out, g = run(ox, room(front), 3)
    assert s.carry[0] == gt.EMPTY
    np.testing.assert_array_equal(g, gt.parse(room(front))[0])


def test_pickup_with_full_hand(ox):
    s, out, g = run(ox, room("Kb"), 3, carry=gt.carry_of(5, 0))
    assert s.carry[0] == gt.carry_of(5, 0)
    assert tuple(g[2, 3]) == (5, 2, 0)


def test_drop_on_empty(ox):
    s, out, g = run(ox, room("."), 4, carry=gt.carry_of(5, 4))
    assert s.carry[0] == gt.EMPTY and tuple(g[2, 3]) == (5, 4, 0)
    assert tuple(out.obs[0, 0, 5, 3]) == (5, 4, 0)   # the key is now ahead


@pytest.mark.parametrize("front", ["#", "Kr", "Dr0", "G"])
def test_drop_blocked(ox, front):
    s, out, g = run(ox, room(front), 4, carry=gt.carry_of(5, 4))
    assert s.carry[0] == gt.carry_of(5, 4)
    np.testing.assert_array_equal(g, gt.parse(room(front))[0])


def test_drop_with_empty_hand(ox):
    s, out, g = run(ox, room("."), 4)
    assert s.carry[0] == gt.EMPTY and tuple(g[2, 3]) == (1, 0, 0)


@pytest.mark.parametrize("door,carry,after", [
    ("Dy2", gt.carry_of(5, 4), 0),     # locked + matching key -> open
    ("Dy2", gt.carry_of(5, 0), 2),     # locked + wrong colour -> stays locked
    ("Dy2", gt.EMPTY, 2),              # locked + empty hand -> stays locked
    ("Dy1", gt.EMPTY, 0),              # closed -> open
    ("Dy0", gt.EMPTY, 1),              # open -> closed
    ("Dy1", gt.carry_of(5, 0), 0),     # closed opens whatever is carried
])
def test_toggle_door(ox, door, carry, after):
    s, out, g = run(ox, room(door), 5, carry=carry)
    assert tuple(g[2, 3]) == (4, 4, after)
    assert s.carry[0] == carry            # the key stays in hand


@pytest.mark.parametrize("front", [".", "#", "Kr", "G"])
def test_toggle_non_door(ox, front):
    s, out, g = run(ox, room(front), 5)
    np.testing.assert_array_equal(g, gt.parse(room(front))[0])


@pytest.mark.parametrize("action", [6, 7, 100, 255])
def test_done_and_out_of_range_are_noops(ox, action):
    s, out, g = run(ox, room("Kr"), action, carry=gt.EMPTY)
    assert (s.x[0], s.y[0], s.dir[0], s.carry[0], s.t[0]) == (2, 2, 0, gt.EMPTY, 1)
    assert out.action[0, 0] == action and out.flags[0, 0] == 0


def test_locked_door_opened_then_walked_through(ox):
    b, s = gt.one_env(ox, room("Dg2"), carry=gt.carry_of(5, 1))
    out = ox.rollout(b, s, 2, np.array([[5], [2]], np.uint8))
    assert (s.x[0], s.y[0]) == (3, 2)
    assert out.flags.tolist() == [[0], [0]]


def test_goal_at_last_step_sets_both_flags(ox):
    T = 7
    s, out, g = run(ox, room("G"), 2, t=T - 1, T=T)
    assert out.flags[0, 0] == 1 | 2
    assert out.reward[0, 0] == np.float32(1) - np.float32(0.9) * (np.float32(T) / np.float32(T))


def test_truncation_then_autoreset(ox):
    b, s = gt.one_env(ox, room("#"), t=98, T=100, seed=5)
    out = ox.rollout(b, s, 3, np.array([[0], [0], [0]], np.uint8))
    assert out.flags[:, 0].tolist() == [0, 2, 4]
    assert out.reward[:, 0].tolist() == [0, 0, 0]
    assert out.action[:, 0].tolist() == [0, 0, 0xFF]
    assert s.t[0] == 0 and s.episode[0] == 1 and s.done_prev[0] == 0
    # the reset state is the family's layout for episode 1
    g1, x1, y1, d1 = ox.layout(1, 6, 5, 0, 1)
    np.testing.assert_array_equal(gt.grid_of(s, 6), g1)
    assert (s.x[0], s.y[0], s.dir[0]) == (x1, y1, d1)
    np.testing.assert_array_equal(out.obs[2, 0], ox.observe(g1, x1, y1, d1))


def test_reset_ignores_action(ox):
    outs = []
    for a in (0, 2, 5):
        b, s = gt.one_env(ox, room("G"), t=3, T=100, seed=9)
        outs.append(ox.rollout(b, s, 2, np.array([[2], [a]], np.uint8)))
    for o in outs[1:]:
        np.testing.assert_array_equal(o.obs, outs[0].obs)
    assert outs[0].flags[:, 0].tolist() == [1, 4]


def test_terminal_obs_shows_agent_on_goal(ox):
    s, out, g = run(ox, room("G"), 2)
    # agent stands on the goal; its own cell shows the (empty) hand
    assert (s.x[0], s.y[0]) == (3, 2)
    assert tuple(out.obs[0, 0, 6, 3]) == (1, 0, 0)
    assert g[2, 3, 0] == 8
