"""Pins for the oracle's whole-grid observations (Table 'observations':
symbolic, the canonical grid encoding [H][W][3], and categorical, the
entity-id grid [H][W]), read as MiniGrid's fully observed encoding: the
agent drawn over its cell as (10, red, heading), the carried object not
shown.  Pinned by hand-worked grids, by agreement with the independently
pinned first-person view at every cell that view sees, and by the
batch layout (records packed like the grids)."""
import json
import os

import numpy as np
import pytest

import gridtools as gt
from test_oracle_views import random_world, world_of_view

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_obs.json")
AGENT = 10


def _cases():
    return json.load(open(GOLDEN))["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"][:2])
def test_hand_worked_full_grids(ox, case):
    g, x, y, d = gt.parse("\n".join(case["picture"]))
    if "agent" in case:
        x, y, d = case["agent"]
    exp = np.stack([np.array(case[k], np.uint8) for k in ("type", "colour", "state")], -1)
    np.testing.assert_array_equal(ox.observe_full(g, x, y, d), exp)
    np.testing.assert_array_equal(ox.observe_full_categorical(g, x, y, d), exp[:, :, 0])


def _check_against_view(ox, g, x, y, d, carry):
    """The whole grid agrees with the first-person view at every cell the
    view sees, and shows exactly one agent: at (x, y), red, its heading."""
    full = ox.observe_full(g, x, y, d)
    S = g.shape[0]
    agents = np.argwhere(full[:, :, 0] == AGENT)
    assert agents.tolist() == [[y, x]]
    assert tuple(full[y, x]) == (AGENT, 0, d)
    view = ox.observe(g, x, y, d, carry)
    seen = 0
    for j in range(7):
        for i in range(7):
            if (i, j) == (3, 6) or view[j, i, 0] == 0:
                continue
            wx, wy = world_of_view(x, y, d, i, j)
            assert 0 <= wx < S and 0 <= wy < S
            np.testing.assert_array_equal(full[wy, wx], view[j, i])
            seen += 1
    assert seen >= 1   # the cell ahead is always visible
    np.testing.assert_array_equal(ox.observe_full_categorical(g, x, y, d), full[:, :, 0])


def test_agrees_with_first_person_view(ox):
    rng = np.random.default_rng(11)
    for _ in range(400):
        S = int(rng.integers(5, 17))
        g, x, y, d = random_world(rng, S)
        carry = int(rng.choice([1, gt.carry_of(5, int(rng.integers(0, 6)))]))
        _check_against_view(ox, g, x, y, d, carry)


def test_carried_object_not_shown(ox):
    g, x, y, d = gt.parse("# # # # #\n# > . . #\n# . . . #\n# . . G #\n# # # # #")
    a = ox.observe_full(g, x, y, d)   # the whole-grid encoding takes no carry
    v = ox.observe(g, x, y, d, gt.carry_of(5, 3))
    assert tuple(v[6, 3]) == (5, 3, 0) and tuple(a[y, x]) == (AGENT, 0, d)


def _mixed_batch(ox, mode, n=24, seed=3):
    rng = np.random.default_rng(seed)
    fam = rng.choice([0, 1, 2, 3, 6], n).astype(np.uint8)
    side = np.where(fam == 2, 9, rng.choice([5, 6, 8], n)).astype(np.uint8)
    par = np.where(fam == 6, 2, 0).astype(np.uint8)
    T = np.full(n, 20, np.int32)
    return ox.Batch(fam, side, T, np.full(n, 77, np.uint64), np.arange(n, dtype=np.uint32), 0,
                    par, mode)


def test_batch_records_are_packed_like_grids(ox):
    """Modes 0, 2 and 3 run the same dynamics; the whole-grid records of env
    i sit at its grid offset (symbolic) or a third of it (categorical), and
    each agrees with that env's first-person record of the same step."""
    outs = {}
    for mode in (0, 2, 3):
        b = _mixed_batch(ox, mode)
        s = ox.State.empty(b)
        first = ox.reset(b, s)
        roll = ox.rollout(b, s, 40)
        outs[mode] = (b, first, roll)
    b2 = outs[2][0]
    assert b2.obs_row_bytes() == b2.grid_bytes() and outs[3][0].obs_row_bytes() == b2.grid_bytes() // 3
    for k in ("reward", "flags", "action"):
        np.testing.assert_array_equal(getattr(outs[0][2], k), getattr(outs[2][2], k))
        np.testing.assert_array_equal(getattr(outs[0][2], k), getattr(outs[3][2], k))
    off = b2.grid_offsets()
    n_agents = 0
    for which in (1, 2):   # the reset row, then every rollout row
        o0, o2, o3 = (outs[m][which].obs for m in (0, 2, 3))
        for r in range(o0.shape[0]):
            for i in range(b2.n):
                S = int(b2.side[i])
                full = ox.full_record(o2[r], 2, int(off[i]), S)
                cat = ox.full_record(o3[r], 3, int(off[i]), S)
                np.testing.assert_array_equal(cat, full[:, :, 0])
                (ay, ax), = np.argwhere(full[:, :, 0] == AGENT)
                d = int(full[ay, ax, 2])
                view = o0[r, i]
                for j in range(7):
                    for ii in range(7):
                        if (ii, j) == (3, 6) or view[j, ii, 0] == 0:
                            continue
                        wx, wy = world_of_view(ax, ay, d, ii, j)
                        np.testing.assert_array_equal(full[wy, wx], view[j, ii])
                n_agents += 1
    assert n_agents == b2.n * 41
