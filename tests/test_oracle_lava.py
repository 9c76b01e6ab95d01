"""Pins for the oracle's lava families (Table 'envs': LavaGap, Crossings,
DistShift with reward R2; Table 'entities': Lava; Tables 'rewards' and
'terminations': on_lava_fall): the structure of every generated layout,
uniformity of every random choice, reachability of the goal, hand-drawn
deterministic layouts, and hand-worked transitions into lava."""
import itertools

import numpy as np
import pytest

import gridtools as gt
from test_oracle_layouts import check_border, chi2_ok

LAVAGAP, CROSSINGS, DISTSHIFT = 3, 4, 5


def layouts(ox, family, side, n, param=0, seed=5):
    return [ox.layout(family, side, seed, i, 0, param) for i in range(n)]


def types(g):
    return g[:, :, 0]


def test_side_limits(ox):
    assert ox.side_ok(LAVAGAP, 5) and not ox.side_ok(LAVAGAP, 4) and not ox.side_ok(LAVAGAP, 33)
    assert ox.side_ok(CROSSINGS, 9, 3) and not ox.side_ok(CROSSINGS, 10, 3)
    assert ox.side_ok(CROSSINGS, 11, 8) and not ox.side_ok(CROSSINGS, 11, 9)
    assert not ox.side_ok(CROSSINGS, 7, 5) and ox.side_ok(CROSSINGS, 7, 4)
    assert not ox.side_ok(CROSSINGS, 9, 0)
    assert ox.side_ok(DISTSHIFT, 6, 1) and ox.side_ok(DISTSHIFT, 8, 2)
    assert not ox.side_ok(DISTSHIFT, 6, 0) and not ox.side_ok(DISTSHIFT, 6, 3)
    assert not ox.side_ok(DISTSHIFT, 5, 1)
    with pytest.raises(ValueError):
        ox.layout(CROSSINGS, 9, 1, 0, 0, 7)


@pytest.mark.parametrize("side", [5, 6, 7, 16])
def test_lavagap_layouts(ox, side):
    n = 12000
    cols, gaps = [], []
    for g, x, y, d in layouts(ox, LAVAGAP, side, n):
        check_border(g)
        t = types(g)
        assert (x, y, d) == (1, 1, 0)
        assert tuple(g[side - 2, side - 2]) == (8, 1, 0)
        lava = np.argwhere(t == 9)
        assert len(lava) == side - 3
        c = int(lava[0][1])
        assert (lava[:, 1] == c).all() and 2 <= c <= side - 3
        assert (g[t == 9] == (9, 0, 0)).all()
        gap = [yy for yy in range(1, side - 1) if t[yy, c] != 9]
        assert len(gap) == 1 and t[gap[0], c] == 1
        # nothing else in the interior
        inner = t[1:-1, 1:-1]
        assert ((inner == 1) | (inner == 9)).sum() == (side - 2) ** 2 - 1
        assert gt.reachable(g, (1, 1), (side - 2, side - 2))
        cols.append(c - 2)
        gaps.append(gap[0] - 1)
    assert chi2_ok(np.bincount(cols, minlength=side - 4))[0]
    assert chi2_ok(np.bincount(gaps, minlength=side - 2))[0]


@pytest.mark.parametrize("side,N", [(9, 1), (9, 2), (9, 3), (11, 5), (7, 4), (13, 8), (5, 2)])
def test_crossings_structure(ox, side, N):
    for g, x, y, d in layouts(ox, CROSSINGS, side, 3000, N):
        check_border(g)
        t = types(g)
        assert (x, y, d) == (1, 1, 0)
        assert tuple(g[side - 2, side - 2]) == (8, 1, 0)
        inner = t[1:-1, 1:-1]
        assert ((inner == 1) | (inner == 9)).sum() == (side - 2) ** 2 - 1
        lava = t == 9
        # lava only on even columns / rows, each lava line a river
        cols = sorted({int(c) for yy, c in np.argwhere(lava) if c % 2 == 0 and
                       lava[1:-1, c].sum() >= side - 3})
        rows = sorted({int(r) for r, xx in np.argwhere(lava) if r % 2 == 0 and
                       lava[r, 1:-1].sum() >= side - 3})
        assert len(cols) + len(rows) == N
        # the rivers: full lines across the interior except exactly one opening each
        for c in cols:
            holes = [yy for yy in range(1, side - 1) if not lava[yy, c]]
            assert len(holes) == 1 and holes[0] not in rows
        for r in rows:
            holes = [xx for xx in range(1, side - 1) if not lava[r, xx]]
            assert len(holes) == 1 and holes[0] not in cols
        # no lava anywhere else
        expect = np.zeros_like(lava)
        for c in cols:
            expect[1:-1, c] = True
        for r in rows:
            expect[r, 1:-1] = True
        assert (lava & ~expect).sum() == 0
        assert (expect & ~lava).sum() == N
        assert gt.reachable(g, (1, 1), (side - 2, side - 2))


def test_crossings_river_subset_uniform(ox):
    side, N = 9, 2          # 6 candidate rivers, C(6, 2) = 15 subsets
    cand = [("c", 2), ("c", 4), ("c", 6), ("r", 2), ("r", 4), ("r", 6)]
    index = {s: i for i, s in enumerate(itertools.combinations(range(6), 2))}
    counts = np.zeros(15, int)
    for g, *_ in layouts(ox, CROSSINGS, side, 15000, N, seed=9):
        lava = types(g) == 9
        chosen = tuple(i for i, (k, v) in enumerate(cand)
                       if (lava[1:-1, v] if k == "c" else lava[v, 1:-1]).sum() >= side - 3)
        counts[index[chosen]] += 1
    assert chi2_ok(counts)[0]


def test_crossings_path_order_and_openings_uniform(ox):
    """One column and one row river: the path crosses the column first with
    probability 1/2, and each opening is uniform along its room side."""
    side, N = 9, 2
    first_east = 0
    col_open, row_open = {}, {}
    n_mixed = 0
    for g, *_ in layouts(ox, CROSSINGS, side, 20000, N, seed=13):
        lava = types(g) == 9
        cols = [c for c in (2, 4, 6) if lava[1:-1, c].sum() >= side - 3]
        rows = [r for r in (2, 4, 6) if lava[r, 1:-1].sum() >= side - 3]
        if len(cols) != 1:
            continue
        n_mixed += 1
        c, r = cols[0], rows[0]
        hy = [yy for yy in range(1, side - 1) if not lava[yy, c]][0]
        hx = [xx for xx in range(1, side - 1) if not lava[r, xx]][0]
        east = hy < r               # crossed the column while still above the row
        assert east == (hx > c)     # then the row opening lies right of the column
        first_east += east
        key = (c, r, east)
        col_open.setdefault(key, []).append(hy)
        row_open.setdefault(key, []).append(hx)
    assert n_mixed > 8000
    p = first_east / n_mixed
    assert abs(p - 0.5) < 6 * np.sqrt(0.25 / n_mixed)
    for (c, r, east), ys in col_open.items():
        lo, hi = (1, r - 1) if east else (r + 1, side - 2)
        assert min(ys) >= lo and max(ys) <= hi
        assert chi2_ok(np.bincount(np.array(ys) - lo, minlength=hi - lo + 1))[0]
    for (c, r, east), xs in row_open.items():
        lo, hi = (c + 1, side - 2) if east else (1, c - 1)
        assert min(xs) >= lo and max(xs) <= hi
        assert chi2_ok(np.bincount(np.array(xs) - lo, minlength=hi - lo + 1))[0]


# DistShift: deterministic, drawn here by hand from the reading (goal at the
# top-right interior cell, lava on row 1 and row 2 (variant 1) or row S-2
# (variant 2) over columns 3..S-3, agent at (1, 1) facing east)
DISTSHIFT_PICTURES = {
    (6, 1): """
# # # # # #
# > . ~ G #
# . . ~ . #
# . . . . #
# . . . . #
# # # # # #
""",
    (6, 2): """
# # # # # #
# > . ~ G #
# . . . . #
# . . . . #
# . . ~ . #
# # # # # #
""",
    (8, 1): """
# # # # # # # #
# > . ~ ~ ~ G #
# . . ~ ~ ~ . #
# . . . . . . #
# . . . . . . #
# . . . . . . #
# . . . . . . #
# # # # # # # #
""",
    (8, 2): """
# # # # # # # #
# > . ~ ~ ~ G #
# . . . . . . #
# . . . . . . #
# . . . . . . #
# . . . . . . #
# . . ~ ~ ~ . #
# # # # # # # #
""",
}


@pytest.mark.parametrize("side,k", list(DISTSHIFT_PICTURES))
def test_distshift_layouts(ox, side, k):
    exp, ex, ey, ed = gt.parse(DISTSHIFT_PICTURES[(side, k)])
    for seed, episode in [(0, 0), (7, 3), (2 ** 40, 9)]:
        g, x, y, d = ox.layout(DISTSHIFT, side, seed, 11, episode, k)
        np.testing.assert_array_equal(g, exp)
        assert (x, y, d) == (ex, ey, ed)


LAVA_ROOM = """
# # # # # #
# . . . . #
# . > ~ . #
# . . . . #
# . . . G #
# # # # # #
"""


@pytest.mark.parametrize("reward_mode", [0, 1])
def test_forward_into_lava(ox, reward_mode):
    b, s = gt.one_env(ox, LAVA_ROOM, t=4, T=100, family=LAVAGAP, reward_mode=reward_mode)
    out = ox.step(b, s, [2])
    assert (s.x[0], s.y[0]) == (3, 2) and s.t[0] == 5
    assert out.flags[0, 0] == 1 and out.reward[0, 0] == np.float32(-1.0)
    assert s.done_prev[0] == 1
    # the agent stands in the lava; its own cell shows the hand, the grid keeps the lava
    assert tuple(out.obs[0, 0, 6, 3]) == (1, 0, 0)
    assert tuple(gt.grid_of(s, 6)[2, 3]) == (9, 0, 0)


def test_lava_at_the_last_step_sets_both_flags(ox):
    b, s = gt.one_env(ox, LAVA_ROOM, t=99, T=100, family=LAVAGAP)
    out = ox.step(b, s, [2])
    assert out.flags[0, 0] == 3 and out.reward[0, 0] == np.float32(-1.0)


@pytest.mark.parametrize("action", [0, 1, 3, 4, 5, 6])
def test_other_actions_leave_lava_alone(ox, action):
    carry = gt.carry_of(5, 1) if action == 4 else gt.EMPTY
    b, s = gt.one_env(ox, LAVA_ROOM, carry=carry, family=LAVAGAP)
    g0 = gt.grid_of(s, 6).copy()
    out = ox.step(b, s, [action])
    np.testing.assert_array_equal(gt.grid_of(s, 6), g0)
    assert s.carry[0] == carry and (s.x[0], s.y[0]) == (2, 2)
    assert out.flags[0, 0] == 0 and out.reward[0, 0] == 0


def test_lava_then_autoreset(ox):
    b, s = gt.one_env(ox, LAVA_ROOM, family=LAVAGAP, seed=21)
    out = ox.rollout(b, s, 2, np.array([[2], [2]], np.uint8))
    assert out.flags[:, 0].tolist() == [1, 4]
    assert out.reward[:, 0].tolist() == [-1.0, 0.0]
    g1, x1, y1, d1 = ox.layout(LAVAGAP, 6, 21, 0, 1)
    np.testing.assert_array_equal(gt.grid_of(s, 6), g1)
    assert (s.x[0], s.y[0], s.dir[0], s.episode[0]) == (x1, y1, d1, 1)


def test_lavagap5_brute_force(ox):
    """Every 6-step action sequence from each LavaGap-5 start: the episode ends
    exactly when the agent stands on the goal (+) or in lava (-1), the agent
    is never in a wall, and lava and walls never change."""
    starts = {}
    for i in range(200):
        g, x, y, d = ox.layout(LAVAGAP, 5, 3, i, 0)
        starts[g.tobytes()] = g
    assert len(starts) == 3                      # c = 2, gap row 1..3
    seqs = np.array(list(itertools.product(range(7), repeat=6)), np.uint8)
    n = len(seqs)
    for g in starts.values():
        fam = np.full(n, LAVAGAP, np.uint8)
        b = ox.Batch(fam, np.full(n, 5, np.uint8), np.full(n, 100, np.int32),
                     np.zeros(n, np.uint64), np.zeros(n, np.uint32))
        s = ox.State.empty(b)
        s.grid[:] = np.tile(g.reshape(-1), n)
        s.x[:] = 1
        s.y[:] = 1
        s.carry[:] = gt.EMPTY
        alive = np.ones(n, bool)
        for k in range(6):
            out = ox.rollout(b, s, 1, seqs[:, k:k + 1].T.copy(), with_obs=False, nthreads=8)
            grids = s.grid.reshape(n, 5, 5, 3)
            cell = grids[np.arange(n), s.y, s.x, 0]
            term = (out.flags[0] & 1) != 0
            live = alive & ((out.flags[0] & 4) == 0)
            assert (cell[live] != gt.WALL).all()
            on_goal, on_lava = cell == gt.GOAL, cell == gt.LAVA
            np.testing.assert_array_equal(term[live], (on_goal | on_lava)[live])
            assert (out.reward[0][live & on_lava] == np.float32(-1)).all()
            assert (out.reward[0][live & on_goal] > 0).all()
            assert (out.reward[0][live & ~term] == 0).all()
            lava0 = g[:, :, 0] == gt.LAVA
            assert (grids[live][:, lava0, 0] == gt.LAVA).all()
            assert (grids[live][:, 0, :, 0] == gt.WALL).all()
            alive &= ~term
