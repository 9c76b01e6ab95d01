"""Pins for the oracle's start-state distribution (reset(key) of Sec.
3.2.2; families of Table 'envs'): structure of every generated layout
and uniformity of every random choice."""
import numpy as np
import pytest

from paper_2407_19396_amd import workloads as wl


def reset_many(ox, family, side, n, seed=11):
    t = wl.uniform_table(n, family, side, seed)
    b = ox.Batch(t.family, t.side, t.max_steps, t.seed, t.rng_id)
    s = ox.State.empty(b)
    out = ox.reset(b, s)
    grids = s.grid.reshape(n, side, side, 3)
    return grids, s, out


def chi2_ok(counts, probs=None):
    counts = np.asarray(counts, float)
    k = len(counts)
    if k == 1:
        return True, 0.0
    probs = np.full(k, 1.0 / k) if probs is None else np.asarray(probs)
    exp = probs * counts.sum()
    stat = ((counts - exp) ** 2 / exp).sum()
    # generous bound: mean k-1, sd sqrt(2(k-1)); 6 sd above the mean
    return stat < (k - 1) + 6 * np.sqrt(2 * (k - 1)), stat


def check_border(g):
    S = g.shape[0]
    for edge in (g[0], g[-1], g[:, 0], g[:, -1]):
        assert (edge == (2, 5, 0)).all()


@pytest.mark.parametrize("side", [4, 5, 6, 8, 16])
def test_empty_layouts(ox, side):
    n = 20000
    grids, s, out = reset_many(ox, 0, side, n)
    inner = side - 2
    pos = np.zeros((inner, inner), int)
    for i in range(n):
        g = grids[i]
        check_border(g)
        assert tuple(g[side - 2, side - 2]) == (8, 1, 0)
        body = g[1:-1, 1:-1].reshape(-1, 3)
        assert (body == (1, 0, 0)).all(axis=1).sum() == inner * inner - 1
        x, y = s.x[i], s.y[i]
        assert 1 <= x <= side - 2 and 1 <= y <= side - 2 and (x, y) != (side - 2, side - 2)
        pos[y - 1, x - 1] += 1
    counts = pos.reshape(-1)[:-1]     # the goal cell is never a start
    assert pos[-1, -1] == 0
    assert chi2_ok(counts)[0]
    assert chi2_ok(np.bincount(s.dir, minlength=4))[0]
    assert (s.t == 0).all() and (s.episode == 0).all() and (s.carry == 1).all()
    assert (out.flags == 4).all() and (out.action == 0xFF).all() and (out.reward == 0).all()


@pytest.mark.parametrize("side", [5, 6, 8, 16])
def test_tworoom_layouts(ox, side):
    n = 20000
    grids, s, _ = reset_many(ox, 1, side, n)
    cols, rows, colours = [], [], []
    key_cells, agent_cells = {}, {}
    for i in range(n):
        g = grids[i]
        check_border(g)
        walls = (g[1:-1, 1:-1, 0] == 2)
        wall_cols = np.where(walls.all(axis=0) | ((g[1:-1, 1:-1, 0] == 2) | (g[1:-1, 1:-1, 0] == 4)).all(axis=0))[0] + 1
        assert len(wall_cols) == 1
        c = int(wall_cols[0])
        assert 2 <= c <= side - 3
        doors = np.argwhere(g[:, :, 0] == 4)
        assert len(doors) == 1 and doors[0][1] == c
        d = int(doors[0][0])
        assert 1 <= d <= side - 3
        colour = int(g[d, c, 1])
        assert g[d, c, 2] == 2 and 0 <= colour <= 5
        keys = np.argwhere(g[:, :, 0] == 5)
        assert len(keys) == 1
        ky, kx = keys[0]
        assert 1 <= kx <= c - 1 and g[ky, kx, 1] == colour
        assert tuple(g[side - 2, side - 2]) == (8, 1, 0)
        x, y = int(s.x[i]), int(s.y[i])
        assert 1 <= x <= c - 1 and 1 <= y <= side - 2 and (x, y) != (kx, ky)
        assert tuple(g[y, x]) == (1, 0, 0)
        # nothing else: all other non-border, non-wall-column cells are empty
        other = np.ones((side, side), bool)
        other[0, :] = other[-1, :] = other[:, 0] = other[:, -1] = False
        other[:, c] = False
        other[ky, kx] = other[side - 2, side - 2] = False
        assert (g[other] == (1, 0, 0)).all()
        cols.append(c); rows.append(d); colours.append(colour)
        key_cells[(c, kx, ky)] = key_cells.get((c, kx, ky), 0) + 1
        agent_cells[(c, x, y)] = agent_cells.get((c, x, y), 0) + 1
    assert chi2_ok(np.bincount(cols)[2:side - 2])[0]
    assert chi2_ok(np.bincount(rows)[1:side - 2])[0]
    assert chi2_ok(np.bincount(colours, minlength=6))[0]
    assert chi2_ok(np.bincount(s.dir, minlength=4))[0]
    # within one wall column the key and the agent are uniform over the left room
    c0 = 2
    kc = [v for (c, _, _), v in key_cells.items() if c == c0]
    ac = [v for (c, _, _), v in agent_cells.items() if c == c0]
    assert len(kc) == (c0 - 1) * (side - 2) and chi2_ok(kc)[0]
    assert len(ac) == (c0 - 1) * (side - 2) and chi2_ok(ac)[0]


@pytest.mark.parametrize("side", [7, 19])
def test_fourrooms_layouts(ox, side):
    n = 20000 if side == 19 else 8000
    grids, s, _ = reset_many(ox, 2, side, n)
    m = side // 2
    gaps = [[], [], [], []]
    goal_cells = np.zeros((side, side), int)
    agent_cells = np.zeros((side, side), int)
    for i in range(n):
        g = grids[i]
        check_border(g)
        col = g[1:-1, m, 0]
        row = g[m, 1:-1, 0]
        assert col[m - 1] == 2 and row[m - 1] == 2
        top, bot = np.where(col[:m - 1] == 1)[0], np.where(col[m:] == 1)[0]
        lef, rig = np.where(row[:m - 1] == 1)[0], np.where(row[m:] == 1)[0]
        for lst, arr in zip(gaps, (top, bot, lef, rig)):
            assert len(arr) == 1 or (len(arr) == 0)
        goals = np.argwhere(g[:, :, 0] == 8)
        assert len(goals) == 1
        gy, gx = goals[0]
        goal_cells[gy, gx] += 1
        # the goal may sit in an opening; count the openings including it
        opening = lambda line, k: line[k] in (1, 8)  # noqa: E731
        segs = [(col, range(0, m - 1)), (col, range(m, side - 2)),
                (row, range(0, m - 1)), (row, range(m, side - 2))]
        for q, (line, rng_) in enumerate(segs):
            ks = [k for k in rng_ if opening(line, k)]
            assert len(ks) == 1
            gaps[q].append(ks[0] - rng_.start)
        x, y = int(s.x[i]), int(s.y[i])
        assert tuple(g[y, x]) == (1, 0, 0) and (x, y) != (gx, gy)
        agent_cells[y, x] += 1
        assert (g[:, :, 0] != 4).all() and (g[:, :, 0] != 5).all()
    for q in range(4):
        assert chi2_ok(np.bincount(gaps[q], minlength=m - 1))[0]
    # goal: uniform over the always-free room cells (openings are free only sometimes)
    rooms = np.ones((side, side), bool)
    rooms[0, :] = rooms[-1, :] = rooms[:, 0] = rooms[:, -1] = False
    rooms[m, :] = rooms[:, m] = False
    assert chi2_ok(goal_cells[rooms])[0]
    assert chi2_ok(agent_cells[rooms])[0]
    assert chi2_ok(np.bincount(s.dir, minlength=4))[0]


def test_layout_depends_on_seed_id_and_episode(ox):
    base = ox.layout(1, 8, 1, 2, 3)
    for args in [(1, 8, 2, 2, 3), (1, 8, 1, 3, 3), (1, 8, 1, 2, 4)]:
        other = ox.layout(*args)
        assert not (np.array_equal(other[0], base[0]) and other[1:] == base[1:])
    again = ox.layout(1, 8, 1, 2, 3)
    np.testing.assert_array_equal(again[0], base[0])
    assert again[1:] == base[1:]


@pytest.mark.parametrize("family,side", [(0, 3), (1, 4), (2, 8), (2, 5), (0, 33)])
def test_invalid_sides_rejected(ox, family, side):
    assert not ox.side_ok(family, side)
    with pytest.raises(ValueError):
        ox.layout(family, side, 0, 0, 0)
