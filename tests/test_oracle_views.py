"""Pins for the oracle's first-person observation (Table 'observations',
symbolic_first_person, R = 7, with MiniGrid's occlusion rule)."""
import json
import os

import numpy as np
import pytest

import gridtools as gt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "views.json")


def _cases():
    return json.load(open(GOLDEN))["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"][:2])
def test_hand_worked_views(ox, case):
    g, x, y, d = gt.parse("\n".join(case["picture"]))
    obs = ox.observe(g, x, y, d, gt.carry_of(*case["carry"]))
    exp = np.stack([np.array(case[k]) for k in ("type", "colour", "state")], -1)
    np.testing.assert_array_equal(obs, exp)


def random_world(rng, S, p_wall=0.25, p_obj=0.1):
    """Random grid with a wall border and random walls, doors, keys, goals."""
    g = np.zeros((S, S, 3), dtype=np.uint8)
    g[:, :] = (1, 0, 0)
    for yy in range(1, S - 1):
        for xx in range(1, S - 1):
            u = rng.random()
            if u < p_wall:
                g[yy, xx] = (2, 5, 0)
            elif u < p_wall + p_obj:
                kind = rng.integers(0, 3)
                c = rng.integers(0, 6)
                g[yy, xx] = [(4, c, rng.integers(0, 3)), (5, c, 0), (8, 1, 0)][kind]
    g[0, :] = g[-1, :] = g[:, 0] = g[:, -1] = (2, 5, 0)
    free = [(xx, yy) for yy in range(1, S - 1) for xx in range(1, S - 1) if g[yy, xx, 0] == 1]
    x, y = free[rng.integers(0, len(free))]
    return g, x, y, int(rng.integers(0, 4))


def world_of_view(x, y, d, i, j):
    f = [(1, 0), (0, 1), (-1, 0), (0, -1)][d]
    r = (-f[1], f[0])
    return x + (i - 3) * r[0] + (6 - j) * f[0], y + (i - 3) * r[1] + (6 - j) * f[1]


def test_rotation_invariance(ox):
    """Turning the whole world with the agent leaves its view unchanged."""
    rng = np.random.default_rng(0)
    for _ in range(300):
        S = int(rng.integers(5, 14))
        g, x, y, d = random_world(rng, S)
        carry = int(rng.choice([1, gt.carry_of(5, int(rng.integers(0, 6)))]))
        o = ox.observe(g, x, y, d, carry)
        g2, x2, y2, d2 = g, x, y, d
        for _ in range(4):
            g2, x2, y2, d2 = gt.rotate_world(g2, x2, y2, d2)
            np.testing.assert_array_equal(ox.observe(g2, x2, y2, d2, carry), o)


def test_mirror_symmetry(ox):
    """Mirroring the world left-right mirrors the view (columns i -> 6-i)."""
    rng = np.random.default_rng(1)
    for _ in range(300):
        S = int(rng.integers(5, 14))
        g, x, y, d = random_world(rng, S)
        o = ox.observe(g, x, y, d)
        gm = g[:, ::-1].copy()
        dm = {0: 2, 2: 0, 1: 1, 3: 3}[d]
        om = ox.observe(gm, S - 1 - x, y, dm)
        np.testing.assert_array_equal(om, o[:, ::-1])


def test_outside_the_border_is_never_seen(ox):
    """Embedding the grid in a larger world full of junk changes nothing:
    sight never crosses the wall border, so cells outside the grid are
    never visible (and reading them as walls is only a convention)."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        S = int(rng.integers(5, 12))
        g, x, y, d = random_world(rng, S)
        big = np.zeros((S + 12, S + 12, 3), dtype=np.uint8)
        junk = rng.integers(0, 3, (S + 12, S + 12))
        big[:, :] = np.array([(1, 0, 0), (8, 1, 0), (4, 2, 0)], dtype=np.uint8)[junk]
        big[6:6 + S, 6:6 + S] = g
        np.testing.assert_array_equal(ox.observe(big, x + 6, y + 6, d), ox.observe(g, x, y, d))


def independent_visibility(g, x, y, d):
    """Visibility written another way: in each row the visible cells are
    the see-through runs touching the row's seeds, widened by one cell on
    each side; the next row's seeds are the three cells ahead of every
    visible see-through cell."""
    S = g.shape[0]
    see = np.zeros((7, 7), bool)
    for j in range(7):
        for i in range(7):
            wx, wy = world_of_view(x, y, d, i, j)
            if 0 <= wx < S and 0 <= wy < S:
                t, s = g[wy, wx, 0], g[wy, wx, 2]
                see[j, i] = not (t == 2 or (t == 4 and s != 0))
    vis = np.zeros((7, 7), bool)
    seeds = {3}
    for j in range(6, -1, -1):
        row = set()
        for s in seeds:
            row.add(s)
            if see[j, s]:
                lo = s
                while lo - 1 >= 0 and see[j, lo - 1]:
                    lo -= 1
                hi = s
                while hi + 1 <= 6 and see[j, hi + 1]:
                    hi += 1
                row.update(range(max(0, lo - 1), min(6, hi + 1) + 1))
        for i in row:
            vis[j, i] = True
        seeds = set()
        for i in row:
            if see[j, i]:
                seeds.update(k for k in (i - 1, i, i + 1) if 0 <= k <= 6)
    return vis


def test_visibility_matches_independent_characterisation(ox):
    rng = np.random.default_rng(3)
    for _ in range(500):
        S = int(rng.integers(5, 16))
        g, x, y, d = random_world(rng, S, p_wall=float(rng.uniform(0.05, 0.5)))
        o = ox.observe(g, x, y, d)
        vis = independent_visibility(g, x, y, d)
        vis_o = o[:, :, 0] != 0
        np.testing.assert_array_equal(vis_o, vis)
        # visible cells show the world cell; the agent cell shows the carry
        for j in range(7):
            for i in range(7):
                if (i, j) == (3, 6):
                    assert tuple(o[j, i]) == (1, 0, 0)
                elif vis[j, i]:
                    wx, wy = world_of_view(x, y, d, i, j)
                    assert tuple(o[j, i]) == tuple(g[wy, wx])
                else:
                    assert tuple(o[j, i]) == (0, 0, 0)


def test_open_field_sees_everything(ox):
    """Deep inside a large empty room all 49 cells are visible empties."""
    S = 20
    g = np.zeros((S, S, 3), dtype=np.uint8)
    g[:, :] = (1, 0, 0)
    g[0, :] = g[-1, :] = g[:, 0] = g[:, -1] = (2, 5, 0)
    for d in range(4):
        o = ox.observe(g, 10, 10, d, gt.carry_of(5, 3))
        exp = np.zeros((7, 7, 3), np.uint8)
        exp[:, :] = (1, 0, 0)
        exp[6, 3] = (5, 3, 0)
        np.testing.assert_array_equal(o, exp)


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"][:2])
def test_hand_worked_categorical_views(ox, case):
    """categorical_first_person (Table 'observations'): the hand-worked
    views' type channel, one byte per cell."""
    g, x, y, d = gt.parse("\n".join(case["picture"]))
    obs = ox.observe_categorical(g, x, y, d, gt.carry_of(*case["carry"]))
    np.testing.assert_array_equal(obs, np.array(case["type"]))


def test_categorical_batches_record_49_bytes(ox):
    """A categorical batch writes 49-byte records at 49 * (row * N + i) and
    its dynamics equal the symbolic batch's (only the record differs)."""
    from paper_2407_19396_amd import workloads as wl
    t = wl.mixed_table(300, seed=5, mix_seed=6)
    outs, states = [], []
    for mode in (0, 1):
        b = ox.Batch(t.family, t.side, t.max_steps, t.seed, t.rng_id, 0, t.param, mode)
        s = ox.State.empty(b)
        first = ox.reset(b, s)
        out = ox.rollout(b, s, 40, None)
        outs.append((first, out))
        states.append(s)
    (f0, o0), (f1, o1) = outs
    assert o1.obs.shape == (40, 300, 7, 7) and f1.obs.shape == (1, 300, 7, 7)
    np.testing.assert_array_equal(o1.obs, o0.obs[..., 0])
    np.testing.assert_array_equal(f1.obs, f0.obs[..., 0])
    for f in ("reward", "flags", "action"):
        np.testing.assert_array_equal(getattr(o1, f), getattr(o0, f))
    for f in ox.STATE_FIELDS:
        np.testing.assert_array_equal(getattr(states[1], f), getattr(states[0], f))
