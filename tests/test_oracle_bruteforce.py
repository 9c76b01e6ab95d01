"""Brute force over every action sequence of length 6 from every start
state of the 5x5 single room and 5x5 two-room layout, checking after each
step invariants that the paper's entities and protocol fix:
agent never inside a wall, exactly one agent, key conservation, a locked
door blocks without its key, counters and flags consistent, autoreset."""
from fractions import Fraction

import numpy as np
import pytest

import enumerate_starts as es

ULP = 2.0 ** -23


def check_step(pre, post, out_obs, rew, flags, act, cfg, family):
    n = pre["x"].shape[0]
    S = 5
    T = cfg["max_steps"]
    g_pre = pre["grid"].reshape(n, S, S, 3)
    g = post["grid"].reshape(n, S, S, 3)
    first = (flags & 4) != 0
    term = (flags & 1) != 0
    trunc = (flags & 2) != 0
    # autoreset exactly after done
    np.testing.assert_array_equal(first, pre["done_prev"] == 1)
    assert (post["t"][first] == 0).all()
    assert (post["episode"][first] == pre["episode"][first] + 1).all()
    assert (act[first] == 0xFF).all() and (rew[first] == 0).all()
    assert not (term[first] | trunc[first]).any()
    nf = ~first
    assert (post["t"][nf] == pre["t"][nf] + 1).all()
    assert (post["episode"][nf] == pre["episode"][nf]).all()
    # I5 / I7: counter range and truncation
    assert ((post["t"] >= 0) & (post["t"] <= T)).all()
    np.testing.assert_array_equal(trunc[nf], post["t"][nf] >= T[nf])
    np.testing.assert_array_equal(post["done_prev"], (term | trunc).astype(np.uint8))
    # I6: reward iff terminated, with the closed-form value
    np.testing.assert_array_equal(rew != 0, term)
    for i in np.where(term)[0][:2000]:
        exact = 1 - Fraction(9, 10) * Fraction(int(post["t"][i]), int(T[i]))
        assert abs(Fraction(float(rew[i])) - exact) <= 3 * ULP
    # I9, I1: heading and position
    assert ((post["dir"] >= 0) & (post["dir"] <= 3)).all()
    x, y = post["x"], post["y"]
    assert ((x >= 1) & (x <= S - 2) & (y >= 1) & (y <= S - 2)).all()
    under = g[np.arange(n), y, x]
    ok_under = (under[:, 0] == 1) | ((under[:, 0] == 4) & (under[:, 2] == 0)) | (under[:, 0] == 8)
    assert ok_under.all()
    on_goal = under[:, 0] == 8
    np.testing.assert_array_equal(on_goal & nf, term)
    # moves are single steps along the heading, only by 'forward'
    moved = nf & ((x != pre["x"]) | (y != pre["y"]))
    assert (act[moved] == 2).all()
    dx = np.array([1, 0, -1, 0])[pre["dir"]]
    dy = np.array([0, 1, 0, -1])[pre["dir"]]
    assert ((x[moved] == pre["x"][moved] + dx[moved]) & (y[moved] == pre["y"][moved] + dy[moved])).all()
    # I4: a locked door ahead blocks forward
    fx, fy = pre["x"] + dx, pre["y"] + dy
    front_pre = g_pre[np.arange(n), fy, fx]
    locked = (front_pre[:, 0] == 4) & (front_pre[:, 2] == 2)
    assert not (moved & locked).any()
    blocked = (front_pre[:, 0] == 2) | (front_pre[:, 0] == 5) | ((front_pre[:, 0] == 4) & (front_pre[:, 2] != 0))
    assert not (moved & blocked).any()
    # I3: key conservation and door count (two-room)
    carry_key = (post["carry"] & 0xFF) == 5
    keys = (g[:, :, :, 0] == 5).sum(axis=(1, 2))
    if family == 1:
        np.testing.assert_array_equal(keys + carry_key, 1)
        assert ((g[:, :, :, 0] == 4).sum(axis=(1, 2)) == 1).all()
        door_colour = g[:, :, :, 1][g[:, :, :, 0] == 4]
        key_colour = np.where(carry_key, (post["carry"] >> 8) & 0xFF, 0)
        kc_grid = np.zeros(n, np.int64)
        has_key = keys == 1
        kc_grid[has_key] = g[:, :, :, 1][g[:, :, :, 0] == 5]
        key_colour = np.where(carry_key, key_colour, kc_grid)
        np.testing.assert_array_equal(door_colour, key_colour)
    else:
        assert (keys == 0).all() and (~carry_key).all()
    # exactly one goal; walls never change within an episode (I12)
    assert ((g[:, :, :, 0] == 8).sum(axis=(1, 2)) == 1).all()
    walls_same = ((g[:, :, :, 0] == 2) == (g_pre[:, :, :, 0] == 2)).all(axis=(1, 2))
    assert walls_same[nf].all()
    # only the front cell changes within an episode
    diff = (g != g_pre).any(axis=3)
    ncell = diff.sum(axis=(1, 2))
    assert (ncell[nf] <= 1).all()
    if nf.any():
        idx = np.where(nf & (ncell == 1))[0]
        assert (diff[idx, fy[idx], fx[idx]]).all()
        assert np.isin(act[idx], (3, 4, 5)).all()
    # I10: the agent's cell shows the carry; the cell ahead is always seen
    obs = out_obs.reshape(n, 7, 7, 3)
    carry3 = np.stack([post["carry"] & 0xFF, (post["carry"] >> 8) & 0xFF, (post["carry"] >> 16) & 0xFF], 1)
    np.testing.assert_array_equal(obs[:, 6, 3], carry3)
    assert (obs[:, 5, 3, 0] != 0).all()
    # I2: one agent; the view never shows an agent or unseen-but-coloured cells
    assert (obs[:, :, :, 0] != 10).all()
    assert ((obs[:, :, :, 0] == 0) <= (obs[:, :, :, 1:] == 0).all(-1)).all()


@pytest.mark.parametrize("case", list(es.CASES))
def test_bruteforce_invariants(ox, case):
    make, L, family, T = es.CASES[case]
    starts = make()
    per_chunk = 8
    total = 0
    for c0 in range(0, len(starts), per_chunk):
        cfg, st, actions = es.batch_arrays(starts[c0:c0 + per_chunk], L, family, T)
        b = ox.Batch(cfg["family"], cfg["side"], cfg["max_steps"], cfg["seed"], cfg["rng_id"])
        s = ox.State(**st)
        for k in range(L):
            pre = {f: getattr(s, f).copy() for f in ("grid", "x", "y", "dir", "t", "carry", "episode", "done_prev")}
            out = ox.rollout(b, s, 1, actions[k:k + 1], nthreads=8)
            post = {f: getattr(s, f) for f in pre}
            # envs sharing the first k+1 actions are in the same state: check one of each
            sel = (np.arange(b.n) % 7 ** L) < 7 ** (k + 1)
            S3 = 75
            sub = lambda d: {f: (v.reshape(b.n, S3)[sel].reshape(-1) if f == "grid" else v[sel])  # noqa: E731
                             for f, v in d.items()}
            csub = {f: v[sel] for f, v in cfg.items()}
            check_step(sub(pre), sub(post), out.obs[0][sel], out.reward[0][sel], out.flags[0][sel],
                       out.action[0][sel], csub, family)
        total += b.n
    assert total == len(starts) * 7 ** L
