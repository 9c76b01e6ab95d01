"""Exhaustive inputs for the brute-force checks: every start state of the
5x5 single room and of the 5x5 two-room key/door layout (and, for the GPU
parity runs, of a 5x5 GoToDoor room and a 5x5 room with one moving ball),
each paired with every action sequence of a given length.  Only inputs are
built here."""
from __future__ import annotations

import itertools

import numpy as np

W, E, G = (2, 5, 0), (1, 0, 0), (8, 1, 0)


def _room(S=5):
    g = np.zeros((S, S, 3), np.uint8)
    g[:, :] = E
    g[0, :] = g[-1, :] = g[:, 0] = g[:, -1] = W
    g[S - 2, S - 2] = G
    return g


def empty5_starts():
    g = _room()
    starts = []
    for y, x, d in itertools.product(range(1, 4), range(1, 4), range(4)):
        if (x, y) == (3, 3):
            continue
        starts.append((g.copy(), x, y, d))
    return starts


def tworoom5_starts(colours=(4,)):
    starts = []
    for d_row, colour, ky, ay, d in itertools.product((1, 2), colours, (1, 2, 3), (1, 2, 3), range(4)):
        if ky == ay:
            continue
        g = _room()
        g[:, 2] = W
        g[d_row, 2] = (4, colour, 2)
        g[ky, 1] = (5, colour, 0)
        starts.append((g, 1, ay, d))
    return starts


def gotodoor5_starts():
    """The 5x5 GoToDoor room with doors at the middle of each wall (top red,
    right green, bottom blue, left purple, all closed): every mission, agent
    cell and heading.  The fifth element is the family bytes (the mission)."""
    starts = []
    for mission, y, x, d in itertools.product(range(4), range(1, 4), range(1, 4), range(4)):
        g = _room()
        g[3, 3] = E                                   # no goal square
        g[0, 2], g[2, 4], g[4, 2], g[2, 0] = (4, 0, 1), (4, 1, 1), (4, 2, 1), (4, 3, 1)
        ob = np.full(16, 0xFF, np.uint8)
        ob[0] = mission
        starts.append((g, x, y, d, ob))
    return starts


def dynobs5_starts():
    """The 5x5 room with the goal at (3, 3) and one blue ball on each free
    interior cell in turn; the agent at (1, 1), every heading."""
    starts = []
    for by, bx, d in itertools.product(range(1, 4), range(1, 4), range(4)):
        if (bx, by) in ((1, 1), (3, 3)):
            continue
        g = _room()
        g[by, bx] = (6, 2, 0)
        ob = np.full(16, 0xFF, np.uint8)
        ob[0], ob[1] = bx, by
        starts.append((g, 1, 1, d, ob))
    return starts


def sequences(length: int) -> np.ndarray:
    """All 7**length action sequences as u8[length][7**length]."""
    n = 7 ** length
    idx = np.arange(n)
    return np.stack([(idx // 7 ** k) % 7 for k in range(length)]).astype(np.uint8)


def batch_arrays(starts, length: int, family: int, T: int, seed: int = 99, param: int = 0):
    """Per-env arrays for every (start, sequence) pair, start-major; a start
    may carry the env's family bytes (obst) as a fifth element."""
    seqs = sequences(length)
    m = seqs.shape[1]
    n = len(starts) * m
    S = starts[0][0].shape[0]
    grid = np.concatenate([np.broadcast_to(s[0].reshape(1, -1), (m, S * S * 3)) for s in starts]).reshape(-1)
    x = np.repeat(np.array([s[1] for s in starts], np.int32), m)
    y = np.repeat(np.array([s[2] for s in starts], np.int32), m)
    d = np.repeat(np.array([s[3] for s in starts], np.int32), m)
    actions = np.tile(seqs, (1, len(starts)))
    cfg = dict(family=np.full(n, family, np.uint8), side=np.full(n, S, np.uint8),
               max_steps=np.full(n, T, np.int32), seed=np.full(n, seed, np.uint64),
               rng_id=np.arange(n, dtype=np.uint32))
    if param:
        cfg["param"] = np.full(n, param, np.uint8)
    state = dict(grid=grid.copy(), x=x, y=y, dir=d, t=np.zeros(n, np.int32),
                 carry=np.ones(n, np.int32), episode=np.zeros(n, np.uint32),
                 done_prev=np.zeros(n, np.uint8))
    if len(starts[0]) > 4:
        state["obst"] = np.concatenate([np.broadcast_to(s[4], (m, 16)) for s in starts]).reshape(-1).copy()
    return cfg, state, actions


CASES = {
    "empty5_T100_L6": (empty5_starts, 6, 0, 100),
    "empty5_T3_L6": (empty5_starts, 6, 0, 3),
    "tworoom5_T250_L6": (tworoom5_starts, 6, 1, 250),
    "tworoom5_T4_L6": (tworoom5_starts, 6, 1, 4),
}

# parity-only cases (GPU against the oracle): (starts, length, family, T, param)
PARITY_CASES = {
    "gotodoor5_T100_L5": (gotodoor5_starts, 5, 7, 100, 0),
    "gotodoor5_T3_L5": (gotodoor5_starts, 5, 7, 3, 0),
    "dynobs5_T100_L6": (dynobs5_starts, 6, 6, 100, 1),
}
