"""Test helpers: build grids from a token picture, inject states, and check
the invariants of the gridworld step.  No dynamics live here; the helpers
only describe inputs and read outputs."""
from __future__ import annotations

import numpy as np

EMPTY, WALL, DOOR, KEY, BALL, GOAL, LAVA = 1, 2, 4, 5, 6, 8, 9
COLOURS = {"r": 0, "g": 1, "b": 2, "p": 3, "y": 4, "e": 5}
DIRS = {">": 0, "v": 1, "<": 2, "^": 3}


def parse(picture: str):
    """Grid [S][S][3] from rows of space-separated tokens:
    ``#`` wall, ``.`` empty, ``G`` goal, ``~`` lava, ``o`` blue ball,
    ``K<c>`` key of colour c,
    ``D<c><s>`` door of colour c in state s (0 open, 1 closed, 2 locked),
    ``> v < ^`` the agent (on an empty cell) facing east/south/west/north.
    Returns (grid, x, y, dir); x, y, dir are None without an agent."""
    rows = [r.split() for r in picture.strip().splitlines()]
    S = len(rows)
    assert all(len(r) == S for r in rows), "picture must be square"
    g = np.zeros((S, S, 3), dtype=np.uint8)
    ax = ay = ad = None
    for y, row in enumerate(rows):
        for x, tok in enumerate(row):
            if tok == "#":
                g[y, x] = (WALL, 5, 0)
            elif tok == ".":
                g[y, x] = (EMPTY, 0, 0)
            elif tok == "G":
                g[y, x] = (GOAL, 1, 0)
            elif tok == "~":
                g[y, x] = (LAVA, 0, 0)
            elif tok == "o":
                g[y, x] = (BALL, 2, 0)
            elif tok[0] == "K":
                g[y, x] = (KEY, COLOURS[tok[1]], 0)
            elif tok[0] == "D":
                g[y, x] = (DOOR, COLOURS[tok[1]], int(tok[2]))
            elif tok in DIRS:
                g[y, x] = (EMPTY, 0, 0)
                ax, ay, ad = x, y, DIRS[tok]
            else:
                raise ValueError(tok)
    return g, ax, ay, ad


def carry_of(type_: int, colour: int = 0, state: int = 0) -> int:
    return type_ | (colour << 8) | (state << 16)


def rotate_world(grid: np.ndarray, x: int, y: int, d: int):
    """Rotate the world a quarter turn clockwise (x, y) -> (S-1-y, x); the
    agent's heading turns with it (d -> d+1)."""
    S = grid.shape[0]
    g2 = np.zeros_like(grid)
    for yy in range(S):
        for xx in range(S):
            g2[xx, S - 1 - yy] = grid[yy, xx]
    return g2, S - 1 - y, x, (d + 1) % 4


def one_env(ox, picture: str, carry: int = EMPTY, t: int = 0, T: int = 100, family: int = 1,
            seed: int = 0, episode: int = 0, reward_mode: int = 0, param: int = 0,
            obst=None, calls: int = 0):
    """A single-env oracle batch whose state is the given picture; obst lists
    the balls' (x, y) in their move order (default: row-major order)."""
    g, x, y, d = parse(picture)
    S = g.shape[0]
    b = ox.Batch(np.array([family], np.uint8), np.array([S], np.uint8), np.array([T], np.int32),
                 np.array([seed], np.uint64), np.array([0], np.uint32), reward_mode,
                 np.array([param], np.uint8))
    if obst is None:
        obst = [(int(bx), int(by)) for by, bx in np.argwhere(g[:, :, 0] == BALL)]
    ob = np.full(16, 0xFF, np.uint8)
    for i, (bx, by) in enumerate(obst):
        ob[2 * i], ob[2 * i + 1] = bx, by
    s = ox.State(g.reshape(-1).copy(), np.array([x], np.int32), np.array([y], np.int32),
                 np.array([d], np.int32), np.array([t], np.int32), np.array([carry], np.int32),
                 np.array([episode], np.uint32), np.array([0], np.uint8),
                 np.array([calls], np.uint32), ob)
    return b, s


def grid_of(state, S: int, off: int = 0) -> np.ndarray:
    return state.grid[off:off + 3 * S * S].reshape(S, S, 3)


def reachable(grid: np.ndarray, start, goal) -> bool:
    """Breadth-first search over cells that are neither wall nor lava."""
    S = grid.shape[0]
    seen = {start}
    todo = [start]
    while todo:
        x, y = todo.pop()
        if (x, y) == goal:
            return True
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            nx, ny = x + dx, y + dy
            if 0 <= nx < S and 0 <= ny < S and (nx, ny) not in seen and \
                    grid[ny, nx, 0] not in (WALL, LAVA):
                seen.add((nx, ny))
                todo.append((nx, ny))
    return False
