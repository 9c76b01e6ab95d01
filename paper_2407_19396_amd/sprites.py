"""A default sprite atlas for the rgb observation functions.

The library draws every cell with the sprite of its symbolic triple
(type, colour, state), from an atlas of 264 sprites of 32 x 32 x 3 bytes
indexed (type * 6 + colour) * 4 + state (the Sprite component of every
entity).  Any atlas of that shape can be passed to ``GridEnv``; this module
draws a plain one from geometric shapes in MiniGrid's six object colours.
It is this package's own drawing, not MiniGrid's or NAVIX's pixel art.
"""
from __future__ import annotations

import numpy as np

SPRITE = 32
N_TYPES, N_COLOURS, N_STATES = 11, 6, 4
N_SPRITES = N_TYPES * N_COLOURS * N_STATES

# red, green, blue, purple, yellow, grey
COLOURS = np.array([(255, 0, 0), (0, 255, 0), (0, 0, 255), (112, 39, 195), (255, 255, 0),
                    (100, 100, 100)], dtype=np.uint8)
LAVA_RGB = np.array((255, 128, 0), dtype=np.uint8)
GRID_LINE = np.array((100, 100, 100), dtype=np.uint8)

UNSEEN, EMPTY, WALL, FLOOR, DOOR, KEY, BALL, BOX, GOAL, LAVA, AGENT = range(11)


def index(type_: int, colour: int, state: int) -> int:
    return (type_ * N_COLOURS + colour) * N_STATES + state


def _coords():
    c = np.arange(SPRITE) + 0.5
    return np.meshgrid(c, c, indexing="xy")   # x (column), y (row), pixel centres


def _with_grid_lines(img: np.ndarray) -> np.ndarray:
    img[0, :] = GRID_LINE
    img[:, 0] = GRID_LINE
    return img


def _disc(cx, cy, r):
    x, y = _coords()
    return (x - cx) ** 2 + (y - cy) ** 2 <= r * r


def _rect(x0, y0, x1, y1):
    x, y = _coords()
    return (x >= x0) & (x < x1) & (y >= y0) & (y < y1)


def _triangle(heading: int):
    """The agent: a triangle pointing east, rotated to the heading
    (0 east, 1 south, 2 west, 3 north)."""
    x, y = _coords()
    u, v = x / SPRITE, y / SPRITE          # east-pointing: tip at (0.88, 0.5), base at u = 0.16
    m = (u >= 0.16) & (np.abs(v - 0.5) <= 0.36 * (0.88 - u) / 0.72)
    return np.rot90(m, k=-heading)        # k = -1 turns east into south (y grows downward)


def sprite(type_: int, colour: int, state: int) -> np.ndarray:
    img = np.zeros((SPRITE, SPRITE, 3), dtype=np.uint8)
    rgb = COLOURS[colour]
    if type_ == UNSEEN:
        return img
    if type_ == WALL:
        img[:] = rgb
        return img
    if type_ == GOAL:
        img[:] = rgb
        return _with_grid_lines(img)
    if type_ == LAVA:
        img[:] = LAVA_RGB
        x, y = _coords()
        for k in range(3):
            wave = np.abs(y - (8 + 8 * k) - 2 * np.sin(x / 4)) < 1.0
            img[wave] = 0
        return _with_grid_lines(img)
    _with_grid_lines(img)
    if type_ == FLOOR:
        img[1:, 1:] = rgb // 2
    elif type_ == DOOR:
        if state == 0:                                   # open: a frame
            img[_rect(1, 1, 32, 32) & ~_rect(4, 4, 29, 29)] = rgb
        elif state == 1:                                 # closed: frame, panel, handle
            img[_rect(1, 1, 32, 32)] = rgb
            img[_rect(4, 4, 29, 29)] = 0
            img[_rect(6, 6, 27, 27)] = rgb // 3
            img[_disc(23, 16, 2)] = rgb
        else:                                            # locked: solid with a keyhole
            img[_rect(1, 1, 32, 32)] = rgb
            img[_disc(16, 13, 3) | _rect(15, 13, 17, 22)] = 0
    elif type_ == KEY:
        img[_disc(16, 9, 5) & ~_disc(16, 9, 2)] = rgb
        img[_rect(15, 13, 18, 28)] = rgb
        img[_rect(18, 20, 22, 22) | _rect(18, 25, 22, 27)] = rgb
    elif type_ == BALL:
        img[_disc(16, 16, 10)] = rgb
    elif type_ == BOX:
        img[_rect(5, 5, 28, 28) & ~_rect(8, 8, 25, 25)] = rgb
        img[_rect(5, 15, 28, 17)] = rgb
    elif type_ == AGENT:
        img[_triangle(state % 4)] = COLOURS[0]
    return img


def default_atlas() -> np.ndarray:
    """u8[264][32][32][3]: sprite (type * 6 + colour) * 4 + state."""
    atlas = np.zeros((N_SPRITES, SPRITE, SPRITE, 3), dtype=np.uint8)
    for t in range(N_TYPES):
        for c in range(N_COLOURS):
            for s in range(N_STATES):
                atlas[index(t, c, s)] = sprite(t, c, s)
    return atlas
