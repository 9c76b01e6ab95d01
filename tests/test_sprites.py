"""The default sprite atlas (paper_2407_19396_amd.sprites): its shape and
indexing, agent sprites that are rotations of one another, and sprites
that tell apart what the symbolic encoding tells apart."""
import numpy as np

from paper_2407_19396_amd import sprites as sp


def test_shape_and_index():
    a = sp.default_atlas()
    assert a.shape == (264, 32, 32, 3) and a.dtype == np.uint8
    assert sp.index(10, 5, 3) == 263 and sp.index(0, 0, 0) == 0
    assert not a[sp.index(sp.UNSEEN, 0, 0)].any()                 # unseen cells are black


def test_agent_headings_are_rotations():
    """The agent's triangle (its red pixels; the grid lines do not turn)
    for heading d is the east-pointing one turned d quarter turns
    clockwise (y grows downward); heading 3 points at the image's top."""
    a = sp.default_atlas()

    def triangle(d):
        img = a[sp.index(sp.AGENT, 0, d)].astype(int)
        return (img[..., 0] == 255) & (img[..., 1] == 0) & (img[..., 2] == 0)

    east = triangle(0)
    assert east.sum() > 100
    for d in range(4):
        np.testing.assert_array_equal(triangle(d), np.rot90(east, k=-d))
    north = triangle(3)
    rows = np.nonzero(north.any(axis=1))[0]
    widths = north.sum(axis=1)
    assert widths[rows[0]] < widths[rows[-1]]        # narrow tip at the top, wide base below


def test_distinct_entities_draw_distinct_sprites():
    a = sp.default_atlas()
    keys = [(sp.EMPTY, 0, 0), (sp.WALL, 5, 0), (sp.GOAL, 1, 0), (sp.LAVA, 0, 0)]
    keys += [(sp.DOOR, c, s) for c in range(6) for s in range(3)]
    keys += [(sp.KEY, c, 0) for c in range(6)] + [(sp.BALL, c, 0) for c in range(6)]
    keys += [(sp.AGENT, 0, d) for d in range(4)]
    imgs = [a[sp.index(*k)].tobytes() for k in keys]
    assert len(set(imgs)) == len(keys)
