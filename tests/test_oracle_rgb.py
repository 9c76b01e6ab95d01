"""Pins for the oracle's RGB observations (Table 'observations': rgb, an
image of 32 pixels per cell side of the whole grid, and rgb_first_person,
the same for the 7 x 7 view; Table 'components': every entity carries a
32 x 32 x 3 sprite).  The sprites are an input atlas indexed by the cell's
symbolic triple, so the images are pinned by decoding: under an atlas whose
every pixel spells out its sprite index and its position in the sprite,
each image pixel must name the triple of its cell in the independently
pinned symbolic views and its own offset inside the cell.  A transposed
sprite, a swapped cell index, a wrong channel order or a wrong agent
heading each fail it."""
import numpy as np
import pytest

import gridtools as gt
from test_oracle_views import random_world

SPRITE = 32
AGENT, RED, NORTH = 10, 0, 3


def coded_atlas() -> np.ndarray:
    """Sprite k's pixel (py, px) = (k & 255, (k >> 8) + 2 py, 64 + px)."""
    k = np.arange(264)[:, None, None]
    py = np.arange(SPRITE)[None, :, None]
    px = np.arange(SPRITE)[None, None, :]
    a = np.zeros((264, SPRITE, SPRITE, 3), np.uint8)
    a[..., 0] = k & 255
    a[..., 1] = (k >> 8) + 2 * py
    a[..., 2] = 64 + px + 0 * k
    return a


def decode(img: np.ndarray):
    """Per pixel: sprite index, row and column inside the sprite."""
    k = img[..., 0].astype(int) + 256 * (img[..., 1].astype(int) & 1)
    return k, img[..., 1].astype(int) >> 1, img[..., 2].astype(int) - 64


def index_of(triples: np.ndarray) -> np.ndarray:
    """Atlas index of each triple, [W][W][3] -> [W][W]."""
    t = triples.astype(int)
    return np.ravel_multi_index((t[..., 0], t[..., 1], t[..., 2]), (11, 6, 4))


def check_image(img: np.ndarray, cells: np.ndarray):
    W = cells.shape[0]
    assert img.shape == (SPRITE * W, SPRITE * W, 3)
    k, py, px = decode(img)
    rows = np.arange(SPRITE * W)
    np.testing.assert_array_equal(py, np.broadcast_to((rows % SPRITE)[:, None], py.shape))
    np.testing.assert_array_equal(px, np.broadcast_to((rows % SPRITE)[None, :], px.shape))
    want = np.repeat(np.repeat(index_of(cells), SPRITE, axis=0), SPRITE, axis=1)
    np.testing.assert_array_equal(k, want)


def test_first_person_image_draws_the_symbolic_view(ox):
    atlas = coded_atlas()
    rng = np.random.default_rng(21)
    for _ in range(60):
        S = int(rng.integers(5, 17))
        g, x, y, d = random_world(rng, S)
        view = ox.observe(g, x, y, d, gt.carry_of(5, int(rng.integers(0, 6))))
        view[6, 3] = (AGENT, RED, NORTH)           # the agent, facing the image's top
        check_image(ox.observe_rgb(g, x, y, d, atlas), view)


def test_whole_grid_image_draws_the_symbolic_grid(ox):
    atlas = coded_atlas()
    rng = np.random.default_rng(22)
    for _ in range(40):
        S = int(rng.integers(5, 17))
        g, x, y, d = random_world(rng, S)
        full = ox.observe_full(g, x, y, d)
        assert tuple(full[y, x]) == (AGENT, RED, d)
        check_image(ox.observe_rgb_full(g, x, y, d, atlas), full)


def test_out_of_range_triples_draw_sprite_zero(ox):
    atlas = coded_atlas()
    cells = np.array([[[10, 5, 3], [11, 0, 0]], [[0, 6, 0], [4, 2, 4]]], np.uint8)
    k, _, _ = decode(ox.render(cells, atlas))
    assert (k[:SPRITE, :SPRITE] == 263).all()
    assert (k[:SPRITE, SPRITE:] == 0).all() and (k[SPRITE:] == 0).all()


def test_pixels_are_copied_not_computed(ox):
    """Any atlas: every 32 x 32 block of the image equals its cell's sprite."""
    rng = np.random.default_rng(5)
    atlas = rng.integers(0, 256, (264, SPRITE, SPRITE, 3), dtype=np.uint8)
    g, x, y, d = gt.parse("# # # # # #\n# > . . . #\n# . Dr1 . . #\n# . . Ky . #\n# . . . G #\n# # # # # #")
    full = ox.observe_full(g, x, y, d)
    img = ox.observe_rgb_full(g, x, y, d, atlas)
    for j in range(6):
        for i in range(6):
            block = img[SPRITE * j:SPRITE * (j + 1), SPRITE * i:SPRITE * (i + 1)]
            np.testing.assert_array_equal(block, atlas[index_of(full[j, i])])


@pytest.mark.parametrize("mode,source", [(4, 0), (5, 2)])
def test_batch_records_render_the_symbolic_records(ox, mode, source):
    """The rgb modes run the same dynamics as the symbolic ones; each rgb
    record is its symbolic record drawn (first person: with the agent's own
    cell as the north-facing agent), at record offsets 1024 times the
    symbolic ones."""
    atlas = coded_atlas()
    rng = np.random.default_rng(8)
    n = 10
    fam = rng.choice([0, 1, 3, 6, 7], n).astype(np.uint8)
    side = rng.choice([5, 6, 8], n).astype(np.uint8)
    par = np.where(fam == 6, 2, 0).astype(np.uint8)
    T = np.full(n, 12, np.int32)
    outs = {}
    for m in (source, mode):
        b = ox.Batch(fam, side, T, np.full(n, 31, np.uint64), np.arange(n, dtype=np.uint32), 0,
                     par, m, atlas if m == mode else None)
        s = ox.State.empty(b)
        outs[m] = (b, ox.reset(b, s), ox.rollout(b, s, 16))
    b = outs[mode][0]
    assert b.obs_row_bytes() == 1024 * outs[source][0].obs_row_bytes()
    for k in ("reward", "flags", "action", "mission"):
        np.testing.assert_array_equal(getattr(outs[source][2], k), getattr(outs[mode][2], k))
    off = b.grid_offsets()
    for which in (1, 2):
        sym, rgb = outs[source][which].obs, outs[mode][which].obs
        for r in range(sym.shape[0]):
            for i in range(n):
                if mode == 4:
                    cells = sym[r, i].copy()
                    cells[6, 3] = (AGENT, RED, NORTH)
                    img = rgb[r, i]
                else:
                    S = int(side[i])
                    cells = ox.full_record(sym[r], 2, int(off[i]), S)
                    img = ox.full_record(rgb[r], 5, int(off[i]), S)
                check_image(img, cells)


def test_rgb_modes_need_an_atlas(ox):
    b = ox.Batch(np.zeros(2, np.uint8), np.full(2, 5, np.uint8), np.full(2, 10, np.int32),
                 np.zeros(2, np.uint64), np.arange(2, dtype=np.uint32), 0, None, 4)
    with pytest.raises(ValueError):
        ox.reset(b, ox.State.empty(b))
