"""Runs every entry point of the CPU oracle on a fixed set of inputs and
saves all outputs and final states to an .npz file.  The sanitizer test
runs it once against the AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle and once against the ordinary build and compares the
files.  Inputs only; no checking here.

    python tests/sanitize_driver.py OUT.npz
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import enumerate_starts as es  # noqa: E402
import oracle as ox  # noqa: E402
from paper_2407_19396_amd import workloads as wl  # noqa: E402


def batch_of(table, obs_mode=0, sprites=None, reward_mode=0):
    return ox.Batch(table.family, table.side, table.max_steps, table.seed, table.rng_id, reward_mode,
                    table.param, obs_mode, sprites)


def main(path):
    out = {}

    def keep(tag, o, s):
        for f in ("obs", "reward", "flags", "action", "mission"):
            v = getattr(o, f)
            if v is not None:
                out[f"{tag}/{f}"] = v
        for f in ox.STATE_FIELDS:
            out[f"{tag}/state_{f}"] = getattr(s, f)

    # every family, all four symbolic / categorical observation modes, the
    # random policy and an external action stream, both reward modes
    table = wl.families_table(120, seed=3, mix_seed=11)
    for mode in (0, 1, 2, 3):
        b = batch_of(table, mode, reward_mode=mode & 1)
        s = ox.State.empty(b)
        ox.reset(b, s)
        keep(f"fam{mode}_policy", ox.rollout(b, s, 96, None, nthreads=2), s)
        acts = wl.random_actions(64, table.n, seed=mode)
        keep(f"fam{mode}_actions", ox.rollout(b, s, 64, acts, rows=17), s)
    # the two image modes on a few envs
    sprites = np.random.default_rng(5).integers(0, 256, (264, 32, 32, 3), dtype=np.uint8)
    small = table.subset(np.arange(0, table.n, 15))
    for mode in (4, 5):
        b = batch_of(small, mode, sprites)
        s = ox.State.empty(b)
        ox.reset(b, s)
        keep(f"rgb{mode}", ox.rollout(b, s, 5, None), s)
    # layouts and observations of every family
    for fam, side, param in ((0, 7, 0), (1, 9, 0), (2, 19, 0), (3, 7, 0), (4, 11, 5), (5, 8, 2),
                             (6, 16, 8), (7, 12, 0), (8, 31, 3)):
        for ep in range(4):
            parts = ox.layout(fam, side, 99, 7, ep, param, with_obst=True)
            out[f"layout{fam}_{ep}"] = np.concatenate([np.ravel(np.asarray(v, dtype=np.int64))
                                                       for v in parts])
    # short exhaustive action sequences from the 5x5 starts
    for name, starts in (("empty5", es.empty5_starts()), ("tworoom5", es.tworoom5_starts())):
        L = 3
        seqs = np.array(np.meshgrid(*[np.arange(7)] * L, indexing="ij")).reshape(L, -1)
        n = len(starts) * seqs.shape[1]
        fam = np.full(n, 0 if name == "empty5" else 1, np.uint8)
        tb = wl.EnvTable(fam, np.full(n, 5, np.uint8), np.full(n, 4, np.int32),
                         np.zeros(n, np.uint64), np.arange(n, dtype=np.uint32), name)
        b = batch_of(tb)
        s = ox.State.empty(b)
        ox.reset(b, s)
        grid = s.grid.reshape(n, 5, 5, 3)
        for k, st in enumerate(starts):
            sl = slice(k * seqs.shape[1], (k + 1) * seqs.shape[1])
            grid[sl] = st[0]
            s.x[sl], s.y[sl], s.dir[sl] = st[1], st[2], st[3]
        acts = np.tile(seqs, (1, len(starts))).astype(np.uint8)
        keep(f"brute_{name}", ox.rollout(b, s, L + 2, np.vstack([acts, acts[:2]])), s)
    np.savez_compressed(path, **out)


if __name__ == "__main__":
    main(sys.argv[1])
