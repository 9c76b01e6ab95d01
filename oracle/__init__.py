"""CPU oracle of the batched gridworld step -- TEST INFRASTRUCTURE ONLY.

Python handle on ``gridworld_oracle.c`` (plain C, built with gcc).  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package; the GPU library never does, and the two share no
code.  See the C file for what each function follows in the NAVIX paper
(arXiv 2407.19396) and how it is pinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gridworld_oracle.c")
_LIB = os.environ.get("OX_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")

# encoding of the oracle (MiniGrid's canonical indices)
EMPTY, WALL, DOOR, KEY, GOAL = 1, 2, 4, 5, 8
OPEN, CLOSED, LOCKED = 0, 1, 2
FLAG_TERMINATED, FLAG_TRUNCATED, FLAG_FIRST = 1, 2, 4
ACTION_NONE = 0xFF
FAMILY_EMPTY, FAMILY_TWOROOM, FAMILY_FOURROOMS = 0, 1, 2
FAMILY_LAVAGAP, FAMILY_CROSSINGS, FAMILY_DISTSHIFT, FAMILY_DYNOBS = 3, 4, 5, 6
BALL, LAVA = 6, 9
MAX_OBST = 8
OBS_BYTES = 147
SPRITE = 32                        # pixels per cell side in the rgb observations
N_SPRITES = 11 * 6 * 4             # atlas entries: (type * 6 + colour) * 4 + state
RGB_FP = (7 * SPRITE, 7 * SPRITE, 3)


SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast math).
    sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build at
    liboracle_san.so instead (load it by setting OX_ORACLE_LIB to its path
    in a process that preloads libasan)."""
    out = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra",
               *(SAN_FLAGS if sanitize else []), "-o", out + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


_lib = None


class _Batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32),
                ("family", ctypes.c_void_p), ("side", ctypes.c_void_p),
                ("max_steps", ctypes.c_void_p), ("seed", ctypes.c_void_p),
                ("rng_id", ctypes.c_void_p), ("grid_off", ctypes.c_void_p),
                ("reward_mode", ctypes.c_int32), ("param", ctypes.c_void_p),
                ("obs_mode", ctypes.c_int32), ("sprites", ctypes.c_void_p)]


STATE_FIELDS = ("grid", "x", "y", "dir", "t", "carry", "episode", "done_prev", "calls", "obst")


class _State(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in STATE_FIELDS]


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("OX_ORACLE_LIB") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.ox_philox4x32_10.argtypes = [P, P, P]
        L.ox_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.ox_uniform.restype = ctypes.c_uint32
        L.ox_policy_action.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
        L.ox_policy_action.restype = ctypes.c_uint32
        L.ox_side_ok.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.ox_side_ok.restype = ctypes.c_int
        L.ox_layout.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_uint32, P, P, P, P, P]
        L.ox_layout.restype = ctypes.c_int
        L.ox_observe.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int32, P]
        L.ox_observe_categorical.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int32, P]
        L.ox_observe_full.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        L.ox_observe_full_categorical.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, P]
        L.ox_render.argtypes = [P, ctypes.c_int, P, P]
        L.ox_observe_rgb.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        L.ox_observe_rgb_full.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          P, P]
        L.ox_goal_reward.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int]
        L.ox_goal_reward.restype = ctypes.c_float
        L.ox_reset.argtypes = [ctypes.POINTER(_Batch), ctypes.POINTER(_State), P, P, P, P, P,
                               ctypes.c_int]
        L.ox_reset.restype = ctypes.c_int
        L.ox_rollout.argtypes = [ctypes.POINTER(_Batch), ctypes.POINTER(_State), ctypes.c_int32,
                                 P, ctypes.c_int32, P, P, P, P, P, ctypes.c_int]
        L.ox_rollout.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- scalars
def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().ox_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(word: int, n: int) -> int:
    return int(lib().ox_uniform(word, n))


def policy_action(seed: int, rng_id: int, call: int) -> int:
    return int(lib().ox_policy_action(seed, rng_id, call))


def side_ok(family: int, side: int, param: int = 0) -> bool:
    return bool(lib().ox_side_ok(family, side, param))


def layout(family: int, side: int, seed: int, rng_id: int, episode: int, param: int = 0,
           with_obst: bool = False):
    """Start state of one env: (grid [S][S][3] uint8, x, y, dir), plus the
    obstacle list u8[16] (x, y per ball, 0xFF unused) with with_obst."""
    g = np.zeros((side, side, 3), dtype=np.uint8)
    ob = np.zeros(2 * MAX_OBST, dtype=np.uint8)
    x, y, d = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int())
    rc = lib().ox_layout(family, side, param, seed, rng_id, episode, _ptr(g),
                         ctypes.addressof(x), ctypes.addressof(y), ctypes.addressof(d), _ptr(ob))
    if rc != 0:
        raise ValueError(f"layout failed ({rc}) for family={family} side={side}")
    if with_obst:
        return g, x.value, y.value, d.value, ob
    return g, x.value, y.value, d.value


def observe(grid: np.ndarray, x: int, y: int, d: int, carry: int = EMPTY) -> np.ndarray:
    """First-person view [7][7][3] (row j, column i, channel) of one env."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    obs = np.zeros((7, 7, 3), dtype=np.uint8)
    lib().ox_observe(_ptr(g), g.shape[0], x, y, d, carry, _ptr(obs))
    return obs


def observe_categorical(grid: np.ndarray, x: int, y: int, d: int, carry: int = EMPTY) -> np.ndarray:
    """categorical_first_person view [7][7] (row j, column i) of one env."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    obs = np.zeros((7, 7), dtype=np.uint8)
    lib().ox_observe_categorical(_ptr(g), g.shape[0], x, y, d, carry, _ptr(obs))
    return obs


def observe_full(grid: np.ndarray, x: int, y: int, d: int) -> np.ndarray:
    """symbolic observation [S][S][3] (row y, column x, channel) of one env."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    obs = np.zeros_like(g)
    lib().ox_observe_full(_ptr(g), g.shape[0], x, y, d, _ptr(obs))
    return obs


def observe_full_categorical(grid: np.ndarray, x: int, y: int, d: int) -> np.ndarray:
    """categorical observation [S][S] (row y, column x) of one env."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    obs = np.zeros(g.shape[:2], dtype=np.uint8)
    lib().ox_observe_full_categorical(_ptr(g), g.shape[0], x, y, d, _ptr(obs))
    return obs


def _atlas(sprites: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(sprites, dtype=np.uint8)
    assert a.shape == (N_SPRITES, SPRITE, SPRITE, 3), a.shape
    return a


def render(cells: np.ndarray, sprites: np.ndarray) -> np.ndarray:
    """Image [32W][32W][3] of W x W symbolic cells [W][W][3] drawn with the
    atlas sprites [264][32][32][3]."""
    c = np.ascontiguousarray(cells, dtype=np.uint8)
    W = c.shape[0]
    assert c.shape == (W, W, 3)
    a = _atlas(sprites)
    img = np.zeros((SPRITE * W, SPRITE * W, 3), dtype=np.uint8)
    lib().ox_render(_ptr(c), W, _ptr(a), _ptr(img))
    return img


def observe_rgb(grid: np.ndarray, x: int, y: int, d: int, sprites: np.ndarray) -> np.ndarray:
    """rgb_first_person image [224][224][3] of one env."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    a = _atlas(sprites)
    img = np.zeros(RGB_FP, dtype=np.uint8)
    lib().ox_observe_rgb(_ptr(g), g.shape[0], x, y, d, _ptr(a), _ptr(img))
    return img


def observe_rgb_full(grid: np.ndarray, x: int, y: int, d: int, sprites: np.ndarray) -> np.ndarray:
    """rgb image [32S][32S][3] of one env's whole grid."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    S = g.shape[0]
    a = _atlas(sprites)
    img = np.zeros((SPRITE * S, SPRITE * S, 3), dtype=np.uint8)
    lib().ox_observe_rgb_full(_ptr(g), S, x, y, d, _ptr(a), _ptr(img))
    return img


def goal_reward(t: int, T: int, reward_mode: int = 0) -> float:
    return float(np.float32(lib().ox_goal_reward(t, T, reward_mode)))


def pack_carry(type_: int, colour: int = 0, state: int = 0) -> int:
    return type_ | (colour << 8) | (state << 16)


# ---------------------------------------------------------------- batches
@dataclass
class Batch:
    family: np.ndarray      # u8[N]
    side: np.ndarray        # u8[N]
    max_steps: np.ndarray   # i32[N]
    seed: np.ndarray        # u64[N]
    rng_id: np.ndarray      # u32[N]
    reward_mode: int = 0
    param: np.ndarray | None = None   # u8[N] family parameter (Crossings N, DistShift k)
    obs_mode: int = 0                 # 0 symbolic_first_person [7][7][3], 1 categorical_first_person
                                      # [7][7], 2 symbolic [S][S][3], 3 categorical [S][S],
                                      # 4 rgb_first_person [224][224][3], 5 rgb [32S][32S][3]
    sprites: np.ndarray | None = None  # modes 4 and 5: the atlas u8[264][32][32][3]

    @property
    def n(self) -> int:
        return int(self.family.shape[0])

    def grid_offsets(self) -> np.ndarray:
        cells = 3 * self.side.astype(np.uint64) ** 2
        off = np.zeros(self.n, dtype=np.uint64)
        if self.n > 1:
            off[1:] = np.cumsum(cells)[:-1]
        return off

    def grid_bytes(self) -> int:
        return int((3 * self.side.astype(np.uint64) ** 2).sum())

    def obs_row_bytes(self) -> int:
        """Bytes of one output row of observations in this batch's mode."""
        return obs_row_bytes(self.obs_mode, self.n, self.grid_bytes())


def obs_row_bytes(obs_mode: int, n: int, grid_bytes: int) -> int:
    """First-person rows hold n records of 147, 49 or 150528 bytes; whole-grid
    rows are packed like the grids: sum 3 S^2 (symbolic), sum S^2
    (categorical) or sum 3072 S^2 bytes (rgb)."""
    return {0: 147 * n, 1: 49 * n, 2: grid_bytes, 3: grid_bytes // 3, 4: 147 * 1024 * n,
            5: 1024 * grid_bytes}[obs_mode]


def full_record(row: np.ndarray, obs_mode: int, grid_off: int, S: int) -> np.ndarray:
    """One env's whole-grid record inside an output row (modes 2, 3 and 5)."""
    if obs_mode == 2:
        return row[grid_off:grid_off + 3 * S * S].reshape(S, S, 3)
    if obs_mode == 5:
        o = 1024 * grid_off
        return row[o:o + 3072 * S * S].reshape(SPRITE * S, SPRITE * S, 3)
    o = grid_off // 3
    return row[o:o + S * S].reshape(S, S)


@dataclass
class State:
    grid: np.ndarray
    x: np.ndarray
    y: np.ndarray
    dir: np.ndarray
    t: np.ndarray
    carry: np.ndarray
    episode: np.ndarray
    done_prev: np.ndarray
    calls: np.ndarray = None      # u32[N] step calls since reset
    obst: np.ndarray = None       # u8[N * 16] obstacle positions (x, y per ball, 0xFF unused)

    def __post_init__(self):
        if self.calls is None:
            self.calls = np.zeros(self.x.shape[0], dtype=np.uint32)
        if self.obst is None:
            self.obst = np.full(self.x.shape[0] * 2 * MAX_OBST, 0xFF, dtype=np.uint8)

    @staticmethod
    def empty(batch: Batch) -> "State":
        n = batch.n
        z = lambda dt: np.zeros(n, dtype=dt)  # noqa: E731
        return State(np.zeros(batch.grid_bytes(), dtype=np.uint8), z(np.int32), z(np.int32),
                     z(np.int32), z(np.int32), z(np.int32), z(np.uint32), z(np.uint8), z(np.uint32),
                     np.full(n * 2 * MAX_OBST, 0xFF, dtype=np.uint8))

    def copy(self) -> "State":
        return State(*(getattr(self, f).copy() for f in STATE_FIELDS))


def _cbatch(b: Batch, keep: list):
    arrs = [np.ascontiguousarray(b.family, dtype=np.uint8),
            np.ascontiguousarray(b.side, dtype=np.uint8),
            np.ascontiguousarray(b.max_steps, dtype=np.int32),
            np.ascontiguousarray(b.seed, dtype=np.uint64),
            np.ascontiguousarray(b.rng_id, dtype=np.uint32),
            b.grid_offsets()]
    param = None if b.param is None else np.ascontiguousarray(b.param, dtype=np.uint8)
    sprites = None if b.sprites is None else _atlas(b.sprites)
    keep.extend(arrs + [param, sprites])
    return _Batch(b.n, *[a.ctypes.data for a in arrs], b.reward_mode,
                  None if param is None else param.ctypes.data, b.obs_mode,
                  None if sprites is None else sprites.ctypes.data)


def _cstate(s: State):
    for f in STATE_FIELDS:
        a = getattr(s, f)
        assert a.flags.c_contiguous, f
    return _State(*[getattr(s, f).ctypes.data for f in STATE_FIELDS])


@dataclass
class Outputs:
    obs: np.ndarray | None   # u8[rows][N][7][7][3], [rows][N][7][7], [rows][N][224][224][3]
                             # or [rows][row bytes] (whole-grid modes)
    reward: np.ndarray       # f32[rows][N]
    flags: np.ndarray        # u8[rows][N]
    action: np.ndarray       # u8[rows][N]
    mission: np.ndarray = None   # u8[rows][N]: GoToDoor's target colour, 0xFF without a mission

    @staticmethod
    def empty(rows: int, n: int, with_obs: bool = True, obs_mode: int = 0,
              row_bytes: int = 0) -> "Outputs":
        """row_bytes: bytes of one observation row in the whole-grid modes."""
        shape = {0: (rows, n, 7, 7, 3), 1: (rows, n, 7, 7),
                 4: (rows, n) + RGB_FP}.get(obs_mode, (rows, row_bytes))
        return Outputs(np.zeros(shape, dtype=np.uint8) if with_obs else None,
                       np.zeros((rows, n), dtype=np.float32),
                       np.zeros((rows, n), dtype=np.uint8),
                       np.zeros((rows, n), dtype=np.uint8),
                       np.zeros((rows, n), dtype=np.uint8))


def reset(batch: Batch, state: State, out: Outputs | None = None, nthreads: int = 0) -> Outputs:
    out = out or Outputs.empty(1, batch.n, obs_mode=batch.obs_mode, row_bytes=batch.obs_row_bytes())
    keep: list = []
    cb = _cbatch(batch, keep)
    cs = _cstate(state)
    rc = lib().ox_reset(ctypes.byref(cb), ctypes.byref(cs), _ptr(out.obs), _ptr(out.reward),
                        _ptr(out.flags), _ptr(out.action), _ptr(out.mission), nthreads)
    if rc != 0:
        raise ValueError(f"oracle reset failed ({rc})")
    return out


def rollout(batch: Batch, state: State, n_steps: int, actions: np.ndarray | None = None,
            rows: int | None = None, with_obs: bool = True, nthreads: int = 0) -> Outputs:
    """Run n_steps steps; step k lands in output row k % rows.  Without
    actions the random policy draws at each env's own call count."""
    rows = n_steps if rows is None else rows
    out = Outputs.empty(rows, batch.n, with_obs, batch.obs_mode, batch.obs_row_bytes())
    if actions is not None:
        actions = np.ascontiguousarray(actions, dtype=np.uint8)
        assert actions.shape == (n_steps, batch.n), actions.shape
    keep: list = []
    cb = _cbatch(batch, keep)
    cs = _cstate(state)
    rc = lib().ox_rollout(ctypes.byref(cb), ctypes.byref(cs), n_steps, _ptr(actions), rows,
                          _ptr(out.obs), _ptr(out.reward), _ptr(out.flags), _ptr(out.action),
                          _ptr(out.mission), nthreads)
    if rc != 0:
        raise ValueError(f"oracle rollout failed ({rc})")
    return out


def step(batch: Batch, state: State, actions: np.ndarray, with_obs: bool = True) -> Outputs:
    """One step for every env with the given actions (u8[N])."""
    a = np.asarray(actions, dtype=np.uint8).reshape(1, batch.n)
    return rollout(batch, state, 1, a, with_obs=with_obs)
