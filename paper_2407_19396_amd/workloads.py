"""Seeded synthetic workloads shared by the GPU path's tests, the oracle's
tests and the benchmark.

This module only *describes inputs*: which family and grid side each env
has, its truncation limit, its RNG seed and id, and external action
streams.  It holds none of the environment dynamics, so both sides of a
parity check can use it without sharing any of the method's arithmetic.

The workloads stand in for the paper's MiniGrid tasks (NAVIX, Table
"envs": Empty-5x5 / 8x8 / 16x16, DoorKey-5x5 ... 16x16, FourRooms, and the
lava tasks LavaGap-S5/6/7, Crossings-S9N1/2/3 and S11N5, DistShift1/2),
which are generated procedurally, so no dataset is involved.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FAMILY_EMPTY, FAMILY_TWOROOM, FAMILY_FOURROOMS = 0, 1, 2
FAMILY_LAVAGAP, FAMILY_CROSSINGS, FAMILY_DISTSHIFT, FAMILY_DYNOBS = 3, 4, 5, 6
FAMILY_GOTODOOR, FAMILY_KEYCORRIDOR = 7, 8
FAMILY_NAMES = {FAMILY_EMPTY: "Empty", FAMILY_TWOROOM: "TwoRoom", FAMILY_FOURROOMS: "FourRooms",
                FAMILY_LAVAGAP: "LavaGap", FAMILY_CROSSINGS: "Crossings",
                FAMILY_DISTSHIFT: "DistShift", FAMILY_DYNOBS: "Dynamic-Obstacles",
                FAMILY_GOTODOOR: "GoToDoor", FAMILY_KEYCORRIDOR: "KeyCorridor"}
N_ACTIONS = 7


def default_max_steps(family: int, side: int) -> int:
    """MiniGrid's default step limits for each family: 4*S^2 (Empty, the
    lava families, Dynamic-Obstacles, GoToDoor), 10*S^2 (DoorKey), 100
    (FourRooms), 30*s^2 for KeyCorridor's rooms of size s = (S + 2) / 3."""
    if family == FAMILY_TWOROOM:
        return 10 * side * side
    if family == FAMILY_FOURROOMS:
        return 100
    if family == FAMILY_KEYCORRIDOR:
        return 30 * ((side + 2) // 3) ** 2
    return 4 * side * side


@dataclass
class EnvTable:
    """Per-env configuration (host arrays)."""
    family: np.ndarray     # u8[N]
    side: np.ndarray       # u8[N]
    max_steps: np.ndarray  # i32[N]
    seed: np.ndarray       # u64[N]
    rng_id: np.ndarray     # u32[N]
    name: str = ""
    param: np.ndarray | None = None   # u8[N]: Crossings rivers, DistShift variant (else 0)

    def __post_init__(self):
        if self.param is None:
            self.param = np.zeros(self.family.shape[0], dtype=np.uint8)

    @property
    def n(self) -> int:
        return int(self.family.shape[0])

    def subset(self, idx) -> "EnvTable":
        idx = np.asarray(idx)
        return EnvTable(self.family[idx].copy(), self.side[idx].copy(), self.max_steps[idx].copy(),
                        self.seed[idx].copy(), self.rng_id[idx].copy(), self.name + "[subset]",
                        self.param[idx].copy())


def _table(family, side, seed: int, name: str, max_steps=None, param=0) -> EnvTable:
    family = np.asarray(family, dtype=np.uint8)
    side = np.asarray(side, dtype=np.uint8)
    n = family.shape[0]
    if max_steps is None:
        max_steps = np.array([default_max_steps(int(f), int(s)) for f, s in zip(family, side)],
                             dtype=np.int32)
    else:
        max_steps = np.broadcast_to(np.asarray(max_steps, dtype=np.int32), (n,)).copy()
    param = np.broadcast_to(np.asarray(param, dtype=np.uint8), (n,)).copy()
    return EnvTable(family, side, max_steps, np.full(n, seed, dtype=np.uint64),
                    np.arange(n, dtype=np.uint32), name, param)


def uniform_table(n: int, family: int, side: int, seed: int = 0, max_steps=None,
                  param: int = 0) -> EnvTable:
    """n envs of one family, side and family parameter."""
    return _table(np.full(n, family), np.full(n, side), seed,
                  f"{FAMILY_NAMES[family]}-{side}x{side}/{param} x{n}", max_steps, param)


# the lava tasks of the paper's environment table: (family, side, param)
LAVA_TASKS = [(FAMILY_LAVAGAP, 5, 0), (FAMILY_LAVAGAP, 6, 0), (FAMILY_LAVAGAP, 7, 0),
              (FAMILY_CROSSINGS, 9, 1), (FAMILY_CROSSINGS, 9, 2), (FAMILY_CROSSINGS, 9, 3),
              (FAMILY_CROSSINGS, 11, 5), (FAMILY_DISTSHIFT, 6, 1), (FAMILY_DISTSHIFT, 8, 2)]


def lava_table(n: int, seed: int = 0, mix_seed: int = 54321) -> EnvTable:
    """The lava tasks in equal shares, drawn i.i.d. per env from a seeded
    generator."""
    rng = np.random.default_rng(mix_seed)
    pick = np.array(LAVA_TASKS)[rng.integers(0, len(LAVA_TASKS), n)]
    return _table(pick[:, 0], pick[:, 1], seed, f"lava x{n}", None, pick[:, 2])


def mixed_table(n: int, seed: int = 0, mix_seed: int = 12345) -> EnvTable:
    """The uneven-size mix: 40 % single rooms and 40 % two-room key/door
    layouts with side uniform over {5, 6, 8, 16}, 20 % 19x19 four-room
    layouts; family and side drawn i.i.d. per env from a seeded generator."""
    rng = np.random.default_rng(mix_seed)
    u = rng.random(n)
    family = np.where(u < 0.4, FAMILY_EMPTY, np.where(u < 0.8, FAMILY_TWOROOM, FAMILY_FOURROOMS))
    side = np.array([5, 6, 8, 16], dtype=np.int64)[rng.integers(0, 4, n)]
    side = np.where(family == FAMILY_FOURROOMS, 19, side)
    return _table(family, side, seed, f"mixed x{n}")


# The five workloads (sizes as stated for the batched step).
def workload_empty5(seed: int = 0) -> EnvTable:
    """16 single rooms 5x5, max_steps 100 (plain step, 100 steps)."""
    return uniform_table(16, FAMILY_EMPTY, 5, seed)


def workload_empty8(seed: int = 0) -> EnvTable:
    """4096 single rooms 8x8, max_steps 256 (plain step, 1000 steps)."""
    return uniform_table(4096, FAMILY_EMPTY, 8, seed)


def workload_tworoom8(seed: int = 0) -> EnvTable:
    """65536 two-room key/door 8x8, max_steps 640 (fused, 2048 steps)."""
    return uniform_table(65536, FAMILY_TWOROOM, 8, seed)


def workload_mixed(seed: int = 0, n: int = 262144) -> EnvTable:
    """262144 envs of uneven sizes (fused persistent launch, 4096 steps)."""
    return mixed_table(n, seed)


# the Dynamic-Obstacles tasks of the paper's environment table: (side, balls)
DYNOBS_TASKS = [(5, 2), (6, 3), (8, 4), (16, 8)]


def dynobs_table(n: int, seed: int = 0, mix_seed: int = 777) -> EnvTable:
    """The Dynamic-Obstacles tasks in equal shares, i.i.d. per env."""
    rng = np.random.default_rng(mix_seed)
    pick = np.array(DYNOBS_TASKS)[rng.integers(0, len(DYNOBS_TASKS), n)]
    return _table(np.full(n, FAMILY_DYNOBS), pick[:, 0], seed, f"dynamic obstacles x{n}", None,
                  pick[:, 1])


def workload_dynobs(seed: int = 0, n: int = 262144) -> EnvTable:
    """262144 envs of the Dynamic-Obstacles tasks (fused, 4096 steps)."""
    return dynobs_table(n, seed)


def workload_lava(seed: int = 0, n: int = 262144) -> EnvTable:
    """262144 envs of the lava tasks (fused persistent launch, 4096 steps)."""
    return lava_table(n, seed)


# the GoToDoor tasks of the paper's environment table: sides
GOTODOOR_SIDES = [5, 6, 8]


def gotodoor_table(n: int, seed: int = 0, mix_seed: int = 999) -> EnvTable:
    """The GoToDoor tasks in equal shares, i.i.d. per env."""
    rng = np.random.default_rng(mix_seed)
    side = np.array(GOTODOOR_SIDES)[rng.integers(0, len(GOTODOOR_SIDES), n)]
    return _table(np.full(n, FAMILY_GOTODOOR), side, seed, f"gotodoor x{n}")


def workload_gotodoor(seed: int = 0, n: int = 262144) -> EnvTable:
    """262144 envs of the GoToDoor tasks (fused, 4096 steps)."""
    return gotodoor_table(n, seed)


# the KeyCorridor tasks of the paper's environment table: (side, rows) for
# S3R1, S3R2, S3R3, S4R3, S5R3, S6R3 (side = 3 * room size - 2)
KEYCORRIDOR_TASKS = [(7, 1), (7, 2), (7, 3), (10, 3), (13, 3), (16, 3)]


def keycorridor_table(n: int, seed: int = 0, mix_seed: int = 1001) -> EnvTable:
    """The KeyCorridor tasks in equal shares, i.i.d. per env."""
    rng = np.random.default_rng(mix_seed)
    pick = np.array(KEYCORRIDOR_TASKS)[rng.integers(0, len(KEYCORRIDOR_TASKS), n)]
    return _table(np.full(n, FAMILY_KEYCORRIDOR), pick[:, 0], seed, f"keycorridor x{n}", None,
                  pick[:, 1])


def workload_keycorridor(seed: int = 0, n: int = 262144) -> EnvTable:
    """262144 envs of the KeyCorridor tasks (fused, 4096 steps)."""
    return keycorridor_table(n, seed)


def families_table(n: int, seed: int = 0, mix_seed: int = 4242) -> EnvTable:
    """Every family in one batch: each env draws a task uniformly from the
    paper's tasks of every family (the uneven mix, the lava, obstacle and
    door tasks)."""
    rng = np.random.default_rng(mix_seed)
    tasks = ([(FAMILY_EMPTY, s, 0) for s in (5, 6, 8, 16)] +
             [(FAMILY_TWOROOM, s, 0) for s in (5, 6, 8, 16)] + [(FAMILY_FOURROOMS, 19, 0)] +
             LAVA_TASKS + [(FAMILY_DYNOBS, s, k) for s, k in DYNOBS_TASKS] +
             [(FAMILY_GOTODOOR, s, 0) for s in GOTODOOR_SIDES] +
             [(FAMILY_KEYCORRIDOR, s, r) for s, r in KEYCORRIDOR_TASKS])
    pick = np.array(tasks)[rng.integers(0, len(tasks), n)]
    return _table(pick[:, 0], pick[:, 1], seed, f"all families x{n}", None, pick[:, 2])


WORKLOAD_STEPS = {"empty5": 100, "empty8": 1000, "tworoom8": 2048, "mixed": 4096, "lava": 4096,
                  "dynobs": 4096, "gotodoor": 4096, "keycorridor": 4096}


def random_actions(n_steps: int, n_envs: int, seed: int) -> np.ndarray:
    """External action stream u8[n_steps][n_envs], uniform over {0..6}."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, N_ACTIONS, size=(n_steps, n_envs), dtype=np.uint8)


@dataclass
class Request:
    """One rollout request of the serving workload."""
    rid: int
    arrival_s: float
    n_envs: int
    n_steps: int
    seed: int
    table: EnvTable


def serving_requests(n_requests: int, rate_per_s: float, master_seed: int = 0,
                     max_envs: int = 8192) -> list[Request]:
    """Poisson arrivals; each request has log-uniform 1..max_envs envs drawn
    from the uneven-size mix, n_steps uniform in [64, 1024] and its own seed."""
    rng = np.random.default_rng(master_seed)
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n_envs = int(min(max_envs, max(1, np.floor(2.0 ** (rng.random() * np.log2(max_envs))))))
        n_steps = int(rng.integers(64, 1025))
        seed = int(rng.integers(0, 2 ** 63))
        table = mixed_table(n_envs, seed=seed, mix_seed=int(rng.integers(0, 2 ** 31)))
        table.name = f"request {rid}"
        reqs.append(Request(rid, t, n_envs, n_steps, seed, table))
    return reqs
