"""GPU parity: the HIP kernels, called through the C-ABI, against the CPU
oracle on the same seeded inputs, element by element and bit-exact (the
whole method is integer except the fp32 reward, whose bits must match)."""
import numpy as np
import pytest

import oracle as ox
import parity as P
from paper_2407_19396_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ge():
    import torch
    from paper_2407_19396_amd import gridenv
    assert torch.cuda.is_available()
    gridenv.load()
    return gridenv


def make(ge, table, reward_mode=0):
    env = ge.GridEnv(table, reward_mode)
    first = ge.Traj.alloc(1, table.n)
    env.reset(first)
    return env, first


def tables():
    return {
        "empty5": wl.workload_empty5(seed=3),
        "empty8": wl.workload_empty8(seed=4),
        "tworoom8": wl.uniform_table(2048, wl.FAMILY_TWOROOM, 8, seed=5),
        "fourrooms19": wl.uniform_table(512, wl.FAMILY_FOURROOMS, 19, seed=6),
        "mixed": wl.mixed_table(3000, seed=7, mix_seed=8),
        "all_sides": all_sides_table(),
        "lava": wl.lava_table(3000, seed=21, mix_seed=22),
        "lava_all": lava_all_table(),
        "dynobs": wl.dynobs_table(3000, seed=41, mix_seed=42),
        "dynobs_all": dynobs_all_table(),
        "gotodoor": wl.gotodoor_table(3000, seed=61, mix_seed=62),
        "gotodoor_all": gotodoor_all_table(),
        "families": wl.families_table(3000, seed=71, mix_seed=72),
        "keycorridor": wl.keycorridor_table(3000, seed=81, mix_seed=82),
        "keycorridor_all": keycorridor_all_table(),
    }


def keycorridor_all_table():
    """Every side 7..31 of KeyCorridor with 1..3 rows of rooms, two envs each."""
    side, rows = [], []
    for S in range(7, 32, 3):
        for R in (1, 2, 3):
            side += [S, S]
            rows += [R, R]
    n = len(side)
    fam = np.full(n, wl.FAMILY_KEYCORRIDOR)
    ms = np.array([wl.default_max_steps(int(f), int(s)) for f, s in zip(fam, side)]) // 8 + 1
    return wl.EnvTable(fam.astype(np.uint8), np.array(side, np.uint8), ms.astype(np.int32),
                       np.full(n, 79, np.uint64), np.arange(n, dtype=np.uint32), "keycorridor all sides",
                       np.array(rows, np.uint8))


def gotodoor_all_table():
    """Every side 5..32 of GoToDoor, three envs each."""
    side = np.repeat(np.arange(5, 33), 3)
    n = len(side)
    fam = np.full(n, wl.FAMILY_GOTODOOR)
    ms = np.array([wl.default_max_steps(int(f), int(s)) for f, s in zip(fam, side)]) // 8 + 1
    return wl.EnvTable(fam.astype(np.uint8), side.astype(np.uint8), ms.astype(np.int32),
                       np.full(n, 78, np.uint64), np.arange(n, dtype=np.uint32), "gotodoor all sides")


def all_sides_table():
    fam, side = [], []
    for s in range(4, 33):
        fam.append(0); side.append(s)
    for s in range(5, 33):
        fam.append(1); side.append(s)
    for s in range(7, 32, 2):
        fam.append(2); side.append(s)
    fam, side = np.array(fam * 3), np.array(side * 3)
    ms = np.array([wl.default_max_steps(int(f), int(s)) for f, s in zip(fam, side)]) // 8 + 1
    return wl.EnvTable(fam.astype(np.uint8), side.astype(np.uint8), ms.astype(np.int32),
                       np.full(len(fam), 77, np.uint64), np.arange(len(fam), dtype=np.uint32), "all sides")


def dynobs_all_table():
    """Every side 5..32 of Dynamic-Obstacles with 1..8 balls, two envs each."""
    side, par = [], []
    for S in range(5, 33):
        for n in range(1, min(8, (S - 2) ** 2 - 2) + 1):
            side.append(S); par.append(n)
    side, par = np.array(side * 2), np.array(par * 2)
    ms = np.array([wl.default_max_steps(6, int(s)) for s in side]) // 16 + 1
    return wl.EnvTable(np.full(len(side), 6, np.uint8), side.astype(np.uint8), ms.astype(np.int32),
                       np.full(len(side), 93, np.uint64), np.arange(len(side), dtype=np.uint32),
                       "dynobs all", par.astype(np.uint8))


def lava_all_table():
    """Every valid (side, parameter) of the lava families, three envs each."""
    fam, side, par = [], [], []
    for S in range(5, 33):
        fam.append(3); side.append(S); par.append(0)
    for S in range(5, 32, 2):
        for N in range(1, min(8, S - 3) + 1):
            fam.append(4); side.append(S); par.append(N)
    for S in range(6, 33):
        for k in (1, 2):
            fam.append(5); side.append(S); par.append(k)
    fam, side, par = np.array(fam * 3), np.array(side * 3), np.array(par * 3)
    ms = np.array([wl.default_max_steps(int(f), int(s)) for f, s in zip(fam, side)]) // 16 + 1
    return wl.EnvTable(fam.astype(np.uint8), side.astype(np.uint8), ms.astype(np.int32),
                       np.full(len(fam), 91, np.uint64), np.arange(len(fam), dtype=np.uint32),
                       "lava all", par.astype(np.uint8))


@pytest.mark.parametrize("name", list(tables()))
def test_reset_parity(ge, name):
    table = tables()[name]
    env, first = make(ge, table)
    b, s, ref = P.oracle_reset(table)
    P.assert_rows_equal(first, ref, what=f"reset {name}")
    P.assert_state_equal(env, s, f"reset {name}")


@pytest.mark.parametrize("name,steps", [("empty5", 100), ("empty8", 300), ("tworoom8", 300),
                                        ("fourrooms19", 250), ("mixed", 300), ("all_sides", 200),
                                        ("lava", 300), ("lava_all", 200), ("dynobs", 300),
                                        ("dynobs_all", 150), ("gotodoor", 300),
                                        ("gotodoor_all", 200), ("families", 300),
                                        ("keycorridor", 300), ("keycorridor_all", 200)])
@pytest.mark.parametrize("policy", [False, True])
def test_plain_step_parity(ge, name, steps, policy):
    import torch
    table = tables()[name]
    env, _ = make(ge, table)
    b, s, _ = P.oracle_reset(table)
    acts = wl.random_actions(steps, table.n, seed=11) if not policy else None
    ref = ox.rollout(b, s, steps, acts, nthreads=8)
    traj = ge.Traj.alloc(steps, table.n)
    dacts = torch.from_numpy(acts).cuda() if acts is not None else None
    for k in range(steps):
        row = traj.row(k)
        env.step(row, dacts[k] if dacts is not None else None)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"plain {name}")
    P.assert_state_equal(env, s, f"plain {name}")


@pytest.mark.parametrize("name,steps", [("empty5", 100), ("empty8", 300), ("tworoom8", 300),
                                        ("fourrooms19", 250), ("mixed", 300), ("all_sides", 200),
                                        ("lava", 300), ("lava_all", 200), ("dynobs", 300),
                                        ("dynobs_all", 150), ("gotodoor", 300),
                                        ("gotodoor_all", 200), ("families", 300),
                                        ("keycorridor", 300), ("keycorridor_all", 200)])
@pytest.mark.parametrize("K", [1, 7, 64])
@pytest.mark.parametrize("policy", [False, True])
def test_fused_rollout_parity(ge, name, steps, K, policy):
    import torch
    table = tables()[name]
    env, _ = make(ge, table)
    b, s, _ = P.oracle_reset(table)
    acts = wl.random_actions(steps, table.n, seed=12) if not policy else None
    ref = ox.rollout(b, s, steps, acts, nthreads=8)
    traj = ge.Traj.alloc(steps, table.n)
    env.rollout(steps, traj, torch.from_numpy(acts).cuda() if acts is not None else None, K=K)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"fused {name} K={K}")
    P.assert_state_equal(env, s, f"fused {name} K={K}")


def test_mixed_calls_share_one_counter(ge):
    """Reset, plain steps and fused chunks interleave and still follow the
    oracle's single call counter for the random policy."""
    import torch
    table = wl.mixed_table(700, seed=31, mix_seed=32)
    env, _ = make(ge, table)
    b, s, _ = P.oracle_reset(table)
    plan = [("step", 1), ("roll", 10), ("step", 1), ("step", 1), ("roll", 37), ("roll", 1), ("step", 1)]
    call = 0
    for kind, n in plan:
        ref = ox.rollout(b, s, n, None, nthreads=8)
        traj = ge.Traj.alloc(n, table.n)
        if kind == "step":
            env.step(traj)
        else:
            env.rollout(n, traj, K=5)
        torch.cuda.synchronize()
        P.assert_rows_equal(traj, ref, what=f"{kind} at call {call}")
        call += n
    P.assert_state_equal(env, s, "interleaved")
    assert (env.state_numpy()["calls"] == call).all()


def test_ring_rows_and_zero_steps(ge):
    import torch
    table = wl.uniform_table(130, wl.FAMILY_TWOROOM, 6, seed=2)
    env, _ = make(ge, table)
    b, s, _ = P.oracle_reset(table)
    traj = ge.Traj.alloc(8, table.n)
    env.rollout(0, traj, K=4)
    torch.cuda.synchronize()
    assert int(traj.flags.sum()) == 0
    ref = ox.rollout(b, s, 21, None, rows=8, nthreads=8)
    env.rollout(21, traj, K=4)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what="ring of 8 rows")
    P.assert_state_equal(env, s, "ring")


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 129])
def test_ragged_batches(ge, n):
    import torch
    table = wl.mixed_table(n, seed=n, mix_seed=n + 1)
    env, first = make(ge, table)
    b, s, ref0 = P.oracle_reset(table)
    P.assert_rows_equal(first, ref0, what=f"reset n={n}")
    ref = ox.rollout(b, s, 40, None, nthreads=8)
    traj = ge.Traj.alloc(40, n)
    env.rollout(40, traj, K=16)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"n={n}")
    P.assert_state_equal(env, s, f"n={n}")


def test_unit_reward_mode(ge):
    import torch
    table = wl.uniform_table(256, wl.FAMILY_EMPTY, 5, seed=9)
    env, _ = make(ge, table, reward_mode=1)
    b, s, _ = P.oracle_reset(table, reward_mode=1)
    ref = ox.rollout(b, s, 200, None, nthreads=8)
    traj = ge.Traj.alloc(200, table.n)
    env.rollout(200, traj, K=32)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what="unit reward")
    assert set(np.unique(ref.reward)) <= {0.0, 1.0} and (ref.reward == 1.0).any()


def test_observations_skipped_when_null(ge):
    import torch
    table = wl.mixed_table(500, seed=4, mix_seed=5)
    env, _ = make(ge, table)
    b, s, _ = P.oracle_reset(table)
    ref = ox.rollout(b, s, 50, None, nthreads=8)
    traj = ge.Traj.alloc(50, table.n, with_obs=False)
    env.rollout(30, traj, K=8)
    row = ge.Traj(None, traj.reward[30:31], traj.flags[30:31], traj.action[30:31], traj.mission[30:31])
    env.step(row)
    env.rollout(19, ge.Traj(None, traj.reward[31:], traj.flags[31:], traj.action[31:], traj.mission[31:]), K=8)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what="no obs")
    P.assert_state_equal(env, s, "no obs")


def test_step_before_reset_is_an_error(ge):
    table = wl.uniform_table(8, wl.FAMILY_EMPTY, 5)
    env = ge.GridEnv(table)
    traj = ge.Traj.alloc(1, 8)
    with pytest.raises(ge.GridEnvError) as ei:
        env.step(traj)
    assert ei.value.status == ge.GX_ESTATE
    with pytest.raises(ge.GridEnvError):
        env.rollout(3, traj)


def test_buffers_too_small_or_mistyped_are_refused(ge):
    """Actions and outputs are checked against the batch before a launch:
    a refused call enqueues nothing, and the state carries on as if it had
    not been made."""
    import torch
    table = wl.uniform_table(70, wl.FAMILY_TWOROOM, 6, seed=4)
    env, _ = make(ge, table)
    b, s, _ = P.oracle_reset(table)
    acts = wl.random_actions(6, table.n, seed=9)
    d = torch.from_numpy(acts).cuda()
    traj = ge.Traj.alloc(6, table.n)
    with pytest.raises(ValueError):
        env.rollout(6, traj, d.long(), K=4)                   # int64 actions
    with pytest.raises(ValueError):
        env.rollout(7, traj, d, K=4)                          # 6 rows of actions for 7 steps
    with pytest.raises(ValueError):
        env.step(traj.row(0), d[0, :69])                      # one env short
    with pytest.raises(ValueError):
        env.rollout(6, ge.Traj.alloc(6, table.n - 1), d, K=4)   # outputs for a smaller batch
    with pytest.raises(ValueError):
        env.rollout(6, ge.Traj.alloc(6, table.n, device="cpu"), d, K=4)   # host outputs
    env.rollout(6, traj, d, K=4)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ox.rollout(b, s, 6, acts, nthreads=8), what="after refused calls")
    P.assert_state_equal(env, s, "after refused calls")


def test_rollouts_are_deterministic(ge):
    import torch
    table = wl.mixed_table(4096, seed=1, mix_seed=2)
    outs = []
    for _ in range(2):
        env, _ = make(ge, table)
        traj = ge.Traj.alloc(64, table.n)
        env.rollout(200, traj, K=50)
        torch.cuda.synchronize()
        outs.append((P.to_np(traj.obs).copy(), P.to_np(traj.flags).copy(), env.state_numpy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    for f in P.FIELDS:
        np.testing.assert_array_equal(outs[0][2][f], outs[1][2][f])


def test_crossings_layouts_many_seeds(ge):
    """Reset of 20000 Crossings envs over every valid (side, rivers), each
    with its own seed: grids, poses and first observations equal the
    oracle's (the device shuffle and path draws are the oracle's)."""
    rng = np.random.default_rng(5)
    combos = [(S, N) for S in range(5, 32, 2) for N in range(1, min(8, S - 3) + 1)]
    pick = np.array(combos)[rng.integers(0, len(combos), 20000)]
    n = len(pick)
    table = wl.EnvTable(np.full(n, 4, np.uint8), pick[:, 0].astype(np.uint8),
                        np.full(n, 50, np.int32), rng.integers(0, 2 ** 63, n).astype(np.uint64),
                        np.arange(n, dtype=np.uint32), "crossings seeds", pick[:, 1].astype(np.uint8))
    env, first = make(ge, table)
    b, s, ref = P.oracle_reset(table)
    P.assert_rows_equal(first, ref, what="crossings reset")
    P.assert_state_equal(env, s, "crossings reset")


def test_unit_reward_mode_lava(ge):
    import torch
    table = wl.lava_table(2048, seed=17, mix_seed=18)
    env, _ = make(ge, table, reward_mode=1)
    b, s, _ = P.oracle_reset(table, reward_mode=1)
    ref = ox.rollout(b, s, 200, None, nthreads=8)
    traj = ge.Traj.alloc(200, table.n)
    env.rollout(200, traj, K=32)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what="unit reward, lava")
    assert set(np.unique(ref.reward)) == {-1.0, 0.0, 1.0}


@pytest.mark.parametrize("name", ["mixed", "lava", "dynobs", "all_sides"])
@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_categorical_observation_parity(ge, name, kernel):
    """categorical_first_person records (49 bytes) through both kernels."""
    import torch
    table = tables()[name]
    env = ge.GridEnv(table, obs_mode=1)
    first = ge.Traj.alloc(1, table.n, obs_mode=1)
    env.reset(first)
    b, s, ref0 = P.oracle_reset(table, obs_mode=1)
    P.assert_rows_equal(first, ref0, what=f"categorical reset {name}")
    steps = 120
    ref = ox.rollout(b, s, steps, None, nthreads=8)
    traj = ge.Traj.alloc(steps, table.n, obs_mode=1)
    if kernel == "fused":
        env.rollout(steps, traj, K=32)
    else:
        for k in range(steps):
            env.step(traj.row(k))
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"categorical {kernel} {name}")
    P.assert_state_equal(env, s, f"categorical {kernel} {name}")


@pytest.mark.parametrize("n", [1, 63, 65, 130])
def test_categorical_ragged(ge, n):
    import torch
    table = wl.mixed_table(n, seed=n + 7, mix_seed=n + 8)
    env = ge.GridEnv(table, obs_mode=1)
    env.reset(ge.Traj.alloc(1, n, obs_mode=1))
    b, s, _ = P.oracle_reset(table, obs_mode=1)
    ref = ox.rollout(b, s, 30, None, nthreads=8)
    traj = ge.Traj.alloc(30, n, obs_mode=1)
    env.rollout(30, traj, K=8)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"categorical n={n}")


@pytest.mark.parametrize("name", ["mixed", "all_sides", "lava", "dynobs_all"])
@pytest.mark.parametrize("kernel", ["plain", "fused"])
@pytest.mark.parametrize("mode", [2, 3])
def test_whole_grid_observation_parity(ge, name, kernel, mode):
    """symbolic (2) and categorical (3) whole-grid records through both
    kernels; each output row starts at a different alignment, so the
    records' unaligned edges are exercised on every row."""
    import torch
    table = tables()[name]
    env = ge.GridEnv(table, obs_mode=mode)
    first = env.traj(1)
    env.reset(first)
    b, s, ref0 = P.oracle_reset(table, obs_mode=mode)
    assert env.info()["obs_row_bytes"] == b.obs_row_bytes()
    P.assert_rows_equal(first, ref0, what=f"grid mode {mode} reset {name}")
    steps = 60
    ref = ox.rollout(b, s, steps, None, nthreads=8)
    traj = env.traj(steps)
    if kernel == "fused":
        env.rollout(steps, traj, K=16)
    else:
        for k in range(steps):
            env.step(traj.row(k))
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"grid mode {mode} {kernel} {name}")
    P.assert_state_equal(env, s, f"grid mode {mode} {kernel} {name}")


@pytest.mark.parametrize("n", [1, 63, 65, 130])
@pytest.mark.parametrize("mode", [2, 3])
def test_whole_grid_ragged_and_ring(ge, n, mode):
    """Ragged batches, and a ring of 7 rows that the 30 steps wrap around
    (launches of K = 8 start mid-ring)."""
    import torch
    table = wl.mixed_table(n, seed=n + 9, mix_seed=n + 10)
    env = ge.GridEnv(table, obs_mode=mode)
    env.reset(env.traj(1))
    b, s, _ = P.oracle_reset(table, obs_mode=mode)
    ref = ox.rollout(b, s, 30, None, rows=7, nthreads=8)
    traj = env.traj(7)
    env.rollout(30, traj, K=8)
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"grid mode {mode} n={n}")


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_gotodoor_done_and_out_of_range_actions(ge, kernel):
    """External actions biased to done, toggle and values >= 7, so that
    on_door_done, toggles of doors on the grid's outer ring (whose view the
    fused kernel reads bounds-checked) and out-of-range actions all occur."""
    import torch
    table = tables()["gotodoor"]
    env, first = make(ge, table)
    b, s, ref0 = P.oracle_reset(table)
    rng = np.random.default_rng(5)
    steps = 200
    acts = rng.choice(np.array([0, 1, 2, 2, 5, 6, 6, 7, 200], np.uint8), size=(steps, table.n))
    ref = ox.rollout(b, s, steps, acts, nthreads=8)
    assert (ref.flags & 1).sum() > 1000 and (ref.reward > 0).sum() > 100
    traj = ge.Traj.alloc(steps, table.n)
    dacts = torch.from_numpy(acts).cuda()
    if kernel == "fused":
        env.rollout(steps, traj, dacts, K=32)
    else:
        for k in range(steps):
            env.step(traj.row(k), dacts[k])
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"gotodoor {kernel}")
    P.assert_state_equal(env, s, f"gotodoor {kernel}")


def largest_tiles_table():
    """Three tiles: 64 envs of side 32 (the largest LDS a tile can take,
    64 KiB of codes), 64 of side 31 (the families that need an odd side),
    and a ragged tile of 5 more of side 32; every family and parameter
    range that those sides allow."""
    big = ([(wl.FAMILY_EMPTY, 32, 0), (wl.FAMILY_TWOROOM, 32, 0), (wl.FAMILY_LAVAGAP, 32, 0),
            (wl.FAMILY_DISTSHIFT, 32, 1), (wl.FAMILY_DISTSHIFT, 32, 2), (wl.FAMILY_GOTODOOR, 32, 0)] +
           [(wl.FAMILY_DYNOBS, 32, k) for k in range(1, 9)])
    odd = ([(wl.FAMILY_FOURROOMS, 31, 0)] + [(wl.FAMILY_CROSSINGS, 31, k) for k in range(1, 9)] +
           [(wl.FAMILY_KEYCORRIDOR, 31, r) for r in (1, 2, 3)])
    tasks = [big[i % len(big)] for i in range(64)] + [odd[i % len(odd)] for i in range(64)] + big[:5]
    fam, side, par = (np.array(c, np.uint8) for c in zip(*tasks))
    n = len(tasks)
    ms = np.array([wl.default_max_steps(int(f), int(s)) for f, s in zip(fam, side)], np.int32)
    return wl.EnvTable(fam, side, ms, np.full(n, 61, np.uint64), np.arange(n, dtype=np.uint32),
                       "largest tiles", par)


@pytest.mark.parametrize("kernel", ["fused", "plain"])
@pytest.mark.parametrize("mode", [0, 2])
def test_largest_tiles(ge, kernel, mode):
    """Tiles at the LDS limit (the fused kernel stages 64 grids of side 32)
    and side-31 grids of every odd-side family, first-person and whole-grid
    records, through both kernels: every record and the state equal the
    oracle's."""
    import torch
    table = largest_tiles_table()
    env = ge.GridEnv(table, obs_mode=mode)
    info = env.info()
    assert info["n_tiles"] == 3 and info["max_tile_cells"] == 64 * 32 * 32
    first = env.traj(1)
    env.reset(first)
    b, s, ref0 = P.oracle_reset(table, obs_mode=mode)
    steps = 60
    traj = env.traj(steps)
    if kernel == "fused":
        env.rollout(steps, traj, K=16)
    else:
        for k in range(steps):
            env.step(traj.row(k))
    ref = ox.rollout(b, s, steps, None, nthreads=8)
    torch.cuda.synchronize()
    P.assert_rows_equal(first, ref0, what=f"reset, largest tiles, mode {mode}")
    P.assert_rows_equal(traj, ref, what=f"{kernel}, largest tiles, mode {mode}")
    P.assert_state_equal(env, s, f"{kernel}, largest tiles")
    env.close()


@pytest.mark.parametrize("blocks", [1, 3])
@pytest.mark.parametrize("tile_envs,mode", [(64, 0), (16, 0), (64, 2)])
def test_persistent_workgroups_many_tiles_each(ge, blocks, tile_envs, mode):
    """Far fewer workgroups than tiles: each workgroup runs many tiles in
    turn, so whatever one tile leaves in LDS (codes, the record stage, the
    write-back's line bitmap, the per-lane cell-written flags) must not leak
    into the next; every family, resets, pickups, toggles and moving balls,
    launches of a few steps and a partial last one."""
    import torch
    table = wl.families_table(700, seed=95, mix_seed=96)
    env = ge.GridEnv(table, obs_mode=mode)
    env.set_tiling(tile_envs)
    env.set_launch(6, blocks)
    assert env.info()["blocks"] == blocks and env.info()["n_tiles"] >= 3 * blocks
    first = env.traj(1)
    env.reset(first)
    b, s, ref0 = P.oracle_reset(table, obs_mode=mode)
    steps = 40
    traj = env.traj(steps)
    env.rollout(steps, traj)
    ref = ox.rollout(b, s, steps, None, nthreads=8)
    torch.cuda.synchronize()
    assert (ref.flags & 4).sum() > 100      # resets happen inside the launches
    P.assert_rows_equal(traj, ref, what=f"{blocks} workgroups, tiles of {tile_envs}, mode {mode}")
    P.assert_state_equal(env, s, f"{blocks} workgroups, tiles of {tile_envs}")
    env.close()


@pytest.mark.parametrize("tile_envs", [1, 13, 16, 32, 48])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_tiling_parity(ge, tile_envs, mode):
    """Tiles of fewer envs than a wave's lanes (env_set_tiling) change only
    how envs map onto waves: every output and the state still equal the
    oracle's, for each record kind, with ragged last tiles and tile sizes
    whose records are not 16-byte aligned."""
    import torch
    table = wl.families_table(1000, seed=91, mix_seed=92)
    env = ge.GridEnv(table, obs_mode=mode)
    env.set_tiling(tile_envs)
    info = env.info()
    assert info["tile_envs"] == tile_envs and info["n_tiles"] == -(-table.n // tile_envs)
    first = env.traj(1)
    env.reset(first)
    b, s, ref0 = P.oracle_reset(table, obs_mode=mode)
    steps = 30
    traj = env.traj(steps)
    env.rollout(steps, traj, K=7)
    ref = ox.rollout(b, s, steps, None, nthreads=8)
    torch.cuda.synchronize()
    P.assert_rows_equal(first, ref0, what=f"reset, tiles of {tile_envs}")
    P.assert_rows_equal(traj, ref, what=f"rollout, tiles of {tile_envs}, mode {mode}")
    P.assert_state_equal(env, s, f"tiles of {tile_envs}")
    env.close()
