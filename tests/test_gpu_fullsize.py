"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the small workloads compared whole, the large ones on a
strided sample of envs whose every record and final state the oracle
recomputes env by env (envs are independent, so a subset is exact)."""
import numpy as np
import pytest

import oracle as ox
import parity as P
from paper_2407_19396_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ge():
    from paper_2407_19396_amd import gridenv as ge
    return ge


@pytest.mark.parametrize("seed", range(5))
def test_empty5_plain_whole(seed):
    """16 single rooms 5x5, 100 plain steps of external random actions."""
    import torch
    ge = _ge()
    table = wl.workload_empty5(seed)
    acts = wl.random_actions(100, table.n, seed)
    env = ge.GridEnv(table)
    first = ge.Traj.alloc(1, table.n)
    env.reset(first)
    b, s, ref0 = P.oracle_reset(table)
    P.assert_rows_equal(first, ref0)
    ref = ox.rollout(b, s, 100, acts)
    traj = ge.Traj.alloc(100, table.n)
    d = torch.from_numpy(acts).cuda()
    for k in range(100):
        env.step(traj.row(k), d[k])
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"empty5 seed {seed}")
    P.assert_state_equal(env, s)


def test_empty8_plain_whole():
    """4096 single rooms 8x8, 1000 plain steps, one launch per step."""
    import torch
    ge = _ge()
    table = wl.workload_empty8(0)
    acts = wl.random_actions(1000, table.n, 0)
    env = ge.GridEnv(table)
    env.reset()
    b, s, _ = P.oracle_reset(table)
    ref = ox.rollout(b, s, 1000, acts, nthreads=16)
    traj = ge.Traj.alloc(1000, table.n)
    d = torch.from_numpy(acts).cuda()
    for k in range(1000):
        env.step(traj.row(k), d[k])
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what="empty8")
    P.assert_state_equal(env, s)


def sampled_run(table, n_steps, K, sample, blocks=0, tile_envs=0, calls=None):
    """Fused rollout of the whole table in calls of at most K steps (the
    bench's launch shape), or in calls of the given step counts; returns
    sampled records and the final state."""
    import torch
    ge = _ge()
    env = ge.GridEnv(table)
    if tile_envs:
        env.set_tiling(tile_envs)
    if blocks:
        env.set_launch(K, blocks)
    env.reset()
    traj = ge.Traj.alloc(K, table.n)
    idx = torch.from_numpy(sample).cuda()
    obs, rew, flg, act = [], [], [], []
    if calls is None:
        calls = [min(K, n_steps - c) for c in range(0, n_steps, K)]
    assert sum(calls) == n_steps and max(calls) <= K
    for k in calls:
        env.rollout(k, traj, K=K)
        obs.append(traj.obs[:k, idx].cpu())
        rew.append(traj.reward[:k, idx].cpu())
        flg.append(traj.flags[:k, idx].cpu())
        act.append(traj.action[:k, idx].cpu())
    torch.cuda.synchronize()
    cat = lambda xs: torch.cat(xs).numpy()  # noqa: E731
    st = env.state_numpy()
    env.close()
    return cat(obs), cat(rew), cat(flg), cat(act), st


def check_sample(table, n_steps, K, stride, blocks=0, tile_envs=0, calls=None, expect_resets=True):
    sample = np.arange(0, table.n, stride)
    obs, rew, flg, act, st = sampled_run(table, n_steps, K, sample, blocks, tile_envs, calls)
    sub = table.subset(sample)
    b, s, _ = P.oracle_reset(sub)
    ref = ox.rollout(b, s, n_steps, None, nthreads=16)
    np.testing.assert_array_equal(flg, ref.flags)
    np.testing.assert_array_equal(act, ref.action)
    np.testing.assert_array_equal(rew.view(np.uint32), ref.reward.view(np.uint32))
    np.testing.assert_array_equal(obs, ref.obs)
    for f in ("x", "y", "dir", "t", "carry", "done_prev"):
        np.testing.assert_array_equal(st[f][sample], getattr(s, f))
    np.testing.assert_array_equal(st["episode"][sample], s.episode)
    offs = np.concatenate([[0], np.cumsum(3 * table.side.astype(np.int64) ** 2)])
    for j, i in enumerate(sample):
        so = P.ox_batch(sub).grid_offsets()[j]
        n3 = 3 * int(table.side[i]) ** 2
        np.testing.assert_array_equal(st["grid"][offs[i]:offs[i] + n3], s.grid[so:so + n3])
    # every env (not only the sample): agents stay inside, counters in range
    assert ((st["t"] >= 0) & (st["t"] <= table.max_steps)).all()
    assert ((st["x"] >= 1) & (st["x"] <= table.side.astype(np.int32) - 2)).all()
    assert ((st["y"] >= 1) & (st["y"] <= table.side.astype(np.int32) - 2)).all()
    if expect_resets:
        assert (st["episode"] > 0).any()


@pytest.mark.parametrize("K,blocks", [(1024, 1024), (64, 0)])
def test_tworoom8_fused_sampled(K, blocks):
    """65536 two-room 8x8 layouts, 2048 steps, fused, random policy, in the
    shape the benchmark's tuner picks (K = 1024, one workgroup per tile) and
    in short launches."""
    check_sample(wl.workload_tworoom8(0), 2048, K, stride=257, blocks=blocks)


@pytest.mark.parametrize("K,blocks", [(1024, 2048), (64, 0)])
def test_mixed_fused_sampled(K, blocks):
    """262144 mixed-size envs, 4096 steps, fused persistent launches, in the
    benchmark's shape (K = 1024, 2048 workgroups: two tiles each) and in
    short launches."""
    check_sample(wl.workload_mixed(0), 4096, K, stride=683, blocks=blocks)


@pytest.mark.parametrize("blocks", [2048, 4096])
def test_mixed_short_run_shape_sampled(blocks):
    """The benchmark's short run (`--steps 20 --warmup 5`): 5 warm-up
    steps, then 20 steps, each one fused launch of the 262144-env mix in the
    shapes the tuner picks from (K = 1024; 2048 persistent workgroups of two
    tiles each, or one workgroup per tile), split as the benchmark splits
    them."""
    check_sample(wl.workload_mixed(0), 25, 1024, stride=683, blocks=blocks, calls=[5, 20])


@pytest.mark.parametrize("family,side", [(wl.FAMILY_EMPTY, 32), (wl.FAMILY_TWOROOM, 32), (wl.FAMILY_EMPTY, 24)])
def test_large_grids_in_tiles_of_32(family, side):
    """65536 envs of side 24 or 32 in the tiling the tuner picks for them
    (32 envs per tile, four workgroups per compute unit), 1024 steps (far
    fewer than T = 4S^2 or 10S^2, so episodes end only at a goal, which the
    random policy may never reach)."""
    check_sample(wl.uniform_table(65536, family, side, seed=3), 1024, 1024, stride=257, blocks=1024, tile_envs=32,
                 expect_resets=False)
