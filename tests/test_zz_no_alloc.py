"""env_rollout_static, the entry point for callers that cannot allocate:
its results equal env_create + env_reset + env_rollout bit for bit, on
consecutive calls whose batches shrink (the second call's tables overwrite
part of the first's in the shared device array), on a continuation without
reset, and in the whole-grid observation mode; oversized batches and the
rgb modes are refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle as ox
import parity as P
from paper_2407_19396_amd import gridenv as ge
from paper_2407_19396_amd import workloads as wl


class Bufs:
    """A state and output rows in device tensors, with no context behind them."""

    def __init__(self, table, rows, obs_mode=0):
        import torch
        n = table.n
        grid_bytes = int(np.sum(3 * table.side.astype(np.int64) ** 2))
        z = lambda dt: torch.zeros(n, dtype=dt, device="cuda")   # noqa: E731
        self.grid = torch.zeros(grid_bytes, dtype=torch.uint8, device="cuda")
        self.x, self.y, self.dir, self.t, self.carry = (z(torch.int32) for _ in range(5))
        self.episode, self.calls = z(torch.int32), z(torch.int32)
        self.done_prev = z(torch.uint8)
        self.obst = torch.full((n * 16,), 0xFF, dtype=torch.uint8, device="cuda")
        row_bytes = {2: grid_bytes, 3: grid_bytes // 3}.get(obs_mode, 0)
        self.first = ge.Traj.alloc(1, n, obs_mode=obs_mode, row_bytes=row_bytes)
        self.traj = ge.Traj.alloc(rows, n, obs_mode=obs_mode, row_bytes=row_bytes)

    def state(self):
        return ge.GxState(*[getattr(self, f).data_ptr() for f in ge.STATE_FIELDS])

    def state_numpy(self):
        return {f: getattr(self, f).cpu().numpy() for f in ge.STATE_FIELDS}


def same_traj(a, b, what):
    for f in ("obs", "reward", "flags", "action", "mission"):
        np.testing.assert_array_equal(P.to_np(getattr(a, f)), P.to_np(getattr(b, f)), err_msg=f"{what}: {f}")


def same_state(env, bufs, what):
    g, s = env.state_numpy(), bufs.state_numpy()
    for f in ge.STATE_FIELDS:
        np.testing.assert_array_equal(g[f].view(np.uint8), s[f].view(np.uint8), err_msg=f"{what}: state {f}")


def run_pair(table, steps, rows, K, obs_mode=0, actions=None):
    """The same reset + rollout through both entry points; returns both."""
    import torch
    env = ge.GridEnv(table, obs_mode=obs_mode)
    first = env.traj(1)
    env.reset(first)
    traj = env.traj(rows)
    act = None if actions is None else torch.from_numpy(actions).to("cuda")
    env.rollout(steps, traj, actions=act, K=K)
    b = Bufs(table, rows, obs_mode)
    ge.env_rollout_static(table, b.state(), True, b.first.c(), steps,
                          act.data_ptr() if act is not None else None, b.traj.c(), K, obs_mode=obs_mode)
    torch.cuda.synchronize()
    same_traj(first, b.first, "reset")
    same_traj(traj, b.traj, "rollout")
    same_state(env, b, "end state")
    return env, b


@pytest.mark.gpu
def test_static_equals_context_on_two_calls_the_second_smaller():
    import torch
    torch.cuda.set_device(0)
    big = wl.families_table(1500, seed=31, mix_seed=32)       # every family, 24 tiles
    env1, b1 = run_pair(big, 70, 32, 16)
    small = wl.families_table(150, seed=33, mix_seed=34)      # 3 tiles, the last ragged
    env2, b2 = run_pair(small, 45, 45, 0)                     # K = 0: 64 steps per launch
    # the second call's outputs also match the oracle
    bo, so, ref0 = P.oracle_reset(small)
    ref = ox.rollout(bo, so, 45, None, nthreads=8)
    P.assert_rows_equal(b2.first, ref0, what="static reset vs oracle")
    P.assert_rows_equal(b2.traj, ref, what="static rollout vs oracle")
    # a continuation of the small batch without reset, external actions
    acts = wl.random_actions(20, small.n, seed=5)
    a = torch.from_numpy(acts).to("cuda")
    t_ctx = env2.traj(20)
    env2.rollout(20, t_ctx, actions=a, K=8)
    ge.env_rollout_static(small, b2.state(), False, None, 20, a.data_ptr(), b2.traj.c(), 8)
    torch.cuda.synchronize()
    same_traj(t_ctx, ge.Traj(b2.traj.obs[:20], b2.traj.reward[:20], b2.traj.flags[:20],
                             b2.traj.action[:20], b2.traj.mission[:20]), "continuation")
    same_state(env2, b2, "continuation end state")
    env1.close()
    env2.close()


@pytest.mark.gpu
def test_static_whole_grid_records():
    import torch
    torch.cuda.set_device(0)
    table = wl.families_table(200, seed=41, mix_seed=42)
    env, b = run_pair(table, 12, 12, 5, obs_mode=2)
    env.close()
    env, b = run_pair(table.subset(np.arange(0, 200, 3)), 9, 9, 4, obs_mode=3)
    env.close()


def test_static_refuses_oversized_and_rgb_batches():
    n = ge.GX_STATIC_MAX_ENVS + 1
    fam = np.zeros(n, np.uint8)
    side = np.full(n, 5, np.uint8)
    ms = np.full(n, 100, np.int32)
    cfg = ge.GxConfig(n, 0, 0, fam.ctypes.data, side.ctypes.data, None, ms.ctypes.data, None, 0, None,
                      None)
    fake = ge.GxState(*([16] * len(ge.STATE_FIELDS)))      # never dereferenced: validation fails first
    tr = ge.GxTraj(16, 16, 16, 16, 1, None)
    L = ge.load()
    rc = L.env_rollout_static(ctypes.byref(cfg), ctypes.byref(fake), 1, None, 1, None, ctypes.byref(tr), 0,
                              None)
    assert rc == ge.GX_ESIZE
    assert "GX_STATIC_MAX_ENVS" in ge.env_strerror(rc)
    cfg.n_envs = 4
    cfg.obs_mode = 4
    rc = L.env_rollout_static(ctypes.byref(cfg), ctypes.byref(fake), 1, None, 1, None, ctypes.byref(tr), 0,
                              None)
    assert rc == ge.GX_EINVAL
