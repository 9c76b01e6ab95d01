"""HIP graph capture of env_rollout (it allocates and synchronises
nothing): every replay, with eager work and synchronisations in between,
equals the same rollout run eagerly and the oracle's rollout continued by
the same number of steps."""
import numpy as np
import pytest

import oracle as ox
import parity as P
from paper_2407_19396_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K", [16, 64])
def test_graph_replays_match_eager(K):
    import torch
    from paper_2407_19396_amd import gridenv as ge
    table = wl.mixed_table(3000, seed=3, mix_seed=4)
    eager = ge.GridEnv(table)
    eager.reset()
    tr_e = ge.Traj.alloc(K, table.n)
    graph = ge.GridEnv(table)
    graph.reset()
    tr_g = ge.Traj.alloc(K, table.n)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graph.rollout(K, tr_g, K=K)
    noise = torch.zeros(1 << 20, device="cuda")
    b, s, _ = P.oracle_reset(table)
    for replay in range(4):
        eager.rollout(K, tr_e, K=K)
        g.replay()
        noise.add_(1.0)                      # eager work between replays
        torch.cuda.synchronize()
        for f in ("obs", "reward", "flags", "action"):
            np.testing.assert_array_equal(P.to_np(getattr(tr_g, f)), P.to_np(getattr(tr_e, f)),
                                          err_msg=f"replay {replay}: {f}")
        se, sg = eager.state_numpy(), graph.state_numpy()
        for f in P.FIELDS:
            np.testing.assert_array_equal(sg[f], se[f], err_msg=f"replay {replay}: state {f}")
        ref = ox.rollout(b, s, K, None, nthreads=16)
        P.assert_rows_equal(tr_g, ref, what=f"replay {replay} vs oracle")
        P.assert_state_equal(graph, s, what=f"replay {replay} vs oracle")
    assert (eager.state_numpy()["calls"] == 4 * K).all()


def test_graph_tworoom8_full_size_against_oracle():
    """The TwoRoom 8x8 workload at full size (65536 envs), its 2048-step
    random-policy rollout captured whole (launches of 512 steps into a
    ring of 512 rows) and replayed twice: after each replay every 64th env's
    records of the last 512 steps and its state equal the oracle's."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    table = wl.workload_tworoom8(seed=0)
    K, steps = 512, 2048
    env = ge.GridEnv(table)
    env.reset()
    traj = env.traj(K)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        env.rollout(steps, traj, K=K)
    pick = np.arange(0, table.n, 64)
    sub = table.subset(pick)
    b, s, _ = P.oracle_reset(sub)
    for replay in range(2):
        g.replay()
        torch.cuda.synchronize()
        ref = ox.rollout(b, s, steps, None, rows=K, nthreads=16)
        view = ge.Traj(traj.obs[:, pick], traj.reward[:, pick], traj.flags[:, pick], traj.action[:, pick])
        P.assert_rows_equal(view, ref, what=f"replay {replay}")
        st = env.state_numpy()
        for f in ("x", "y", "dir", "t", "carry", "episode", "done_prev", "calls"):
            r = getattr(s, f)
            a = st[f][pick]
            a = a.view(r.dtype) if a.dtype.itemsize == r.dtype.itemsize else a.astype(r.dtype)
            np.testing.assert_array_equal(a, r, err_msg=f"replay {replay}: state {f}")
    env.close()


@pytest.mark.parametrize("mode", [4, 5])
def test_rgb_graph_replays_match_eager(mode):
    """The rgb path (fused launches, index passes and draws, no allocation)
    captured whole: every replay equals the eager rollout."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    table = wl.mixed_table(200, seed=5, mix_seed=6)
    sprites = np.random.default_rng(mode).integers(0, 256, (264, 32, 32, 3), dtype=np.uint8)
    eager = ge.GridEnv(table, obs_mode=mode, sprites=sprites)
    eager.reset()
    tr_e = eager.traj(6)
    graph = ge.GridEnv(table, obs_mode=mode, sprites=sprites)
    graph.reset()
    tr_g = graph.traj(6)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graph.rollout(10, tr_g, K=4)         # three fused launches, the ring wrapped
    noise = torch.zeros(1 << 20, device="cuda")
    for replay in range(3):
        eager.rollout(10, tr_e, K=4)
        g.replay()
        noise.add_(1.0)
        torch.cuda.synchronize()
        for f in ("obs", "reward", "flags", "action", "mission"):
            np.testing.assert_array_equal(P.to_np(getattr(tr_g, f)), P.to_np(getattr(tr_e, f)),
                                          err_msg=f"replay {replay}: {f}")
        se, sg = eager.state_numpy(), graph.state_numpy()
        for f in P.FIELDS:
            np.testing.assert_array_equal(sg[f], se[f], err_msg=f"replay {replay}: state {f}")
