"""Parity on injected states that random rollouts rarely reach: closed and
open doors, keys of every colour (matching or not) in hand or on the
floor, several doors and keys, agents next to goals, and so on.  The state
buffers belong to the caller, so both sides start from the same picture."""
import numpy as np
import pytest

import oracle as ox
import parity as P
from paper_2407_19396_amd import workloads as wl

pytestmark = pytest.mark.gpu


def random_state(rng, S):
    g = np.zeros((S, S, 3), np.uint8)
    g[:, :] = (1, 0, 0)
    for y in range(1, S - 1):
        for x in range(1, S - 1):
            u = rng.random()
            c = int(rng.integers(0, 6))
            if u < 0.15:
                g[y, x] = (2, 5, 0)
            elif u < 0.25:
                g[y, x] = (4, c, int(rng.integers(0, 3)))
            elif u < 0.35:
                g[y, x] = (5, c, 0)
            elif u < 0.38:
                g[y, x] = (8, 1, 0)
    g[0, :] = g[-1, :] = g[:, 0] = g[:, -1] = (2, 5, 0)
    free = [(x, y) for y in range(1, S - 1) for x in range(1, S - 1) if g[y, x, 0] == 1]
    x, y = free[int(rng.integers(0, len(free)))]
    carry = 1 if rng.random() < 0.5 else (5 | (int(rng.integers(0, 6)) << 8))
    return g, x, y, int(rng.integers(0, 4)), carry


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_injected_state_parity(seed, kernel):
    import torch
    from paper_2407_19396_amd import gridenv as ge
    rng = np.random.default_rng(seed)
    n = 2000
    fam = rng.choice([0, 1], n).astype(np.uint8)
    side = rng.choice([5, 6, 8, 11, 16], n).astype(np.uint8)
    T = rng.integers(5, 60, n).astype(np.int32)
    table = wl.EnvTable(fam, side, T, np.full(n, 1234 + seed, np.uint64), np.arange(n, dtype=np.uint32))
    grids, xs, ys, ds, cs = [], [], [], [], []
    for i in range(n):
        g, x, y, d, c = random_state(rng, int(side[i]))
        grids.append(g.reshape(-1)); xs.append(x); ys.append(y); ds.append(d); cs.append(c)
    st = dict(grid=np.concatenate(grids), x=np.array(xs, np.int32), y=np.array(ys, np.int32),
              dir=np.array(ds, np.int32), t=rng.integers(0, 5, n).astype(np.int32),
              carry=np.array(cs, np.int32), episode=rng.integers(0, 9, n).astype(np.uint32),
              done_prev=np.zeros(n, np.uint8))
    steps = 80
    acts = wl.random_actions(steps, n, seed=seed + 100)
    b = P.ox_batch(table)
    s = ox.State(**{k: v.copy() for k, v in st.items()})
    ref = ox.rollout(b, s, steps, acts, nthreads=16)
    env = ge.GridEnv(table)
    env.reset()
    env.load_state(st)
    traj = ge.Traj.alloc(steps, n)
    dacts = torch.from_numpy(acts).cuda()
    if kernel == "fused":
        env.rollout(steps, traj, dacts, K=13)
    else:
        for k in range(steps):
            env.step(traj.row(k), dacts[k])
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"injected seed {seed} {kernel}")
    P.assert_state_equal(env, s, f"injected seed {seed} {kernel}")
    env.close()


def random_dynobs_state(rng, S, n):
    """A Dynamic-Obstacles state: n balls on random empty interior cells, in
    a random list order, some walls, the goal, the agent anywhere free."""
    g = np.zeros((S, S, 3), np.uint8)
    g[:, :] = (1, 0, 0)
    for y in range(1, S - 1):
        for x in range(1, S - 1):
            if rng.random() < 0.12:
                g[y, x] = (2, 5, 0)
    g[0, :] = g[-1, :] = g[:, 0] = g[:, -1] = (2, 5, 0)
    g[S - 2, S - 2] = (8, 1, 0)
    free = [(x, y) for y in range(1, S - 1) for x in range(1, S - 1) if g[y, x, 0] == 1]
    n = min(n, len(free) - 1)         # the list must hold exactly the balls on the grid
    pick = rng.permutation(len(free))[:n + 1]
    ax, ay = free[pick[0]]
    ob = np.full(16, 0xFF, np.uint8)
    for b, i in enumerate(pick[1:]):
        bx, by = free[i]
        g[by, bx] = (6, 2, 0)
        ob[2 * b], ob[2 * b + 1] = bx, by
    return g, ax, ay, int(rng.integers(0, 4)), ob, n


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_injected_dynobs_parity(seed, kernel):
    """Crowded Dynamic-Obstacles states (balls next to each other, to walls
    and to the agent, in random list order) under random actions 0..6."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    rng = np.random.default_rng(100 + seed)
    n = 1500
    side = rng.choice([5, 6, 7, 9, 16], n).astype(np.uint8)
    nb = np.array([rng.integers(1, min(8, (int(s) - 2) ** 2 - 2) + 1) for s in side], np.uint8)
    T = rng.integers(5, 60, n).astype(np.int32)
    parts = [random_dynobs_state(rng, int(side[i]), int(nb[i])) for i in range(n)]
    nb = np.array([p[5] for p in parts], np.uint8)
    assert (nb >= 1).all()
    table = wl.EnvTable(np.full(n, 6, np.uint8), side, T, np.full(n, 99 + seed, np.uint64),
                        np.arange(n, dtype=np.uint32), "injected dynobs", nb)
    st = dict(grid=np.concatenate([p[0].reshape(-1) for p in parts]),
              x=np.array([p[1] for p in parts], np.int32), y=np.array([p[2] for p in parts], np.int32),
              dir=np.array([p[3] for p in parts], np.int32), t=rng.integers(0, 5, n).astype(np.int32),
              carry=np.ones(n, np.int32), episode=rng.integers(0, 9, n).astype(np.uint32),
              done_prev=np.zeros(n, np.uint8), calls=rng.integers(0, 1000, n).astype(np.uint32),
              obst=np.concatenate([p[4] for p in parts]))
    steps = 60
    acts = wl.random_actions(steps, n, seed=seed + 200)
    b = P.ox_batch(table)
    s = ox.State(**{k: v.copy() for k, v in st.items()})
    ref = ox.rollout(b, s, steps, acts, nthreads=16)
    env = ge.GridEnv(table)
    env.reset()
    env.load_state(st)
    traj = ge.Traj.alloc(steps, n)
    dacts = torch.from_numpy(acts).cuda()
    if kernel == "fused":
        env.rollout(steps, traj, dacts, K=11)
    else:
        for k in range(steps):
            env.step(traj.row(k), dacts[k])
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"injected dynobs seed {seed} {kernel}")
    P.assert_state_equal(env, s, f"injected dynobs seed {seed} {kernel}")
    env.close()


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_malformed_obstacle_lists(kernel):
    """Obstacle lists with entries off the interior (more balls asked than
    listed): both sides leave those entries alone, nothing outside any grid
    changes, and results still match."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    rng = np.random.default_rng(7)
    n = 800
    side = rng.choice([5, 6, 9], n).astype(np.uint8)
    parts = [random_dynobs_state(rng, int(side[i]), int(rng.integers(1, 4))) for i in range(n)]
    placed = np.array([p[5] for p in parts])
    nb = np.minimum(placed + rng.integers(1, 4, n), 8).astype(np.uint8)
    nb = np.minimum(nb, (side.astype(int) - 2) ** 2 - 2).astype(np.uint8)
    obst = np.concatenate([p[4] for p in parts])
    for i in range(n):                      # a few junk entries past the real balls
        if placed[i] < 8 and rng.random() < 0.5:
            obst[16 * i + 2 * placed[i]] = rng.choice([0, 200])
    T = np.full(n, 1000, np.int32)
    table = wl.EnvTable(np.full(n, 6, np.uint8), side, T, np.full(n, 5, np.uint64),
                        np.arange(n, dtype=np.uint32), "malformed lists", nb)
    st = dict(grid=np.concatenate([p[0].reshape(-1) for p in parts]),
              x=np.array([p[1] for p in parts], np.int32), y=np.array([p[2] for p in parts], np.int32),
              dir=np.array([p[3] for p in parts], np.int32), t=np.zeros(n, np.int32),
              carry=np.ones(n, np.int32), episode=np.zeros(n, np.uint32),
              done_prev=np.zeros(n, np.uint8), calls=np.zeros(n, np.uint32), obst=obst)
    acts = np.zeros((20, n), np.uint8)      # turning in place: episodes do not end
    b = P.ox_batch(table)
    s = ox.State(**{k: v.copy() for k, v in st.items()})
    ref = ox.rollout(b, s, 20, acts, nthreads=16)
    env = ge.GridEnv(table)
    env.reset()
    env.load_state(st)
    traj = ge.Traj.alloc(20, n)
    dacts = torch.from_numpy(acts).cuda()
    if kernel == "fused":
        env.rollout(20, traj, dacts, K=7)
    else:
        for k in range(20):
            env.step(traj.row(k), dacts[k])
    torch.cuda.synchronize()
    P.assert_rows_equal(traj, ref, what=f"malformed lists {kernel}")
    P.assert_state_equal(env, s, f"malformed lists {kernel}")
    env.close()
