"""Brute force on the GPU: every action sequence of length 6 from every
5x5 start (single room and two-room key/door, with and without early
truncation; and of length 5 or 6 from the 5x5 GoToDoor and one-ball
Dynamic-Obstacles starts), each sequence one env, compared with the oracle
step by step (plain kernel and fused kernel)."""
import numpy as np
import pytest

import enumerate_starts as es
import oracle as ox
import parity as P
from paper_2407_19396_amd import workloads as wl

pytestmark = pytest.mark.gpu


CASES = {k: v + (0,) for k, v in es.CASES.items()} | es.PARITY_CASES


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_bruteforce_parity(case, kernel):
    import torch
    from paper_2407_19396_amd import gridenv as ge
    make, L, family, T, param = CASES[case]
    starts = make()
    per_chunk = 16
    for c0 in range(0, len(starts), per_chunk):
        cfg, st, actions = es.batch_arrays(starts[c0:c0 + per_chunk], L, family, T, param=param)
        table = wl.EnvTable(cfg["family"], cfg["side"], cfg["max_steps"], cfg["seed"], cfg["rng_id"], "",
                            cfg.get("param"))
        b = ox.Batch(cfg["family"], cfg["side"], cfg["max_steps"], cfg["seed"], cfg["rng_id"], 0,
                     cfg.get("param"))
        s = ox.State(**{k: v.copy() for k, v in st.items()})
        ref = ox.rollout(b, s, L, actions, nthreads=16)
        env = ge.GridEnv(table)
        env.reset()                      # enables stepping; the state is then replaced
        env.load_state(st)
        dacts = torch.from_numpy(actions).cuda()
        traj = ge.Traj.alloc(L, table.n)
        if kernel == "fused":
            env.rollout(L, traj, dacts, K=L)
        else:
            for k in range(L):
                env.step(traj.row(k), dacts[k])
        torch.cuda.synchronize()
        P.assert_rows_equal(traj, ref, what=f"{case} {kernel} starts {c0}..")
        P.assert_state_equal(env, s, f"{case} {kernel}")
        env.close()
