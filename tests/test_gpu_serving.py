"""Serving (continuous batching): a request's results are the same alone and
in a mix of requests admitted while others run, and equal the oracle's
reset + rollout of the request's own envs."""
import numpy as np
import pytest

import oracle as ox
import parity as P
from paper_2407_19396_amd import workloads as wl

pytestmark = pytest.mark.gpu


def requests(n, seed):
    reqs = wl.serving_requests(n, rate_per_s=1.0, master_seed=seed, max_envs=600)
    rng = np.random.default_rng(seed)
    for r in reqs:
        r.n_steps = int(rng.integers(20, 150))
    return reqs


def alloc(ge, r):
    stride = ge.padded_stride(r.n_envs)
    return ge.Traj.alloc(r.n_steps, stride), stride


def run_alone(ge, r, K):
    import torch
    srv = ge.Server(max_tiles=16)
    out, stride = alloc(ge, r)
    h = srv.admit(r.table, r.n_steps, out, stride)
    assert h is not None
    done = []
    while not done:
        done = srv.step(K)
    torch.cuda.synchronize()
    srv.release(h)
    srv.close()
    return out


def run_mix(ge, reqs, K, max_tiles, per_step=8):
    """Admit a few requests before every step (as arrivals would), retrying
    those that do not fit until tiles free up."""
    import torch
    srv = ge.Server(max_tiles=max_tiles)
    outs, waiting, live = {}, list(range(len(reqs))), {}
    busy_seen = False
    while waiting or live:
        for _ in range(per_step):
            if not waiting:
                break
            i = waiting[0]
            out, stride = alloc(ge, reqs[i])
            h = srv.admit(reqs[i].table, reqs[i].n_steps, out, stride)
            if h is None:
                busy_seen = True
                break
            waiting.pop(0)
            outs[i] = out
            live[h] = i
        fin = srv.step(K)
        if fin:
            torch.cuda.synchronize()
            for h in fin:
                srv.release(h)
                live.pop(h)
    torch.cuda.synchronize()
    info = srv.info()
    srv.close()
    return outs, busy_seen, info


def oracle_of(r):
    b = ox.Batch(r.table.family, r.table.side, r.table.max_steps,
                 np.full(r.n_envs, r.seed, np.uint64), np.arange(r.n_envs, dtype=np.uint32), 0,
                 r.table.param)
    s = ox.State.empty(b)
    ox.reset(b, s)
    return ox.rollout(b, s, r.n_steps, None, nthreads=16)


def crop(out, n):
    from paper_2407_19396_amd import gridenv as ge
    return ge.Traj(out.obs[:, :n], out.reward[:, :n], out.flags[:, :n], out.action[:, :n])


@pytest.mark.parametrize("K", [16, 64])
def test_alone_equals_mix_equals_oracle(K):
    from paper_2407_19396_amd import gridenv as ge
    reqs = requests(40, seed=K)
    outs, busy_seen, info = run_mix(ge, reqs, K, max_tiles=16)
    assert busy_seen, "the mix never filled the server; the test would not exercise admission"
    assert info["live_requests"] == 0 and info["free_tiles"] == info["max_tiles"]
    for i in (0, 7, 19, 33, 39):
        alone = run_alone(ge, reqs[i], K)
        a, m = crop(alone, reqs[i].n_envs), crop(outs[i], reqs[i].n_envs)
        for f in ("obs", "reward", "flags", "action"):
            np.testing.assert_array_equal(P.to_np(getattr(a, f)), P.to_np(getattr(m, f)),
                                          err_msg=f"request {i} {f}: alone != mix")
    for i in range(0, 40, 3):
        P.assert_rows_equal(crop(outs[i], reqs[i].n_envs), oracle_of(reqs[i]), what=f"request {i}")


def test_busy_and_release():
    import torch
    from paper_2407_19396_amd import gridenv as ge
    srv = ge.Server(max_tiles=2)
    t = wl.mixed_table(100, seed=3, mix_seed=4)
    out, stride = ge.Traj.alloc(10, 112), 112
    h = srv.admit(t, 10, out, stride)
    assert h is not None
    t2 = wl.mixed_table(10, seed=5, mix_seed=6)
    out2 = ge.Traj.alloc(10, 16)
    assert srv.admit(t2, 10, out2, 16) is None            # both tiles taken
    with pytest.raises(ge.GridEnvError) as ei:
        srv.release(h)                                    # not finished yet
    assert ei.value.status == ge.GX_ESTATE
    fin = srv.step(64)
    assert fin == [h]
    torch.cuda.synchronize()
    srv.release(h)
    assert srv.admit(t2, 10, out2, 16) is not None
    assert srv.step(64) != []
    torch.cuda.synchronize()
    srv.close()


def test_release_needs_the_returned_handle():
    """A request whose last step is launched but whose handle no step call
    has returned yet cannot be released; the next step call returns it
    (without a launch, nothing else being live) and then it can."""
    import ctypes
    import torch
    from paper_2407_19396_amd import gridenv as ge
    srv = ge.Server(max_tiles=2)
    t = wl.mixed_table(20, seed=21, mix_seed=22)
    out = ge.Traj.alloc(8, 32)
    h = srv.admit(t, 8, out, 32)
    assert h is not None
    n = ctypes.c_int32(-1)
    fin = (ctypes.c_int32 * 1)()
    rc = ge.load().env_server_step(srv.ptr, 64, ge._stream_ptr(None), fin, 0, ctypes.byref(n))
    assert rc == ge.GX_OK and n.value == 0
    torch.cuda.synchronize()
    with pytest.raises(ge.GridEnvError) as ei:
        srv.release(h)
    assert ei.value.status == ge.GX_ESTATE
    assert srv.step(64) == [h]
    torch.cuda.synchronize()
    srv.release(h)
    assert srv.info()["free_tiles"] == 2
    P.assert_rows_equal(crop(out, 20), oracle_of(wl.Request(0, 0.0, 20, 8, int(t.seed[0]), t)),
                        what="released request")
    srv.close()


def test_native_loop_with_more_finishing_requests_than_4096():
    """4500 one-env requests arriving together all finish in the same
    launch; the loop collects every handle and completes."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    reqs = []
    for i in range(4500):
        t = wl.mixed_table(1, seed=1000 + i, mix_seed=i)
        reqs.append(wl.Request(i, 0.0, 1, 4, int(t.seed[0]), t))
    srv = ge.Server(max_tiles=4608)
    budget = srv.info()["device_bytes"] + (256 << 20)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    res = ge.serve_run(srv, reqs, 16, budget, arena, keep_obs=False)
    assert res["completed"] == len(reqs)
    assert res["launches"] == 1
    assert res["env_steps"] == 4 * len(reqs)
    info = srv.info()
    assert info["live_requests"] == 0 and info["free_tiles"] == 4608
    srv.close()


def test_native_serving_loop_completes_everything():
    import torch
    from paper_2407_19396_amd import gridenv as ge
    reqs = wl.serving_requests(300, rate_per_s=3000.0, master_seed=7, max_envs=2048)
    srv = ge.Server(max_tiles=256)
    budget = 2 << 30
    arena = torch.empty(budget - srv.info()["device_bytes"], dtype=torch.uint8, device="cuda")
    res = ge.serve_run(srv, reqs, 32, budget, arena)
    assert res["completed"] == len(reqs)
    assert res["env_steps"] == sum(r.n_envs * r.n_steps for r in reqs)
    assert (res["admit_s"] >= res["arrival_s"] - 1e-9).all()
    assert (res["done_s"] > res["admit_s"]).all()
    # every launch advances some request: no more launches than request chunks
    assert 0 < res["launches"] <= sum(-(-r.n_steps // 32) for r in reqs)
    assert res["host_latency_s"] is None
    info = srv.info()
    assert info["live_requests"] == 0 and info["free_tiles"] == 256
    srv.close()


def test_host_delivery_of_scalar_outputs():
    """With a host arena every request's reward, flags and action reach
    pinned host memory after its device completion; a lone request's copy
    sits at the arena's start (reward, then flags and action at 256-byte
    aligned offsets) and equals the oracle's rollout."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    srv = ge.Server(max_tiles=64)
    budget = 1 << 30
    arena = torch.empty(budget - srv.info()["device_bytes"], dtype=torch.uint8, device="cuda")
    host = torch.empty(64 << 20, dtype=torch.uint8, pin_memory=True)
    # one request alone: its delivered outputs are checked against the oracle
    t = wl.mixed_table(100, seed=11, mix_seed=12)
    r = wl.Request(0, 0.0, 100, 70, int(t.seed[0]), t)
    res = ge.serve_run(srv, [r], 16, budget, arena, keep_obs=False, host_arena=host)
    assert res["completed"] == 1
    assert res["host_done_s"][0] >= res["done_s"][0] > 0
    stride = ge.padded_stride(r.n_envs)
    recs = stride * r.n_steps
    up = lambda x: (x + 255) // 256 * 256  # noqa: E731
    h = host.numpy()
    reward = h[:4 * recs].view(np.float32).reshape(r.n_steps, stride)[:, :r.n_envs]
    flags = h[up(4 * recs):up(4 * recs) + recs].reshape(r.n_steps, stride)[:, :r.n_envs]
    action = h[up(4 * recs) + up(recs):up(4 * recs) + up(recs) + recs].reshape(r.n_steps, stride)[:, :r.n_envs]
    ref = oracle_of(r)
    np.testing.assert_array_equal(reward.view(np.uint32), ref.reward.view(np.uint32))
    np.testing.assert_array_equal(flags, ref.flags)
    np.testing.assert_array_equal(action, ref.action)
    # a Poisson mix through a small host arena: everything is delivered
    reqs = wl.serving_requests(200, rate_per_s=3000.0, master_seed=9, max_envs=1024)
    res = ge.serve_run(srv, reqs, 32, budget, arena, keep_obs=True, host_arena=host)
    assert res["completed"] == len(reqs)
    assert (res["host_done_s"] >= res["done_s"]).all() and (res["done_s"] > res["admit_s"]).all()
    assert (res["host_latency_s"] > 0).all()
    info = srv.info()
    assert info["live_requests"] == 0 and info["free_tiles"] == 64
    srv.close()


def test_lava_and_obstacle_requests_equal_oracle():
    """Requests of the lava and Dynamic-Obstacles tasks through the server
    (admission resets them on the device) equal the oracle's reset +
    rollout."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(8):
        n = int(rng.integers(1, 300))
        make = wl.lava_table if i % 2 == 0 else wl.dynobs_table
        t = make(n, seed=int(rng.integers(0, 2 ** 62)), mix_seed=i)
        reqs.append(wl.Request(i, 0.0, n, int(rng.integers(20, 120)), int(t.seed[0]), t))
    outs, _, info = run_mix(ge, reqs, 32, max_tiles=10)
    assert info["live_requests"] == 0
    for i, r in enumerate(reqs):
        P.assert_rows_equal(crop(outs[i], r.n_envs), oracle_of(r), what=f"lava request {i}")


def test_requests_of_every_family_equal_oracle():
    """Requests mixing every family (GoToDoor and KeyCorridor included) through
    the server equal the oracle's reset + rollout."""
    from paper_2407_19396_amd import gridenv as ge
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(8):
        n = int(rng.integers(1, 300))
        make = [wl.families_table, wl.gotodoor_table, wl.keycorridor_table][i % 3]
        t = make(n, seed=int(rng.integers(0, 2 ** 62)), mix_seed=100 + i)
        reqs.append(wl.Request(i, 0.0, n, int(rng.integers(20, 120)), int(t.seed[0]), t))
    outs, _, info = run_mix(ge, reqs, 32, max_tiles=10)
    assert info["live_requests"] == 0
    for i, r in enumerate(reqs):
        P.assert_rows_equal(crop(outs[i], r.n_envs), oracle_of(r), what=f"family request {i}")
