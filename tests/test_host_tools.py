"""Host-side logic that needs no GPU: launch-shape candidates of the
autotuner, the profile summary reader, and the workload generators."""
import numpy as np
import pytest

from paper_2407_19396_amd import autotune, profiling
from paper_2407_19396_amd import workloads as wl


def test_block_candidates_include_full_occupancy_and_whole_rounds():
    c = autotune.block_candidates(n_tiles=4096, lds_bytes=18432, cus=256)
    assert 2048 in c                      # 8 per CU fill the LDS and make exactly 2 rounds
    assert 4096 in c                      # one workgroup per tile
    assert all(b <= 8 * 256 or b == 4096 for b in c)
    assert 4096 // 3 + 1 in c or 1366 in c
    c = autotune.block_candidates(n_tiles=10, lds_bytes=18432, cus=256)
    assert max(c) == 10                   # never more workgroups than tiles


def test_resident_blocks_by_lds():
    # side-32 grids in tiles of 32 envs: 39 760 B a workgroup, four per CU
    assert autotune.resident_blocks(n_tiles=2048, lds_bytes=39760, cus=256) == 1024
    assert autotune.resident_blocks(n_tiles=700, lds_bytes=39760, cus=256) == 700
    assert autotune.resident_blocks(n_tiles=10**6, lds_bytes=100, cus=256) == 16 * 256   # wave cap
    assert autotune.resident_blocks(n_tiles=10**6, lds_bytes=200_000, cus=256) == 256    # at least one


def test_traffic_is_read_only_for_the_same_kernel(tmp_path):
    p = tmp_path / "k.txt"
    h = profiling.kernel_source_hash()
    p.write_text(f"# x\nmachine: traffic_bytes_per_launch=123 K=512 envs=262144 kernel={h} avg_ns=1\n")
    assert profiling.traffic_bytes(str(p), 512, 262144) == 123.0
    assert profiling.traffic_bytes(str(p), 256, 262144) is None
    assert profiling.traffic_bytes(str(p), 512, 1000) is None
    p.write_text("machine: traffic_bytes_per_launch=123 K=512 envs=262144 kernel=0000 avg_ns=1\n")
    assert profiling.traffic_bytes(str(p), 512, 262144) is None
    assert profiling.traffic_bytes(str(tmp_path / "missing.txt"), 512, 262144) is None


def test_mixed_workload_composition():
    t = wl.workload_mixed(seed=0)
    assert t.n == 262144
    frac = np.bincount(t.family, minlength=3) / t.n
    assert abs(frac[0] - 0.4) < 0.01 and abs(frac[1] - 0.4) < 0.01 and abs(frac[2] - 0.2) < 0.01
    assert set(np.unique(t.side[t.family != 2])) == {5, 6, 8, 16}
    assert set(np.unique(t.side[t.family == 2])) == {19}
    assert (t.max_steps[t.family == 0] == 4 * t.side[t.family == 0].astype(int) ** 2).all()
    assert (t.max_steps[t.family == 1] == 10 * t.side[t.family == 1].astype(int) ** 2).all()
    assert (t.max_steps[t.family == 2] == 100).all()


def test_serving_requests_shape():
    reqs = wl.serving_requests(3000, rate_per_s=1000.0, master_seed=1)
    n = np.array([r.n_envs for r in reqs])
    steps = np.array([r.n_steps for r in reqs])
    arr = np.array([r.arrival_s for r in reqs])
    assert n.min() >= 1 and n.max() <= 8192 and 700 < n.mean() < 1150   # log-uniform, E ~ 909
    assert steps.min() >= 64 and steps.max() <= 1024
    assert (np.diff(arr) > 0).all() and 2.5 < arr[-1] < 3.5            # Poisson at 1000/s
    assert all(r.table.n == r.n_envs and (r.table.seed == r.seed).all() for r in reqs[:50])
    assert len({r.seed for r in reqs}) == len(reqs)


def test_kernel_hash_ignores_comments_but_not_code(tmp_path):
    a, b = tmp_path / "a.hip", tmp_path / "b.h"
    a.write_text("int f(int x) { return x + 1; }  // one\n/* block */\n")
    b.write_text("struct S { int y; };\n")
    h = profiling.kernel_source_hash((str(a), str(b)))
    a.write_text("// a new comment\nint f(int x)   {\n  return x + 1;  /* two */ }\n")
    assert profiling.kernel_source_hash((str(a), str(b))) == h
    a.write_text("int f(int x) { return x + 2; }\n")
    assert profiling.kernel_source_hash((str(a), str(b))) != h
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("struct S { long y; };\n")
    assert profiling.kernel_source_hash((str(a), str(b))) != h


def _write_csv(path, header, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_render_summary_leaves_out_the_reset_launch(tmp_path):
    """Synthetic rocprofv3 CSVs: two 16-row renderer launches and a one-row
    launch (after a reset) that must not count; the copy probe calibrates."""
    K, envs = 16, 1024
    algo = K * envs * (147 + 7 + 224 * 224 * 3 + 7)
    tr = tmp_path / "trace"
    tr.mkdir()
    _write_csv(tr / "t_kernel_trace.csv", ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [[1, "k_render<false>", 0, 100_000], [2, "k_fused<false>", 100_000, 110_000],
                [3, "k_sprite_ids<false>", 110_000, 111_000], [4, "k_render<false>", 111_000, 2_111_000],
                [5, "k_render<false>", 2_200_000, 4_200_000]])
    for kind, counter, copy_kib, render_kib in (("fetch", "FETCH_SIZE", 512, 100.0),
                                                 ("write", "WRITE_SIZE", 1024, algo / 1024)):
        d = tmp_path / kind
        d.mkdir()
        _write_csv(d / "c_counter_collection.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
                   [[1, "__amd_rocclr_copyBuffer", counter, copy_kib],
                    [2, "k_render<false>", counter, render_kib / 16],
                    [3, "k_render<false>", counter, render_kib],
                    [4, "k_render<false>", counter, render_kib]])
    text = profiling.render_summary(str(tr), str(tmp_path / "fetch"), str(tmp_path / "write"), 1 << 20,
                                    K, envs, "cmd")
    assert "16-row launches: 2, average 2000.0 us" in text
    assert f"achieved: {algo / 2_000_000:.1f} GB/s" in text
    # fetch is scaled x2 by the copy probe (512 KiB for 1 MiB), write x1
    assert f"fetch {2 * 100.0 * 1024 / 1e6:.1f} MB" in text


def test_traffic_lookup_is_per_kernel(tmp_path):
    p = tmp_path / "k.txt"
    h = profiling.kernel_source_hash()
    p.write_text(f"machine: name=k_plain traffic_bytes_per_launch=77 K=1 envs=64 kernel={h} avg_ns=1 median_ns=1\n")
    assert profiling.traffic_bytes(str(p), 1, 64, "k_plain") == 77.0
    assert profiling.traffic_bytes(str(p), 1, 64, "k_fused") is None


def _bench():
    import importlib.util
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_launch_accounting():
    b = _bench()
    assert b.chunks(20, 1024) == [20]
    assert b.chunks(4096, 1024) == [1024] * 4
    assert b.chunks(2500, 1024) == [1024, 1024, 452]
    # a 20-step launch counts 20 steps of records and the state once
    n, g = 262144, 116_778_432
    per = b.fused_bytes(n, g, 20)
    assert per == n * 20 * 153 + 2 * (g + b.STATE_BYTES_PER_ENV * n)
    r = b.roofline_entry(per, 0.25)
    assert 0 < r["frac"] <= 1 and abs(r["achieved"] - per / 0.25e-3 / 1e9) < 1e-6
    with pytest.raises(SystemExit):
        b.roofline_entry(b.fused_bytes(n, g, 1024), 0.25)     # 1024 steps of bytes in a 20-step time
    # counter traffic below the algorithmic bytes is explained on the line
    assert "traffic_note" in b.roofline_entry(per, 0.25, 0.9 * per, kernel="k_fused")
    assert "traffic_note" not in b.roofline_entry(per, 0.25, 1.01 * per, kernel="k_fused")


def test_serving_summary_splits_runs(tmp_path):
    rows = ["Kernel_Name,Start_Timestamp,End_Timestamp"]
    name = "void gx::k_fused<false, true, 0>(gx::FusedArgs)"
    t = 0
    for run in range(2):
        for k in range(5):
            rows.append(f'"{name}",{t},{t + 1_000_000}')
            t += 1_010_000                       # 1 ms launches, 10 us apart
        t += 500_000_000                         # half a second idle between runs
    d = tmp_path / "trace"
    d.mkdir()
    (d / "run_kernel_trace.csv").write_text("\n".join(rows) + "\n")
    text = profiling.serving_summary(str(d), "cmd")
    assert text.count("## run") == 2
    assert "serving launches: 5" in text and "(99.2 % of the span)" in text


def test_buffer_checks_of_the_binding():
    """The binding refuses, before any kernel sees it, a buffer of the wrong
    type, too short for the batch, not contiguous or on another device."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    cpu = torch.device("cpu")
    ge.check_buffer(torch.zeros(4, 10, dtype=torch.uint8), "a", torch.uint8, 40, cpu)
    ge.check_buffer(torch.zeros(4, 10, dtype=torch.uint8)[1], "a", torch.uint8, 10, cpu)   # a row
    bad = [(torch.zeros(40, dtype=torch.int64), torch.uint8, 40, cpu),          # type
           (torch.zeros(39, dtype=torch.uint8), torch.uint8, 40, cpu),          # length
           (torch.zeros(10, 4, dtype=torch.uint8).t(), torch.uint8, 40, cpu),   # layout
           (torch.zeros(40, dtype=torch.uint8), torch.uint8, 40, torch.device("cuda"))]   # device
    for t, dt, n, dev in bad:
        with pytest.raises(ValueError):
            ge.check_buffer(t, "a", dt, n, dev)
    rows, n = 3, 5
    tr = ge.Traj.alloc(rows, n, device="cpu")
    ge.check_traj(tr, n, n * ge.OBS_BYTES, cpu)
    with pytest.raises(ValueError):
        ge.check_traj(tr, n + 1, (n + 1) * ge.OBS_BYTES, cpu)                  # a bigger batch
    with pytest.raises(ValueError):
        ge.check_traj(tr, n, n * ge.OBS_BYTES, cpu, stride=8)                  # a wider request row
    tr2 = ge.Traj(tr.obs, tr.reward.double(), tr.flags, tr.action)
    with pytest.raises(ValueError):
        ge.check_traj(tr2, n, n * ge.OBS_BYTES, cpu)                           # reward not f32
    # a check holds for the buffers it saw, in the rows too, until a buffer
    # is replaced
    key = (n, n * ge.OBS_BYTES, cpu)
    assert tr.checked_view(key) is None
    g = tr.mark_checked(key)
    assert tr.checked_view(key) is g and tr.checked_view((n + 1,) + key[1:]) is None
    r1 = tr.row(1)
    assert r1.checked_view(key) is not None
    assert r1.reward.data_ptr() == tr.reward[1].data_ptr() and r1.rows == 1
    r1.flags = torch.zeros(1, n, dtype=torch.uint8)
    assert r1.checked_view(key) is None
    tr.flags = torch.zeros(rows, n, dtype=torch.uint8)
    assert tr.checked_view(key) is None
    r1b = tr.row(1)
    assert r1b.checked_view(key) is None
    assert r1b.flags.data_ptr() == tr.flags[1].data_ptr()


def _oracle_snapshot(table, steps):
    """What bench.snapshot would hold after a reset and `steps` steps, made
    by the oracle itself in the GPU's layout."""
    import oracle as ox
    b = ox.Batch(table.family, table.side, table.max_steps, table.seed, table.rng_id, 0, table.param)
    s = ox.State.empty(b)
    ox.reset(b, s, nthreads=4)
    out = ox.rollout(b, s, steps, None, rows=1, nthreads=4)
    state = {f: getattr(s, f).copy() for f in ("grid", "x", "y", "dir", "t", "carry", "episode",
                                               "done_prev", "calls", "obst")}
    last = {f: getattr(out, f)[0].copy() for f in ("obs", "reward", "flags", "action")}
    last["mission"] = out.mission[0].copy() if out.mission is not None else None
    return {"state": state, "last": last}


def test_bench_oracle_check_of_the_timed_run():
    """The bench's check passes a run that is the oracle's, over every env
    and over an even sample, and names what differs in one that is not."""
    b = _bench()
    table = wl.mixed_table(300, seed=5, mix_seed=6)
    snap = _oracle_snapshot(table, 13)
    whole = b.oracle_parity(table, snap, 13, 0)
    assert whole["bit_exact"] and whole["envs"] == 300 and whole["mismatch"] == []
    part = b.oracle_parity(table, snap, 13, 0, max_env_steps=13 * 100)
    assert part["bit_exact"] and part["envs"] == 100
    # one grid byte of the last env and one observation byte of env 0
    snap["state"]["grid"][-1] ^= 1
    snap["last"]["obs"][0, 3, 3, 0] ^= 1
    bad = b.oracle_parity(table, snap, 13, 0)
    assert not bad["bit_exact"] and bad["mismatch"] == ["grid", "last row obs"]
    # a different step count is a different run
    assert not b.oracle_parity(table, _oracle_snapshot(table, 12), 13, 0)["bit_exact"]
