#!/usr/bin/env python3
"""Throughput of the batched gridworld step on one MI355X.

Workload: 262144 envs of uneven sizes (40 % single rooms and 40 % two-room
key/door layouts with side in {5, 6, 8, 16}, 20 % 19x19 four-room
layouts), uniform random actions drawn on the device, every env-step
writing its record (147-byte observation, fp32 reward, flags, action) to
an HBM trajectory ring.  One benchmark "step" is one environment step of
the whole batch; the fused persistent kernel runs K of them per launch.

Reported beside it on the same input: the plain one-launch-per-step
kernel, per-launch latency percentiles, five repeats of the timed rollout,
the dominant kernel's roofline position (with the HBM traffic of the
committed rocprofv3 summary when it was taken of this kernel's code), the
native serving loop at three offered loads, and the CPU oracle's rate on
its whole job and on one thread.  --workload and --obs select the other
task mixes and observation functions.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
OBS = 147
RECORD_BYTES = OBS + 4 + 1 + 1          # obs + reward + flags + action per env-step
STATE_BYTES_PER_ENV = 4 * 5 + 4 + 1 + 4 + 16  # x, y, dir, t, carry + episode + done_prev + calls + obstacles


WORKLOADS = {
    "mixed": "mixed uneven sizes: {n} envs (40% Empty S in {5,6,8,16}, 40% TwoRoom key/door "
             "S in {5,6,8,16}, 20% FourRooms 19x19), random policy on device, trajectory ring in HBM",
    "tworoom8": "65536 TwoRoom key/door 8x8, T=640, random policy on device, trajectory ring in HBM",
    "empty8": "4096 Empty 8x8, T=256, random policy on device, trajectory ring in HBM",
    "empty5": "16 Empty 5x5, T=100, random policy on device, trajectory ring in HBM",
    "lava": "lava tasks: {n} envs in equal shares of LavaGap S5/S6/S7, Crossings S9N1/S9N2/S9N3/"
            "S11N5, DistShift1 (6x6), DistShift2 (8x8), random policy on device, trajectory ring in HBM",
    "dynobs": "Dynamic-Obstacles tasks: {n} envs in equal shares of 5x5 (2 balls), 6x6 (3), 8x8 (4), "
              "16x16 (8), random policy on device, trajectory ring in HBM",
    "gotodoor": "GoToDoor tasks: {n} envs in equal shares of 5x5, 6x6, 8x8, random policy on device, "
                "trajectory ring in HBM",
    "keycorridor": "KeyCorridor tasks: {n} envs in equal shares of S3R1, S3R2, S3R3, S4R3, S5R3, S6R3, "
                   "random policy on device, trajectory ring in HBM",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


OBS_MODES = {"symbolic": 0, "categorical": 1, "symbolic_grid": 2, "categorical_grid": 3,
             "rgb_first_person": 4, "rgb": 5}
RGB_SCALE = 1024   # rgb bytes per symbolic byte (32 x 32 pixels per cell)
RING_BUDGET = 64 << 30   # bytes of HBM the trajectory ring of one launch may take


def fused_bytes(n_envs: int, grid_bytes: int, k: int, obs_bytes: int = OBS) -> float:
    """Algorithmic HBM bytes of one fused launch of k steps: every record
    written once, the state (grids + scalars) read and written once."""
    record = obs_bytes + 4 + 1 + 1
    return n_envs * k * record + 2.0 * (grid_bytes + STATE_BYTES_PER_ENV * n_envs)


def rgb_path_bytes(n_envs: int, grid_bytes: int, k: int, sym_bytes: float) -> float:
    """Algorithmic HBM bytes of one chunk of the rgb path: the fused launch
    with its symbolic records staged, then the renderer reading them (with
    the 7 scalar bytes) and writing the images (and the scalars)."""
    render = n_envs * k * (sym_bytes + 7 + RGB_SCALE * sym_bytes + 7)
    return fused_bytes(n_envs, grid_bytes, k, sym_bytes) + render


def cpu_baseline(table, n_envs: int, n_steps: int, obs_mode: int = 0, sprites=None) -> dict:
    import oracle as ox
    sub = table.subset(np.arange(n_envs))
    b = ox.Batch(sub.family, sub.side, sub.max_steps, sub.seed, sub.rng_id, 0, sub.param, obs_mode,
                 sprites)
    s = ox.State.empty(b)
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    rows = 1 if obs_mode >= 4 else 16   # rgb records are 1024 times larger
    ox.reset(b, s, nthreads=threads)
    t0 = time.perf_counter()
    ox.rollout(b, s, n_steps, None, rows=rows, nthreads=threads)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, over 1 / threads of the envs
    n1 = max(1, n_envs // threads)
    sub1 = table.subset(np.arange(n1))
    b1 = ox.Batch(sub1.family, sub1.side, sub1.max_steps, sub1.seed, sub1.rng_id, 0, sub1.param, obs_mode,
                  sprites)
    s1 = ox.State.empty(b1)
    ox.reset(b1, s1)
    t1 = time.perf_counter()
    ox.rollout(b1, s1, n_steps, None, rows=rows)
    dt1 = time.perf_counter() - t1
    return {"value": n_envs * n_steps / dt, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_envs} envs of the same mix, {n_steps} steps, random policy, "
                      f"observations on, {dt:.1f} s",
            "single_thread": {"value": n1 * n_steps / dt1, "cores": 1,
                              "sample": f"first {n1} envs, {n_steps} steps, {dt1:.1f} s"}}


def run_serving(capacity: float, n_requests: int, loads, K: int, budget_gib: int,
                inflight: int = 2) -> list:
    """Poisson serving at fractions of the measured fused capacity."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    from paper_2407_19396_amd import workloads as wl

    probe = wl.serving_requests(4000, rate_per_s=1.0, master_seed=12345)
    ework = float(np.mean([r.n_envs * r.n_steps for r in probe]))
    srv = ge.Server(max_tiles=16384, max_side=19)
    budget = budget_gib << 30
    arena = torch.empty(budget - srv.info()["device_bytes"], dtype=torch.uint8, device="cuda")
    out = []
    for load in loads:
        rate = load * capacity / ework
        reqs = wl.serving_requests(n_requests, rate, master_seed=int(load * 1000))
        res = ge.serve_run(srv, reqs, K, budget, arena, max_inflight=inflight)
        lat = res["latency_s"] * 1e3
        wait = (res["admit_s"] - res["arrival_s"]) * 1e3
        rec = {"load": load, "requests": n_requests, "completed": res["completed"],
               "rate_req_per_s": rate, "mean_env_steps_per_request": ework,
               "env_steps_per_s": res["env_steps"] / res["wall_s"], "wall_s": res["wall_s"],
               "launches": res["launches"],
               "host_s": {"admit": res["host_admit_s"], "step": res["host_step_s"],
                          "wait": res["host_wait_s"]},
               "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
               "admission_wait_ms": {"p50": float(np.percentile(wait, 50)),
                                     "p99": float(np.percentile(wait, 99))}}
        log(f"[bench] serving load {load}: {rec['env_steps_per_s'] / 1e9:.2f} G env-steps/s, "
            f"latency p50 {rec['latency_ms']['p50']:.1f} ms p99 {rec['latency_ms']['p99']:.1f} ms")
        out.append(rec)
    srv.close()
    del arena
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4096, help="timed environment steps of the batch")
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of the same rollout, reported as median / min / max")
    ap.add_argument("--workload", default="mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--envs", type=int, default=0, help="override the workload's env count")
    ap.add_argument("--K", type=int, default=0, help="steps fused per launch (0: autotune)")
    ap.add_argument("--blocks", type=int, default=0, help="persistent workgroups (0: autotune or default)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner, use library defaults")
    ap.add_argument("--ring", type=int, default=0, help="trajectory ring rows (0: K)")
    ap.add_argument("--plain-steps", type=int, default=512)
    ap.add_argument("--obs", default="symbolic", choices=list(OBS_MODES),
                    help="observation function: symbolic (147 B) or categorical (49 B) first person, "
                         "the whole grid: symbolic_grid (3 S^2 B) or categorical_grid (S^2 B), or "
                         "images drawn with the default sprites: rgb_first_person (150528 B) or rgb "
                         "(3072 S^2 B); the rgb modes default to 16384 envs and K = 16")
    ap.add_argument("--graph", action="store_true",
                    help="capture the timed rollout in a HIP graph and time its replay")
    ap.add_argument("--plain-actions", action="store_true",
                    help="plain steps take an external action buffer instead of the device policy")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-envs", type=int, default=0, help="CPU oracle sample envs (0: all)")
    ap.add_argument("--cpu-steps", type=int, default=0, help="CPU oracle sample steps (0: --steps)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per serving load level (0: skip serving)")
    ap.add_argument("--serve-K", type=int, default=256)
    ap.add_argument("--serve-inflight", type=int, default=2, help="launches enqueued ahead of the device")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95")
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the environment "
              "batch would shard by env id with no exchange, see the design notes.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_19396_amd import gridenv as ge
    from paper_2407_19396_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {n} bytes read and {n} bytes written by one copy kernel")
        del src, dst
    make = {"mixed": lambda: wl.workload_mixed(seed=0, n=args.envs or 262144),
            "tworoom8": lambda: wl.workload_tworoom8(seed=0),
            "empty8": lambda: wl.workload_empty8(seed=0),
            "empty5": lambda: wl.workload_empty5(seed=0),
            "lava": lambda: wl.workload_lava(seed=0, n=args.envs or 262144),
            "dynobs": lambda: wl.workload_dynobs(seed=0, n=args.envs or 262144),
            "gotodoor": lambda: wl.workload_gotodoor(seed=0, n=args.envs or 262144),
            "keycorridor": lambda: wl.workload_keycorridor(seed=0, n=args.envs or 262144)}[args.workload]
    obs_mode = OBS_MODES[args.obs]
    rgb = obs_mode >= 4
    if rgb and not args.envs:
        args.envs = 16384          # a step writes 2.5 GB of first-person images at this size
    table = make()
    if args.envs and args.workload not in ("mixed", "lava", "dynobs", "gotodoor", "keycorridor"):
        table = table.subset(np.arange(args.envs) % table.n)
    sprites = None
    if rgb:
        from paper_2407_19396_amd.sprites import default_atlas
        sprites = default_atlas()
    env = ge.GridEnv(table, obs_mode=obs_mode, sprites=sprites)
    # observation bytes per env-step (the mean record size in the whole-grid modes)
    obs_bytes = env.info()["obs_row_bytes"] / table.n
    first = env.traj(1)
    stream = torch.cuda.current_stream()
    tuned = None
    if rgb:
        # launches of K steps, each drawn by the renderer right after
        env.set_launch(args.K or 16, args.blocks)
    elif args.K or args.blocks or args.no_tune:
        env.set_launch(args.K or env.info()["k_default"], args.blocks)
    else:
        from paper_2407_19396_amd import autotune
        # K up to 1024, as long as a ring of K rows stays within RING_BUDGET
        row_bytes = table.n * (obs_bytes + 6)
        Ks = [k for k in (128, 256, 512, 1024) if k * row_bytes <= RING_BUDGET] or [128]
        probe = env.traj(max(Ks))
        env.reset(first)
        tuned = autotune.tune(env, probe, Ks=tuple(Ks), log=log)
        del probe
        log(f"[bench] autotuned K={tuned['K']} blocks={tuned['blocks']}")
    info = env.info()
    K = info["k_default"]
    ring = args.ring or K
    log(f"[bench] {table.name}: grid {info['grid_bytes'] / 1e6:.1f} MB, tiles {info['n_tiles']}, "
        f"LDS/WG {info['lds_bytes']} B, blocks {info['blocks']}, K {K}, ring {ring}")
    traj = env.traj(ring)
    env.reset(first)
    # warmup (also advances episodes away from the synchronous start)
    env.rollout(args.warmup, traj, K=K)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # timed fused run (optionally as the replay of a captured graph)
    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            env.rollout(args.steps, traj, K=K)
        graph.replay()                      # one untimed replay
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        log("[bench] rollout captured in a HIP graph")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    if graph is not None:
        graph.replay()
    else:
        env.rollout(args.steps, traj, K=K)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    launches = -(-args.steps // K)
    env_steps = table.n * args.steps
    value = env_steps / (ms / 1e3)
    log(f"[bench] fused: {args.steps} steps in {ms:.1f} ms ({wall * 1e3:.1f} ms wall), "
        f"{value / 1e9:.2f} G env-steps/s")

    # the same timed rollout repeated, for its spread
    reps = []
    for _ in range(args.repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        if graph is not None:
            graph.replay()
        else:
            env.rollout(args.steps, traj, K=K)
        b.record(stream)
        b.synchronize()
        reps.append(env_steps / (a.elapsed_time(b) / 1e3))
    # per-launch latency of the fused kernel
    lat = []
    for _ in range(min(64, max(8, launches))):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        env.rollout(K, traj, K=K)
        b.record(stream)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    lat = np.array(lat)

    # plain kernel on the same input, writing a ring of the same size
    plain_rate = None
    plain_lat = None
    if args.plain_steps > 0:
        rows = [traj.row(r) for r in range(traj.rows)]
        acts = None
        if args.plain_actions:
            acts = torch.from_numpy(wl.random_actions(args.plain_steps, table.n, seed=1)).to(dev)
        for k in range(8):
            env.step(rows[k % len(rows)])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for k in range(args.plain_steps):
            env.step(rows[k % len(rows)], acts[k] if acts is not None else None)
        b.record(stream)
        torch.cuda.synchronize()
        pms = a.elapsed_time(b)
        plain_rate = table.n * args.plain_steps / (pms / 1e3)
        pl = []
        for k in range(64):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            env.step(rows[k % len(rows)])
            b.record(stream)
            b.synchronize()
            pl.append(a.elapsed_time(b))
        plain_lat = np.array(pl)
        log(f"[bench] plain: {plain_rate / 1e9:.2f} G env-steps/s, launch p50 "
            f"{np.percentile(plain_lat, 50) * 1e3:.1f} us")

    per_launch_ms = ms / launches
    if rgb:
        bytes_launch = rgb_path_bytes(table.n, info["grid_bytes"], K, obs_bytes / RGB_SCALE)
    else:
        bytes_launch = fused_bytes(table.n, info["grid_bytes"], K, obs_bytes)
    achieved = bytes_launch / (per_launch_ms / 1e3) / 1e9
    from paper_2407_19396_amd import profiling
    traffic = None
    if args.workload == "mixed" and args.steps % K == 0 and obs_mode == 0:
        traffic = profiling.traffic_bytes(os.path.join(ROOT, "profiles", "k_fused_mixed262144.txt"),
                                          K, table.n)
    serving = None
    if args.serve_requests > 0 and args.workload == "mixed" and obs_mode == 0:
        del traj, env
        torch.cuda.empty_cache()
        loads = tuple(float(x) for x in args.serve_loads.split(","))
        serving = run_serving(value, args.serve_requests, loads, args.serve_K,
                              args.serve_budget_gib, args.serve_inflight)
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a sample")
        if rgb:   # the oracle draws every pixel: a smaller sample
            cpu = cpu_baseline(table, min(args.cpu_envs or 4096, table.n), args.cpu_steps or 1024,
                               obs_mode, sprites)
        else:
            cpu = cpu_baseline(table, min(args.cpu_envs or table.n, table.n), args.cpu_steps or args.steps)
        log(f"[bench] cpu oracle: {cpu['value'] / 1e6:.2f} M env-steps/s on {cpu['cores']} threads")

    out = {
        "metric": "env-steps/sec on 1 MI355X, fused multi-size vs plain step; p50/p99 latency",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].replace("{n}", str(table.n)),
                   "n_envs": table.n, "K": K, "ring_rows": ring, "blocks": info["blocks"],
                   "lds_bytes_per_wg": info["lds_bytes"], "global_batch": table.n,
                   "autotuned": tuned is not None, "hip_graph": graph is not None,
                   "observation": args.obs},
        "fused_launch_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "repeats": None if not reps else {"n": len(reps), "median": float(np.median(reps)),
                                          "min": float(np.min(reps)), "max": float(np.max(reps))},
        "plain": None if plain_rate is None else {
            "value": plain_rate, "unit": "env-steps/s", "steps": args.plain_steps,
            "launch_ms": {"p50": float(np.percentile(plain_lat, 50)),
                          "p99": float(np.percentile(plain_lat, 99))},
            "fused_over_plain": value / plain_rate},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_fused + k_sprite_ids + k_render" if rgb else "k_fused",
                     "bytes_per_launch": bytes_launch,
                     "launch_ms": per_launch_ms},
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
