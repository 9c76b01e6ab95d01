#!/usr/bin/env python3
"""Throughput of the batched gridworld step on one MI355X.

Workload: 262144 envs of uneven sizes (40 % single rooms and 40 % two-room
key/door layouts with side in {5, 6, 8, 16}, 20 % 19x19 four-room
layouts), uniform random actions drawn on the device, every env-step
writing its record (147-byte observation, fp32 reward, flags, action) to
an HBM trajectory ring.  One benchmark "step" is one environment step of
the whole batch; the fused persistent kernel runs K of them per launch.

Reported beside it on the same input: the plain one-launch-per-step
kernel, per-launch latency percentiles, the dominant kernel's roofline
position and the CPU oracle's rate on a bounded sample.
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
STATE_BYTES_PER_ENV = 4 * 5 + 4 + 1      # x, y, dir, t, carry + episode + done_prev


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def fused_bytes(n_envs: int, grid_bytes: int, k: int) -> float:
    """Algorithmic HBM bytes of one fused launch of k steps: every record
    written once, the state (grids + scalars) read and written once."""
    return n_envs * k * RECORD_BYTES + 2.0 * (grid_bytes + STATE_BYTES_PER_ENV * n_envs)


def cpu_baseline(table, n_envs: int, n_steps: int) -> dict:
    import oracle as ox
    from paper_2407_19396_amd import workloads as wl
    sub = table.subset(np.arange(n_envs))
    b = ox.Batch(sub.family, sub.side, sub.max_steps, sub.seed, sub.rng_id)
    s = ox.State.empty(b)
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    ox.reset(b, s, nthreads=threads)
    t0 = time.perf_counter()
    ox.rollout(b, s, n_steps, None, rows=16, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n_envs * n_steps / dt, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_envs} envs of the same mix, {n_steps} steps, random policy, "
                      f"observations on, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4096, help="timed environment steps of the batch")
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--envs", type=int, default=262144)
    ap.add_argument("--K", type=int, default=0, help="steps fused per launch (0: library default)")
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--ring", type=int, default=0, help="trajectory ring rows (0: K)")
    ap.add_argument("--plain-steps", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-envs", type=int, default=32768)
    ap.add_argument("--cpu-steps", type=int, default=512)
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
    table = wl.workload_mixed(seed=0, n=args.envs)
    env = ge.GridEnv(table)
    if args.K or args.blocks:
        env.set_launch(args.K or env.info()["k_default"], args.blocks)
    info = env.info()
    K = info["k_default"]
    ring = args.ring or K
    log(f"[bench] {table.name}: grid {info['grid_bytes'] / 1e6:.1f} MB, tiles {info['n_tiles']}, "
        f"LDS/WG {info['lds_bytes']} B, blocks {info['blocks']}, K {K}, ring {ring}")
    traj = ge.Traj.alloc(ring, table.n)
    first = ge.Traj.alloc(1, table.n)
    stream = torch.cuda.current_stream()
    env.reset(first)
    # warmup (also advances episodes away from the synchronous start)
    env.rollout(args.warmup, traj, K=K)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # timed fused run
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
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

    # plain kernel on the same input
    plain_rate = None
    plain_lat = None
    if args.plain_steps > 0:
        row = ge.Traj.alloc(1, table.n)
        for _ in range(8):
            env.step(row)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.plain_steps):
            env.step(row)
        b.record(stream)
        torch.cuda.synchronize()
        pms = a.elapsed_time(b)
        plain_rate = table.n * args.plain_steps / (pms / 1e3)
        pl = []
        for _ in range(64):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            env.step(row)
            b.record(stream)
            b.synchronize()
            pl.append(a.elapsed_time(b))
        plain_lat = np.array(pl)
        log(f"[bench] plain: {plain_rate / 1e9:.2f} G env-steps/s")

    per_launch_ms = ms / launches
    bytes_launch = fused_bytes(table.n, info["grid_bytes"], K)
    achieved = bytes_launch / (per_launch_ms / 1e3) / 1e9
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a sample")
        cpu = cpu_baseline(table, min(args.cpu_envs, table.n), args.cpu_steps)
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
        "config": {"workload": "mixed uneven sizes: 262144 envs (40% Empty S in {5,6,8,16}, 40% "
                               "TwoRoom key/door S in {5,6,8,16}, 20% FourRooms 19x19), random "
                               "policy on device, trajectory ring in HBM",
                   "n_envs": table.n, "K": K, "ring_rows": ring, "blocks": info["blocks"],
                   "lds_bytes_per_wg": info["lds_bytes"], "global_batch": table.n},
        "fused_launch_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "plain": None if plain_rate is None else {
            "value": plain_rate, "unit": "env-steps/s", "steps": args.plain_steps,
            "launch_ms": {"p50": float(np.percentile(plain_lat, 50)),
                          "p99": float(np.percentile(plain_lat, 99))},
            "fused_over_plain": value / plain_rate},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_fused", "bytes_per_launch": bytes_launch,
                     "launch_ms": per_launch_ms},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    env.close()


if __name__ == "__main__":
    main()
