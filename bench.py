#!/usr/bin/env python3
"""Throughput of the batched gridworld step on one MI355X.

Workload: 262144 envs of uneven sizes (40 % single rooms and 40 % two-room
key/door layouts with side in {5, 6, 8, 16}, 20 % 19x19 four-room
layouts), uniform random actions drawn on the device, every env-step
writing its record (147-byte symbolic first-person observation, fp32
reward, flags, action) to an HBM trajectory ring.  One benchmark "step" is
one environment step of the whole batch; the fused persistent kernel runs
K of them per launch.  Before the timed region: the autotuner (or its cached
choice), about 0.3 s of untimed rollouts of the timed length, a reset, and
the --warmup steps.

Reported beside it:
  * roofline: the fused launches of the timed region (algorithmic bytes of
    the steps they ran over their HIP-event time) and, under steady_state,
    launches of K steps; each with the calibrated HBM traffic of the
    committed rocprofv3 summary taken of that launch shape and kernel code;
  * the plain one-launch-per-step kernel on the same input, per-launch
    latency percentiles, five repeats of the timed rollout;
  * configs: the smaller workloads as their own legs -- 16 Empty 5x5 and
    4096 Empty 8x8 through the plain kernel with external uniform actions
    (per-launch latency), 65536 TwoRoom 8x8 through the fused kernel with
    the rollout captured in a HIP graph and its replay timed;
  * serving: the native Poisson loop -- its capacity from a saturated run,
    then 0.5 / 0.8 / 0.95 of it, with results left in HBM (device-ready
    latency) and with each request's scalar outputs delivered to pinned host
    memory (host-ready latency, anchored on the delivering loop's own
    saturated capacity);
  * cpu_baseline: the oracle on the host's cores on a bounded sample, and
    under parity the timed run itself checked against the oracle: the state
    and the last output row of every env (or of an even sample when that is
    too much CPU work), bit for bit; a mismatch ends the run with an error
    after the line is printed.
--workload and --obs select the other task mixes and observation functions.
"""
from __future__ import annotations

import argparse
import glob
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
# plain kernel per env-step: state and tables read (x, y, dir, t, carry, episode, done_prev, calls,
# meta, max_steps, seed, rng_id, grid_off), the view's cells, the state written, the record
PLAIN_READ = 4 * 5 + 4 + 1 + 4 + 4 + 4 + 8 + 4 + 8
PLAIN_WRITE = 4 * 5 + 4 + 1 + 4


WORKLOADS = {
    "mixed": "mixed uneven sizes: {n} envs (40% Empty S in {5,6,8,16}, 40% TwoRoom key/door "
             "S in {5,6,8,16}, 20% FourRooms 19x19), random policy on device, trajectory ring in HBM",
    "tworoom8": "65536 TwoRoom key/door 8x8, T=640, random policy on device, trajectory ring in HBM",
    "empty8": "4096 Empty 8x8, T=256, random policy on device, trajectory ring in HBM",
    "empty24": "{n} Empty 24x24, T=2304, random policy on device, trajectory ring in HBM",
    "empty32": "{n} Empty 32x32, T=4096, random policy on device, trajectory ring in HBM",
    "tworoom32": "{n} TwoRoom key/door 32x32, T=10240, random policy on device, trajectory ring in HBM",
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


# observation functions by the names of the paper's table of observations
OBS_MODES = {"symbolic_first_person": 0, "categorical_first_person": 1, "symbolic": 2, "categorical": 3,
             "rgb_first_person": 4, "rgb": 5}
RGB_SCALE = 1024   # rgb bytes per symbolic byte (32 x 32 pixels per cell)
RING_BUDGET = 64 << 30   # bytes of HBM the trajectory ring of one launch may take


def fused_bytes(n_envs: int, grid_bytes: int, k: int, obs_bytes: float = OBS) -> float:
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


def chunks(steps: int, K: int) -> list:
    """Steps run by each fused launch of a rollout of `steps` steps."""
    return [K] * (steps // K) + ([steps % K] if steps % K else [])


def profile_traffic(workload: str, k: int, n_envs: int, kernel: str = "k_fused"):
    """Calibrated HBM bytes of one k-step launch of a kernel from the
    committed rocprofv3 summaries of this workload, or None."""
    from paper_2407_19396_amd import profiling
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_{workload}{n_envs}_*.txt"))):
        t = profiling.traffic_bytes(path, k, n_envs, kernel)
        if t is not None:
            return t
    return None


def roofline_entry(bytes_per_launch: float, launch_ms: float, traffic=None, **extra) -> dict:
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    frac = achieved / HBM_PEAK_GBS
    if not frac <= 1.0:
        raise SystemExit(f"bench.py: roofline fraction {frac:.3f} > 1 ({bytes_per_launch:.4g} B in "
                         f"{launch_ms:.4g} ms): the byte or time accounting is wrong")
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac,
           "traffic": traffic, "bytes_per_launch": bytes_per_launch, "launch_ms": launch_ms, **extra}
    if traffic is not None and traffic < bytes_per_launch and extra.get("kernel") == "k_fused":
        out["traffic_note"] = ("below the algorithmic bytes: the state term counts every grid written "
                               "back, the kernel writes back only the grids that changed")
    return out


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(table, n_envs: int, n_steps: int, obs_mode: int = 0, sprites=None) -> dict:
    import oracle as ox
    sub = table.subset(np.arange(n_envs))
    b = ox.Batch(sub.family, sub.side, sub.max_steps, sub.seed, sub.rng_id, 0, sub.param, obs_mode,
                 sprites)
    s = ox.State.empty(b)
    threads = host_threads()
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


def snapshot(env, traj, row: int, with_obs: bool) -> dict:
    """Host copy of the state and of output row `row` (the timed rollout's
    last step; its observations only if with_obs), taken before later runs
    move them on."""
    last = {f: (None if getattr(traj, f) is None else getattr(traj, f)[row].cpu().numpy())
            for f in ("reward", "flags", "action", "mission")}
    last["obs"] = traj.obs[row].cpu().numpy() if with_obs and traj.obs is not None else None
    return {"state": env.state_numpy(), "last": last}


def oracle_parity(table, snap: dict, n_steps: int, obs_mode: int, max_env_steps: float = 2e8) -> dict:
    """The timed run against the oracle: every env (or an even sample of
    them when that is more than max_env_steps of CPU work) reset and stepped
    n_steps times by the random policy, as the GPU did since the rollout's
    reset; its state and last output row compared bit for bit (first-person
    observations included)."""
    import oracle as ox
    n = table.n
    n_check = int(min(n, max(64, max_env_steps // max(1, n_steps))))
    idx = np.unique(np.linspace(0, n - 1, n_check).round().astype(np.int64))
    sub = table.subset(idx)
    check_obs = obs_mode in (0, 1)
    b = ox.Batch(sub.family, sub.side, sub.max_steps, sub.seed, sub.rng_id, 0, sub.param,
                 obs_mode if check_obs else 0)
    s = ox.State.empty(b)
    threads = host_threads()
    t0 = time.perf_counter()
    ox.reset(b, s, nthreads=threads)
    ref = ox.rollout(b, s, n_steps, None, rows=1, with_obs=check_obs, nthreads=threads)
    dt = time.perf_counter() - t0
    g = snap["state"]
    sides = table.side.astype(np.int64)
    off = np.concatenate([[0], np.cumsum(3 * sides * sides)])
    gpu = {"grid": np.concatenate([g["grid"][off[i]:off[i + 1]] for i in idx]),
           "obst": g["obst"].reshape(n, -1)[idx].reshape(-1)}
    for f in ("x", "y", "dir", "t", "carry", "episode", "done_prev", "calls"):
        gpu[f] = g[f][idx]
    bad = [f for f in gpu if not np.array_equal(gpu[f].view(getattr(s, f).dtype), getattr(s, f))]
    last = snap["last"]
    for f in ("reward", "flags", "action", "mission"):
        r = getattr(ref, f)
        if last[f] is not None and r is not None:
            a = last[f][idx]
            if not np.array_equal(a.view(np.uint8), r[0].view(np.uint8)):
                bad.append(f"last row {f}")
    if check_obs and last["obs"] is not None and not np.array_equal(last["obs"][idx], ref.obs[0]):
        bad.append("last row obs")
    return {"envs": int(len(idx)), "of": n, "steps_since_reset": n_steps,
            "compared": "state and the last output row" + (" with observations" if check_obs else ""),
            "bit_exact": not bad, "mismatch": bad, "oracle_s": round(dt, 2)}


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def serving_run(ge, wl, srv, n_requests, rate, K, budget, arena, inflight, host=None, seed=0) -> dict:
    reqs = wl.serving_requests(n_requests, rate, master_seed=seed)
    res = ge.serve_run(srv, reqs, K, budget, arena, max_inflight=inflight, host_arena=host)
    lat = res["latency_s"] * 1e3
    wait = (res["admit_s"] - res["arrival_s"]) * 1e3
    rec = {"requests": n_requests, "completed": res["completed"], "rate_req_per_s": rate,
           "env_steps_per_s": res["env_steps"] / res["wall_s"], "wall_s": res["wall_s"],
           "launches": res["launches"],
           "host_s": {"admit": res["host_admit_s"], "step": res["host_step_s"], "wait": res["host_wait_s"]},
           "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
           "admission_wait_ms": {"p50": pct(wait, 50), "p99": pct(wait, 99)}}
    if host is not None:
        hl = res["host_latency_s"] * 1e3
        rec["host_latency_ms"] = {"p50": pct(hl, 50), "p99": pct(hl, 99)}
    return rec


def run_serving(n_requests: int, loads, K: int, budget_gib: int, inflight: int = 2) -> dict:
    """Poisson serving: capacity from a saturated run (every request arrives
    at once), then fractions of it; once with results left in HBM, once
    with every request's scalar outputs delivered to pinned host memory."""
    import torch
    from paper_2407_19396_amd import gridenv as ge
    from paper_2407_19396_amd import workloads as wl

    probe = wl.serving_requests(4000, rate_per_s=1.0, master_seed=12345)
    ework = float(np.mean([r.n_envs * r.n_steps for r in probe]))
    srv = ge.Server(max_tiles=16384, max_side=19)
    budget = budget_gib << 30
    arena = torch.empty(budget - srv.info()["device_bytes"], dtype=torch.uint8, device="cuda")
    host = torch.empty(4 << 30, dtype=torch.uint8, pin_memory=True)
    out = {"K": K, "budget_gib": budget_gib, "mean_env_steps_per_request": ework,
           "request_mix": "log-uniform 1..8192 envs of the mixed workload, n_steps uniform 64..1024"}
    for name, h in (("device", None), ("host", host)):
        sat = serving_run(ge, wl, srv, n_requests, 1e9, K, budget, arena, inflight, h, seed=4321)
        cap = sat["env_steps_per_s"]
        log(f"[bench] serving ({name}-ready results) capacity: {cap / 1e9:.2f} G env-steps/s")
        levels = []
        for load in loads:
            rec = serving_run(ge, wl, srv, n_requests, load * cap / ework, K, budget, arena, inflight, h,
                              seed=int(load * 1000))
            rec["load"] = load
            key = "host_latency_ms" if h is not None else "latency_ms"
            log(f"[bench] serving load {load} ({name}): {rec['env_steps_per_s'] / 1e9:.2f} G env-steps/s, "
                f"latency p50 {rec[key]['p50']:.1f} ms p99 {rec[key]['p99']:.1f} ms")
            levels.append(rec)
        out[name] = {"capacity_env_steps_per_s": cap, "saturated": sat, "loads": levels}
    out["host"]["delivered"] = "reward, flags and action of every env-step (6 B) to pinned host memory; " \
                               "observations stay in HBM"
    srv.close()
    del arena, host
    return out


def plain_leg(ge, wl, table, n_steps: int, seed: int) -> dict:
    """A workload through the plain kernel, one launch per step, external
    uniform actions: rate over all launches and per-launch latency."""
    import torch
    env = ge.GridEnv(table)
    traj = env.traj(n_steps)
    rows = [traj.row(k) for k in range(n_steps)]
    acts = torch.from_numpy(wl.random_actions(n_steps, table.n, seed=seed)).to("cuda")
    stream = torch.cuda.current_stream()
    env.reset()
    for k in range(min(8, n_steps)):
        env.step(rows[k], acts[k])
    env.reset()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for k in range(n_steps):
        env.step(rows[k], acts[k])
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    lat = []
    env.reset()
    for k in range(n_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        env.step(rows[k], acts[k])
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    env.close()
    return {"value": table.n * n_steps / (ms / 1e3), "unit": "env-steps/s", "steps": n_steps,
            "kernel": "k_plain", "ms": ms, "launch_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)}}


def graph_leg(ge, wl, table, n_steps: int, warmup: int) -> dict:
    """A workload through the fused kernel with the on-device policy, K
    autotuned, the whole rollout captured in a HIP graph and its replay
    timed; per-chunk latency from eager launches of K steps."""
    import torch
    from paper_2407_19396_amd import autotune
    env = ge.GridEnv(table)
    Ks = tuple(k for k in (64, 128, 256, 512, 1024, 2048) if k <= n_steps)
    probe = env.traj(max(Ks))
    env.reset()
    tuned = autotune.tune(env, probe, Ks=Ks, steps=max(Ks), log=None)
    del probe
    K = env.info()["k_default"]
    traj = env.traj(K)
    env.reset()
    env.rollout(warmup, traj, K=K)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        env.rollout(n_steps, traj, K=K)
    graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    reps = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        graph.replay()
        b.record(stream)
        b.synchronize()
        reps.append(a.elapsed_time(b))
    ms = float(np.median(reps))
    lat = []
    for _ in range(16):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        env.rollout(K, traj, K=K)
        b.record(stream)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    info = env.info()
    cs = chunks(n_steps, K)
    total = sum(fused_bytes(table.n, info["grid_bytes"], k) for k in cs)
    roof = roofline_entry(total / len(cs), ms / len(cs), None, kernel="k_fused", launches=len(cs),
                          steps_per_launch=K, timing="median of 5 graph replays")
    env.close()
    del graph
    return {"value": table.n * n_steps / (ms / 1e3), "unit": "env-steps/s", "steps": n_steps, "K": K,
            "blocks": info["blocks"], "tile_envs": info["tile_envs"], "autotuned": True,
            "cached_tuning": bool(tuned.get("cached")),
            "hip_graph": True, "replay_ms": ms, "replay_ms_range": [min(reps), max(reps)],
            "chunk_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)}, "roofline": roof}


def run_configs(steps_c3: int, seed: int = 0) -> dict:
    from paper_2407_19396_amd import gridenv as ge
    from paper_2407_19396_amd import workloads as wl
    out = {}
    t = wl.workload_empty5(seed=seed)
    out["empty5_plain"] = {"workload": "16 Empty 5x5, T=100, 100 steps of external uniform actions, "
                                       "plain kernel (one launch per step)", **plain_leg(ge, wl, t, 100, 1)}
    t = wl.workload_empty8(seed=seed)
    out["empty8_plain"] = {"workload": "4096 Empty 8x8, T=256, 1000 steps of external uniform actions, "
                                       "plain kernel (one launch per step)", **plain_leg(ge, wl, t, 1000, 2)}
    t = wl.workload_tworoom8(seed=seed)
    out["tworoom8_graph"] = {"workload": f"65536 TwoRoom key/door 8x8, T=640, {steps_c3} steps, random "
                                         "policy on device, fused kernel, rollout captured in a HIP graph",
                             **graph_leg(ge, wl, t, steps_c3, 256)}
    for k, v in out.items():
        log(f"[bench] {k}: {v['value'] / 1e9:.3f} G env-steps/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4096, help="timed environment steps of the batch")
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of the same rollout, reported as median / min / max")
    ap.add_argument("--workload", default="mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0,
                    help="master seed of the workloads: keys every env's layouts and random policy "
                         "(the mix of families and sizes stays the same)")
    ap.add_argument("--envs", type=int, default=0, help="override the workload's env count")
    ap.add_argument("--K", type=int, default=0, help="steps fused per launch (0: autotune)")
    ap.add_argument("--blocks", type=int, default=0, help="persistent workgroups (0: autotune or default)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner, use library defaults")
    ap.add_argument("--tile-envs", type=int, default=0, help="envs per fused tile (0: autotune or 64)")
    ap.add_argument("--ring", type=int, default=0, help="trajectory ring rows (0: K)")
    ap.add_argument("--plain-steps", type=int, default=512)
    ap.add_argument("--latency-launches", type=int, default=-1,
                    help="launches of K steps timed one by one for the per-launch latency and the "
                         "steady-state roofline (-1: 8 to 64; 0: skip)")
    ap.add_argument("--obs", default="symbolic_first_person", choices=list(OBS_MODES),
                    help="observation function (the paper's names): symbolic_first_person (147 B) or "
                         "categorical_first_person (49 B), the whole grid: symbolic (3 S^2 B) or "
                         "categorical (S^2 B), or images drawn with the default sprites: "
                         "rgb_first_person (150528 B) or rgb (3072 S^2 B); the rgb modes default to "
                         "16384 envs and K = 16")
    ap.add_argument("--graph", action="store_true",
                    help="capture the timed rollout in a HIP graph and time its replay")
    ap.add_argument("--plain-actions", action="store_true",
                    help="plain steps take an external action buffer instead of the device policy")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the small-workload legs (Empty 5x5 and 8x8 plain, TwoRoom 8x8 graph)")
    ap.add_argument("--c3-steps", type=int, default=2048, help="steps of the TwoRoom 8x8 graph leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-envs", type=int, default=0, help="CPU oracle sample envs (0: all)")
    ap.add_argument("--cpu-steps", type=int, default=2048,
                    help="CPU oracle sample steps (about 10 s on 16 host threads for the mixed batch)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per serving run (0: skip serving)")
    ap.add_argument("--serve-K", type=int, default=256)
    ap.add_argument("--serve-inflight", type=int, default=2, help="launches enqueued ahead of the device")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95")
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the environment "
              "batch would shard by env id (each GPU steps its own envs; nothing is exchanged "
              "between them), so one GPU's share is what is measured.", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be at least 1 and --warmup at least 0")

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
    make = {"mixed": lambda: wl.workload_mixed(seed=args.seed, n=args.envs or 262144),
            "tworoom8": lambda: wl.workload_tworoom8(seed=args.seed),
            "empty8": lambda: wl.workload_empty8(seed=args.seed),
            "empty5": lambda: wl.workload_empty5(seed=args.seed),
            "empty24": lambda: wl.uniform_table(args.envs or 65536, wl.FAMILY_EMPTY, 24, seed=args.seed),
            "empty32": lambda: wl.uniform_table(args.envs or 65536, wl.FAMILY_EMPTY, 32, seed=args.seed),
            "tworoom32": lambda: wl.uniform_table(args.envs or 65536, wl.FAMILY_TWOROOM, 32, seed=args.seed),
            "lava": lambda: wl.workload_lava(seed=args.seed, n=args.envs or 262144),
            "dynobs": lambda: wl.workload_dynobs(seed=args.seed, n=args.envs or 262144),
            "gotodoor": lambda: wl.workload_gotodoor(seed=args.seed, n=args.envs or 262144),
            "keycorridor": lambda: wl.workload_keycorridor(seed=args.seed, n=args.envs or 262144)}[args.workload]
    obs_mode = OBS_MODES[args.obs]
    rgb = obs_mode >= 4
    if rgb and not args.envs:
        args.envs = 16384          # a step writes 2.5 GB of first-person images at this size
    table = make()
    if args.envs and args.workload not in ("mixed", "lava", "dynobs", "gotodoor", "keycorridor", "empty24",
                                           "empty32", "tworoom32"):
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
    elif args.K or args.blocks or args.no_tune or args.tile_envs:
        if args.tile_envs:
            env.set_tiling(args.tile_envs)
        env.set_launch(args.K or env.info()["k_default"], args.blocks)
    else:
        from paper_2407_19396_amd import autotune
        # K up to 1024, as long as a ring of K rows stays within RING_BUDGET
        row_bytes = table.n * (obs_bytes + 6)
        Ks = [k for k in (128, 256, 512, 1024) if k * row_bytes <= RING_BUDGET] or [128]
        probe = env.traj(max(Ks))
        env.reset(first)
        tuned = autotune.tune(env, probe, Ks=tuple(Ks), steps=args.steps, log=log)
        del probe
        log(f"[bench] autotuned tile_envs={tuned['tile_envs']} K={tuned['K']} blocks={tuned['blocks']}")
    info = env.info()
    K = info["k_default"]
    ring = args.ring or K
    log(f"[bench] {table.name}: grid {info['grid_bytes'] / 1e6:.1f} MB, tiles {info['n_tiles']}, "
        f"LDS/WG {info['lds_bytes']} B, blocks {info['blocks']}, K {K}, ring {ring}")
    traj = env.traj(ring)
    if not np.any(table.family == 7):
        traj.mission = None       # the mission output only carries GoToDoor's target
    # about 0.3 s of untimed rollouts of the timed length first, so that the
    # GPU runs at its working clocks whether or not the tuner has just run
    # (a cached tuning leaves it idle until here); they launch exactly what
    # the timed region launches, so a kernel trace of the run holds launches
    # of that one shape; the reset below starts the measured sequence afresh
    env.reset(first)
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < 0.3:
        env.rollout(args.steps, traj, K=K)
        torch.cuda.synchronize()
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
    # every step since the reset before the warmup (the graph's untimed
    # replay included), for the oracle's check of the timed run
    since_reset = args.warmup + args.steps * (2 if graph is not None else 1)
    snap = None if args.no_cpu else snapshot(env, traj, (args.steps - 1) % ring, obs_mode in (0, 1))
    timed_chunks = chunks(args.steps, K)
    env_steps = table.n * args.steps
    value = env_steps / (ms / 1e3)
    log(f"[bench] fused: {args.steps} steps in {ms:.3f} ms ({wall * 1e3:.1f} ms wall), "
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
    # per-launch latency of the fused kernel at K steps per launch
    lat = []
    n_lat = args.latency_launches if args.latency_launches >= 0 else min(64, max(8, len(timed_chunks)))
    for _ in range(n_lat):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        env.rollout(K, traj, K=K)
        b.record(stream)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    lat = np.array(lat)

    # plain kernel on the same input, writing a ring of the same size
    plain = None
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
        plain = {"value": plain_rate, "unit": "env-steps/s", "steps": args.plain_steps,
                 "launch_ms": {"p50": pct(pl, 50), "p99": pct(pl, 99)},
                 "fused_over_plain": value / plain_rate}
        if obs_mode == 0:
            # algorithmic bytes of a plain step: state, view cells (at most 49 in the grid), record
            cells = float(np.mean(np.minimum(49, table.side.astype(np.int64) ** 2)))
            per_step = table.n * (PLAIN_READ + 3 * cells + PLAIN_WRITE + RECORD_BYTES)
            plain["roofline"] = roofline_entry(per_step, pms / args.plain_steps,
                                               profile_traffic(args.workload, 1, table.n, "k_plain"),
                                               kernel="k_plain", bytes_per_env_step=per_step / table.n)
        log(f"[bench] plain: {plain_rate / 1e9:.2f} G env-steps/s, launch p50 "
            f"{plain['launch_ms']['p50'] * 1e3:.1f} us")

    # roofline of the dominant kernel over the timed region: the algorithmic
    # bytes of the steps each launch ran (the state term once per launch)
    def launch_bytes(k):
        if rgb:
            return rgb_path_bytes(table.n, info["grid_bytes"], k, obs_bytes / RGB_SCALE)
        return fused_bytes(table.n, info["grid_bytes"], k, obs_bytes)

    def traffic_of(ks):
        if rgb or obs_mode != 0:
            return None
        ts = [profile_traffic(args.workload, k, table.n) for k in ks]
        return None if any(t is None for t in ts) else sum(ts) / len(ts)

    kernel = "k_fused + k_sprite_ids + k_render" if rgb else "k_fused"
    roof = roofline_entry(sum(launch_bytes(k) for k in timed_chunks) / len(timed_chunks),
                          ms / len(timed_chunks), traffic_of(timed_chunks), kernel=kernel,
                          launches=len(timed_chunks), steps_per_launch=sorted(set(timed_chunks)),
                          timing="HIP events around the timed rollout")
    if len(lat):
        roof["steady_state"] = roofline_entry(launch_bytes(K), float(np.mean(lat)), traffic_of([K]),
                                              steps_per_launch=K, launches=len(lat),
                                              timing="HIP events around each launch of K steps, mean")

    del traj, env, first
    torch.cuda.empty_cache()
    configs = None
    if not args.no_configs and args.workload == "mixed" and obs_mode == 0:
        configs = run_configs(args.c3_steps, args.seed)
    serving = None
    if args.serve_requests > 0 and args.workload == "mixed" and obs_mode == 0:
        loads = tuple(float(x) for x in args.serve_loads.split(","))
        serving = run_serving(args.serve_requests, loads, args.serve_K, args.serve_budget_gib,
                              args.serve_inflight)
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a sample")
        if rgb:   # the oracle draws every pixel: a smaller sample
            cpu = cpu_baseline(table, min(args.cpu_envs or 4096, table.n), min(args.cpu_steps, 1024),
                               obs_mode, sprites)
        else:
            cpu = cpu_baseline(table, min(args.cpu_envs or table.n, table.n), args.cpu_steps, obs_mode)
        log(f"[bench] cpu oracle: {cpu['value'] / 1e6:.2f} M env-steps/s on {cpu['cores']} threads")
        cpu["parity"] = oracle_parity(table, snap, since_reset, obs_mode)
        snap = None
        par = cpu["parity"]
        log(f"[bench] timed run vs oracle ({par['envs']} of {par['of']} envs, {since_reset} steps): "
            + ("bit-exact" if par["bit_exact"] else f"MISMATCH in {', '.join(par['mismatch'])}"))

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
                   "tile_envs": info["tile_envs"],
                   "lds_bytes_per_wg": info["lds_bytes"], "max_tile_cells": info["max_tile_cells"],
                   "global_batch": table.n, "autotuned": tuned is not None,
                   "hip_graph": graph is not None, "observation": args.obs, "seed": args.seed},
        "fused_launch_ms": {"K": K, "p50": pct(lat, 50), "p99": pct(lat, 99)} if len(lat) else None,
        "repeats": None if not reps else {"n": len(reps), "median": float(np.median(reps)),
                                          "min": float(np.min(reps)), "max": float(np.max(reps)),
                                          "values": [float(r) for r in reps]},
        "plain": plain,
        "roofline": roof,
        "configs": configs,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if cpu is not None and not cpu["parity"]["bit_exact"]:
        sys.exit("bench: the timed run does not match the oracle")


if __name__ == "__main__":
    main()
