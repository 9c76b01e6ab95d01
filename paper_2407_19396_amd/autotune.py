"""Launch-shape autotuner for the fused rollout kernel.

The fused kernel's speed depends on three choices the library cannot know
in advance: the envs per tile (one env per lane; fewer than a wave's 64
lanes need less LDS per workgroup, so more workgroups fit a compute unit,
which pays for large grids), K, the steps fused per launch (longer chunks amortise loading and
storing each tile's grids, shorter ones bound the latency of a chunk), and
the number of workgroups (one per tile lets the hardware start each tile
wherever a workgroup slot frees up; fewer are persistent and take their
tiles in whole rounds, so a count that does not divide the tile count
leaves the last round partly idle, which matters most for short rollouts,
where the grids' staging is a large share of a launch).
``tune`` times rollouts of the actual batch and length for each candidate
and keeps the fastest, caching the choice on disk per device, batch
composition and rollout length.

Tuning steps the envs: call it before the real run and reset afterwards.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gridenv", "autotune.json")


def batch_key(table, device_name: str, obs_mode: int = 0, reward_mode: int = 0, Ks=()) -> str:
    """Cache key of a tuning: the device, the batch's composition (families,
    sides, parameters, limits), the observation and reward modes (each
    observation mode runs its own kernel variant), the K candidates and the
    kernel's code, so that an edited kernel is tuned afresh."""
    from .profiling import kernel_source_hash
    h = hashlib.sha256()
    for a in (table.family, table.side, table.param, table.max_steps):
        h.update(np.ascontiguousarray(a).tobytes())
    ks = ",".join(str(k) for k in Ks)
    return (f"{device_name}|{table.n}|{h.hexdigest()[:16]}|obs{obs_mode}|rew{reward_mode}|K{ks}|"
            f"code{kernel_source_hash()}")


def resident_blocks(n_tiles: int, lds_bytes: int, cus: int, lds_per_cu: int = 160 * 1024) -> int:
    """The most workgroups that are resident at once by LDS (at most 16 per
    compute unit), or the tile count if that is smaller."""
    fit = max(1, min(16, lds_per_cu // max(1, lds_bytes)))
    return min(n_tiles, fit * cus)


def block_candidates(n_tiles: int, lds_bytes: int, cus: int, lds_per_cu: int = 160 * 1024) -> list[int]:
    """Workgroup counts worth trying: the largest that fits the LDS of every
    CU, smaller ones, those that make every workgroup take the same number
    of tiles, and one workgroup per tile.  With more tiles than fit at once
    the last gives up persistence: a later workgroup starts wherever an
    earlier one has finished, instead of each workgroup taking its next tile
    in turn, which balances short rollouts of tiles with uneven work."""
    fit = max(1, min(16, lds_per_cu // max(1, lds_bytes)))
    out = {n_tiles}
    for p in range(max(1, fit - 2), fit + 1):
        out.add(min(n_tiles, p * cus))
    for rounds in range(1, 9):
        b = -(-n_tiles // rounds)
        if b <= fit * cus:
            out.add(b)
    return sorted(out)


def _time_rollout(env, traj, steps: int, K: int, stream, budget_ms: float = 30.0) -> float:
    """Mean milliseconds of a `steps`-step rollout at K steps per launch:
    one untimed run, then enough timed runs to fill about budget_ms."""
    import torch
    env.rollout(steps, traj, K=K)
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    env.rollout(steps, traj, K=K)
    z.record(stream)
    z.synchronize()
    one = max(a.elapsed_time(z), 1e-3)
    reps = int(min(50, max(1, budget_ms // one)))
    if reps == 1:
        return one
    a.record(stream)
    for _ in range(reps):
        env.rollout(steps, traj, K=K)
    z.record(stream)
    z.synchronize()
    return a.elapsed_time(z) / reps


def tune(env, traj, Ks=(128, 256, 512), steps: int = 0, tile_envs=(64, 32, 16), use_cache: bool = True,
         log=None) -> dict:
    """Pick the envs per tile, K and the workgroup count for rollouts of
    `steps` steps (0: one launch of each candidate K, the steady state).

    First the envs per tile (each tiling at one workgroup per tile and at
    the count resident at once by LDS, K the largest candidate: large grids
    can run a tiling faster in persistent workgroups), then K x workgroups
    for the best tiling.  When `steps` is shorter than every candidate K,
    all of them run the same single launch, so only the workgroup count is
    searched (at the largest K, which later full launches then use)."""
    import torch

    dev = torch.cuda.current_device()
    props = torch.cuda.get_device_properties(dev)
    Ks = [k for k in Ks if k <= traj.rows]
    Es = [e for e in tile_envs if 1 <= e <= 64]
    if not Ks or not Es:
        raise ValueError(f"nothing to tune: no K candidate fits a ring of {traj.rows} rows "
                         f"or no envs per tile in 1..64 (Ks {Ks}, tile_envs {tuple(tile_envs)})")
    key = (batch_key(env.table, props.name, env.obs_mode, env.reward_mode, Ks) +
           f"|steps{steps}|E{','.join(str(e) for e in Es)}")
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            with open(CACHE) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache and cache[key].get("K") in Ks and cache[key].get("tile_envs") in Es:
        best = cache[key]
        env.set_tiling(best["tile_envs"])
        env.set_launch(best["K"], best["blocks"])
        return best | {"cached": True}

    search = [max(Ks)] if 0 < steps <= min(Ks) else Ks
    stream = torch.cuda.current_stream()
    results = []

    def trial(E, K, b):
        n = steps if steps > 0 else K
        env.set_launch(K, b)
        ms = _time_rollout(env, traj, n, K, stream)
        r = {"tile_envs": E, "K": K, "blocks": b, "lds_bytes": env.info()["lds_bytes"],
             "rate": env.n * n / (ms / 1e3)}
        results.append(r)
        if log:
            log(f"[autotune] E={E} K={K} blocks={b} ({n}-step rollouts): {r['rate'] / 1e9:.2f} G env-steps/s")
        return r

    # stage 1: envs per tile
    firsts = []
    for E in Es:
        env.set_tiling(E)
        info = env.info()
        counts = sorted({info["blocks"], resident_blocks(info["n_tiles"], info["lds_bytes"],
                                                         props.multi_processor_count)})
        firsts.append(max((trial(E, max(search), b) for b in counts), key=lambda r: r["rate"]))
    E = max(firsts, key=lambda r: r["rate"])["tile_envs"]
    # stage 2: K x workgroups at that tiling
    env.set_tiling(E)
    info = env.info()
    for K in search:
        for b in block_candidates(info["n_tiles"], info["lds_bytes"], props.multi_processor_count):
            trial(E, K, b)
    best = max((r for r in results if r["tile_envs"] == E), key=lambda r: r["rate"])
    env.set_launch(best["K"], best["blocks"])
    if use_cache:
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            cache[key] = {k: best[k] for k in ("tile_envs", "K", "blocks", "lds_bytes", "rate")} | {"steps": steps}
            # written whole and then renamed, so a concurrent reader sees the
            # old file or the new one
            tmp = f"{CACHE}.{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, CACHE)
        except OSError:
            pass
    return best | {"cached": False, "trials": results, "steps": steps}
