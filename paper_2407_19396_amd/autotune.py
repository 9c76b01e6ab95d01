"""Launch-shape autotuner for the fused rollout kernel.

The fused kernel's speed depends on two choices the library cannot know in
advance: K, the steps fused per launch (longer chunks amortise loading and
storing each tile's grids, shorter ones bound the latency of a chunk), and
the number of persistent workgroups (more hide latency better, but tiles
are handed out in whole rounds, so a count that does not divide the tile
count leaves the last round partly idle).  ``tune`` times short rollouts
of the actual batch for each candidate and keeps the fastest, caching the
choice on disk per device and batch composition.

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


def block_candidates(n_tiles: int, lds_bytes: int, cus: int, lds_per_cu: int = 160 * 1024) -> list[int]:
    """Workgroup counts worth trying: the largest that fits the LDS of every
    CU, smaller ones, and those that make every workgroup take the same
    number of tiles."""
    fit = max(1, min(16, lds_per_cu // max(1, lds_bytes)))
    out = set()
    for p in range(max(1, fit - 2), fit + 1):
        out.add(min(n_tiles, p * cus))
    for rounds in range(1, 9):
        b = -(-n_tiles // rounds)
        if b <= fit * cus:
            out.add(b)
    return sorted(out)


def tune(env, traj, Ks=(128, 256, 512), steps: int = 1024, use_cache: bool = True, log=None) -> dict:
    import torch
    from . import gridenv as ge

    dev = torch.cuda.current_device()
    props = torch.cuda.get_device_properties(dev)
    Ks = [k for k in Ks if k <= traj.rows]
    key = batch_key(env.table, props.name, env.obs_mode, env.reward_mode, Ks)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache and cache[key].get("K") in Ks:
        best = cache[key]
        env.set_launch(best["K"], best["blocks"])
        return best | {"cached": True}

    info = env.info()
    blocks = block_candidates(info["n_tiles"], info["lds_bytes"], props.multi_processor_count)
    results = []
    stream = torch.cuda.current_stream()
    for K in Ks:
        for b in blocks:
            env.set_launch(K, b)
            env.rollout(K, traj, K=K)          # warm this shape
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            n = max(K, (steps // K) * K)
            a.record(stream)
            env.rollout(n, traj, K=K)
            z.record(stream)
            z.synchronize()
            rate = env.n * n / (a.elapsed_time(z) / 1e3)
            results.append({"K": K, "blocks": b, "rate": rate})
            if log:
                log(f"[autotune] K={K} blocks={b}: {rate / 1e9:.2f} G env-steps/s")
    best = max(results, key=lambda r: r["rate"])
    env.set_launch(best["K"], best["blocks"])
    if use_cache:
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            cache[key] = {"K": best["K"], "blocks": best["blocks"], "rate": best["rate"]}
            json.dump(cache, open(CACHE, "w"), indent=1)
        except OSError:
            pass
    return best | {"cached": False, "trials": results}
