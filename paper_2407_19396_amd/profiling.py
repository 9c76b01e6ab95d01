"""rocprofv3 summaries for the step kernels.

``summarize`` turns the CSV output of a kernel-trace run and of FETCH_SIZE /
WRITE_SIZE (and optional SQ) counter runs into a short text summary for
``profiles/``.  The HBM byte counters are calibrated against a plain
device-to-device copy of known size recorded in the same runs (the copy
reads and writes exactly that many bytes).  The summary ends with one
machine-readable line that ``traffic_bytes`` reads back for the benchmark;
it is ignored once the kernel's code has changed (comments and layout
aside).

    python -m paper_2407_19396_amd.profiling --trace DIR --fetch DIR --write DIR
        [--sq DIR] --copy-bytes N --K K --envs N [--kernel k_plain] --command "..." -o profiles/x.txt

``render_summary`` covers the rgb path: the renderer's launches of K rows
(the one-row launch after a reset left out) against their algorithmic bytes,
with its calibrated HBM traffic, and the fused launches beside them.

    python -m paper_2407_19396_amd.profiling --render-trace DIR --fetch DIR --write DIR
        --copy-bytes N --K K --envs N --command "..." -o profiles/z.txt

``serving_summary`` reads the kernel trace of a serving run instead: how
busy the device was between the first and the last serving launch, and the
launches' durations and gaps.

    python -m paper_2407_19396_amd.profiling --serving-trace DIR --command "..." -o profiles/y.txt

``store_ceilings`` measures, without a profiler, what plain fills and copies
and the fused kernel's own record store pattern reach on the GPU.

    python -m paper_2407_19396_amd.profiling --ceilings -o profiles/hbm_store_ceilings.txt
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")
KERNEL_SOURCES = (KERNEL_SOURCE, os.path.join(HERE, "csrc", "launch.h"))
COPY_KERNEL = "copyBuffer"
FUSED = "k_fused"
PLAIN = "k_plain"
RENDER = "k_render"
RGB_FIRST_PERSON_BYTES = 224 * 224 * 3
RENDER_SOURCES = (os.path.join(HERE, "csrc", "render.hip"), os.path.join(HERE, "csrc", "render.h"))


def _code_only(text: str) -> str:
    """The source without its comments and with blank space collapsed: a
    change to either leaves the compiled kernel as it was."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(paths=KERNEL_SOURCES) -> str:
    """Hash of the kernel's code: the kernel source and the launch header."""
    h = hashlib.sha256()
    for p in ([paths] if isinstance(paths, str) else paths):
        with open(p) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def _one(pattern: str) -> str:
    """The first file matching dir/pattern, in dir or below it (rocprofv3
    may add host and process subdirectories)."""
    d, base = os.path.split(pattern)
    hits = sorted(glob.glob(pattern)) or sorted(glob.glob(os.path.join(d, "**", base), recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def _counters(directory: str) -> dict:
    """{(kernel key, counter): [values per dispatch]}"""
    path = _one(os.path.join(directory, "*counter_collection.csv"))
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        key = FUSED if FUSED in name else PLAIN if PLAIN in name else COPY_KERNEL if COPY_KERNEL in name else None
        if key:
            out[(key, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return out


def _stats(directory: str) -> dict:
    path = _one(os.path.join(directory, "*kernel_stats.csv"))
    out = {}
    for r in csv.DictReader(open(path)):
        name = r["Name"]
        key = FUSED if FUSED in name else PLAIN if PLAIN in name else None
        if key:
            out[key] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                        "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
    return out


def _mean(xs):
    return sum(xs) / len(xs)


def _median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def summarize(trace: str, fetch: str, write: str, sq, copy_bytes: int, K: int,
              envs: int, command: str, source=KERNEL_SOURCES, kernel_name: str = FUSED,
              workload: str = "mixed", valu: str | None = None) -> str:
    """Summary of one kernel's launches (kernel_name: k_fused, launches of K
    steps; or k_plain, one step per launch).  sq: a directory or a list of
    directories of SQ counter runs; valu: a run of rocprofv3's derived
    VALUBusy and VALUUtilization (percentages: the share of the time the
    SIMDs' vector ALUs are busy, and the share of lanes active when they
    are); source: the sources the profiled library was built from.  Counters
    are the median over the kernel's dispatches (a k_plain run also holds a
    few reset launches, which the median leaves out)."""
    kernel = kernel_source_hash(source)
    st = _stats(trace)
    fc, wc = _counters(fetch), _counters(write)
    copy_fetch = _mean(fc[(COPY_KERNEL, "FETCH_SIZE")]) * 1024
    copy_write = _mean(wc[(COPY_KERNEL, "WRITE_SIZE")]) * 1024
    f_scale, w_scale = copy_bytes / copy_fetch, copy_bytes / copy_write
    k_fetch = _median(fc[(kernel_name, "FETCH_SIZE")]) * 1024 * f_scale
    k_write = _median(wc[(kernel_name, "WRITE_SIZE")]) * 1024 * w_scale
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            for r in _dispatches(trace, "*kernel_trace.csv", kernel_name, None)]
    shape = f"launches of K = {K} steps" if kernel_name == FUSED else "one step per launch"
    lines = [
        f"# {kernel_name} on the {workload} {envs}-env workload, {shape} (rocprofv3)",
        "",
        f"command: {command}",
        f"kernel code sha256[:16] (kernels.hip + launch.h, comments aside): {kernel}",
        f"steps per launch K = {K}, envs = {envs}",
        "",
        "## kernel trace (--kernel-trace --stats)",
    ]
    for k in (FUSED, PLAIN):
        if k in st:
            s_ = st[k]
            lines.append(f"{k}: calls {s_['calls']}, average {s_['avg_ns'] / 1e3:.1f} us, "
                         f"min {s_['min_ns'] / 1e3:.1f} us, max {s_['max_ns'] / 1e3:.1f} us")
    if durs:
        lines.append(f"{kernel_name} median dispatch (kernel trace): {_median(durs) / 1e3:.1f} us "
                     f"over {len(durs)} dispatches")
    lines += [
        "",
        "## HBM traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE; KiB per dispatch)",
        f"copy probe of {copy_bytes} bytes: FETCH_SIZE {copy_fetch / 1024:.0f} KiB, "
        f"WRITE_SIZE {copy_write / 1024:.0f} KiB -> scale fetch x{f_scale:.3f}, write x{w_scale:.3f}",
        f"{kernel_name} per launch (median): fetch {k_fetch / 1e6:.2f} MB, write {k_write / 1e6:.2f} MB (scaled)",
    ]
    if sq:
        wave_steps = envs / 64 * K
        lines += ["", "## SQ counters per launch, median (and per wave-step of 64 env-steps)"]
        for d in ([sq] if isinstance(sq, str) else sq):
            qc = _counters(d)
            for (k, c), v in sorted(qc.items()):
                if k == kernel_name:
                    m = _median(v)
                    lines.append(f"{c}: {m:.4g} ({m / wave_steps:.1f} per wave-step)")
    if valu:
        lines += ["", "## vector ALU (--pmc VALUBusy VALUUtilization), median over dispatches"]
        for (k, c), v in sorted(_counters(valu).items()):
            if k == kernel_name:
                lines.append(f"{c}: {_median(v):.1f} %")
    avg = st.get(kernel_name, {}).get("avg_ns", 0)
    lines += ["", f"machine: name={kernel_name} traffic_bytes_per_launch={k_fetch + k_write:.0f} K={K} "
                  f"envs={envs} kernel={kernel} avg_ns={avg:.0f} median_ns={_median(durs) if durs else 0:.0f}"]
    return "\n".join(lines) + "\n"


def traffic_bytes(profile_path: str, K: int, envs: int, kernel_name: str = FUSED) -> float | None:
    """Calibrated HBM bytes per launch of a kernel from a committed summary,
    or None if it is missing or was taken for another kernel source, K or
    size."""
    if not os.path.exists(profile_path):
        return None
    for line in open(profile_path):
        if line.startswith("machine:"):
            kv = dict(tok.split("=", 1) for tok in line.split()[1:])
            if (kv.get("name", FUSED) == kernel_name and kv.get("kernel") == kernel_source_hash()
                    and int(kv["K"]) == K and int(kv["envs"]) == envs):
                return float(kv["traffic_bytes_per_launch"])
    return None


def _dispatches(directory: str, pattern: str, key: str, column: str) -> list:
    """Per-dispatch values of one kernel, in dispatch order."""
    path = _one(os.path.join(directory, pattern))
    rows = [r for r in csv.DictReader(open(path)) if key in r["Kernel_Name"]]
    if "Dispatch_Id" in (rows[0] if rows else {}):
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows if column is None else [float(r[column]) for r in rows]


def render_summary(trace: str, fetch: str, write: str, copy_bytes: int, K: int, envs: int,
                   command: str) -> str:
    """The rgb first-person path: renderer launches of K rows each."""
    tr = _dispatches(trace, "*kernel_trace.csv", RENDER, None)
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in tr]
    full = [d for d in dur if d > 0.5 * max(dur)]          # the one-row reset launch left out
    fused = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
             for r in _dispatches(trace, "*kernel_trace.csv", FUSED, None)]
    ids = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
           for r in _dispatches(trace, "*kernel_trace.csv", "k_sprite_ids", None)]
    fc, wc = _counters(fetch), _counters(write)
    f_scale = copy_bytes / (_mean(fc[(COPY_KERNEL, "FETCH_SIZE")]) * 1024)
    w_scale = copy_bytes / (_mean(wc[(COPY_KERNEL, "WRITE_SIZE")]) * 1024)
    rf = _dispatches(fetch, "*counter_collection.csv", RENDER, "Counter_Value")
    rw = _dispatches(write, "*counter_collection.csv", RENDER, "Counter_Value")
    big_f = [v for v, w in zip(rf, rw) if w > 0.5 * max(rw)]
    big_w = [w for w in rw if w > 0.5 * max(rw)]
    r_fetch = _mean(big_f) * 1024 * f_scale
    r_write = _mean(big_w) * 1024 * w_scale
    algo = K * envs * (147 + 7 + RGB_FIRST_PERSON_BYTES + 7)
    avg = _mean(full)
    h = hashlib.sha256()
    for p in RENDER_SOURCES:
        h.update(_code_only(open(p).read()).encode())
    lines = [
        f"# k_render, rgb_first_person, {envs} mixed envs, launches of K = {K} rows (rocprofv3)",
        "",
        f"command: {command}",
        f"renderer code sha256[:16] (render.hip + render.h, comments aside): {h.hexdigest()[:16]}",
        "",
        "## kernel trace (--kernel-trace)",
        f"k_render, {K}-row launches: {len(full)}, average {avg / 1e3:.1f} us "
        f"(min {min(full) / 1e3:.1f}, max {max(full) / 1e3:.1f})",
        f"k_fused (fills the staging ring): {len(fused)} launches, average {_mean(fused) / 1e3:.1f} us",
        f"k_sprite_ids (the renderer's index pass, K rows): average {_mean(sorted(ids)[1:] or ids) / 1e3:.1f} us",
        f"algorithmic bytes per k_render launch: {algo} (K x envs x (147 + 7 read, 150528 + 7 written))",
        f"achieved: {algo / avg:.1f} GB/s = {algo / avg / 8000.0:.3f} of 8000 GB/s",
        "",
        "## HBM traffic per K-row launch (--pmc FETCH_SIZE, then --pmc WRITE_SIZE)",
        f"copy probe of {copy_bytes} bytes -> scale fetch x{f_scale:.3f}, write x{w_scale:.3f}",
        f"k_render: fetch {r_fetch / 1e6:.1f} MB, write {r_write / 1e6:.1f} MB (scaled); "
        f"traffic / algorithmic bytes = {(r_fetch + r_write) / algo:.3f}",
    ]
    return "\n".join(lines) + "\n"


def _is_serving_launch(name: str) -> bool:
    # the serving variant of the fused kernel: template arguments <false, true, ...>
    return FUSED in name and ("<false, true" in name or "ILb0ELb1E" in name)


def serving_summary(trace: str, command: str, split_ms: float = 20.0) -> str:
    """Device occupancy of serving runs from their --kernel-trace CSV: the
    serving launches, split into runs wherever the device sat idle for more
    than split_ms (a bench invocation serves several runs in a row)."""
    rows = list(csv.DictReader(open(_one(os.path.join(trace, "*kernel_trace.csv")))))
    spans = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)
    serve = [(a, b) for a, b, n in spans if _is_serving_launch(n)]
    if not serve:
        raise ValueError("no serving launches in the trace")
    runs, cur = [], [serve[0]]
    for a, b in serve[1:]:
        if (a - cur[-1][1]) / 1e6 > split_ms:
            runs.append(cur)
            cur = []
        cur.append((a, b))
    runs.append(cur)
    pct = lambda xs, q: xs[min(len(xs) - 1, int(q * (len(xs) - 1) + 0.5))]  # noqa: E731
    lines = [
        "# serving launches of k_fused (rocprofv3 --kernel-trace)",
        "",
        f"command: {command}",
        f"kernel code sha256[:16] (kernels.hip + launch.h, comments aside): {kernel_source_hash()}",
        f"runs: the serving launches split wherever the device was idle for more than {split_ms:g} ms",
    ]
    for k, run in enumerate(runs):
        t0, t1 = run[0][0], max(b for _, b in run)
        dur = sorted((b - a) / 1e6 for a, b in run)
        gaps = sorted((run[i + 1][0] - run[i][1]) / 1e3 for i in range(len(run) - 1)) or [0.0]
        others = collections.defaultdict(float)
        for a, b, n in spans:
            if a >= t0 and b <= t1 and not _is_serving_launch(n):
                others[n.split("(")[0][:60]] += (b - a) / 1e6
        busy = sum(dur)
        lines += [
            "",
            f"## run {k + 1}",
            f"serving launches: {len(run)}; span {(t1 - t0) / 1e6:.1f} ms; busy {busy:.1f} ms "
            f"({100.0 * busy / max((t1 - t0) / 1e6, 1e-9):.1f} % of the span)",
            f"launch duration ms: p50 {pct(dur, 0.5):.3f}, p99 {pct(dur, 0.99):.3f}, max {dur[-1]:.3f}",
            f"gap between launches us: p50 {pct(gaps, 0.5):.1f}, max {gaps[-1]:.1f}",
            "other kernels inside the span (ms): " +
            (", ".join(f"{kk} {v:.2f}" for kk, v in sorted(others.items(), key=lambda kv: -kv[1])) or "none"),
        ]
    return "\n".join(lines) + "\n"


def store_ceilings(n_envs: int = 262144, K: int = 1024, blocks: int = 2048, reps: int = 5) -> str:
    """Write bandwidths this GPU reaches with no environment work: torch's
    fill_ (write only) and copy_ (read + write) of large buffers, and the
    fused rollout's record store pattern (gx_probe_record_stores): its
    pieces as the fused kernel writes them (ending on 64-byte boundaries of
    the output), with non-temporal and with ordinary stores, and as two
    halves of each tile's block; each timed with HIP events (median of
    `reps` runs after one warm run)."""
    import ctypes
    import statistics
    import torch
    from . import gridenv

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            out.append(a.elapsed_time(b))
        return statistics.median(out)

    lines = ["# HBM store ceilings on this GPU (HIP events, median of %d runs)" % reps, ""]
    buf = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")
    ms = timed(lambda: buf.fill_(7))
    lines.append(f"torch fill_ of {buf.numel()} bytes: {ms:.3f} ms, {buf.numel() / ms / 1e6:.1f} GB/s (written)")
    half = buf.numel() // 2
    src, dst = buf[:half], buf[half:]
    ms = timed(lambda: dst.copy_(src))
    lines.append(f"torch copy_ of {half} bytes: {ms:.3f} ms, {2 * half / ms / 1e6:.1f} GB/s (read + written)")
    del buf, src, dst
    torch.cuda.empty_cache()

    L = gridenv.load()
    fn = L.gx_probe_record_stores
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    fn.argtypes = [P, P, P, P, I64, I32, I32, I32, I32, I32, P]
    fn.restype = ctypes.c_int
    obs = torch.empty(K * n_envs * 147, dtype=torch.uint8, device="cuda")
    rew = torch.empty(K * n_envs, dtype=torch.float32, device="cuda")
    flg = torch.empty(K * n_envs, dtype=torch.uint8, device="cuda")
    act = torch.empty(K * n_envs, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    # launches of K steps over a ring of K rows, and of 256 steps over a ring
    # of 256 rows, where the two piece patterns differ most
    for k, nt, aligned in ((K, 1, 1), (K, 0, 1), (K, 1, 0), (256, 1, 1), (256, 1, 0)):
        algo = k * n_envs * (147 + 4 + 1 + 1)

        def run(k=k, nt=nt, aligned=aligned):
            rc = fn(obs.data_ptr(), rew.data_ptr(), flg.data_ptr(), act.data_ptr(), n_envs, k, k, blocks, nt,
                    aligned, stream)
            if rc != 0:
                raise RuntimeError(f"gx_probe_record_stores failed: {rc}")
        ms = timed(run)
        pieces = "pieces ending on 64-byte boundaries" if aligned else "two 4704-byte halves per tile"
        lines.append(f"record store pattern of k_fused ({n_envs} envs, {k} steps over {k} rows, {blocks} "
                     f"workgroups, {pieces}, {'non-temporal' if nt else 'ordinary'} stores): {ms:.3f} ms for "
                     f"{algo} bytes, {algo / ms / 1e6:.1f} GB/s")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ceilings", action="store_true",
                    help="measure the HBM store ceilings on the current GPU (no profiler needed)")
    ap.add_argument("--serving-trace", help="kernel trace directory of a serving run")
    ap.add_argument("--render-trace", help="kernel trace directory of an rgb_first_person run")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq", action="append", help="SQ counter run directory (repeatable)")
    ap.add_argument("--valu", help="run directory of --pmc VALUBusy VALUUtilization")
    ap.add_argument("--source", nargs="+", default=list(KERNEL_SOURCES),
                    help="kernel source and launch header the profiled build used")
    ap.add_argument("--copy-bytes", type=int)
    ap.add_argument("--K", type=int)
    ap.add_argument("--envs", type=int)
    ap.add_argument("--kernel", default=FUSED, choices=(FUSED, PLAIN), help="kernel to summarise")
    ap.add_argument("--workload", default="mixed", help="workload name for the title")
    ap.add_argument("--command", default="")
    ap.add_argument("-o", "--out", required=True)
    a = ap.parse_args()
    if a.ceilings:
        text = (store_ceilings() + "\ncommand: python3 -m paper_2407_19396_amd.profiling --ceilings -o <file>\n")
    elif not a.command:
        ap.error("--command is needed")
    elif a.serving_trace:
        text = serving_summary(a.serving_trace, a.command)
    elif a.render_trace:
        if not (a.fetch and a.write and a.copy_bytes and a.K and a.envs):
            ap.error("--fetch, --write, --copy-bytes, --K and --envs are needed")
        text = render_summary(a.render_trace, a.fetch, a.write, a.copy_bytes, a.K, a.envs, a.command)
    else:
        if not (a.trace and a.fetch and a.write and a.copy_bytes and a.K and a.envs):
            ap.error("--trace, --fetch, --write, --copy-bytes, --K and --envs are needed")
        text = summarize(a.trace, a.fetch, a.write, a.sq, a.copy_bytes, a.K, a.envs, a.command, a.source,
                         a.kernel, a.workload, a.valu)
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
