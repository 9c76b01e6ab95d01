"""ctypes binding of libgridenv.so (C-ABI in include/gridenv.h).

Argument marshalling only: every step of the environment runs in the
library's gfx950 kernels.  torch provides device memory (tensors) and the
HIP stream.  The functions keep the C names; ``GridEnv`` bundles a context
with its state tensors.  A missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import workloads

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgridenv.so")

GX_OK, GX_EINVAL, GX_ENOMEM, GX_EDEVICE, GX_ESTATE, GX_EBUSY, GX_ESIZE = 0, -1, -2, -3, -4, -5, -6
GX_STATIC_MAX_ENVS = 262144
OBS_BYTES = 147
RGB_FIRST_PERSON = (224, 224, 3)
EXPORTS = ("env_create", "env_sizes", "env_info", "env_reset", "env_step", "env_rollout",
           "env_set_launch", "env_set_tiling", "env_destroy", "env_strerror",
           "env_server_create", "env_server_admit", "env_server_step", "env_server_release",
           "env_server_info", "env_server_destroy", "env_serve_run", "env_rollout_static")


class GxConfig(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("reward_mode", ctypes.c_int32), ("obs_mode", ctypes.c_int32),
                ("family", ctypes.c_void_p), ("side", ctypes.c_void_p), ("param", ctypes.c_void_p),
                ("max_steps", ctypes.c_void_p), ("seed", ctypes.c_void_p),
                ("seed_all", ctypes.c_uint64), ("rng_id", ctypes.c_void_p),
                ("sprites", ctypes.c_void_p)]


STATE_FIELDS = ("grid", "x", "y", "dir", "t", "carry", "episode", "done_prev", "calls", "obst")


class GxState(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in STATE_FIELDS]


class GxTraj(ctypes.Structure):
    _fields_ = [("obs", ctypes.c_void_p), ("reward", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("action", ctypes.c_void_p),
                ("rows", ctypes.c_int32), ("mission", ctypes.c_void_p)]


class GxInfo(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("max_tile_cells", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("k_default", ctypes.c_int32),
                ("grid_bytes", ctypes.c_uint64), ("obs_row_bytes", ctypes.c_uint64),
                ("tile_envs", ctypes.c_int32)]


class GxRequest(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("family", ctypes.c_void_p), ("side", ctypes.c_void_p), ("param", ctypes.c_void_p),
                ("max_steps", ctypes.c_void_p),
                ("obs", ctypes.c_void_p), ("reward", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("action", ctypes.c_void_p), ("stride", ctypes.c_int32)]


class GxServerInfo(ctypes.Structure):
    _fields_ = [("max_tiles", ctypes.c_int32), ("free_tiles", ctypes.c_int32),
                ("live_requests", ctypes.c_int32), ("max_side", ctypes.c_int32),
                ("device_bytes", ctypes.c_uint64)]


class GxServeItem(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("n_envs", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("env_offset", ctypes.c_int64)]


class GxServeOpts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("max_inflight", ctypes.c_int32), ("keep_obs", ctypes.c_int32),
                ("budget_bytes", ctypes.c_uint64), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_uint64), ("host_arena", ctypes.c_void_p),
                ("host_arena_bytes", ctypes.c_uint64), ("host_done_s", ctypes.c_void_p)]


class GxServeStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("env_steps", ctypes.c_uint64),
                ("completed", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("admit_s", ctypes.c_double), ("step_s", ctypes.c_double), ("wait_s", ctypes.c_double)]


class GridEnvError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status} ({env_strerror(status)})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2407_19396_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    L.env_create.argtypes = [ctypes.POINTER(GxConfig), ctypes.POINTER(P)]
    L.env_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(I32)]
    L.env_info.argtypes = [P, ctypes.POINTER(GxInfo)]
    L.env_reset.argtypes = [P, ctypes.POINTER(GxState), ctypes.POINTER(GxTraj), P]
    L.env_step.argtypes = [P, ctypes.POINTER(GxState), P, ctypes.POINTER(GxTraj), P]
    L.env_rollout.argtypes = [P, ctypes.POINTER(GxState), I32, P, ctypes.POINTER(GxTraj), I32, P]
    L.env_set_launch.argtypes = [P, I32, I32]
    L.env_set_tiling.argtypes = [P, I32]
    L.env_destroy.argtypes = [P]
    L.env_server_create.argtypes = [I32, I32, I32, ctypes.POINTER(P)]
    L.env_server_admit.argtypes = [P, ctypes.POINTER(GxRequest), ctypes.POINTER(I32)]
    L.env_server_step.argtypes = [P, I32, P, ctypes.POINTER(I32), I32, ctypes.POINTER(I32)]
    L.env_server_release.argtypes = [P, I32]
    L.env_server_info.argtypes = [P, ctypes.POINTER(GxServerInfo)]
    L.env_server_destroy.argtypes = [P]
    L.env_serve_run.argtypes = [P, ctypes.POINTER(GxServeItem), I32, P, P, P, P,
                                ctypes.POINTER(GxServeOpts), P, P, P, ctypes.POINTER(GxServeStats)]
    L.env_rollout_static.argtypes = [ctypes.POINTER(GxConfig), ctypes.POINTER(GxState), I32,
                                     ctypes.POINTER(GxTraj), I32, P, ctypes.POINTER(GxTraj), I32, P]
    L.env_strerror.argtypes = [ctypes.c_int]
    L.env_strerror.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f != "env_strerror":
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(fn: str, status: int):
    if status != GX_OK:
        raise GridEnvError(fn, status)


def env_strerror(status: int) -> str:
    return load().env_strerror(status).decode()


def _stream_ptr(stream) -> int | None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


# --------------------------------------------------------------- C names
def env_create(table: workloads.EnvTable, reward_mode: int = 0, obs_mode: int = 0,
               sprites: np.ndarray | None = None) -> int:
    """sprites: the atlas u8[264][32][32][3] of the rgb modes (4, 5)."""
    cfg, keep = _config(table, reward_mode, obs_mode, sprites)
    ctx = ctypes.c_void_p()
    _check("env_create", load().env_create(ctypes.byref(cfg), ctypes.byref(ctx)))
    del keep
    return ctx.value


def _config(table: workloads.EnvTable, reward_mode: int, obs_mode: int, sprites=None):
    """The gx_config of a table, and the host arrays it points into."""
    fam = np.ascontiguousarray(table.family, np.uint8)
    side = np.ascontiguousarray(table.side, np.uint8)
    ms = np.ascontiguousarray(table.max_steps, np.int32)
    seed = np.ascontiguousarray(table.seed, np.uint64)
    rid = np.ascontiguousarray(table.rng_id, np.uint32)
    par = np.ascontiguousarray(table.param, np.uint8)
    atlas = None
    if sprites is not None:
        atlas = np.ascontiguousarray(sprites, np.uint8)
        if atlas.shape != (264, 32, 32, 3):
            raise ValueError(f"sprite atlas must be [264][32][32][3], got {atlas.shape}")
    cfg = GxConfig(table.n, reward_mode, obs_mode, fam.ctypes.data, side.ctypes.data, par.ctypes.data,
                   ms.ctypes.data, seed.ctypes.data, 0, rid.ctypes.data,
                   atlas.ctypes.data if atlas is not None else None)
    return cfg, (fam, side, ms, seed, rid, par, atlas)


def env_rollout_static(table: workloads.EnvTable, state: GxState, reset: bool, first: GxTraj | None,
                       n_steps: int, actions_ptr: int | None, traj: GxTraj | None, K: int = 0,
                       reward_mode: int = 0, obs_mode: int = 0, stream=None):
    """env_create + (env_reset) + env_rollout of `table` without any
    allocation: the library's fixed tables hold up to GX_STATIC_MAX_ENVS envs."""
    cfg, keep = _config(table, reward_mode, obs_mode)
    _check("env_rollout_static",
           load().env_rollout_static(ctypes.byref(cfg), ctypes.byref(state), 1 if reset else 0,
                                     ctypes.byref(first) if first is not None else None, n_steps,
                                     actions_ptr, ctypes.byref(traj) if traj is not None else None, K,
                                     _stream_ptr(stream)))
    del keep


def env_sizes(ctx: int) -> tuple[int, int]:
    gb, n = ctypes.c_size_t(), ctypes.c_int32()
    _check("env_sizes", load().env_sizes(ctx, ctypes.byref(gb), ctypes.byref(n)))
    return gb.value, n.value


def env_info(ctx: int) -> dict:
    info = GxInfo()
    _check("env_info", load().env_info(ctx, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in GxInfo._fields_}


def env_reset(ctx: int, state: GxState, first: GxTraj | None, stream=None):
    _check("env_reset", load().env_reset(ctx, ctypes.byref(state),
                                         ctypes.byref(first) if first is not None else None,
                                         _stream_ptr(stream)))


def env_step(ctx: int, state: GxState, actions_ptr: int | None, out: GxTraj, stream=None):
    _check("env_step", load().env_step(ctx, ctypes.byref(state), actions_ptr, ctypes.byref(out),
                                       _stream_ptr(stream)))


def env_rollout(ctx: int, state: GxState, n_steps: int, actions_ptr: int | None, traj: GxTraj,
                K: int = 0, stream=None):
    _check("env_rollout", load().env_rollout(ctx, ctypes.byref(state), n_steps, actions_ptr,
                                             ctypes.byref(traj), K, _stream_ptr(stream)))


def env_set_launch(ctx: int, K: int, blocks: int = 0):
    _check("env_set_launch", load().env_set_launch(ctx, K, blocks))


def env_set_tiling(ctx: int, tile_envs: int):
    _check("env_set_tiling", load().env_set_tiling(ctx, tile_envs))


def env_destroy(ctx: int):
    _check("env_destroy", load().env_destroy(ctx))


# --------------------------------------------------------------- tensors
def check_buffer(t, what: str, dtype, numel: int, device) -> None:
    """A tensor whose pointer a kernel is given: contiguous, of `dtype`, on
    `device` and at least `numel` elements long (the kernels index it by the
    batch size and the step count alone, so a shorter one would be read or
    written past its end)."""
    on_device = t.is_cuda if device.type == "cuda" else t.device.type == device.type
    if (t.dtype is not dtype or t.numel() < numel or not t.is_contiguous() or not on_device
            or (device.index is not None and t.device.index != device.index)):
        raise ValueError(f"{what}: need a contiguous {dtype} tensor on {device} with at least {numel} "
                         f"elements, got {t.dtype} {tuple(t.shape)} on {t.device}"
                         f"{'' if t.is_contiguous() else ' (not contiguous)'}")


def check_traj(tr: "Traj", n: int, obs_row_bytes: int, device, stride: int | None = None) -> None:
    """Output rows for a batch of n envs: reward, flags, action (and mission,
    if given) of rows x stride records (stride = n unless given), obs (if
    given) of rows x obs_row_bytes bytes."""
    import torch
    recs = tr.rows * (n if stride is None else stride)
    check_buffer(tr.reward, "reward", torch.float32, recs, device)
    check_buffer(tr.flags, "flags", torch.uint8, recs, device)
    check_buffer(tr.action, "action", torch.uint8, recs, device)
    if tr.mission is not None:
        check_buffer(tr.mission, "mission", torch.uint8, recs, device)
    if tr.obs is not None:
        check_buffer(tr.obs, "obs", torch.uint8, tr.rows * obs_row_bytes, device)


@dataclass
class Traj:
    """Device output rows: obs u8 [rows][N][7][7][3] (mode 0), [rows][N][7][7]
    (mode 1), [rows][N][224][224][3] (mode 4) or [rows][row_bytes]
    (whole-grid modes 2, 3 and 5, records packed like the grids), or None;
    reward f32, flags u8, action u8 [rows][N]."""
    obs: object
    reward: object
    flags: object
    action: object
    mission: object = None   # u8 [rows][N]: the episode's mission (GoToDoor colour, else 0xFF)

    # A check (check_traj) holds for the buffers it saw: the record of the
    # last one keeps those tensors and their C view, and a buffer replaced
    # since is checked again.
    def _buffers(self) -> tuple:
        return (self.obs, self.reward, self.flags, self.action, self.mission)

    def checked_view(self, key) -> GxTraj | None:
        """The C view, if these buffers were checked for `key`."""
        ck = self.__dict__.get("_ck")
        if ck is None or ck[0] != key:
            return None
        b = ck[1]
        if (b[0] is self.obs and b[1] is self.reward and b[2] is self.flags and b[3] is self.action
                and b[4] is self.mission):
            return ck[2]
        return None

    def mark_checked(self, key) -> GxTraj:
        g = self.c()
        self.__dict__["_ck"] = (key, self._buffers(), g)
        return g

    @staticmethod
    def alloc(rows: int, n: int, device="cuda", with_obs: bool = True, obs_mode: int = 0,
              row_bytes: int = 0) -> "Traj":
        import torch
        shape = {0: (rows, n, 7, 7, 3), 1: (rows, n, 7, 7),
                 4: (rows, n) + RGB_FIRST_PERSON}.get(obs_mode, (rows, row_bytes))
        return Traj(torch.zeros(shape, dtype=torch.uint8, device=device) if with_obs else None,
                    torch.zeros((rows, n), dtype=torch.float32, device=device),
                    torch.zeros((rows, n), dtype=torch.uint8, device=device),
                    torch.zeros((rows, n), dtype=torch.uint8, device=device),
                    torch.zeros((rows, n), dtype=torch.uint8, device=device))

    @property
    def rows(self) -> int:
        return int(self.reward.shape[0])

    def row(self, k: int) -> "Traj":
        """Row k alone, as a one-row Traj (e.g. the output of one env_step)."""
        sl = lambda t: None if t is None else t[k:k + 1]   # noqa: E731
        r = Traj(sl(self.obs), sl(self.reward), sl(self.flags), sl(self.action), sl(self.mission))
        # one row of checked rows holds the same records per row
        ck = self.__dict__.get("_ck")
        if ck is not None and self.checked_view(ck[0]) is not None:
            r.mark_checked(ck[0])
        return r

    def c(self) -> GxTraj:
        return GxTraj(self.obs.data_ptr() if self.obs is not None else None, self.reward.data_ptr(),
                      self.flags.data_ptr(), self.action.data_ptr(), self.rows,
                      self.mission.data_ptr() if self.mission is not None else None)


class GridEnv:
    """A batch of envs on the current HIP device with its state tensors."""

    FIELDS = STATE_FIELDS

    def __init__(self, table: workloads.EnvTable, reward_mode: int = 0, device="cuda", obs_mode: int = 0,
                 sprites: np.ndarray | None = None):
        """obs_mode 4 (rgb_first_person) and 5 (rgb) draw with `sprites`, an
        atlas u8[264][32][32][3]; None takes sprites.default_atlas()."""
        import torch
        self.table = table
        self.obs_mode = obs_mode
        self.reward_mode = reward_mode
        self.device = torch.device(device)
        if obs_mode >= 4 and sprites is None:
            from .sprites import default_atlas
            sprites = default_atlas()
        self.ctx = env_create(table, reward_mode, obs_mode, sprites)
        grid_bytes, n = env_sizes(self.ctx)
        self.n = n
        dev = self.device
        self.grid = torch.zeros(max(grid_bytes, 1), dtype=torch.uint8, device=dev)
        self.x = torch.zeros(n, dtype=torch.int32, device=dev)
        self.y = torch.zeros(n, dtype=torch.int32, device=dev)
        self.dir = torch.zeros(n, dtype=torch.int32, device=dev)
        self.t = torch.zeros(n, dtype=torch.int32, device=dev)
        self.carry = torch.zeros(n, dtype=torch.int32, device=dev)
        self.episode = torch.zeros(n, dtype=torch.int32, device=dev)   # uint32 bits
        self.done_prev = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.calls = torch.zeros(n, dtype=torch.int32, device=dev)        # uint32 bits
        self.obst = torch.full((n * 16,), 0xFF, dtype=torch.uint8, device=dev)
        self._cstate = None
        self._row_bytes = int(self.info()["obs_row_bytes"])
        self._key = (self.n, self._row_bytes, self.device)
        self._u8 = torch.uint8

    def state(self) -> GxState:
        """The C view of the state tensors (built once: the tensors are
        allocated here and only ever written in place)."""
        if self._cstate is None:
            self._cstate = GxState(*[getattr(self, f).data_ptr() for f in self.FIELDS])
        return self._cstate

    def traj(self, rows: int, with_obs: bool = True) -> Traj:
        """Output rows shaped for this context's observation mode (checked
        for it from the start, and so are their rows)."""
        tr = Traj.alloc(rows, self.n, self.device, with_obs, self.obs_mode, self._row_bytes)
        check_traj(tr, self.n, self._row_bytes, self.device)
        tr.mark_checked(self._key)
        return tr

    def _out(self, tr: Traj) -> GxTraj:
        """The C view of output rows, their sizes checked against this batch
        (once per set of buffers and batch shape)."""
        g = tr.checked_view(self._key)
        if g is None:
            check_traj(tr, self.n, self._row_bytes, self.device)
            g = tr.mark_checked(self._key)
        return g

    def _actions(self, actions, n_steps: int) -> int | None:
        """Pointer of external actions u8 [n_steps][N], or None (the on-device
        random policy)."""
        if actions is None:
            return None
        check_buffer(actions, "actions", self._u8, n_steps * self.n, self.device)
        return actions.data_ptr()

    def reset(self, first: Traj | None = None, stream=None):
        env_reset(self.ctx, self.state(), self._out(first) if first is not None else None, stream)

    def step(self, out: Traj, actions=None, stream=None):
        env_step(self.ctx, self.state(), self._actions(actions, 1), self._out(out), stream)

    def rollout(self, n_steps: int, traj: Traj, actions=None, K: int = 0, stream=None):
        env_rollout(self.ctx, self.state(), n_steps, self._actions(actions, n_steps), self._out(traj), K,
                    stream)

    def set_launch(self, K: int, blocks: int = 0):
        env_set_launch(self.ctx, K, blocks)

    def set_tiling(self, tile_envs: int):
        env_set_tiling(self.ctx, tile_envs)

    def info(self) -> dict:
        return env_info(self.ctx)

    def state_numpy(self) -> dict:
        out = {f: getattr(self, f).cpu().numpy() for f in self.FIELDS}
        out["episode"] = out["episode"].view(np.uint32)
        out["calls"] = out["calls"].view(np.uint32)
        return out

    def load_state(self, st: dict):
        """Copy a host state (dict of numpy arrays) into the device tensors."""
        import torch
        for f in self.FIELDS:
            if f in st:
                a = np.ascontiguousarray(st[f])
            elif f == "obst":
                a = np.full(self.n * 16, 0xFF, np.uint8)
            else:
                a = np.zeros(self.n, np.uint32)
            if f in ("episode", "calls"):
                a = a.astype(np.uint32).view(np.int32)
            t = torch.from_numpy(a.copy()).to(self.device)
            getattr(self, f).copy_(t.view(getattr(self, f).shape))

    def close(self):
        if self.ctx:
            env_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- serving
def padded_stride(n_envs: int) -> int:
    """Row stride (envs) of a request's outputs: a multiple of 16 keeps every
    64-env tile's records 16-byte aligned."""
    return -(-n_envs // 16) * 16


class Server:
    """Continuous-batching server (env_server_* of the C-ABI)."""

    def __init__(self, max_tiles: int, max_side: int = 19, reward_mode: int = 0):
        self.ptr = ctypes.c_void_p()
        _check("env_server_create", load().env_server_create(max_tiles, max_side, reward_mode,
                                                              ctypes.byref(self.ptr)))
        # at most max_tiles requests are live, so one step call returns every
        # finished handle
        self._fin = (ctypes.c_int32 * max_tiles)()

    def admit(self, table: workloads.EnvTable, n_steps: int, out: Traj, stride: int) -> int | None:
        """Queue a request for the envs of `table` (its first seed keys them
        all); returns its handle, or None when no tiles are free now.
        `out` holds at least n_steps rows of `stride` records."""
        import torch
        if out.rows < n_steps or stride < table.n:
            raise ValueError(f"request outputs: need {n_steps} rows of stride >= {table.n}, "
                             f"got {out.rows} rows of stride {stride}")
        check_traj(out, table.n, stride * OBS_BYTES, torch.device("cuda"), stride=stride)
        fam = np.ascontiguousarray(table.family, np.uint8)
        side = np.ascontiguousarray(table.side, np.uint8)
        ms = np.ascontiguousarray(table.max_steps, np.int32)
        par = np.ascontiguousarray(table.param, np.uint8)
        req = GxRequest(table.n, n_steps, int(table.seed[0]), fam.ctypes.data, side.ctypes.data,
                        par.ctypes.data, ms.ctypes.data,
                        out.obs.data_ptr() if out.obs is not None else None,
                        out.reward.data_ptr(), out.flags.data_ptr(), out.action.data_ptr(), stride)
        h = ctypes.c_int32()
        rc = load().env_server_admit(self.ptr, ctypes.byref(req), ctypes.byref(h))
        if rc == GX_EBUSY:
            return None
        _check("env_server_admit", rc)
        return h.value

    def step(self, K: int, stream=None) -> list[int]:
        n = ctypes.c_int32()
        _check("env_server_step", load().env_server_step(self.ptr, K, _stream_ptr(stream), self._fin,
                                                         len(self._fin), ctypes.byref(n)))
        return [self._fin[i] for i in range(n.value)]

    def release(self, handle: int):
        _check("env_server_release", load().env_server_release(self.ptr, handle))

    def info(self) -> dict:
        i = GxServerInfo()
        _check("env_server_info", load().env_server_info(self.ptr, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in GxServerInfo._fields_}

    def close(self):
        if self.ptr:
            _check("env_server_destroy", load().env_server_destroy(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_run(server: Server, requests: list, K: int, budget_bytes: int, arena, keep_obs: bool = True,
              max_inflight: int = 2, stream=None, host_arena=None) -> dict:
    """Run a Poisson serving workload (workloads.serving_requests) through
    the native serving loop; returns throughput and per-request latencies.
    host_arena: a pinned host uint8 tensor to deliver each request's scalar
    outputs to (latency then also to the host), or None."""
    n = len(requests)
    items = (GxServeItem * max(n, 1))()
    fam, side, par, ms = [], [], [], []
    off = 0
    for i, r in enumerate(requests):
        items[i] = GxServeItem(r.arrival_s, r.n_envs, r.n_steps, r.seed, off)
        fam.append(r.table.family)
        side.append(r.table.side)
        par.append(r.table.param)
        ms.append(r.table.max_steps)
        off += r.n_envs
    fam = np.ascontiguousarray(np.concatenate(fam), np.uint8)
    side = np.ascontiguousarray(np.concatenate(side), np.uint8)
    par = np.ascontiguousarray(np.concatenate(par), np.uint8)
    ms = np.ascontiguousarray(np.concatenate(ms), np.int32)
    admit = np.zeros(n, np.float64)
    done = np.zeros(n, np.float64)
    host_done = np.full(n, -1.0, np.float64)
    if host_arena is not None and not host_arena.is_pinned():
        raise ValueError("host_arena must be pinned host memory")
    opts = GxServeOpts(K, max_inflight, 1 if keep_obs else 0, budget_bytes, arena.data_ptr(),
                       arena.numel() * arena.element_size(),
                       host_arena.data_ptr() if host_arena is not None else None,
                       host_arena.numel() * host_arena.element_size() if host_arena is not None else 0,
                       host_done.ctypes.data if host_arena is not None else None)
    st = GxServeStats()
    _check("env_serve_run", load().env_serve_run(server.ptr, items, n, fam.ctypes.data, side.ctypes.data,
                                                 par.ctypes.data, ms.ctypes.data, ctypes.byref(opts),
                                                 _stream_ptr(stream),
                                                 admit.ctypes.data, done.ctypes.data, ctypes.byref(st)))
    arrival = np.array([r.arrival_s for r in requests])
    return {"wall_s": st.wall_s, "env_steps": st.env_steps, "completed": st.completed,
            "launches": st.launches, "host_admit_s": st.admit_s, "host_step_s": st.step_s,
            "host_wait_s": st.wait_s, "arrival_s": arrival, "admit_s": admit, "done_s": done,
            "latency_s": done - arrival,
            "host_done_s": host_done if host_arena is not None else None,
            "host_latency_s": host_done - arrival if host_arena is not None else None}
