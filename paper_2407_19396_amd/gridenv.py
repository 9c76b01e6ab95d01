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

GX_OK, GX_EINVAL, GX_ENOMEM, GX_EDEVICE, GX_ESTATE = 0, -1, -2, -3, -4
OBS_BYTES = 147
EXPORTS = ("env_create", "env_sizes", "env_info", "env_reset", "env_step", "env_rollout",
           "env_set_launch", "env_destroy", "env_strerror")


class GxConfig(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("reward_mode", ctypes.c_int32),
                ("family", ctypes.c_void_p), ("side", ctypes.c_void_p),
                ("max_steps", ctypes.c_void_p), ("seed", ctypes.c_void_p),
                ("seed_all", ctypes.c_uint64), ("rng_id", ctypes.c_void_p)]


class GxState(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in
                ("grid", "x", "y", "dir", "t", "carry", "episode", "done_prev")]


class GxTraj(ctypes.Structure):
    _fields_ = [("obs", ctypes.c_void_p), ("reward", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("action", ctypes.c_void_p),
                ("rows", ctypes.c_int32)]


class GxInfo(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("max_tile_cells", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("k_default", ctypes.c_int32),
                ("grid_bytes", ctypes.c_uint64), ("calls", ctypes.c_uint64)]


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
    L.env_destroy.argtypes = [P]
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
def env_create(table: workloads.EnvTable, reward_mode: int = 0) -> int:
    fam = np.ascontiguousarray(table.family, np.uint8)
    side = np.ascontiguousarray(table.side, np.uint8)
    ms = np.ascontiguousarray(table.max_steps, np.int32)
    seed = np.ascontiguousarray(table.seed, np.uint64)
    rid = np.ascontiguousarray(table.rng_id, np.uint32)
    cfg = GxConfig(table.n, reward_mode, fam.ctypes.data, side.ctypes.data, ms.ctypes.data,
                   seed.ctypes.data, 0, rid.ctypes.data)
    ctx = ctypes.c_void_p()
    _check("env_create", load().env_create(ctypes.byref(cfg), ctypes.byref(ctx)))
    return ctx.value


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


def env_destroy(ctx: int):
    _check("env_destroy", load().env_destroy(ctx))


# --------------------------------------------------------------- tensors
@dataclass
class Traj:
    """Device output rows: obs [rows][N][7][7][3] u8 (or None), reward f32,
    flags u8, action u8 [rows][N]."""
    obs: object
    reward: object
    flags: object
    action: object

    @staticmethod
    def alloc(rows: int, n: int, device="cuda", with_obs: bool = True) -> "Traj":
        import torch
        return Traj(torch.zeros((rows, n, 7, 7, 3), dtype=torch.uint8, device=device) if with_obs else None,
                    torch.zeros((rows, n), dtype=torch.float32, device=device),
                    torch.zeros((rows, n), dtype=torch.uint8, device=device),
                    torch.zeros((rows, n), dtype=torch.uint8, device=device))

    @property
    def rows(self) -> int:
        return int(self.reward.shape[0])

    def c(self) -> GxTraj:
        return GxTraj(self.obs.data_ptr() if self.obs is not None else None, self.reward.data_ptr(),
                      self.flags.data_ptr(), self.action.data_ptr(), self.rows)


class GridEnv:
    """A batch of envs on the current HIP device with its state tensors."""

    FIELDS = ("grid", "x", "y", "dir", "t", "carry", "episode", "done_prev")

    def __init__(self, table: workloads.EnvTable, reward_mode: int = 0, device="cuda"):
        import torch
        self.table = table
        self.device = torch.device(device)
        self.ctx = env_create(table, reward_mode)
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

    def state(self) -> GxState:
        return GxState(*[getattr(self, f).data_ptr() for f in self.FIELDS])

    def reset(self, first: Traj | None = None, stream=None):
        env_reset(self.ctx, self.state(), first.c() if first is not None else None, stream)

    def step(self, out: Traj, actions=None, stream=None):
        env_step(self.ctx, self.state(), actions.data_ptr() if actions is not None else None,
                 out.c(), stream)

    def rollout(self, n_steps: int, traj: Traj, actions=None, K: int = 0, stream=None):
        env_rollout(self.ctx, self.state(), n_steps,
                    actions.data_ptr() if actions is not None else None, traj.c(), K, stream)

    def set_launch(self, K: int, blocks: int = 0):
        env_set_launch(self.ctx, K, blocks)

    def info(self) -> dict:
        return env_info(self.ctx)

    def state_numpy(self) -> dict:
        out = {f: getattr(self, f).cpu().numpy() for f in self.FIELDS}
        out["episode"] = out["episode"].view(np.uint32)
        return out

    def load_state(self, st: dict):
        """Copy a host state (dict of numpy arrays) into the device tensors."""
        import torch
        for f in self.FIELDS:
            a = np.ascontiguousarray(st[f])
            if f == "episode":
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
