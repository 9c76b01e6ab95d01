"""Host-side checks of the C-ABI: the library loads, exports every entry
point the public header declares, and rejects bad arguments before any
device work (these paths never touch a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2407_19396_amd import gridenv as ge

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gridenv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(env_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert declared_functions() == sorted(ge.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ge.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror():
    assert ge.env_strerror(0) == "ok"
    assert "invalid" in ge.env_strerror(ge.GX_EINVAL)
    assert ge.env_strerror(-99) == "unknown status"


def _cfg(family, side, max_steps, n=None, reward_mode=0, param=None, obs_mode=0):
    family = np.asarray(family, np.uint8)
    side = np.asarray(side, np.uint8)
    max_steps = np.asarray(max_steps, np.int32)
    param = None if param is None else np.asarray(param, np.uint8)
    keep = (family, side, max_steps, param)
    n = len(family) if n is None else n
    return ge.GxConfig(n, reward_mode, obs_mode, family.ctypes.data, side.ctypes.data,
                       None if param is None else param.ctypes.data, max_steps.ctypes.data,
                       None, 0, None), keep


@pytest.mark.parametrize("family,side,T,n,mode,param", [
    ([0], [3], [10], None, 0, None),          # Empty needs side >= 4
    ([1], [4], [10], None, 0, None),          # TwoRoom needs side >= 5
    ([2], [8], [10], None, 0, None),          # FourRooms needs an odd side
    ([2], [5], [10], None, 0, None),          # FourRooms needs side >= 7
    ([0], [33], [10], None, 0, None),         # side <= 32
    ([9], [8], [10], None, 0, None),          # unknown family
    ([6], [8], [10], None, 0, None),          # Dynamic-Obstacles needs 1..8 balls
    ([6], [5], [10], None, 0, [8]),           # ... and two free interior cells
    ([7], [4], [10], None, 0, None),          # GoToDoor needs side >= 5
    ([8], [8], [10], None, 0, [1]),           # KeyCorridor side is 3 s - 2
    ([8], [10], [10], None, 0, [0]),          # KeyCorridor needs 1..3 rows
    ([8], [10], [10], None, 0, [4]),
    ([3], [4], [10], None, 0, None),          # LavaGap needs side >= 5
    ([4], [9], [10], None, 0, None),          # Crossings needs N >= 1 (NULL param: 0)
    ([4], [10], [10], None, 0, [2]),          # Crossings needs an odd side
    ([4], [9], [10], None, 0, [7]),           # Crossings needs N <= S - 3
    ([4], [31], [10], None, 0, [9]),          # Crossings needs N <= 8
    ([5], [8], [10], None, 0, [0]),           # DistShift variant 1 or 2
    ([5], [5], [10], None, 0, [1]),           # DistShift needs side >= 6
    ([0], [8], [0], None, 0, None),           # max_steps >= 1
    ([0], [8], [10], 0, 0, None),             # n_envs >= 1
    ([0], [8], [10], None, 2, None),          # reward mode 0 or 1
])
def test_create_rejects_bad_configs(family, side, T, n, mode, param):
    lib = ge.load()
    cfg, keep = _cfg(family, side, T, n, mode, param)
    ctx = ctypes.c_void_p(1)
    assert lib.env_create(ctypes.byref(cfg), ctypes.byref(ctx)) == ge.GX_EINVAL
    assert ctx.value is None


@pytest.mark.parametrize("obs_mode", [-1, 6, 99, 4, 5])
def test_create_rejects_bad_observation_modes(obs_mode):
    """Unknown modes, and the rgb modes (4, 5) without a sprite atlas."""
    lib = ge.load()
    cfg, keep = _cfg([0], [8], [10], obs_mode=obs_mode)
    ctx = ctypes.c_void_p(1)
    assert lib.env_create(ctypes.byref(cfg), ctypes.byref(ctx)) == ge.GX_EINVAL
    assert ctx.value is None


def test_null_arguments_are_rejected():
    lib = ge.load()
    assert lib.env_create(None, None) == ge.GX_EINVAL
    ctx = ctypes.c_void_p()
    assert lib.env_create(None, ctypes.byref(ctx)) == ge.GX_EINVAL
    st, tr = ge.GxState(), ge.GxTraj()
    assert lib.env_sizes(None, None, None) == ge.GX_EINVAL
    assert lib.env_info(None, None) == ge.GX_EINVAL
    assert lib.env_reset(None, ctypes.byref(st), None, None) == ge.GX_EINVAL
    assert lib.env_step(None, ctypes.byref(st), None, ctypes.byref(tr), None) == ge.GX_EINVAL
    assert lib.env_rollout(None, ctypes.byref(st), 1, None, ctypes.byref(tr), 0, None) == ge.GX_EINVAL
    assert lib.env_set_launch(None, 4, 0) == ge.GX_EINVAL
    assert lib.env_destroy(None) == ge.GX_EINVAL


def test_store_probe_is_exported_and_validates_before_any_launch():
    """The measurement tool of include/gridenv_probe.h: exported, and bad
    arguments are refused before anything is launched."""
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "gridenv_probe.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(gx_[a-z_]+)\s*\(", text)))
    assert names == ["gx_probe_record_stores"]
    lib = ctypes.CDLL(ge.LIB_PATH)
    fn = lib.gx_probe_record_stores
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    fn.argtypes = [P, P, P, P, I64, I32, I32, I32, I32, I32, P]
    fn.restype = ctypes.c_int
    assert fn(16, 16, 16, 16, 100, 1, 1, 1, 1, 1, None) == -1      # n_envs not a multiple of 64
    assert fn(None, 16, 16, 16, 64, 1, 1, 1, 1, 1, None) == -1     # missing buffer
    assert fn(16, 16, 16, 16, 64, 0, 1, 1, 1, 1, None) == -1       # no rows
    assert fn(24, 16, 16, 16, 64, 1, 1, 1, 1, 1, None) == -1       # observations not 16-byte aligned
