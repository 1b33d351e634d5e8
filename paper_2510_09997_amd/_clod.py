"""ctypes binding of libclod (include/clod.h).  Argument marshalling only: every step of the
render path runs in the HIP library; torch supplies device memory and streams.

The functions keep the C names; they take torch tensors (device memory) and raise
``ClodError`` on a non-zero status.  Importing this module does not load the library;
the first call does, and fails loudly if libclod.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclod.so")

CLOD_OK, CLOD_E_ARG, CLOD_E_CAPACITY, CLOD_E_HIP, CLOD_E_UNSUPPORTED, CLOD_E_BUSY = 0, -1, -2, -3, -4, -5
MAX_VIEWS = 1024
LOD_SCRATCH_BYTES = 64 << 20   # library scratch of clod_lod_count_noalloc (per GPU)
SERVER_SLOTS, SERVER_MAX_VIEWS = 16, 16
ABI_VERSION = 13


class ClodError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libclod status {status}: {msg}")
        self.status = status


class CapacityError(ClodError):
    pass


class BusyError(ClodError):
    pass


P = ctypes.c_void_p


class clod_scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mean", P), ("log_scale", P), ("quat", P), ("opacity", P), ("decay", P), ("sh", P),
                ("sh_packed", P)]


class clod_scene_grad(ctypes.Structure):
    _fields_ = [("mean", P), ("log_scale", P), ("quat", P), ("opacity", P), ("decay", P), ("sh", P)]


class clod_view(ctypes.Structure):
    _fields_ = [("W", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("c", ctypes.c_float * 3),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("s_v", ctypes.c_float),
                ("budget", ctypes.c_int64), ("frame_width", ctypes.c_int32), ("frame_height", ctypes.c_int32),
                ("vx", ctypes.c_int32), ("vy", ctypes.c_int32)]


class clod_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 7), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("reserved", ctypes.c_int32), ("step", ctypes.c_int64)]


class clod_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_float), ("eps", ctypes.c_float), ("near_z", ctypes.c_float),
                ("guard", ctypes.c_float), ("dilation", ctypes.c_float), ("bg", ctypes.c_float * 3)]


class clod_batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_views", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("views_host", P), ("views_dev", P), ("params", clod_params),
                ("ws", P), ("ws_bytes", ctypes.c_size_t), ("dup", P), ("dup_bytes", ctypes.c_size_t)]


assert ctypes.sizeof(clod_view) == 112

EXPORTS = ["clod_ws_bytes", "clod_dup_bytes", "clod_dup_capacity", "clod_project", "clod_bin_sort",
           "clod_render_fwd", "clod_render_bwd", "clod_lod_count", "clod_loss", "clod_read_info",
           "clod_inspect", "clod_last_error", "clod_abi_version", "clod_adam_step", "clod_lod_count_noalloc",
           "clod_server_start", "clod_server_submit", "clod_server_poll", "clod_server_clock", "clod_server_stop",
           "clod_server_stage_times", "clod_scene_reorder_ws_bytes", "clod_scene_reorder"]

SEC_KEYS, SEC_VALUES, SEC_RANGES, SEC_REC, SEC_ALPHA = 0, 1, 2, 3, 4
SEC_FLAGS, SEC_DMAX, SEC_GSCREEN, SEC_HEADER = 6, 7, 9, 10

_lib = None


def load(path: str = LIB_PATH):
    """Loads libclod.so (no fallback: raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2510_09997_amd/build.py "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    i64, i32, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    L.clod_ws_bytes.argtypes = [i64, i32, P]; L.clod_ws_bytes.restype = sz
    L.clod_dup_bytes.argtypes = [i64]; L.clod_dup_bytes.restype = sz
    L.clod_dup_capacity.argtypes = [sz]; L.clod_dup_capacity.restype = i64
    L.clod_project.argtypes = [P, P, P, P, P]; L.clod_project.restype = i32
    L.clod_bin_sort.argtypes = [P, P, P]; L.clod_bin_sort.restype = i32
    L.clod_render_fwd.argtypes = [P, P, P, P, P, P]; L.clod_render_fwd.restype = i32
    L.clod_render_bwd.argtypes = [P, P, P, P, P, P, i32, P, P, P]; L.clod_render_bwd.restype = i32
    L.clod_lod_count.argtypes = [P, P, P, P]; L.clod_lod_count.restype = i32
    L.clod_lod_count_noalloc.argtypes = [P, i32, P, P, P, P, P]; L.clod_lod_count_noalloc.restype = i32
    L.clod_scene_reorder_ws_bytes.argtypes = [i64]; L.clod_scene_reorder_ws_bytes.restype = sz
    L.clod_scene_reorder.argtypes = [P, P, P, P, sz, P]; L.clod_scene_reorder.restype = i32
    L.clod_loss.argtypes = [P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, P, sz, P, P, P, P]
    L.clod_loss.restype = i32
    L.clod_read_info.argtypes = [P, P, P]; L.clod_read_info.restype = i32
    L.clod_adam_step.argtypes = [i64, i32, P, P, P, P, P, P]; L.clod_adam_step.restype = i32
    L.clod_inspect.argtypes = [P, i32, P, P]; L.clod_inspect.restype = i32
    L.clod_last_error.argtypes = []; L.clod_last_error.restype = ctypes.c_char_p
    L.clod_abi_version.argtypes = []; L.clod_abi_version.restype = i32
    L.clod_server_start.argtypes = [i32, ctypes.c_double, P, P, P]; L.clod_server_start.restype = i32
    L.clod_server_submit.argtypes = [P, P, P, P, P, P, P]; L.clod_server_submit.restype = i32
    L.clod_server_poll.argtypes = [P, i64, P, P]; L.clod_server_poll.restype = i32
    L.clod_server_clock.argtypes = [P, P]; L.clod_server_clock.restype = i32
    L.clod_server_stop.argtypes = [P, P]; L.clod_server_stop.restype = i32
    L.clod_server_stage_times.argtypes = [P, i64, P, P, i32, P]; L.clod_server_stage_times.restype = i32
    if L.clod_abi_version() != ABI_VERSION:
        raise RuntimeError("libclod ABI version mismatch")
    _lib = L
    return L


def _check(status: int):
    if status != CLOD_OK:
        msg = load().clod_last_error().decode()
        if status == CLOD_E_CAPACITY:
            raise CapacityError(status, msg)
        if status == CLOD_E_BUSY:
            raise BusyError(status, msg)
        raise ClodError(status, msg)


F32, I32, I64 = torch.float32, (torch.int32, torch.uint32), torch.int64


def _ptr(t, dtype=None) -> int | None:
    """Device address of a contiguous tensor (or a raw address); with `dtype` (a dtype or a
    tuple of accepted dtypes) the tensor's element type is checked against the C type the
    entry point reads or writes."""
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if dtype is not None:
            ok = dtype if isinstance(dtype, tuple) else (dtype,)
            if t.dtype not in ok:
                raise TypeError(f"tensor of dtype {t.dtype} where the C ABI expects {ok[0]}")
        return t.data_ptr()
    return int(t)


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# ------------------------------------------------------------------------------- structs

def make_scene(planes: dict) -> clod_scene:
    """planes: dict of contiguous float32 device tensors in the C layout (see clod.h)."""
    s = clod_scene()
    s.n = int(planes["n"])
    s.sh_degree = int(planes["sh_degree"])
    for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh"):
        setattr(s, k, _ptr(planes[k], F32))
    s.sh_packed = _ptr(planes.get("sh_packed"), F32)
    return s


def make_grad(planes: dict) -> clod_scene_grad:
    g = clod_scene_grad()
    for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh"):
        setattr(g, k, _ptr(planes[k], F32))
    return g


def make_views(views) -> ctypes.Array:
    """Host array of clod_view from objects with W, t, c, fx, fy, cx, cy, width, height, s_v
    (and optionally budget)."""
    arr = (clod_view * len(views))()
    for j, v in enumerate(views):
        cv = arr[j]
        W = np.asarray(v.W, dtype=np.float32).reshape(9)
        for k in range(9):
            cv.W[k] = float(W[k])
        for k in range(3):
            cv.t[k] = float(np.float32(v.t[k]))
            cv.c[k] = float(np.float32(v.c[k]))
        cv.fx, cv.fy, cv.cx, cv.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
        cv.width, cv.height = int(v.width), int(v.height)
        cv.s_v = float(v.s_v)
        cv.budget = int(getattr(v, "budget", 0))
        cv.frame_width = int(getattr(v, "frame_width", 0))
        cv.frame_height = int(getattr(v, "frame_height", 0))
        cv.vx, cv.vy = int(getattr(v, "vx", 0)), int(getattr(v, "vy", 0))
    return arr


def views_to_device(arr: ctypes.Array, device="cuda") -> torch.Tensor:
    raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def make_params(tau=1.0 / 255.0, eps=1e-6, near=0.2, guard=1.3, dilation=0.3, bg=(0.0, 0.0, 0.0)) -> clod_params:
    p = clod_params()
    p.tau, p.eps, p.near_z, p.guard, p.dilation = tau, eps, near, guard, dilation
    for k in range(3):
        p.bg[k] = float(bg[k])
    return p


# ------------------------------------------------------------------------------- entry points

def clod_ws_bytes(n: int, views_host) -> int:
    return int(load().clod_ws_bytes(n, len(views_host), ctypes.cast(views_host, P)))


def clod_dup_bytes(capacity: int) -> int:
    return int(load().clod_dup_bytes(capacity))


def clod_dup_capacity(nbytes: int) -> int:
    return int(load().clod_dup_capacity(nbytes))


def clod_project(scene: clod_scene, batch: clod_batch, counts=None, stream=None, eta=None):
    _check(load().clod_project(ctypes.byref(scene), ctypes.byref(batch), _ptr(counts, I64), _ptr(eta, F32),
                               _stream(stream)))


def clod_bin_sort(batch: clod_batch, sync_count: bool = False, stream=None) -> int | None:
    n = ctypes.c_int64(0)
    _check(load().clod_bin_sort(ctypes.byref(batch), ctypes.byref(n) if sync_count else None, _stream(stream)))
    return int(n.value) if sync_count else None


def clod_render_fwd(batch: clod_batch, rgb, T, last, pairs=None, stream=None):
    _check(load().clod_render_fwd(ctypes.byref(batch), _ptr(rgb, F32), _ptr(T, F32), _ptr(last, I32), _ptr(pairs, I64),
                                  _stream(stream)))


def clod_render_bwd(scene: clod_scene, batch: clod_batch, T, last, dL_drgb, dL_deta, accumulate: bool,
                    grad: clod_scene_grad, stream=None, pairs=None):
    _check(load().clod_render_bwd(ctypes.byref(scene), ctypes.byref(batch), _ptr(T, F32), _ptr(last, I32),
                                  _ptr(dL_drgb, F32), _ptr(dL_deta, F32), int(bool(accumulate)), ctypes.byref(grad),
                                  _ptr(pairs, I64), _stream(stream)))


def clod_lod_count(scene: clod_scene, batch: clod_batch, counts, stream=None):
    _check(load().clod_lod_count(ctypes.byref(scene), ctypes.byref(batch), _ptr(counts, I64), _stream(stream)))


def clod_lod_count_noalloc(scene: clod_scene, views_host, views_dev, params: clod_params, counts, stream=None):
    """clod_lod_count without a workspace (library scratch; see clod.h)."""
    _check(load().clod_lod_count_noalloc(ctypes.byref(scene), len(views_host), ctypes.cast(views_host, P),
                                         _ptr(views_dev, torch.uint8), ctypes.byref(params), _ptr(counts, I64),
                                         _stream(stream)))



def clod_scene_reorder_ws_bytes(n: int) -> int:
    return int(load().clod_scene_reorder_ws_bytes(int(n)))


def clod_scene_reorder(src: clod_scene, dst: clod_scene_grad, perm, ws, stream=None):
    """Spatial (Morton) order of src's Gaussians into dst's planes; perm[j] = original index."""
    _check(load().clod_scene_reorder(ctypes.byref(src), ctypes.byref(dst), _ptr(perm, I32), _ptr(ws, torch.uint8),
                                     ws.numel() if isinstance(ws, torch.Tensor) else 0, _stream(stream)))


ADAM_GROUPS = ("mean", "log_scale", "quat", "opacity", "decay", "sh_dc", "sh_rest")


def make_adam(lrs: dict, t: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15) -> clod_adam:
    """Hyperparameters of step t >= 1 (the library forms the bias corrections)."""
    hp = clod_adam()
    for j, k in enumerate(ADAM_GROUPS):
        hp.lr[j] = float(lrs[k])
    hp.beta1, hp.beta2, hp.eps = float(beta1), float(beta2), float(eps)
    hp.step = int(t)
    return hp


def clod_adam_step(n: int, sh_degree: int, param: clod_scene_grad, grad: clod_scene_grad, m: clod_scene_grad,
                   v: clod_scene_grad, hp: clod_adam, stream=None):
    _check(load().clod_adam_step(int(n), int(sh_degree), ctypes.byref(param), ctypes.byref(grad), ctypes.byref(m),
                                 ctypes.byref(v), ctypes.byref(hp), _stream(stream)))


def clod_loss(batch: clod_batch, rgb, target, s_max: float, lambda_reg: float, loss, dL_drgb, dL_deta,
              stream=None, lambda_dssim: float = 0.0, ssim_scratch=None):
    nbytes = 0 if ssim_scratch is None else ssim_scratch.numel() * ssim_scratch.element_size()
    _check(load().clod_loss(ctypes.byref(batch), _ptr(rgb, F32), _ptr(target, F32), float(s_max), float(lambda_reg),
                            float(lambda_dssim), _ptr(ssim_scratch, F32), nbytes, _ptr(loss, F32), _ptr(dL_drgb, F32),
                            _ptr(dL_deta, F32), _stream(stream)))


def clod_read_info(batch: clod_batch, stream=None) -> dict:
    out = (ctypes.c_int64 * 4)()
    _check(load().clod_read_info(ctypes.byref(batch), out, _stream(stream)))
    return dict(n_dup=int(out[0]), overflow=bool(out[1]), capacity=int(out[2]), passes=int(out[3]))


def clod_inspect(batch: clod_batch, section: int) -> tuple[int, int]:
    """(device address, element count) of an intermediate section (see clod.h)."""
    ptr = ctypes.c_void_p(0)
    cnt = ctypes.c_int64(0)
    _check(load().clod_inspect(ctypes.byref(batch), int(section), ctypes.byref(ptr), ctypes.byref(cnt)))
    return int(ptr.value or 0), int(cnt.value)


# ------------------------------------------------------------------------------- persistent server

def clod_server_start(workers: int = 0, max_seconds: float = 60.0, stream=None) -> tuple[int, int]:
    """Launches the resident serving kernel on `stream`; returns (handle, workers used)."""
    h = ctypes.c_void_p(0)
    used = ctypes.c_int32(0)
    _check(load().clod_server_start(int(workers), float(max_seconds), _stream(stream), ctypes.byref(h),
                                    ctypes.byref(used)))
    return int(h.value), int(used.value)


def clod_server_submit(server: int, scene: clod_scene, batch: clod_batch, rgb, T, last) -> int:
    seq = ctypes.c_int64(-1)
    _check(load().clod_server_submit(P(server), ctypes.byref(scene), ctypes.byref(batch), _ptr(rgb, F32), _ptr(T, F32),
                                     _ptr(last, I32), ctypes.byref(seq)))
    return int(seq.value)


def clod_server_poll(server: int, seq: int) -> dict | None:
    """None while job `seq` runs, else {overflow, n_dup, t_ns} (device clock since start)."""
    done = ctypes.c_int32(0)
    info = (ctypes.c_int64 * 3)()
    _check(load().clod_server_poll(P(server), int(seq), ctypes.byref(done), info))
    if not done.value:
        return None
    return dict(overflow=bool(info[0]), n_dup=int(info[1]), t_ns=int(info[2]))


def clod_server_clock(server: int) -> int:
    ns = ctypes.c_int64(0)
    _check(load().clod_server_clock(P(server), ctypes.byref(ns)))
    return int(ns.value)


def clod_server_stop(server: int) -> int:
    st = ctypes.c_int32(0)
    _check(load().clod_server_stop(P(server), ctypes.byref(st)))
    return int(st.value)


def clod_server_stage_times(server: int, seq: int, max_entries: int = 96) -> list[tuple[int, int]]:
    """[(stage kind, ns since start when it opened)] of a completed job, then (0, completion ns)."""
    ns = (ctypes.c_int64 * max_entries)()
    kinds = (ctypes.c_int32 * max_entries)()
    cnt = ctypes.c_int32(0)
    _check(load().clod_server_stage_times(P(server), int(seq), ns, kinds, int(max_entries), ctypes.byref(cnt)))
    return [(int(kinds[k]), int(ns[k])) for k in range(cnt.value)]
