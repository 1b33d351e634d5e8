"""Host-side checks of libclod that need no GPU: the library loads, exports every entry
point the header declares, sizes its workspaces consistently and rejects invalid
arguments before launching anything."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_09997_amd import _clod as C, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "clod.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(clod_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    lib = C.load()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(C.EXPORTS)
    assert lib.clod_abi_version() == C.ABI_VERSION


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(C.clod_view) == 112
    assert ctypes.sizeof(C.clod_params) == 32
    assert ctypes.sizeof(C.clod_scene) == 8 + 4 + 4 + 7 * 8
    assert C.clod_batch.ws.offset % 8 == 0


def test_workspace_sizes_are_consistent():
    views = C.make_views([synth.look_at((0, 0, -3), width=w, height=h) for w, h in ((256, 256), (100, 75))])
    a = C.clod_ws_bytes(1000, views)
    b = C.clod_ws_bytes(2000, views)
    assert a > 0 and b > a
    assert C.clod_ws_bytes(0, views) > 0
    for cap in (1, 1000, 123457, 10 ** 7):
        nb = C.clod_dup_bytes(cap)
        assert nb % 256 == 0 and nb >= 16 * cap   # two ping-pong copies of uint32 keys and values
        assert C.clod_dup_capacity(nb) >= cap
        assert C.clod_dup_capacity(nb - 256) < cap or nb == C.clod_dup_bytes(C.clod_dup_capacity(nb - 256))


FAKE = 1 << 20          # never dereferenced: every case below fails validation first

# The cases that hand the library the fake device address run only where no GPU is visible:
# should host validation ever regress, a launch on a GPU would dereference it.  (Counting devices
# does not initialise the GPU.)
no_gpu_only = pytest.mark.skipif(__import__("torch").cuda.device_count() > 0,
                                 reason="fake device addresses are only passed where no GPU is visible")


def fake_batch(views, n=10, **over):
    arr = C.make_views(views)
    b = C.clod_batch()
    b.n = n
    b.n_views = len(views)
    b.views_host = ctypes.cast(arr, C.P)
    b.views_dev = FAKE
    b.params = C.make_params()
    b.ws = FAKE
    b.ws_bytes = C.clod_ws_bytes(n, arr)
    b.dup = FAKE
    b.dup_bytes = C.clod_dup_bytes(1000)
    for k, v in over.items():
        setattr(b, k, v)
    return b, arr


def fake_scene(n=10, deg=0):
    s = C.clod_scene()
    s.n, s.sh_degree = n, deg
    for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh"):
        setattr(s, k, FAKE)
    return s


def call_project(scene, batch):
    return C.load().clod_project(ctypes.byref(scene), ctypes.byref(batch), None, None, None)


@no_gpu_only
@pytest.mark.parametrize("case", [
    "sv_below_one", "sv_nan", "n_negative", "degree_4", "null_mean", "zero_views", "eps_zero",
    "tau_negative", "ws_small", "ws_misaligned", "bad_width", "centre_mismatch", "n_mismatch",
    "viewport_unaligned", "viewport_exceeds_frame", "origin_without_frame", "negative_budget",
])
def test_invalid_arguments_are_rejected_before_launch(case):
    v = synth.look_at((0, 0, -3), width=64, height=48)
    scene = fake_scene()
    views = [v]
    kw = {}
    if case == "sv_below_one":
        views = [synth.look_at((0, 0, -3), width=64, height=48, s_v=0.5)]
    elif case == "sv_nan":
        views = [synth.look_at((0, 0, -3), width=64, height=48, s_v=float("nan"))]
    elif case == "n_negative":
        scene = fake_scene(n=-1)
    elif case == "degree_4":
        scene = fake_scene(deg=4)
    elif case == "null_mean":
        scene.mean = None
    elif case == "bad_width":
        bad = synth.look_at((0, 0, -3), width=64, height=48)
        bad.width = 0
        views = [bad]
    elif case == "centre_mismatch":
        bad = synth.look_at((0, 0, -3), width=64, height=48)
        bad.c = np.array([0.0, 0.0, 3.0], np.float32)
        views = [bad]
    if case == "viewport_unaligned":
        views = [synth.viewport(synth.look_at((0, 0, -3), width=128, height=96), 8, 0, 64, 48)]
    elif case == "viewport_exceeds_frame":
        views = [synth.viewport(synth.look_at((0, 0, -3), width=128, height=96), 96, 0, 64, 48)]
    elif case == "origin_without_frame":
        bad = synth.look_at((0, 0, -3), width=64, height=48)
        bad.vx = 16
        views = [bad]
    elif case == "negative_budget":
        bad = synth.look_at((0, 0, -3), width=64, height=48)
        bad.budget = -1
        views = [bad]
    batch, arr = fake_batch(views)
    if case == "zero_views":
        batch.n_views = 0
    elif case == "eps_zero":
        batch.params.eps = 0.0
    elif case == "tau_negative":
        batch.params.tau = -1.0
    elif case == "ws_small":
        batch.ws_bytes = 16
    elif case == "ws_misaligned":
        batch.ws = FAKE + 4
    elif case == "n_mismatch":
        batch.n = 11
    st = call_project(scene, batch)
    assert st == C.CLOD_E_ARG, (case, st)
    assert C.load().clod_last_error().decode() != ""


@no_gpu_only
def test_other_entry_points_validate_arguments():
    v = synth.look_at((0, 0, -3), width=64, height=48, s_v=0.9)
    batch, arr = fake_batch([v])
    lib = C.load()
    n = ctypes.c_int64(0)
    assert lib.clod_bin_sort(ctypes.byref(batch), ctypes.byref(n), None) == C.CLOD_E_ARG
    assert lib.clod_render_fwd(ctypes.byref(batch), FAKE, FAKE, FAKE, None, None) == C.CLOD_E_ARG
    g = C.clod_scene_grad()
    assert lib.clod_render_bwd(ctypes.byref(fake_scene()), ctypes.byref(batch), FAKE, FAKE, FAKE, None, 0,
                               ctypes.byref(g), None, None) == C.CLOD_E_ARG
    assert lib.clod_lod_count(ctypes.byref(fake_scene()), ctypes.byref(batch), FAKE, None) == C.CLOD_E_ARG
    assert lib.clod_loss(ctypes.byref(batch), FAKE, FAKE, ctypes.c_float(8.0), ctypes.c_float(1.0),
                         ctypes.c_float(0.0), None, 0, FAKE, FAKE, FAKE, None) == C.CLOD_E_ARG
    ok_batch, arr2 = fake_batch([synth.look_at((0, 0, -3), width=64, height=48, s_v=4.0)])
    # s_max below a view's s_v is an argument error.
    assert lib.clod_loss(ctypes.byref(ok_batch), FAKE, FAKE, ctypes.c_float(2.0), ctypes.c_float(1.0),
                         ctypes.c_float(0.0), None, 0, FAKE, FAKE, FAKE, None) == C.CLOD_E_ARG
    ok8, arr3 = fake_batch([synth.look_at((0, 0, -3), width=64, height=48, s_v=1.0)])
    # D-SSIM weight outside [0, 1], or a positive weight without a large enough scratch buffer.
    for lam, scratch, nbytes in ((1.5, FAKE, 1 << 30), (0.2, None, 0), (0.2, FAKE, 36 * 64 * 48 - 4)):
        assert lib.clod_loss(ctypes.byref(ok8), FAKE, FAKE, ctypes.c_float(8.0), ctypes.c_float(1.0),
                             ctypes.c_float(lam), scratch, nbytes, FAKE, FAKE, FAKE, None) == C.CLOD_E_ARG, lam
    # Missing gradient planes.
    assert lib.clod_render_bwd(ctypes.byref(fake_scene()), ctypes.byref(ok_batch), FAKE, FAKE, FAKE, None, 0,
                               ctypes.byref(g), None, None) == C.CLOD_E_ARG
    # Unknown inspection section.
    p, c = ctypes.c_void_p(0), ctypes.c_int64(0)
    assert lib.clod_inspect(ctypes.byref(ok_batch), 99, ctypes.byref(p), ctypes.byref(c)) == C.CLOD_E_ARG


def _fake_planes():
    g = C.clod_scene_grad()
    for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh"):
        setattr(g, k, FAKE)
    return g


@pytest.mark.parametrize("case", ["n_negative", "degree_4", "null_hp", "lr_negative", "lr_nan", "beta_one",
                                  "eps_zero", "step_zero", "step_negative", "null_plane"])
@no_gpu_only
def test_adam_step_rejects_invalid_arguments_before_launch(case):
    lib = C.load()
    p, g, m, v = (_fake_planes() for _ in range(4))
    hp = C.make_adam({k: 1e-3 for k in C.ADAM_GROUPS}, t=1)
    n, deg = 10, 3
    if case == "n_negative":
        n = -1
    elif case == "degree_4":
        deg = 4
    elif case == "lr_negative":
        hp.lr[3] = -1.0
    elif case == "lr_nan":
        hp.lr[0] = float("nan")
    elif case == "beta_one":
        hp.beta2 = 1.0
    elif case == "eps_zero":
        hp.eps = 0.0
    elif case == "step_zero":
        hp.step = 0
    elif case == "step_negative":
        hp.step = -3
    elif case == "null_plane":
        m.sh = None
    hp_ref = None if case == "null_hp" else ctypes.byref(hp)
    st = lib.clod_adam_step(n, deg, ctypes.byref(p), ctypes.byref(g), ctypes.byref(m), ctypes.byref(v), hp_ref, None)
    assert st == C.CLOD_E_ARG, (case, st)
    # n = 0 is a valid no-op (nothing launched).
    assert lib.clod_adam_step(0, 3, ctypes.byref(p), ctypes.byref(g), ctypes.byref(m), ctypes.byref(v),
                              ctypes.byref(C.make_adam({k: 1e-3 for k in C.ADAM_GROUPS}, t=1)), None) == C.CLOD_OK


@no_gpu_only
def test_noalloc_lod_count_rejects_inputs_beyond_its_scratch_before_launch():
    lib = C.load()
    # 17M Gaussians: the work list alone (4 bytes per Gaussian) exceeds the 64 MiB scratch.
    vs = [synth.look_at((0, 0, -3), width=16, height=16)]
    arr = C.make_views(vs)
    scene = fake_scene(n=17_000_000)
    p = C.make_params()
    st = lib.clod_lod_count_noalloc(ctypes.byref(scene), len(vs), ctypes.cast(arr, C.P), FAKE, ctypes.byref(p),
                                    FAKE, None)
    assert st == C.CLOD_E_ARG and b"scratch" in lib.clod_last_error()
    # Other argument errors are caught first, as in clod_lod_count.
    one = C.make_views([synth.look_at((0, 0, -3), width=16, height=16, s_v=0.5)])
    st = lib.clod_lod_count_noalloc(ctypes.byref(fake_scene()), 1, ctypes.cast(one, C.P), FAKE, ctypes.byref(p),
                                    FAKE, None)
    assert st == C.CLOD_E_ARG
    assert lib.clod_lod_count_noalloc(ctypes.byref(fake_scene()), 0, ctypes.cast(one, C.P), FAKE,
                                      ctypes.byref(p), FAKE, None) == C.CLOD_E_ARG


def test_scene_reorder_workspace_sizes():
    a, b = C.clod_scene_reorder_ws_bytes(1000), C.clod_scene_reorder_ws_bytes(3_000_000)
    assert a % 256 == 0 and b % 256 == 0 and b > a >= 3 * 4 * 1000
    assert C.clod_scene_reorder_ws_bytes(-1) == 0 and C.clod_scene_reorder_ws_bytes(1 << 31) == 0


@pytest.mark.parametrize("case", ["null_dst", "null_perm", "null_plane", "overlap", "no_ws", "misaligned_ws",
                                  "small_ws", "too_many", "degree_4"])
@no_gpu_only
def test_scene_reorder_rejects_invalid_arguments_before_launch(case):
    n = 1000
    src = fake_scene(n, 3)
    dst = C.clod_scene_grad()
    for j, k in enumerate(("mean", "log_scale", "quat", "opacity", "decay", "sh")):
        setattr(dst, k, (1 << 30) + j * (1 << 20))
    perm, ws, nbytes = 1 << 29, 1 << 28, C.clod_scene_reorder_ws_bytes(n)
    dst_arg = ctypes.byref(dst)
    if case == "null_dst":
        dst_arg = None
    elif case == "null_perm":
        perm = None
    elif case == "null_plane":
        dst.quat = None
    elif case == "overlap":
        dst.sh = FAKE + 4 * n
    elif case == "no_ws":
        ws = None
    elif case == "misaligned_ws":
        ws += 16
    elif case == "small_ws":
        nbytes -= 256
    elif case == "too_many":
        src.n = 1 << 31
    elif case == "degree_4":
        src.sh_degree = 4
    assert C.load().clod_scene_reorder(ctypes.byref(src), dst_arg, perm, ws, nbytes, None) == C.CLOD_E_ARG, case


def test_scene_order_refuses_host_planes():
    """The reorder runs on device planes only: a scene kept in host memory is refused before any
    library call."""
    from paper_2510_09997_amd.render import Scene
    sc = synth.make_scene(100, 0, "uniform", seed=0)
    with pytest.raises(ValueError):
        Scene(sc, device="cpu", spatial_order=True)
