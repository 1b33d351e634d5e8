"""Persistent serving launch (clod_server_*): jobs run by the resident kernel give the same bytes
as the per-stage launches of clod_project / clod_bin_sort / clod_render_fwd, whether a request
is rendered alone or inside a mixed batch, with several jobs in flight at once; a 4K request
inside a 720p / 4K / 1080p job and a frame with very long tile lists are checked against the
oracle.  Also: stop on request, the
kernel's own deadline, overflow and resubmission, and the argument checks."""
import ctypes
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_09997_amd import _clod as C, synth
from paper_2510_09997_amd.render import Batch, Scene
from paper_2510_09997_amd.serve import serve

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def same_bits(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def per_stage(sc, scene, views):
    b = Batch(sc["n"], views)
    b.project(scene)
    b.bin_sort()
    return b.render_fwd()


class Job:
    """One job submitted straight through the C ABI, with its own buffers."""

    def __init__(self, srv, scene, n, views, dup_pairs=None):
        px = sum(v.width * v.height for v in views)
        self.views = views
        self.vh = C.make_views(views)
        self.ws = torch.empty(C.clod_ws_bytes(n, self.vh), dtype=torch.uint8, device="cuda")
        cap = dup_pairs if dup_pairs is not None else 16 * px + 65536
        self.dup = torch.empty(C.clod_dup_bytes(cap), dtype=torch.uint8, device="cuda")
        self.rgb = torch.empty(3 * px, dtype=torch.float32, device="cuda")
        self.T = torch.empty(px, dtype=torch.float32, device="cuda")
        self.last = torch.empty(px, dtype=torch.int32, device="cuda")
        self.n, self.scene, self.srv = n, scene, srv

    def batch(self):
        b = C.clod_batch()
        b.n, b.n_views = self.n, len(self.views)
        b.views_host = ctypes.cast(self.vh, C.P)
        b.views_dev = None
        b.params = C.make_params()
        b.ws, b.ws_bytes = self.ws.data_ptr(), self.ws.numel()
        b.dup, b.dup_bytes = self.dup.data_ptr(), self.dup.numel()
        return b

    def submit(self):
        self.seq = C.clod_server_submit(self.srv, self.scene.c_struct(), self.batch(), self.rgb, self.T, self.last)
        return self.seq

    def wait(self, timeout_s=60.0):
        t0 = time.perf_counter()
        while True:
            info = C.clod_server_poll(self.srv, self.seq)
            if info is not None:
                return info
            assert time.perf_counter() - t0 < timeout_s, f"job {self.seq} not done after {timeout_s} s"
            time.sleep(1e-4)

    def view_out(self, k):
        off = sum(v.width * v.height for v in self.views[:k])
        px = self.views[k].width * self.views[k].height
        return self.rgb[3 * off:3 * (off + px)], self.T[off:off + px], self.last[off:off + px]


def start(max_seconds=60.0):
    torch.cuda.synchronize()
    srv, workers = C.clod_server_start(0, max_seconds, torch.cuda.Stream())
    log(f"  server started with {workers} workers")
    return srv


def test_stop_on_request_and_argument_checks():
    log("case: persistent start / stop / checks")
    sc = synth.make_scene(2000, 3, "uniform", seed=3)
    plain = Scene(sc)
    packed = Scene(sc, packed_sh=True)
    job = Job(None, plain, sc["n"], [synth.look_at((0.0, 0.0, -3.0), width=64, height=48)])
    many = Job(None, packed, sc["n"], [synth.look_at((0.0, 0.0, -3.0), width=32, height=32)] * (C.SERVER_MAX_VIEWS + 1))
    srv = start()
    try:
        job.srv = many.srv = srv
        with pytest.raises(C.ClodError):          # plane-major SH only: the server needs packed SH
            job.submit()
        with pytest.raises(C.ClodError):          # more views than a job may carry
            many.submit()
    finally:
        status = C.clod_server_stop(srv)
    assert status == 1
    torch.cuda.synchronize()


def test_deadline_ends_the_kernel_by_itself():
    """max_seconds bounds every wait of the resident kernel: with no stop request it ends on
    its own, and stop reports the deadline."""
    log("case: persistent deadline")
    srv = start(max_seconds=0.5)
    time.sleep(1.5)
    with pytest.raises(C.ClodError, match="status 2"):
        C.clod_server_stop(srv)
    torch.cuda.synchronize()


def test_jobs_in_flight_match_per_stage_launches_and_4k_matches_oracle():
    """3M Gaussians resident.  Jobs in flight together: a 4K view alone, the same 4K view
    between a 720p and a 1080p request, and four small mixed jobs.  Every view of every job is
    byte-identical to the per-stage launches of the same batch, the 4K view of the mix to the
    4K view alone, and the 4K view to the oracle, pixel by pixel."""
    log("case: persistent 3M, 4K alone / in mix, small jobs")
    sc = synth.make_scene(3_000_000, 3, "mixture", seed=0)
    scene = Scene(sc, packed_sh=True)
    n = sc["n"]
    v4k = synth.look_at((2.0, 1.5, -7.0), width=3840, height=2160, s_v=1.7)
    v720 = synth.look_at((-9.0, 4.0, 12.0), width=1280, height=720, s_v=5.0)
    v1080 = synth.look_at((15.0, -2.0, -20.0), width=1920, height=1080, s_v=1.0)
    small = synth.poisson_requests(7, 10, rate_hz=1e4, resolutions=((320, 180), (480, 270), (640, 360)))
    groups = [[v4k], [v720, v4k, v1080]] + [[r.view for r in small[j:j + k]] for j, k in ((0, 1), (1, 3), (4, 2), (6, 4))]
    jobs = [Job(None, scene, n, g) for g in groups]   # every buffer allocated before the kernel starts
    srv = start()
    try:
        for j in jobs:
            j.srv = srv
            j.submit()
        infos = [j.wait() for j in jobs]
    finally:
        C.clod_server_stop(srv)
    torch.cuda.synchronize()
    for j, info in zip(jobs, infos):
        log(f"  job {j.seq}: {len(j.views)} views, pairs {info['n_dup']}, done at {info['t_ns'] / 1e6:.3f} ms")
        assert not info["overflow"]
        rgb, T, last = per_stage(sc, scene, j.views)
        assert same_bits(j.rgb, rgb) and same_bits(j.T, T) and torch.equal(j.last, last), j.seq
    a4k, m4k = jobs[0].view_out(0), jobs[1].view_out(1)
    for a, m in zip(a4k, m4k):
        assert torch.equal(a.view(torch.int32), m.view(torch.int32))
    o = O.render32(sc, v4k)
    rgb, T, last = m4k
    assert np.array_equal(last.cpu().numpy().reshape(o["last"].shape), o["last"])
    assert np.array_equal(T.cpu().numpy().reshape(o["T"].shape).view(np.uint32), o["T"].view(np.uint32))
    assert np.array_equal(rgb.cpu().numpy().reshape(o["rgb"].shape).view(np.uint32), o["rgb"].view(np.uint32))
    assert infos[1]["n_dup"] >= infos[0]["n_dup"]


def test_very_long_tile_lists_in_a_job_match_per_stage_and_oracle():
    """A dense cluster seen from far away (two tile lists of more than 65,536 entries beside
    short ones): the job's stages include the per-entry block masks of the very long tiles and
    the 4x4-block blend; the result is byte-identical to the per-stage launches and to the
    oracle."""
    log("case: persistent very long tile lists")
    dense = synth.make_scene(380_000, 0, "uniform", seed=33, log_scale_mean=-5.0)
    spread = synth.make_scene(20_000, 0, "uniform", seed=34, log_scale_mean=-2.5)
    spread["mean"] = (spread["mean"] * np.float32(12.0)).astype(np.float32)
    sc = dict(n=400_000, sh_degree=0, **{k: np.ascontiguousarray(np.concatenate([dense[k], spread[k]], axis=-1))
                                        for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh")})
    scene = Scene(sc, packed_sh=True)
    view = synth.look_at((0.0, 0.0, -40.0), width=96, height=80, s_v=1.0)
    job = Job(None, scene, sc["n"], [view], dup_pairs=1 << 22)
    srv = start()
    try:
        job.srv = srv
        job.submit()
        info = job.wait()
    finally:
        C.clod_server_stop(srv)
    torch.cuda.synchronize()
    assert not info["overflow"]
    o = O.render32(sc, view)
    lists = np.diff(o["tile_off"])
    log(f"  pairs {info['n_dup']}, longest list {lists.max()}, lists >= 65536: {(lists >= 65536).sum()}")
    assert (lists >= 65536).sum() >= 2 and info["n_dup"] == o["entries"].size
    rgb, T, last = per_stage(sc, scene, [view])
    assert same_bits(job.rgb, rgb) and same_bits(job.T, T) and torch.equal(job.last, last)
    assert np.array_equal(job.last.cpu().numpy().reshape(o["last"].shape), o["last"])
    assert np.array_equal(job.T.cpu().numpy().reshape(o["T"].shape).view(np.uint32), o["T"].view(np.uint32))
    assert np.array_equal(job.rgb.cpu().numpy().reshape(o["rgb"].shape).view(np.uint32), o["rgb"].view(np.uint32))


def test_overflowing_job_completes_flagged_and_resubmits():
    log("case: persistent overflow")
    sc = synth.make_scene(200_000, 3, "mixture", seed=4)
    scene = Scene(sc, packed_sh=True)
    views = [synth.look_at((0.5, -0.3, -4.0), width=640, height=480, s_v=1.2)]
    job = Job(None, scene, sc["n"], views, dup_pairs=1000)
    big = torch.empty(C.clod_dup_bytes(16 * 640 * 480), dtype=torch.uint8, device="cuda")
    srv = start()
    try:
        job.srv = srv
        job.submit()
        info = job.wait()
        assert info["overflow"] and 1000 < info["n_dup"] <= 16 * 640 * 480
        job.dup = big
        job.submit()
        info2 = job.wait()
    finally:
        C.clod_server_stop(srv)
    torch.cuda.synchronize()
    assert not info2["overflow"] and info2["n_dup"] == info["n_dup"]
    rgb, T, last = per_stage(sc, scene, views)
    assert same_bits(job.rgb, rgb) and same_bits(job.T, T) and torch.equal(job.last, last)


def test_scheduler_stream_alone_equals_mix_in_persistent_mode():
    """The continuous-batching scheduler driving the resident kernel: 24 requests of mixed
    resolution, pose and s_v batched up to six per job with up to eight jobs in flight; each
    request's image equals the per-stage render of that request alone."""
    log("case: persistent scheduler stream")
    sc = synth.make_scene(300_000, 3, "mixture", seed=2)
    scene = Scene(sc, packed_sh=True)
    reqs = synth.poisson_requests(5, 24, rate_hz=4000.0, resolutions=((320, 180), (480, 270), (960, 540)))
    recs, ex, sch = serve(scene, reqs, mode="persistent", budget_bytes=1 << 32, max_batch=6, max_inflight=8,
                          keep_outputs=True)
    log(f"  batches {sch.batches}, workers {ex.workers}, retries {ex.retries}")
    assert sch.batches < len(reqs)
    assert any(sum(1 for r in recs if r.batch == b) > 1 for b in range(sch.batches))
    assert all(np.isfinite(r.done_s) and r.done_s > r.admitted_s - 1e-3 for r in recs)
    for r in reqs:
        rgb, T, last = per_stage(sc, scene, [r.view])
        mrgb, mT, mlast = ex.outputs[r.rid]
        assert same_bits(rgb, mrgb) and same_bits(T, mT) and torch.equal(last, mlast), r.rid
