"""Parity at the benchmark's full sizes, in the launch configurations bench.py times.

* Serving headline: 3,000,000 Gaussians (degree 3, 64-cluster mixture, per-Gaussian SH copy,
  stored in Morton order as the benchmark stores its serving scenes; the oracle runs on the
  stored planes),
  the five LoD frames s_v = 1, 2, 4, 8, 16 of one pose as one batch at 1920x1080: counts, pair
  count, last-contributor indices, transmittance and colour of every pixel of every frame
  bit-identical to the oracle.
* Training step: 1,000,000 Gaussians at 1297x840 (L1 + point-count regulariser) and the
  16-view step over 2,000,000 Gaussians (640x480 / 1297x840 / 1920x1080), both scenes stored in
  Morton order as the benchmark stores them: counts bit-identical;
  for sampled Gaussians every parameter gradient within 1e-4 of FP64 autograd restricted to
  the tiles they cover.
* Continuous-LoD sweep: 6,000,000 Gaussians, 64 distances log-spaced in [2, 200] along one ray
  and the virtual sweep s_v = D_k / 2 at the nearest pose, each sweep's counts from one launch:
  bit-identical to the oracle on eight sampled distances of each sweep (the oracle takes about
  two seconds per 6M view), and never rising along the virtual sweep at all 64."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_09997_amd import _clod as C, synth
from paper_2510_09997_amd.render import Batch, Scene
from paper_2510_09997_amd.train import MultiViewTrainer

from helpers import check_grads, gpu_forward, params_struct, stored_planes

pytestmark = pytest.mark.gpu

SV_SWEEP = (1.0, 2.0, 4.0, 8.0, 16.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    C.load()


def log(*a):
    print(*a, flush=True)


def test_headline_batch_full_size_bitexact():
    log("case: 3M, five LoD frames at 1080p in one packed-SH batch, scene in Morton order")
    scene = Scene(synth.make_scene(3_000_000, 3, "mixture", seed=0), packed_sh=True, spatial_order=True)
    sc = stored_planes(scene)
    views = [synth.look_at((6.0, -3.5, -9.0), width=1920, height=1080, s_v=s) for s in SV_SWEEP]
    g = gpu_forward(sc, views, scene=scene)
    total = 0
    for v, view in enumerate(views):
        r = O.render32(sc, view)
        log(f"  s_v = {view.s_v:g}: counts {g['counts'][v].tolist()}, pairs {r['entries'].size}")
        assert np.array_equal(g["counts"][v], r["counts"]), (v, g["counts"][v], r["counts"])
        assert np.array_equal(g["last"][v], r["last"]), v
        assert np.array_equal(g["T"][v].view(np.uint32), r["T"].view(np.uint32)), v
        assert np.array_equal(g["rgb"][v].view(np.uint32), r["rgb"].view(np.uint32)), v
        total += r["entries"].size
    assert g["D"] == total
    # Fewer primitives are kept as the virtual distance grows.
    assert np.all(np.diff(g["counts"][:, 1]) <= 0)


def _images_bitexact(g, v, r):
    assert np.array_equal(g["counts"][v], r["counts"]), (v, g["counts"][v], r["counts"])
    assert np.array_equal(g["last"][v], r["last"]), v
    assert np.array_equal(g["T"][v].view(np.uint32), r["T"].view(np.uint32)), v
    assert np.array_equal(g["rgb"][v].view(np.uint32), r["rgb"].view(np.uint32)), v


def test_4k_request_alone_and_in_mixed_serving_batch_bitexact():
    """The serving stream's 3840x2160 requests (32,400 tiles per view) over the resident 3M scene:
    a 4K view rendered alone and inside a batch with a 1280x720 and a 1920x1080 request, every
    pixel of every view bit-identical to the oracle, and the 4K frame of the mix byte for byte
    the frame rendered alone."""
    log("case: 3M, 4K alone and in a 720p / 4K / 1080p batch, scene in Morton order")
    scene = Scene(synth.make_scene(3_000_000, 3, "mixture", seed=0), packed_sh=True, spatial_order=True)
    sc = stored_planes(scene)
    v4k = synth.look_at((2.0, 1.5, -7.0), width=3840, height=2160, s_v=1.7)
    v720 = synth.look_at((-9.0, 4.0, 12.0), width=1280, height=720, s_v=5.0)
    v1080 = synth.look_at((15.0, -2.0, -20.0), width=1920, height=1080, s_v=1.0)
    alone = gpu_forward(sc, [v4k], scene=scene)
    r4k = O.render32(sc, v4k)
    log(f"  4K alone: counts {alone['counts'][0].tolist()}, pairs {alone['D']}")
    _images_bitexact(alone, 0, r4k)
    assert alone["D"] == r4k["entries"].size
    del alone["batch"]
    mixed = gpu_forward(sc, [v720, v4k, v1080], scene=scene)
    log(f"  mix: counts {mixed['counts'].tolist()}, pairs {mixed['D']}")
    _images_bitexact(mixed, 1, r4k)
    for v, view in ((0, v720), (2, v1080)):
        _images_bitexact(mixed, v, O.render32(sc, view))
    for key in ("last", "T", "rgb"):
        assert np.array_equal(mixed[key][1].view(np.uint32), alone[key][0].view(np.uint32)), key


def test_lod_sweep_6m_frames_bitexact_at_four_distances():
    """Frames of the continuous-LoD sweep (6M Gaussians, 1920x1080, camera at D_k = 2 100^(k/63)
    on the -z axis) at k = 0, 21, 42, 56, 63: the far frames hold the longest tile lists of any
    workload (at k = 56 and 63 lists of 65,536 entries or more, walked compacted per 4x4 block).
    Counts, pair count, last index, T and colour of every pixel bit-identical."""
    log("case: 6M LoD sweep frames, scene in Morton order")
    scene = Scene(synth.make_scene(6_000_000, 3, "mixture", seed=0), packed_sh=True, spatial_order=True)
    sc = stored_planes(scene)
    ds = synth.sweep_distances(64, 2.0, 200.0)
    for k in (0, 21, 42, 56, 63):
        view = synth.look_at((0.0, 0.0, -float(ds[k])), width=1920, height=1080)
        g = gpu_forward(sc, [view], scene=scene)
        r = O.render32(sc, view)
        lists = np.diff(r["tile_off"])
        log(f"  k={k} d={ds[k]:.2f}: counts {g['counts'][0].tolist()}, pairs {g['D']}, longest list {lists.max()}")
        _images_bitexact(g, 0, r)
        assert g["D"] == r["entries"].size
        del g


def test_lod_sweep_6m_counts_sampled_bitexact_and_monotone():
    log("case: 6M LoD sweep, 64 distances")
    sc = synth.make_scene(6_000_000, 3, "mixture", seed=0)
    scene = Scene(sc)
    ds = synth.sweep_distances(64, 2.0, 200.0)
    ray = [synth.look_at((0.0, 0.0, -float(d)), width=1920, height=1080) for d in ds]
    virt = [synth.look_at((0.0, 0.0, -2.0), width=1920, height=1080, s_v=float(d / 2.0)) for d in ds]
    sample = [0, 9, 18, 27, 36, 45, 54, 63]
    for name, views in (("ray", ray), ("virtual", virt)):
        b = Batch(sc["n"], views, params_struct(None))
        cnt = b.lod_count(scene).cpu().numpy()
        del b
        for k in sample:
            want = O.view_pass(sc, views[k])["counts"]
            log(f"  {name} k={k}: {cnt[k].tolist()}")
            assert np.array_equal(cnt[k], want), (name, k, cnt[k], want)
        if name == "virtual":
            assert np.all(np.diff(cnt[:, 1]) <= 0) and np.all(np.diff(cnt[:, 2]) <= 0)
            assert cnt[0, 1] > cnt[-1, 1]


def _sampled_gradient_parity(sc, views, pix, counts, dL, deta, got, rng, per_view_min=1, samples=12):
    """Counts bit-exact per view; for sampled rendered Gaussians (no frustum argmax) the
    gradients summed over the views against FP64 autograd over the tiles they cover."""
    vps = [O.render32(sc, v) for v in views]
    for j, vp in enumerate(vps):
        assert np.array_equal(counts[j], vp["counts"]), (j, counts[j], vp["counts"])
    rendered = np.stack([(vp["flags"] & 4) > 0 for vp in vps])
    argmaxes = {vp["argmax"] for vp in vps}
    cand = np.array([g for g in np.nonzero(rendered.sum(0) >= per_view_min)[0] if g not in argmaxes])
    sample = rng.choice(cand, size=min(samples, cand.size), replace=False)
    want = {k: np.zeros(got[k][..., sample].shape) for k in got}
    S = {k: np.zeros(got[k][..., sample].shape) for k in got}
    for j, (view, vp) in enumerate(zip(views, vps)):
        TW = (view.width + 15) // 16
        tiles = set()
        for g in sample:
            if vp["flags"][g] & 4:
                x0, x1, y0, y1 = vp["rect"][g]
                tiles.update(int(ty * TW + tx) for ty in range(y0, y1) for tx in range(x0, x1))
        h, w = view.height, view.width
        a = int(pix[j])
        gv = dL[3 * a:3 * a + 3 * h * w].reshape(3, h, w)
        ref = O.fp64_grads(sc, view, vp, gv, float(deta[j]), tiles=sorted(tiles), abs_terms=True)
        for k in want:
            want[k] += ref[k][..., sample]
            S[k] += ref["abs"][k][..., sample]
    check_grads({k: got[k][..., sample] for k in got}, want, S, 1e-4, log=log)


def test_training_step_1m_full_size_sampled_gradients():
    log("case: 1M single-view training step at 1297x840, scene in Morton order")
    scene = Scene(synth.make_scene(1_000_000, 3, "mixture", seed=0), spatial_order=True)
    sc = stored_planes(scene)
    view = synth.random_views(0, 1, radius=(4.0, 6.0), resolutions=((1297, 840),), sv_range=(1.0, 8.0))[0]
    target = torch.from_numpy(synth.random_target(0, 840, 1297).reshape(-1)).cuda()
    b = Batch(sc["n"], [view], params_struct(None))
    b.project(scene)
    b.bin_sort()
    rgb, T, last = b.render_fwd()
    _, dL, deta = b.loss(rgb, target, 8.0, 1.0)
    grads = b.render_bwd(scene, T, last, dL, deta)
    torch.cuda.synchronize()
    _sampled_gradient_parity(sc, [view], b.pix_base, b.counts.cpu().numpy(), dL.cpu().numpy(), deta.cpu().numpy(),
                             {k: v.cpu().numpy() for k, v in grads.items()}, np.random.default_rng(1))


def test_sixteen_view_step_2m_full_size_sampled_gradients():
    log("case: 2M 16-view training step, scene in Morton order")
    scene = Scene(synth.make_scene(2_000_000, 3, "mixture", seed=0), spatial_order=True)
    sc = stored_planes(scene)
    res = ((640, 480), (1297, 840), (1920, 1080))
    views = synth.random_views(7, 16, radius=(4.0, 6.0), resolutions=res, sv_range=(1.0, 8.0))
    tr = MultiViewTrainer(scene, views, s_max=8.0)
    tr.set_target(torch.rand(3 * tr.batch.pixels, device="cuda", generator=torch.Generator("cuda").manual_seed(0), dtype=torch.float32))
    tr.step()
    assert not tr.overflowed()
    torch.cuda.synchronize()
    _sampled_gradient_parity(sc, views, tr.batch.pix_base, tr.batch.counts.cpu().numpy(), tr.dL.cpu().numpy(), tr.deta.cpu().numpy(),
                             {k: v.cpu().numpy() for k, v in tr.grads.items()}, np.random.default_rng(2),
                             per_view_min=2)
