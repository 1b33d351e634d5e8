"""Benchmark of the CLoD-GS render path on one MI355X.

Headline: 1080p frames/s at 3,000,000 Gaussians (SH degree 3, 64-cluster mixture) across
the LoD sweep s_v in {1, 2, 4, 8, 16}.  One step renders the five LoD frames of one random
pose (radius U(3, 30), direction uniform) as one batched pass of the forward path
(clod_project, clod_bin_sort, clod_render_fwd).  Inputs are resident in HBM before timing.
The timed steps run pipelined over three streams, each with its own workspace (the overlap
a continuous-batching server gets); the same steps also run once sequentially on one stream,
which gives the per-stage times and the roofline of the blend launched alone.

Also reported on the same line: the plain per-request path (one view per pass), the
training step (1,000,000 Gaussians, 1297x840, forward + loss + backward, ms/iter), the
roofline of the dominant kernel (timed with events around its own launch on the stream it
runs on) and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-train]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU peak without packed FP32: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s;
# a fused multiply-add counts 2 flops -> 78.6 TFLOP/s.
VALU_PEAK_TFLOPS = 78.6
SV_SWEEP = (1.0, 2.0, 4.0, 8.0, 16.0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic HBM bytes of the path (what the method must move, not what a design moves):
# N Gaussians, R rendered (view, Gaussian) records, D tile pairs, P pixels, SH degree 3.
#   forward  = 20 N (means, opacity, decay: read once per batch) + 280 R (scale, rotation and 48
#              SH coefficients read, 52-byte record written, 8-byte scan entry) + 84 D (keys
#              written, one sort pass read + write, ranges, record and index reads of the blend)
#              + 20 P (colour, T, last index written)
#   backward = 20 P (dL/dC, T, last read) + 76 D (records re-read, screen-space partials
#              accumulated) + 36 R (partials read) + 480 N (all parameters read, all gradients
#              written: the point-count term reaches every Gaussian)
#   loss     = 36 P (rendered colour and target read, dL/dC written)
def fwd_bytes(N, R, D, P):
    return 20 * N + 280 * R + 84 * D + 20 * P


def bwd_bytes(N, R, D, P):
    return 20 * P + 76 * D + 36 * R + 480 * N


LOSS_BYTES_PER_PIXEL = 36
# Flops per pair of the adjoint loop's live pairs (power, alpha, transmittance recovery, colour
# dot product, the nine partial sums and the colour recurrence).
FLOPS_PER_PAIR_BWD = 45


def pose_views(seed: int, k: int, width=1920, height=1080, radius=(3.0, 30.0)):
    from paper_2510_09997_amd import synth
    rng = np.random.default_rng(seed + 1000)
    dirs = synth.unit_vectors(rng, k)
    radii = rng.uniform(radius[0], radius[1], size=k)
    return [[synth.look_at(dirs[j] * radii[j], width=width, height=height, s_v=s) for s in SV_SWEEP]
            for j in range(k)]


class StepTables:
    """Per-step view tables uploaded to HBM before timing (host copies kept for launch geometry)."""

    def __init__(self, per_step_views):
        import torch
        from paper_2510_09997_amd import _clod as C
        self.host = [C.make_views(vs) for vs in per_step_views]
        self.dev = [C.views_to_device(h, "cuda") for h in self.host]
        torch.cuda.synchronize()


def run_serving(args, torch, C, Batch, Scene, synth):
    n = 3_000_000
    log(f"[bench] scene: {n} Gaussians, SH degree 3, mixture")
    sc = synth.make_scene(n, 3, "mixture", seed=0)
    # Static scene: stored in Morton order of the means (clod_scene_reorder), per-Gaussian SH copy.
    scene = Scene(sc, packed_sh=True, spatial_order=True)
    del sc
    K, W = args.steps, args.warmup
    # Timed poses depend on K only (warm-up poses are drawn apart), so any warm-up count times
    # the same launches.
    steps = pose_views(7, W) + pose_views(0, K)
    tables = StepTables(steps)
    # Batched path: one Batch with five 1080p views; capacity sized by a sizing pass.
    b = Batch(n, steps[0])
    dmax = 0
    for j in range(K + W):
        b.views_host, b.views_dev = tables.host[j], tables.dev[j]
        b.project(scene)
        dmax = max(dmax, b.bin_sort())
    cap = int(dmax * 1.1) + 4096
    b._alloc_dup(cap)
    log(f"[bench] max pairs per 5-frame step {dmax}, capacity {cap}")
    pairs = torch.zeros(3, dtype=torch.int64, device="cuda")
    # Pipelined serving: consecutive steps rotate over NS streams, each with its own batch
    # workspace and output buffers, so one step's projection and binning (latency-bound, few
    # waves) overlap the previous step's blend (issue-bound).  Slot 0 also runs the sequential
    # pass that times each stage in isolation.
    NS = max(1, args.streams)
    slots = [b] + [Batch(n, steps[0], dup_capacity=cap) for _ in range(NS - 1)]
    outs = [(torch.empty(3 * b.pixels, device="cuda", dtype=torch.float32), torch.empty(b.pixels, device="cuda", dtype=torch.float32),
             torch.empty(b.pixels, dtype=torch.int32, device="cuda")) for _ in range(NS)]
    streams = [torch.cuda.Stream() for _ in range(NS)]
    rgb, T, last = outs[0]
    scs = scene.c_struct()

    def step(j, ev=None, slot=0, stream=None):
        sb = slots[slot]
        sb.views_host, sb.views_dev = tables.host[j], tables.dev[j]
        bs = sb.c_struct()
        C.clod_project(scs, bs, sb.counts, stream=stream)
        if ev is not None:
            ev[0].record()
        C.clod_bin_sort(bs, sync_count=False, stream=stream)
        if ev is not None:
            ev[1].record()
        C.clod_render_fwd(bs, *outs[slot], None, stream=stream)
        if ev is not None:
            ev[2].record()

    def pipelined(j0, count):
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for k in range(count):
            i = k % NS
            step(j0 + k, slot=i, stream=streams[i])
        for st in streams:
            cur.wait_stream(st)

    if args.profile == "timed-blend":
        # Only the launches whose blend time the roofline uses: the timed steps, one after the
        # other on one stream (the sequential pass below), for hardware counters of exactly them.
        evp = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
        for k in range(K):
            evp[k][3].record()
            step(W + k, evp[k])
        torch.cuda.synchronize()
        blend = sum(e[1].elapsed_time(e[2]) for e in evp) / K
        return dict(profile="timed-blend", blend_fwd_ms=blend, steps=K), scene, b, steps
    pipelined(0, max(W, NS))
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # Sequential pass over the timed steps (one stream, events around every stage).
    start.record()
    for k in range(K):
        evs[k][3].record()
        step(W + k, evs[k])
    end.record()
    torch.cuda.synchronize()
    seq_ms = start.elapsed_time(end)
    # Headline timed region: the same K steps, pipelined over the NS streams.
    start.record()
    pipelined(W, K)
    end.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    for sb in slots:
        info = C.clod_read_info(sb.c_struct())
        assert not info["overflow"], "duplicate buffer overflow inside the timed region"
    # Each slot's output of its last pipelined step against a sequential re-render of the same
    # step on the default stream (untimed): the overlap must not change a single byte.
    identical = True
    for i in range(NS):
        ks = [k for k in range(K) if k % NS == i]
        if not ks:
            continue
        got = [o.clone() for o in outs[i]]
        step(W + ks[-1], slot=i)
        torch.cuda.synchronize()
        identical = identical and all(torch.equal(a, b_) for a, b_ in zip(got, outs[i]))
    proj_ms = sum(e[3].elapsed_time(e[0]) for e in evs) / K
    sort_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / K
    blend_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / K
    frames = len(SV_SWEEP) * K
    # Work counters of the blend, from an untimed re-run of the timed steps (the timed
    # launches carry no counters, so their duration is the blend kernel alone).
    pairs_per_step = None
    dups, rend = [], []
    if not args.no_count:
        for k in range(K):
            b.views_host, b.views_dev = tables.host[W + k], tables.dev[W + k]
            bs = b.c_struct()
            C.clod_project(scs, bs, b.counts)
            C.clod_bin_sort(bs, sync_count=False)
            C.clod_render_fwd(bs, rgb, T, last, pairs)
            dups.append(C.clod_read_info(bs)["n_dup"])
            rend.append(int(b.counts[:, 2].sum().item()))
        torch.cuda.synchronize()
        pairs_per_step = (pairs.cpu().numpy() / K).tolist()
    res = dict(total_ms=total_ms, ms_per_step=total_ms / K, fps=frames / (total_ms / 1e3), streams=NS,
               pipelined_identical=identical,
               sequential_fps=frames / (seq_ms / 1e3), sequential_ms_per_step=seq_ms / K,
               stage_ms=dict(project=proj_ms, bin_sort=sort_ms, blend_fwd=blend_ms),
               pairs_per_step=pairs_per_step, max_dup=dmax, blend_launches=K,
               dup_per_step=float(np.mean(dups)) if dups else None, pixels_per_step=b.pixels,
               rendered_per_step=float(np.mean(rend)) if rend else None)
    if dups:
        nb = fwd_bytes(n, res["rendered_per_step"], res["dup_per_step"], b.pixels)
        res["hbm"] = {"algorithmic_bytes_per_step": int(nb),
                      "frac_pipelined": round(nb / (res["ms_per_step"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                      "frac_sequential": round(nb / (res["sequential_ms_per_step"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
    # Per-view kept counts of the last step (mask counts fall with s_v).
    res["counts_last_step"] = b.counts.cpu().numpy().tolist()

    if args.no_plain:
        return res, scene, b, steps
    # Plain per-request path: one view per pass, same frames.
    single = [Batch(n, [steps[0][i]], dup_capacity=cap) for i in range(len(SV_SWEEP))]
    singles_host = [[C.make_views([v]) for v in vs] for vs in steps]
    singles_dev = [[C.views_to_device(h, "cuda") for h in hs] for hs in singles_host]
    outs = [(torch.empty(3 * sb.pixels, device="cuda", dtype=torch.float32), torch.empty(sb.pixels, device="cuda", dtype=torch.float32),
             torch.empty(sb.pixels, dtype=torch.int32, device="cuda")) for sb in single]

    def plain(j):
        for i, sb in enumerate(single):
            sb.views_host, sb.views_dev = singles_host[j][i], singles_dev[j][i]
            bs = sb.c_struct()
            C.clod_project(scene.c_struct(), bs, sb.counts)
            C.clod_bin_sort(bs, sync_count=False)
            C.clod_render_fwd(bs, *outs[i], None)

    for j in range(W):
        plain(j)
    torch.cuda.synchronize()
    start.record()
    for k in range(K):
        plain(W + k)
    end.record()
    torch.cuda.synchronize()
    plain_ms = start.elapsed_time(end)
    res["plain_fps"] = frames / (plain_ms / 1e3)
    res["plain_ms_per_step"] = plain_ms / K
    return res, scene, b, steps


def run_train(args, torch, C, Batch, Scene, synth):
    n = 1_000_000
    log(f"[bench] training: {n} Gaussians, SH degree 3, 1297x840")
    sc = synth.make_scene(n, 3, "mixture", seed=0)
    scene = Scene(sc, spatial_order=True)   # stored in Morton order of the means (clod_scene_reorder)
    del sc
    K, W = args.train_steps, 5
    views = synth.random_views(0, K + W, radius=(4.0, 6.0), resolutions=((1297, 840),), sv_range=(1.0, 8.0))
    hosts = [C.make_views([v]) for v in views]
    devs = [C.views_to_device(h, "cuda") for h in hosts]
    target = torch.from_numpy(synth.random_target(0, 840, 1297).reshape(-1)).cuda()
    b = Batch(n, [views[0]])
    dmax = 0
    for j in range(K + W):
        b.views_host, b.views_dev = hosts[j], devs[j]
        b.project(scene)
        dmax = max(dmax, b.bin_sort())
    b._alloc_dup(int(dmax * 1.1) + 4096)
    grads = scene.zeros_like()
    rgb = torch.empty(3 * b.pixels, device="cuda", dtype=torch.float32)
    T = torch.empty(b.pixels, device="cuda", dtype=torch.float32)
    last = torch.empty(b.pixels, dtype=torch.int32, device="cuda")
    loss = torch.empty(1, device="cuda", dtype=torch.float32)
    dL = torch.empty_like(rgb)
    deta = torch.empty(1, device="cuda", dtype=torch.float32)
    gs = C.make_grad(grads)

    def it(j, ev=None):
        b.views_host, b.views_dev = hosts[j], devs[j]
        bs = b.c_struct()
        s = scene.c_struct()
        C.clod_project(s, bs, b.counts)
        C.clod_bin_sort(bs, sync_count=False)
        C.clod_render_fwd(bs, rgb, T, last, None)
        C.clod_loss(bs, rgb, target, 8.0, 1.0, loss, dL, deta)
        if ev is not None:
            ev[0].record()
        C.clod_render_bwd(s, bs, T, last, dL, deta, False, gs)
        if ev is not None:
            ev[1].record()

    for j in range(W):
        it(j)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    per = []
    for k in range(K):
        evs[k][2].record()
        it(W + k, evs[k])
    end.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(end)
    it_ms = [evs[k][2].elapsed_time(evs[k + 1][2]) for k in range(K - 1)] + [evs[K - 1][2].elapsed_time(end)]
    bwd_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / K
    info = C.clod_read_info(b.c_struct())
    assert not info["overflow"]
    res = dict(ms_per_iter=total / K, p50_ms=float(np.percentile(it_ms, 50)), p99_ms=float(np.percentile(it_ms, 99)),
               bwd_ms=bwd_ms, max_dup=dmax)
    # Work of the timed iterations, from an untimed re-run of the first ten of them: records,
    # tile pairs and the pairs of both per-pixel loops (the kernels count them exactly).
    fp = torch.zeros(3, dtype=torch.int64, device="cuda")
    bp = torch.zeros(3, dtype=torch.int64, device="cuda")
    R, D, S = [], [], min(K, 10)
    for k in range(S):
        b.views_host, b.views_dev = hosts[W + k], devs[W + k]
        bs = b.c_struct()
        s = scene.c_struct()
        C.clod_project(s, bs, b.counts)
        C.clod_bin_sort(bs, sync_count=False)
        C.clod_render_fwd(bs, rgb, T, last, fp)
        C.clod_loss(bs, rgb, target, 8.0, 1.0, loss, dL, deta)
        C.clod_render_bwd(s, bs, T, last, dL, deta, False, gs, pairs=bp)
        D.append(C.clod_read_info(bs)["n_dup"])
        R.append(int(b.counts[0, 2].item()))
    torch.cuda.synchronize()
    Rm, Dm, P = float(np.mean(R)), float(np.mean(D)), b.pixels
    fb, bb = fwd_bytes(n, Rm, Dm, P), bwd_bytes(n, Rm, Dm, P)
    tot = fb + bb + LOSS_BYTES_PER_PIXEL * P
    fpairs, bpairs = (fp.cpu().numpy() / S).tolist(), (bp.cpu().numpy() / S).tolist()
    res.update(rendered=Rm, pairs=Dm, pixels=P, fwd_pairs=fpairs, bwd_pairs=bpairs,
               hbm={"algorithmic_bytes_per_iter": int(tot), "fwd_bytes": int(fb), "bwd_bytes": int(bb),
                    "frac": round(tot / (res["ms_per_iter"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                    "bwd_frac": round(bb / (bwd_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)},
               bwd_alu={"flops_per_pair": FLOPS_PER_PAIR_BWD, "live_pairs": bpairs[1],
                        "tflops_over_clod_render_bwd": round(FLOPS_PER_PAIR_BWD * bpairs[1] / (bwd_ms * 1e-3) / 1e12, 3)})
    return res


def run_multiview_train(args, torch, C, Scene, synth):
    """16 views per step (resolutions among 640x480, 1297x840, 1920x1080, fixed per view slot;
    poses radius U(4, 6), s_v log-uniform [1, 8] redrawn every step), 2M Gaussians, forward +
    loss + backward captured once in a graph and replayed."""
    from paper_2510_09997_amd.train import MultiViewTrainer
    n = 2_000_000
    sc = synth.make_scene(n, 3, "mixture", seed=0)
    scene = Scene(sc, spatial_order=True)   # stored in Morton order of the means (clod_scene_reorder)
    del sc
    res = ((640, 480), (1297, 840), (1920, 1080))
    K, W = args.train_steps, 5
    first = synth.random_views(7, 16, radius=(4.0, 6.0), resolutions=res, sv_range=(1.0, 8.0))
    slots = [(v.width, v.height) for v in first]
    sets = [first]
    for j in range(1, K + W):
        vs = synth.random_views(7 + 31 * j, 16, radius=(4.0, 6.0), resolutions=((640, 480),), sv_range=(1.0, 8.0))
        sets.append([synth.look_at(v.c, width=w, height=h, s_v=v.s_v) for v, (w, h) in zip(vs, slots)])
    tr = MultiViewTrainer(scene, first, s_max=8.0, dup_capacity=1)
    dmax = tr.size_capacity(sets)
    tables = [C.views_to_device(C.make_views(vs), "cuda") for vs in sets]
    tr.set_target(torch.rand(3 * tr.batch.pixels, device="cuda", generator=torch.Generator("cuda").manual_seed(0), dtype=torch.float32))
    eager = args.profile == "multiview-eager"
    if not eager:
        tr.capture()
    for j in range(W):
        tr.set_views_dev(tables[j])
        tr.step()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    evs[0].record()
    for k in range(K):
        tr.set_views_dev(tables[W + k])
        tr.step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    per = [evs[k].elapsed_time(evs[k + 1]) for k in range(K)]
    assert not tr.overflowed(), "duplicate buffer overflow inside the timed region"
    # Records and tile pairs of the timed steps (untimed eager re-run of the first five).
    R, D = [], []
    graph, tr.graph = tr.graph, None
    for k in range(min(K, 5)):
        tr.set_views_dev(tables[W + k])
        tr.step()
        D.append(tr.n_dup())
        R.append(int(tr.batch.counts[:, 2].sum().item()))
    tr.graph = graph
    Rm, Dm, P = float(np.mean(R)), float(np.mean(D)), tr.batch.pixels
    step_bytes = fwd_bytes(n, Rm, Dm, P) + bwd_bytes(n, Rm, Dm, P) + LOSS_BYTES_PER_PIXEL * P
    hbm = {"algorithmic_bytes_per_step": int(step_bytes), "rendered": Rm, "pairs": Dm,
           "frac": round(step_bytes / (float(np.mean(per)) * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
    if eager:
        return dict(ms_per_step=float(np.mean(per)), p50_ms=float(np.percentile(per, 50)), eager=True, views=16,
                    gaussians=n, pixels_per_step=P, hbm=hbm)
    # The same step with the full 3DGS rendering loss (0.8 L1 + 0.2 D-SSIM), re-captured.
    tr.lambda_dssim = 0.2
    tr.capture()
    torch.cuda.synchronize()
    d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    d0.record()
    for k in range(K):
        tr.set_views_dev(tables[W + k])
        tr.step()
    d1.record()
    torch.cuda.synchronize()
    dssim_ms = d0.elapsed_time(d1) / K
    # Fused Adam over all 2M x 60 parameters (one launch per step, outside the graph since its
    # learning rates and bias corrections change every step).
    from paper_2510_09997_amd.train import DEFAULT_LRS, FusedAdam
    opt = FusedAdam(scene)
    for _ in range(3):
        opt.step(tr.grads, DEFAULT_LRS)
    torch.cuda.synchronize()
    reps = 20
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record()
    for _ in range(reps):
        opt.step(tr.grads, DEFAULT_LRS)
    a1.record()
    torch.cuda.synchronize()
    adam_ms = a0.elapsed_time(a1) / reps
    nparam = sum(v.numel() for v in scene.t.values())
    adam_bytes = 28 * nparam   # read parameter, gradient, m, v; write parameter, m, v
    return dict(ms_per_step=float(np.mean(per)), p50_ms=float(np.percentile(per, 50)),
                p99_ms=float(np.percentile(per, 99)), views=16, gaussians=n, max_dup=dmax,
                pixels_per_step=tr.batch.pixels, ms_per_step_with_dssim=dssim_ms, adam_ms=adam_ms, adam_params=nparam,
                adam_hbm_frac=adam_bytes / (adam_ms * 1e-3) / 8e12, hbm=hbm)


def run_budget_sweep(args, torch, C, Batch, scene, pose):
    """Primitive budget -> frames/s: one 1080p view (a headline pose, s_v = 1) rendered with
    the K largest alpha'' kept, K from 25,000 to all 3,000,000 (the selection of the paper's
    quality/speed comparisons)."""
    import dataclasses
    n = scene.n
    out = {"budgets": [], "kept": [], "rendered": [], "fps": []}
    budgets = [25_000, 50_000, 100_000, 200_000, 400_000, 800_000, 1_600_000, n]
    b = Batch(n, [dataclasses.replace(pose, budget=budgets[0])])
    rgb = torch.empty(3 * b.pixels, device="cuda", dtype=torch.float32)
    T = torch.empty(b.pixels, device="cuda", dtype=torch.float32)
    last = torch.empty(b.pixels, dtype=torch.int32, device="cuda")
    for k in budgets:
        b.update_views([dataclasses.replace(pose, budget=k)])
        b.project(scene)
        b.bin_sort()
        bs = b.c_struct()
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            C.clod_project(scene.c_struct(), bs, b.counts)
            C.clod_bin_sort(bs, sync_count=False)
            C.clod_render_fwd(bs, rgb, T, last, None)
        e1.record()
        torch.cuda.synchronize()
        cnt = b.counts.cpu().numpy()[0]
        out["budgets"].append(int(k))
        out["kept"].append(int(cnt[1]))
        out["rendered"].append(int(cnt[2]))
        out["fps"].append(round(reps / (e0.elapsed_time(e1) / 1e3), 2))
    return out


def run_strips(args, torch, C, Batch, scene, pose, synth):
    """Spatially varying s_v: a 1080p frame rendered as four vertical strips at s_v = 8, 4, 2, 1
    (the layout of the paper's DLoD/CLoD comparison), as one batch of viewports, against the
    whole frame at s_v = 1.  Frames/s and per-strip kept counts."""
    out = {}
    for name, views in (("uniform", [pose]), ("strips", synth.strips(pose, [8.0, 4.0, 2.0, 1.0]))):
        b = Batch(scene.n, views)
        b.project(scene)
        b.bin_sort()
        rgb = torch.empty(3 * b.pixels, device="cuda", dtype=torch.float32)
        T = torch.empty(b.pixels, device="cuda", dtype=torch.float32)
        last = torch.empty(b.pixels, dtype=torch.int32, device="cuda")
        bs = b.c_struct()
        reps = 10
        for _ in range(2):
            C.clod_project(scene.c_struct(), bs, b.counts)
            C.clod_bin_sort(bs, sync_count=False)
            C.clod_render_fwd(bs, rgb, T, last, None)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            C.clod_project(scene.c_struct(), bs, b.counts)
            C.clod_bin_sort(bs, sync_count=False)
            C.clod_render_fwd(bs, rgb, T, last, None)
        e1.record()
        torch.cuda.synchronize()
        out[name + "_fps"] = round(reps / (e0.elapsed_time(e1) / 1e3), 2)
        out[name + "_kept"] = b.counts.cpu().numpy()[:, 1].tolist()
        del b
    out["strip_s_v"] = [8.0, 4.0, 2.0, 1.0]
    return out


def run_lod_sweep(args, torch, C, Batch, Scene, synth):
    """6M Gaussians, 1920x1080, 64 camera distances log-spaced in [2, 200] along one ray
    (looking at the origin from -z): kept-primitive counts of all 64 views in one launch, and
    frames/s of the forward render at each distance; also the virtual sweep s_v = D_k / 2 at
    the nearest pose."""
    n = 6_000_000
    sc = synth.make_scene(n, 3, "mixture", seed=0)
    # Static scene: stored in Morton order of the means (clod_scene_reorder), per-Gaussian SH copy.
    scene = Scene(sc, packed_sh=True, spatial_order=True)
    del sc
    ds = synth.sweep_distances(64, 2.0, 200.0)
    ray = [synth.look_at((0.0, 0.0, -float(d)), width=1920, height=1080) for d in ds]
    virt = [synth.look_at((0.0, 0.0, -2.0), width=1920, height=1080, s_v=float(d / 2.0)) for d in ds]
    out = {"distances": [round(float(d), 3) for d in ds]}
    for name, views in (("ray", ray), ("virtual", virt)):
        b = Batch(n, views)
        b.lod_count(scene)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cnt = b.lod_count(scene)
        e1.record()
        torch.cuda.synchronize()
        out[name + "_counts_ms"] = round(e0.elapsed_time(e1), 4)
        out[name + "_counts"] = cnt.cpu().numpy().tolist()
        del b
    # Frames per distance (one view per pass), capacity sized per pose.
    fps = []
    b = Batch(n, [ray[0]])
    rgb = torch.empty(3 * b.pixels, device="cuda", dtype=torch.float32)
    T = torch.empty(b.pixels, device="cuda", dtype=torch.float32)
    last = torch.empty(b.pixels, dtype=torch.int32, device="cuda")
    stage = {"project": [], "bin_sort": [], "blend_fwd": []}
    work = {"rendered": [], "pairs": [], "longest_list": [], "evaluated": [], "blended": []}
    pairs = torch.zeros(3, dtype=torch.int64, device="cuda")
    for k, v in enumerate(ray):
        b.update_views([v])
        b.project(scene)
        b.bin_sort()
        bs = b.c_struct()
        reps = 3
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
        for r in range(reps):
            ev[r][0].record()
            C.clod_project(scene.c_struct(), bs, None)
            ev[r][1].record()
            C.clod_bin_sort(bs, sync_count=False)
            ev[r][2].record()
            C.clod_render_fwd(bs, rgb, T, last, None)
            ev[r][3].record()
        torch.cuda.synchronize()
        fps.append(round(reps / (ev[0][0].elapsed_time(ev[-1][3]) / 1e3), 2))
        for j, key in enumerate(("project", "bin_sort", "blend_fwd")):
            stage[key].append(round(float(np.mean([e[j].elapsed_time(e[j + 1]) for e in ev])), 4))
        # Work of the frame (untimed counting re-run of the blend).
        pairs.zero_()
        C.clod_render_fwd(bs, rgb, T, last, pairs)
        rg = b.section(C.SEC_RANGES).view(-1, 2).to(torch.int64)
        pc = pairs.cpu().numpy()
        work["rendered"].append(int(b.counts[0, 2].item()))
        work["pairs"].append(int(C.clod_read_info(bs)["n_dup"]))
        work["longest_list"].append(int((rg[:, 1] - rg[:, 0]).max().item()))
        work["evaluated"].append(int(pc[0]))
        work["blended"].append(int(pc[2]))
    out["ray_fps"] = fps
    out["ray_stage_ms"] = stage
    out["ray_work"] = work
    return out


def run_serve_stream(args, torch, Scene, synth):
    """Request streams over the resident 3M scene, resolutions uniform over {720p, 1080p, 4K},
    s_v log-uniform in [1, 16], served three ways: plain (one forward render per request, in
    arrival order), multi-stream continuous batching (host-launched stages on three streams)
    and the persistent serving kernel (up to eight batches in flight inside one resident
    kernel).  The plain path's capacity is measured first (every request queued at once); the
    overload stream then arrives at 1.25 times that rate, a light stream at 200 requests/s.
    Latency is measured from arrival to the device completion of the request's batch."""
    from paper_2510_09997_amd.serve import serve, summarize
    n = 3_000_000
    sc = synth.make_scene(n, 3, "mixture", seed=0)
    # Static scene: stored in Morton order of the means (clod_scene_reorder), per-Gaussian SH copy.
    scene = Scene(sc, packed_sh=True, spatial_order=True)
    del sc
    budget = 24 << 30
    inflight = {"plain": 1, "continuous": 3, "persistent": 8}

    def run(reqs, mode, warm):
        recs, ex, sch = serve(scene, reqs, mode=mode, budget_bytes=budget, max_batch=8, max_inflight=inflight[mode])
        s = summarize(recs, first=warm)
        s["retries"] = ex.retries
        s["batches"] = sch.batches
        s["peak_hbm_gib"] = round(sch.peak_in_use / 2 ** 30, 3)
        if mode == "persistent":
            s["workers"] = ex.workers
        torch.cuda.synchronize()
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}

    out = {"persistent_timeline": server_timeline(torch, scene, synth)}
    burst = synth.poisson_requests(2, args.serve_capacity_requests, rate_hz=1e9)
    cap = run(burst, "plain", 0)
    capacity = cap["frames_per_s"]
    out["plain_capacity_fps"] = round(capacity, 2)
    log(f"[bench] serve: plain capacity {capacity:.1f} frames/s")
    rate = 1.25 * capacity
    warm = args.serve_warmup
    over = synth.poisson_requests(1, warm + args.serve_requests, rate_hz=rate)
    light = synth.poisson_requests(3, warm + args.serve_light_requests, rate_hz=200.0)
    out["overload"] = {"rate_hz": round(rate, 2), "requests": args.serve_requests}
    out["light"] = {"rate_hz": 200.0, "requests": args.serve_light_requests}
    for name, reqs in (("overload", over), ("light", light)):
        for mode in ("plain", "continuous", "persistent"):
            out[name][mode] = run(reqs, mode, warm)
            log(f"[bench] serve {name} {mode}: {out[name][mode]}")
    return out


STAGE_NAMES = ["end", "view_setup", "fill", "frustum_max", "fold", "classify", "project", "select_hist",
               "select_pick", "scan_reduce", "scan_partials", "compact", "radix_up", "radix_scan", "radix_down",
               "emit_reduce", "emit_partials", "emit_offsets", "emit", "ranges", "tile_count", "tile_scatter", "blend",
               "reduce_pairs", "long_mask"]


def server_timeline(torch, scene, synth, reps=12):
    """One job at a time through the resident serving kernel (1080p, 4K) at 3M Gaussians: the
    median time from each stage's opening to the next one's, against the same job launched
    stage by stage (events around ten back-to-back jobs on one stream)."""
    import ctypes
    from paper_2510_09997_amd import _clod as C
    from paper_2510_09997_amd.render import Batch
    n = scene.n
    cases = {"1920x1080": synth.look_at((4.0, 1.0, -9.0), width=1920, height=1080, s_v=1.0),
             "3840x2160": synth.look_at((2.0, 1.5, -7.0), width=3840, height=2160, s_v=1.7)}
    out = {}
    for name, view in cases.items():
        b = Batch(n, [view])
        for _ in range(3):
            b.project(scene); b.bin_sort(); b.render_fwd()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.project(scene); b.bin_sort(sync=False); b.render_fwd()
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"per_stage_launches_ms": round(e0.elapsed_time(e1) / 10, 4)}
        del b
    bufs = {}
    for name, view in cases.items():
        px = view.width * view.height
        vh = C.make_views([view])
        cb = C.clod_batch()
        ws = torch.empty(C.clod_ws_bytes(n, vh), dtype=torch.uint8, device="cuda")
        dup = torch.empty(C.clod_dup_bytes(16 * px + 65536), dtype=torch.uint8, device="cuda")
        o = (torch.empty(3 * px, device="cuda"), torch.empty(px, device="cuda"),
             torch.empty(px, dtype=torch.int32, device="cuda"))
        cb.n, cb.n_views, cb.views_host, cb.views_dev, cb.params = n, 1, ctypes.cast(vh, C.P), None, C.make_params()
        cb.ws, cb.ws_bytes, cb.dup, cb.dup_bytes = ws.data_ptr(), ws.numel(), dup.data_ptr(), dup.numel()
        bufs[name] = (vh, ws, dup, o, cb)
    torch.cuda.synchronize()
    srv, workers = C.clod_server_start(0, 60.0, torch.cuda.Stream())
    try:
        t0 = time.perf_counter()
        while C.clod_server_clock(srv) < 0:
            assert time.perf_counter() - t0 < 30.0, "serving kernel did not start"
            time.sleep(1e-4)
        for name in cases:
            _, _, _, o, cb = bufs[name]
            tot, per = [], {}
            for rep in range(reps):
                seq = C.clod_server_submit(srv, scene.c_struct(), cb, *o)
                t0 = time.perf_counter()
                while C.clod_server_poll(srv, seq) is None:
                    assert time.perf_counter() - t0 < 30.0, "serving job did not complete"
                tl = C.clod_server_stage_times(srv, seq)
                if rep < 2:
                    continue
                tot.append((tl[-1][1] - tl[0][1]) / 1e6)
                for j in range(len(tl) - 1):
                    per.setdefault(f"{j:02d}_{STAGE_NAMES[tl[j][0]]}", []).append((tl[j + 1][1] - tl[j][1]) / 1e3)
            out[name].update(persistent_job_ms=round(float(np.median(tot)), 4), workers=workers,
                             stage_us={k: round(float(np.median(v)), 1) for k, v in per.items()})
            log(f"[bench] persistent timeline {name}: job {np.median(tot):.3f} ms vs "
                f"{out[name]['per_stage_launches_ms']:.3f} ms launched stage by stage")
    finally:
        C.clod_server_stop(srv)
    torch.cuda.synchronize()
    return out


def cpu_info() -> dict:
    """Host CPU of the run: usable cores (affinity), logical CPUs and the model name."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count(), "model": model}


def cpu_baseline(timed_steps, poses=3):
    """The oracle (binary32 contract, OpenMP over tiles) on a bounded sample of the headline
    workload: the five LoD frames of each of the first three timed poses (about 10 s of CPU
    work); also the small parity scene (10,000 Gaussians, 256x256)."""
    from oracle import oracle as O
    from paper_2510_09997_amd import synth
    sc = synth.make_scene(3_000_000, 3, "mixture", seed=0)
    frames = [view for vs in timed_steps[:poses] for view in vs]
    t0 = time.perf_counter()
    for view in frames:
        O.render32(sc, view)
    dt = time.perf_counter() - t0
    svs = ", ".join(f"{v:g}" for v in SV_SWEEP)
    sc1 = synth.make_scene(10_000, 0, "uniform", seed=0)
    v1 = synth.look_at((0.0, 0.0, -3.0), width=256, height=256)
    t1 = []
    for _ in range(3):
        t = time.perf_counter()
        O.render32(sc1, v1)
        t1.append(time.perf_counter() - t)
    return dict(value=round(len(frames) / dt, 4), unit="frames/s", cores=O.num_threads(), kind="oracle",
                sample=f"{len(frames)} frames of 1920x1080 at 3M Gaussians (the first {poses} timed poses, s_v = "
                       f"{svs} each): {dt:.1f} s",
                small_scene_ms=round(1e3 * float(np.median(t1)), 3), cpu=cpu_info())


def cpu_suite(one_core: bool) -> dict:
    """The oracle on the parity configurations (median of three runs where cheap): the 10,000-
    Gaussian scene; one forward + backward of the 1M training configuration with the FP64
    gradient oracle; the LoD-sweep frames at 6M, k = 0, 21, 42, 63 (one core: k = 0 and 63, and
    the backward at 648x420, a quarter of the pixels, to stay within a few minutes)."""
    import torch
    from oracle import oracle as O
    from paper_2510_09997_amd import synth
    if one_core:
        torch.set_num_threads(1)
    out = {"threads": O.num_threads(), "torch_threads": torch.get_num_threads(), "cpu": cpu_info()}

    def timed(f, reps):
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    sc1 = synth.make_scene(10_000, 0, "uniform", seed=0)
    v1 = synth.look_at((0.0, 0.0, -3.0), width=256, height=256)
    out["c1_fwd_ms"] = round(1e3 * timed(lambda: O.render32(sc1, v1), 3), 3)
    log(f"[cpu] c1 forward {out['c1_fwd_ms']} ms")
    sc2 = synth.make_scene(1_000_000, 3, "mixture", seed=0)
    w, h = (648, 420) if one_core else (1297, 840)
    v2 = synth.look_at((1.5, 2.0, -4.5), width=w, height=h, s_v=2.0)
    out["c2_resolution"] = [w, h]
    out["c2_fwd_s"] = round(timed(lambda: O.render32(sc2, v2), 1 if one_core else 3), 3)
    log(f"[cpu] c2 forward {out['c2_fwd_s']} s")
    vp = O.render32(sc2, v2)
    g = np.random.default_rng(1).normal(size=(3, h, w))
    out["c2_bwd_fp64_s"] = round(timed(lambda: O.fp64_grads(sc2, v2, vp, g, 0.5), 1), 3)
    out["c2_fwd_bwd_s"] = round(out["c2_fwd_s"] + out["c2_bwd_fp64_s"], 3)
    log(f"[cpu] c2 FP64 backward {out['c2_bwd_fp64_s']} s")
    del sc2, vp, g
    sc4 = synth.make_scene(6_000_000, 3, "mixture", seed=0)
    ds = synth.sweep_distances(64, 2.0, 200.0)
    out["c4_frame_s"] = {}
    for k in ((0, 63) if one_core else (0, 21, 42, 63)):
        v = synth.look_at((0.0, 0.0, -float(ds[k])), width=1920, height=1080)
        out["c4_frame_s"][str(k)] = round(timed(lambda: O.render32(sc4, v), 1), 3)
        log(f"[cpu] c4 k={k} {out['c4_frame_s'][str(k)]} s")
    return out


# Algorithmic work of the blend: 18 flops per evaluated (pixel, entry) pair of the per-pixel
# loop (the contract's iteration count, counted exactly by the kernel and equal to the
# oracle's).  FP32 vector peak of MI355X: 256 CUs x 128 lanes x 2 flops x 2.4 GHz.
FLOPS_PER_PAIR = 18
FP32_VECTOR_PEAK_TFLOPS = 157.3
# HBM bytes per launch of the dominant kernel: rocprofv3 FETCH_SIZE and WRITE_SIZE over the 20
# timed launches (bench.py --profile timed-blend runs exactly those launches; the timed poses do
# not depend on the warm-up count), each scaled by the same counter's reading for a 1 GiB device
# copy (profiles/k_blend_fwd_serve1080p_3M_hbm.txt).  Emptied whenever the kernel changes.
TRAFFIC = {"k_blend_fwd": 944650690}


def probe_copy(torch):
    """One 1 GiB device-to-device copy: the reference reading for the HBM byte counters."""
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--train-steps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-multiview", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-budget", action="store_true", help="skip the primitive-budget sweep")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-request comparison path")
    ap.add_argument("--no-count", action="store_true", help="skip the untimed work-counting re-run")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run a 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--streams", type=int, default=3,
                    help="streams the headline serving steps are pipelined over (1 = sequential)")
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--serve-light-requests", type=int, default=1000)
    ap.add_argument("--serve-capacity-requests", type=int, default=600)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--profile", choices=("timed-blend", "multiview-eager", "train"), default=None,
                    help="run one part only (for rocprofv3): the headline's timed launches, the 16-view "
                         "step without the graph, or the 1M training iterations")
    ap.add_argument("--cpu-suite", choices=("all", "one"), default=None,
                    help="time the oracle on the parity configurations on all cores or one core, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.cpu_suite:
        if args.cpu_suite == "one":
            os.environ["OMP_NUM_THREADS"] = "1"   # before any OpenMP runtime starts
        print(json.dumps({"cpu_suite": args.cpu_suite, **cpu_suite(args.cpu_suite == "one")}), flush=True)
        return
    import torch
    from paper_2510_09997_amd import _clod as C, synth
    from paper_2510_09997_amd.render import Batch, Scene
    C.load()
    assert torch.cuda.is_available()
    if args.profile == "multiview-eager":
        res = run_multiview_train(args, torch, C, Scene, synth)
        if args.probe_copy:
            probe_copy(torch)
        print(json.dumps({"profile": args.profile, **res}), flush=True)
        return
    if args.profile == "train":
        print(json.dumps({"profile": args.profile, **run_train(args, torch, C, Batch, Scene, synth)}), flush=True)
        return
    serve, scene, b, steps = run_serving(args, torch, C, Batch, Scene, synth)
    if args.profile == "timed-blend":
        if args.probe_copy:
            probe_copy(torch)
        print(json.dumps(serve), flush=True)
        return
    log(f"[bench] serving: {serve['fps']:.1f} frames/s batched, {serve.get('plain_fps', float('nan')):.1f} plain; "
        f"stages {serve['stage_ms']}")
    budget = None
    if not args.no_budget:
        budget = run_budget_sweep(args, torch, C, Batch, scene, steps[min(10, len(steps) - 1)][0])
        log(f"[bench] budget sweep fps: {dict(zip(budget['budgets'], budget['fps']))}")
    strips = None
    if not args.no_budget:
        strips = run_strips(args, torch, C, Batch, scene, steps[min(10, len(steps) - 1)][0], synth)
        log(f"[bench] strips: {strips}")
    del scene, b
    torch.cuda.empty_cache()
    train = None
    if not args.no_train:
        train = run_train(args, torch, C, Batch, Scene, synth)
        log(f"[bench] train: {train['ms_per_iter']:.2f} ms/iter")
    # Roofline of the dominant kernel of the headline workload (the forward blend, one launch
    # per step, timed with events around its own launch on the stream it runs on).
    blend_ms = serve["stage_ms"]["blend_fwd"]
    e, x, bl = serve["pairs_per_step"] or (float("nan"),) * 3
    flops = FLOPS_PER_PAIR * e
    achieved = flops / (blend_ms * 1e-3) / 1e12
    # Bytes the blend must move per launch: 40 B per tile pair (record fields and sorted index),
    # 8 B per tile range, 20 B per pixel of output (colour, T, last index).
    alg_bytes = None
    if serve["dup_per_step"] is not None:
        alg_bytes = int(40 * serve["dup_per_step"] + 8 * 5 * 8160 + 20 * serve["pixels_per_step"])
    out = {
        "metric": "1080p frames/s at 3M Gaussians across LoD distances; fwd+bwd ms/iter; p99 ms",
        "value": round(serve["fps"], 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(serve["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 64-cluster mixture scenes; random poses)",
        "config": {"workload": "serve-1080p-3M-lod-sweep", "gaussians": 3_000_000, "sh_degree": 3,
                   "resolution": [1920, 1080], "s_v": list(SV_SWEEP), "frames_per_step": len(SV_SWEEP),
                   "pose_radius": [3.0, 30.0], "streams": serve["streams"]},
        "pipelined_matches_sequential": serve["pipelined_identical"],
        "sequential_fps": round(serve["sequential_fps"], 2),
        "plain_path_fps": round(serve["plain_fps"], 2) if "plain_fps" in serve else None,
        "stage_ms": {k: round(v, 4) for k, v in serve["stage_ms"].items()},
        "pairs_per_step": {"evaluated": e, "exp_evaluated": x, "blended": bl},
        "roofline": {"kernel": "k_blend_fwd", "bound": "alu",
                     "achieved": None if math.isnan(achieved) else round(achieved, 3),
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": None if math.isnan(achieved) else round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": TRAFFIC.get("k_blend_fwd"),
                     "algorithmic_bytes": alg_bytes,
                     "avg_launch_ms": round(blend_ms, 4)},
        "dup_per_step": serve["dup_per_step"],
        "rendered_per_step": serve.get("rendered_per_step"),
        "hbm_served_step": serve.get("hbm"),
    }
    if train is not None:
        out["fwd_bwd_ms_per_iter"] = round(train["ms_per_iter"], 3)
        out["fwd_bwd_p50_ms"] = round(train["p50_ms"], 3)
        out["fwd_bwd_p99_ms"] = round(train["p99_ms"], 3)
        out["train_config"] = {"gaussians": 1_000_000, "sh_degree": 3, "resolution": [1297, 840],
                               "s_v": "log-uniform [1, 8]", "loss": "L1 + point-count regulariser"}
        out["train_work"] = {k: train[k] for k in ("bwd_ms", "rendered", "pairs", "pixels", "fwd_pairs", "bwd_pairs",
                                                   "hbm", "bwd_alu")}
    if budget is not None:
        out["budget_sweep"] = budget
    if strips is not None:
        out["spatial_sv_strips"] = strips
    if not args.no_multiview:
        torch.cuda.empty_cache()
        mv = run_multiview_train(args, torch, C, Scene, synth)
        log(f"[bench] 16-view train step: {mv['ms_per_step']:.2f} ms")
        out["multiview_train"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in mv.items()}
    if not args.no_sweep:
        torch.cuda.empty_cache()
        sw = run_lod_sweep(args, torch, C, Batch, Scene, synth)
        log(f"[bench] LoD sweep fps (k=0,21,42,63): {[sw['ray_fps'][k] for k in (0, 21, 42, 63)]}")
        out["lod_sweep"] = sw
    if args.probe_copy:
        probe_copy(torch)
    if not args.no_serve:
        torch.cuda.empty_cache()
        st = run_serve_stream(args, torch, Scene, synth)
        out["serve_stream"] = {"resolutions": ["1280x720", "1920x1080", "3840x2160"], "s_v": "log-uniform [1, 16]",
                               "gaussians": 3_000_000, **st}
        out["p99_ms"] = st["light"]["continuous"]["p99_ms"]
        out["p50_ms"] = st["light"]["continuous"]["p50_ms"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(steps[len(steps) - args.steps:])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
