"""Continuous-batching render server over a device-resident scene.

Requests (pose, resolution, virtual distance scale s_v) arrive over time.  The scheduler
admits arrived requests in FIFO order into the next batch while an HBM budget and a slot
limit allow, and launches each batch as one batched pass of the render path (one launch per
stage covering every request of the batch, whatever their resolutions and LoD scales) on one
of several streams, so a batch admitted while earlier ones are still on the GPU overlaps them
on the device.  Memory of a batch returns to the budget when its completion event fires.

The plain path serves one request per forward render, in arrival order.

The persistent path hands each admitted batch to the resident serving kernel of libclod
(clod_server_*): no kernel launches per batch, and the stages of successive batches overlap
inside the one kernel.  Its device memory is one arena carved per batch on the host, so nothing
is allocated while the kernel runs.

The scheduling core (``Scheduler``) is independent of the GPU: ``GpuExecutor`` runs batches
through libclod; tests drive the same core with a CPU stand-in executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class RequestRecord:
    rid: int
    arrival_s: float
    width: int
    height: int
    s_v: float
    admitted_s: float = float("nan")
    done_s: float = float("nan")
    batch: int = -1


class Scheduler:
    """FIFO admission under an HBM budget and a per-batch slot limit.

    ``cost(req)`` gives a request's device bytes while it is in flight.  A batch is launched
    when at least one request has arrived and it fits; a request that does not fit waits (it
    is never dropped) until in-flight batches complete and release their bytes.
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 8, max_inflight: int = 3):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.in_use = 0
        self.peak_in_use = 0
        self.batches = 0

    def run(self, requests, clock=time.perf_counter, sleep=time.sleep, poll_s: float = 50e-6):
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        recs = {r.rid: RequestRecord(r.rid, r.arrival_s, r.view.width, r.view.height, r.view.s_v) for r in reqs}
        for r in reqs:
            c = self.ex.cost(r)
            if c > self.budget:
                raise ValueError(f"request {r.rid} needs {c} bytes, more than the whole budget {self.budget}")
        pending = collections.deque(reqs)
        inflight = collections.deque()          # (handle, [requests], bytes)
        if hasattr(self.ex, "prepare"):
            self.ex.prepare(reqs, self.max_batch, self.budget)
        # The executor's time origin precedes the host origin (completion times are measured
        # from it), so latencies are never understated.
        self.ex.start()
        t0 = clock()
        while pending or inflight:
            now = clock() - t0
            # Retire completed batches (in launch order per stream is not required).
            for item in list(inflight):
                h, rs, nbytes = item
                done_at = self.ex.poll(h)
                if done_at is not None:
                    inflight.remove(item)
                    self.in_use -= nbytes
                    for r in rs:
                        recs[r.rid].done_s = done_at
            # Admit arrived requests into one batch.
            if pending and pending[0].arrival_s <= now and len(inflight) < self.max_inflight:
                batch, nbytes = [], 0
                while (pending and pending[0].arrival_s <= now and len(batch) < self.max_batch
                       and self.in_use + nbytes + self.ex.cost(pending[0]) <= self.budget):
                    r = pending.popleft()
                    batch.append(r)
                    nbytes += self.ex.cost(r)
                if batch:
                    self.in_use += nbytes
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    assert self.in_use <= self.budget
                    h = self.ex.launch(batch)
                    for r in batch:
                        recs[r.rid].admitted_s = now
                        recs[r.rid].batch = self.batches
                    self.batches += 1
                    inflight.append((h, batch, nbytes))
                    continue
            # Nothing to launch: wait for the next arrival or a completion.
            if not inflight and pending:
                wait = pending[0].arrival_s - (clock() - t0)
                if wait > 0:
                    sleep(min(wait, 1e-3))
            else:
                sleep(poll_s)
        self.ex.finish()
        return [recs[r.rid] for r in reqs]


def summarize(records, first: int = 0) -> dict:
    rs = records[first:]
    lat = np.array([(r.done_s - r.arrival_s) * 1e3 for r in rs])
    span = max(r.done_s for r in rs) - min(r.arrival_s for r in rs)
    return dict(requests=len(rs), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()), frames_per_s=len(rs) / span,
                megapixels_per_s=sum(r.width * r.height for r in rs) / span / 1e6)


class GpuExecutor:
    """Renders a batch of requests as one batched pass (clod_project, clod_bin_sort,
    clod_render_fwd) on a rotating set of streams, with per-stream reusable workspaces."""

    def __init__(self, scene, params=None, streams: int = 3, dup_per_pixel: float = 12.0,
                 keep_outputs: bool = False):
        import torch
        from . import _clod as C
        self.torch, self.C = torch, C
        self.scene = scene
        self.params = params if params is not None else C.make_params()
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.next = 0
        self.dup_per_pixel = dup_per_pixel
        self.keep = keep_outputs
        self.outputs = {}
        self.ws = [None] * streams
        self.dup = [None] * streams
        self.retries = 0
        self.t0_event = None

    # Device bytes of one request while in flight: per-(view, Gaussian) workspace (flags,
    # alpha'', depth, 64-byte record, rectangle, tiles touched, backward partials), outputs
    # and an estimate of its tile pairs (16 bytes each).
    def cost(self, req) -> int:
        n = self.scene.n
        px = req.view.width * req.view.height
        return int(n * 121 + px * (20 + 12) + 16 * self.dup_per_pixel * px)

    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.streams[0])
        self.t0_event.synchronize()

    def _buffers(self, slot, ws_bytes, dup_cap):
        # Called inside the slot's stream context: the caching allocator ties the blocks to
        # that stream, and every batch holding them keeps a reference until it is retired.
        torch, C = self.torch, self.C
        if self.ws[slot] is None or self.ws[slot].numel() < ws_bytes:
            self.ws[slot] = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        nb = C.clod_dup_bytes(dup_cap)
        if self.dup[slot] is None or self.dup[slot].numel() < nb:
            self.dup[slot] = torch.empty(nb, dtype=torch.uint8, device="cuda")
        return self.ws[slot], self.dup[slot]

    def _batch_struct(self, views_host, views_dev, ws, dup):
        C = self.C
        b = C.clod_batch()
        b.n = self.scene.n
        b.n_views = len(views_host)
        b.views_host = C.ctypes.cast(views_host, C.P)
        b.views_dev = views_dev.data_ptr()
        b.params = self.params
        b.ws = ws.data_ptr()
        b.ws_bytes = ws.numel()
        b.dup = dup.data_ptr()
        b.dup_bytes = dup.numel()
        return b

    def launch(self, batch):
        torch, C = self.torch, self.C
        slot = self.next
        self.next = (self.next + 1) % len(self.streams)
        st = self.streams[slot]
        views = [r.view for r in batch]
        vh = C.make_views(views)
        pixels = sum(v.width * v.height for v in views)
        # A slot's workspaces are reused by its next batch, which is ordered after this one on
        # the same stream.
        with torch.cuda.stream(st):
            ws, dup = self._buffers(slot, C.clod_ws_bytes(self.scene.n, vh), int(self.dup_per_pixel * pixels) + 65536)
            vd = C.views_to_device(vh, "cuda")
            rgb = torch.empty(3 * pixels, device="cuda", dtype=torch.float32)
            T = torch.empty(pixels, device="cuda", dtype=torch.float32)
            last = torch.empty(pixels, dtype=torch.int32, device="cuda")
            bs = self._batch_struct(vh, vd, ws, dup)
            C.clod_project(self.scene.c_struct(), bs, None, st)
            C.clod_bin_sort(bs, False, st)
            C.clod_render_fwd(bs, rgb, T, last, None, st)
            hdr = self._header_copy(bs, ws, st)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
        return dict(ev=ev, batch=batch, slot=slot, vh=vh, vd=vd, out=(rgb, T, last), bs=bs, stream=st,
                    ws=ws, dup=dup, hdr=hdr)

    def _header_copy(self, bs, ws, st):
        # Asynchronous copy of {D, overflow} to pinned host memory, read once the event fires.
        torch, C = self.torch, self.C
        ptr, _ = C.clod_inspect(bs, C.SEC_HEADER)
        off = ptr - ws.data_ptr()
        hdr = torch.empty(16, dtype=torch.uint8, pin_memory=True)
        hdr.copy_(ws[off:off + 16], non_blocking=True)
        return hdr

    def poll(self, h):
        if not h["ev"].query():
            return None
        C = self.C
        n_dup, overflow = (int(x) for x in h["hdr"].view(self.torch.int64).tolist())
        if overflow:
            # Grow this slot's duplicate buffer and re-run the batch (rare; counted).  The
            # batch gets a workspace of its own: later batches may already use the slot's.
            self.retries += 1
            torch = self.torch
            st = h["stream"]
            with torch.cuda.stream(st):
                ws = torch.empty(h["ws"].numel(), dtype=torch.uint8, device="cuda")
                dup = torch.empty(C.clod_dup_bytes(int(n_dup * 1.25) + 65536), dtype=torch.uint8, device="cuda")
                self.dup[h["slot"]] = dup
                bs = self._batch_struct(h["vh"], h["vd"], ws, dup)
                C.clod_project(self.scene.c_struct(), bs, None, st)
                C.clod_bin_sort(bs, False, st)
                C.clod_render_fwd(bs, *h["out"], None, st)
                h["hdr"] = self._header_copy(bs, ws, st)
                h["ev"].record(st)
            h.update(bs=bs, ws=ws, dup=dup)
            return None
        done = self.t0_event.elapsed_time(h["ev"]) / 1e3
        if self.keep:
            # Copies on the stream that owns the outputs (ordered before any reuse of their
            # memory by the slot's next batch), finished before the handle is dropped.
            rgb, T, last = h["out"]
            off = 0
            with self.torch.cuda.stream(h["stream"]):
                for r in h["batch"]:
                    px = r.view.width * r.view.height
                    self.outputs[r.rid] = (rgb[3 * off:3 * (off + px)].clone(), T[off:off + px].clone(),
                                           last[off:off + px].clone())
                    off += px
            h["stream"].synchronize()
        return done

    def finish(self):
        self.torch.cuda.synchronize()


class Arena:
    """First-fit sub-allocation of one device buffer (256-byte aligned blocks)."""

    def __init__(self, nbytes: int):
        self.size = int(nbytes)
        self.free = [(0, self.size)]   # sorted, coalesced (offset, size)

    def alloc(self, nbytes: int) -> int | None:
        need = (int(nbytes) + 255) & ~255
        for j, (off, sz) in enumerate(self.free):
            if sz >= need:
                if sz == need:
                    del self.free[j]
                else:
                    self.free[j] = (off + need, sz - need)
                return off
        return None

    def release(self, off: int, nbytes: int):
        need = (int(nbytes) + 255) & ~255
        blocks = sorted(self.free + [(off, need)])
        merged = []
        for o, z in blocks:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + z)
            else:
                merged.append((o, z))
        self.free = merged


def _out_bytes(pixels: int) -> int:
    a = lambda x: (x + 255) & ~255
    return a(12 * pixels) + a(4 * pixels) + a(4 * pixels)


def _out_views(mem, off: int, pixels: int, torch):
    """rgb (float32 [3 pixels]), T (float32), last (int32) carved from a uint8 device buffer."""
    a = lambda x: (x + 255) & ~255
    o_t, o_l = off + a(12 * pixels), off + a(12 * pixels) + a(4 * pixels)
    return (mem[off:off + 12 * pixels].view(torch.float32), mem[o_t:o_t + 4 * pixels].view(torch.float32),
            mem[o_l:o_l + 4 * pixels].view(torch.int32))


class PersistentExecutor:
    """Serves batches through the resident serving kernel (clod_server_*).

    ``prepare`` allocates, before the kernel starts, one device arena for the workspaces,
    duplicate buffers and outputs of the batches in flight (the admission budget plus one
    largest batch of slack), and with ``keep_outputs`` one output set per request; batches
    then take and return arena blocks on the host only."""

    def __init__(self, scene, params=None, dup_per_pixel: float = 12.0, keep_outputs: bool = False,
                 workers: int = 0, max_seconds: float = 120.0):
        import torch
        from . import _clod as C
        if scene.sh_packed is None:
            raise ValueError("the persistent server reads packed SH coefficients: build the Scene with packed_sh=True")
        self.torch, self.C = torch, C
        self.scene = scene
        self.params = params if params is not None else C.make_params()
        self.dup_per_pixel = dup_per_pixel
        self.keep = keep_outputs
        self.workers_req = workers
        self.max_seconds = max_seconds
        self.outputs = {}
        self.retries = 0
        self.server = None
        self.workers = 0
        self.arena = None
        self.mem = None
        self.req_out = {}
        self.stream = torch.cuda.Stream()
        self.origin_ns = 0

    def cost(self, req) -> int:
        n = self.scene.n
        px = req.view.width * req.view.height
        return int(n * 121 + px * (20 + 12) + 16 * self.dup_per_pixel * px)

    def _batch_bytes(self, views, pixels):
        C = self.C
        vh = C.make_views(views)
        ws = C.clod_ws_bytes(self.scene.n, vh)
        dup = C.clod_dup_bytes(int(self.dup_per_pixel * pixels) + 65536)
        out = _out_bytes(pixels)
        return vh, ws, dup, out

    def prepare(self, requests, max_batch: int, budget: int):
        torch = self.torch
        big = sorted(requests, key=lambda r: r.view.width * r.view.height)[-max_batch:]
        _, ws, dup, out = self._batch_bytes([r.view for r in big], sum(r.view.width * r.view.height for r in big))
        total = int(budget) + ws + dup + out
        self.arena = Arena(total)
        self.mem = torch.empty(total, dtype=torch.uint8, device="cuda")
        if self.keep:
            for r in requests:
                px = r.view.width * r.view.height
                self.req_out[r.rid] = (torch.empty(3 * px, dtype=torch.float32, device="cuda"),
                                       torch.empty(px, dtype=torch.float32, device="cuda"),
                                       torch.empty(px, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()

    def start(self):
        import time
        C = self.C
        self.server, self.workers = C.clod_server_start(self.workers_req, self.max_seconds, self.stream)
        t0 = time.perf_counter()
        while C.clod_server_clock(self.server) < 0:
            if time.perf_counter() - t0 > 30.0:
                raise RuntimeError("the serving kernel did not start within 30 s")
            time.sleep(1e-4)
        self.origin_ns = C.clod_server_clock(self.server)

    def _take(self, nbytes):
        off = self.arena.alloc(nbytes)
        if off is None:
            raise RuntimeError(f"serving arena exhausted ({nbytes} bytes requested)")
        return off

    def _submit(self, h):
        C = self.C
        b = C.clod_batch()
        b.n = self.scene.n
        b.n_views = len(h["vh"])
        b.views_host = C.ctypes.cast(h["vh"], C.P)
        b.views_dev = None
        b.params = self.params
        base = self.mem.data_ptr()
        b.ws, b.ws_bytes = base + h["blocks"]["ws"][0], h["blocks"]["ws"][1]
        b.dup, b.dup_bytes = base + h["blocks"]["dup"][0], h["blocks"]["dup"][1]
        rgb, T, last = h["out"]
        h["seq"] = C.clod_server_submit(self.server, self.scene.c_struct(), b, rgb, T, last)

    def launch(self, batch):
        views = [r.view for r in batch]
        pixels = sum(v.width * v.height for v in views)
        vh, ws, dup, out = self._batch_bytes(views, pixels)
        blocks = {"ws": (self._take(ws), ws), "dup": (self._take(dup), dup)}
        if self.keep and len(batch) == 1:
            outs = self.req_out[batch[0].rid]   # rendered in place
        else:
            # A batch renders into one output set (requests back to back); with keep_outputs the
            # requests' parts are copied out at completion.
            blocks["out"] = (self._take(out), out)
            outs = _out_views(self.mem, blocks["out"][0], pixels, self.torch)
        h = dict(batch=batch, vh=vh, blocks=blocks, out=outs, pixels=pixels)
        self._submit(h)
        return h

    def poll(self, h):
        C = self.C
        info = C.clod_server_poll(self.server, h["seq"])
        if info is None:
            return None
        if info["overflow"]:
            # Larger duplicate buffer from the arena, then the same job again.
            self.retries += 1
            off, nb = h["blocks"]["dup"]
            self.arena.release(off, nb)
            nb = C.clod_dup_bytes(int(info["n_dup"] * 1.25) + 65536)
            h["blocks"]["dup"] = (self._take(nb), nb)
            self._submit(h)
            return None
        if self.keep and "out" in h["blocks"]:
            # Device-to-device copies into each request's own outputs (after completion).
            rgb, T, last = h["out"]
            off = 0
            with self.torch.cuda.stream(self.stream_copy()):
                for r in h["batch"]:
                    px = r.view.width * r.view.height
                    d = self.req_out[r.rid]
                    d[0].copy_(rgb[3 * off:3 * (off + px)], non_blocking=True)
                    d[1].copy_(T[off:off + px], non_blocking=True)
                    d[2].copy_(last[off:off + px], non_blocking=True)
                    off += px
            self._copy_stream.synchronize()
        if self.keep:
            for r in h["batch"]:
                self.outputs[r.rid] = self.req_out[r.rid]
        for off, nb in h["blocks"].values():
            self.arena.release(off, nb)
        return (info["t_ns"] - self.origin_ns) / 1e9

    def stream_copy(self):
        if not hasattr(self, "_copy_stream"):
            self._copy_stream = self.torch.cuda.Stream()
        return self._copy_stream

    def finish(self):
        if self.server is not None:
            status = self.C.clod_server_stop(self.server)
            self.server = None
            if status != 1:
                raise RuntimeError(f"serving kernel ended with status {status}")
        self.torch.cuda.synchronize()


class PlainExecutor(GpuExecutor):
    """The plain path: one request per forward render, on one stream, in arrival order."""

    def __init__(self, scene, params=None, dup_per_pixel: float = 12.0, keep_outputs: bool = False):
        super().__init__(scene, params, streams=1, dup_per_pixel=dup_per_pixel, keep_outputs=keep_outputs)


def serve(scene, requests, mode: str = "continuous", budget_bytes: int = 24 << 30, max_batch: int = 8,
          max_inflight: int = 3, params=None, keep_outputs: bool = False):
    """Serves ``requests`` (synth.Request) in real time; returns (records, executor)."""
    if mode == "continuous":
        ex = GpuExecutor(scene, params, streams=max_inflight, keep_outputs=keep_outputs)
        sch = Scheduler(ex, budget_bytes, max_batch=max_batch, max_inflight=max_inflight)
    elif mode == "plain":
        ex = PlainExecutor(scene, params, keep_outputs=keep_outputs)
        sch = Scheduler(ex, budget_bytes, max_batch=1, max_inflight=1)
    elif mode == "persistent":
        ex = PersistentExecutor(scene, params, keep_outputs=keep_outputs)
        sch = Scheduler(ex, budget_bytes, max_batch=max_batch, max_inflight=max_inflight)
    else:
        raise ValueError(mode)
    try:
        recs = sch.run(requests)
    finally:
        if mode == "persistent" and ex.server is not None:
            ex.finish()
    return recs, ex, sch
