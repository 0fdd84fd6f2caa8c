"""Continuous-batching render server for a resident scene.

Requests (a camera of any size) arrive at any time.  A scheduler thread
admits queued requests into a batch while the batch has fewer than
`max_batch` views and the estimated device memory of everything in flight
stays within `mem_budget`; it launches the batch as ONE sss_project +
sss_bin_sort + sss_render_fwd sequence over all its views, on the next of
`n_streams` streams, and goes on admitting: the next batch's projection and
sort run on another stream while the previous batch still rasterizes.  A
completion thread waits for each batch's event, hands every request its
image (a [H, W, 3] device tensor) and releases the batch's memory, which lets
the scheduler admit more.  A request that arrives while nothing is queued or
in flight is launched at once by the submitting thread (a batch of one),
without a hand-over to the scheduler.

Nothing on the launch path waits for the device: the bin sort's kernels
read its counts on the device and write them straight into the stream's
pinned host buffer.  The completion thread checks them after the batch's
event; a batch whose pair lists outgrew its stream's capacity is rendered
again with a larger one before its results are handed out (the capacity
only grows, and `warmup` sizes it up front).  A resolved future keeps its
request (`future.request`: submit and completion times, pixels), but the
request no longer refers to the future, so an image is freed as soon as the
caller drops the future.

Each view is rendered independently inside a batch (its own tiles, ranks
ordered by depth within the view), so a request's image is bit-identical
alone and in any mix.

Streams: a request's image is complete when its future resolves.  It may be
read on the server's consumer stream (by default the stream that was
current when the server was created, normally the default stream) with no
further synchronisation: the server records that stream on the image's
memory, so the memory is not reused by a later batch before the consumer
stream's work queued up to the image's release has run.  To read an image
on any other stream, call `image.record_stream(that_stream)` first.

`PlainRenderer` is the baseline: one request per launch sequence, FIFO, one
stream, same kernels.
"""
from __future__ import annotations

import collections
import functools
import math
import threading
import time
from concurrent.futures import Future

import torch

from . import sss

_REC = sss.RECORD_BYTES


class _Req:
    __slots__ = ("cam", "t_submit", "future", "pixels", "t_done")

    def __init__(self, cam):
        self.cam = cam
        self.t_submit = time.perf_counter()
        self.future = Future()
        self.future.request = self
        self.pixels = int(cam["width"]) * int(cam["height"])
        self.t_done = None


class _Slot:
    """Per-stream scratch buffers that only grow (projection outputs, bins,
    the pair list and sort workspace, per-pixel side outputs), reused by every
    batch launched on the stream; images handed to callers are allocated per
    batch."""

    def __init__(self):
        self.binner = sss.BinSorter(0, no_wait=True)
        self.buf = {}
        self.views = {}
        self.host_counts = None
        self.host_np = None          # numpy view of host_counts
        self.event = None

    def take(self, name, shape, dtype, device):
        v = self.views.get((name, shape))
        if v is not None:
            return v
        numel = int(math.prod(shape))
        b = self.buf.get(name)
        if b is None or b.numel() < numel:
            # grow with headroom, so a run of slightly larger batches does
            # not allocate every time; views of the old buffer are dropped
            grown = numel if b is None else max(numel, b.numel() + b.numel() // 4)
            b = torch.empty(max(grown, 1), dtype=dtype, device=device)
            self.buf[name] = b
            self.views = {k: t for k, t in self.views.items() if k[0] != name}
        v = b[:numel].view(shape)
        if len(self.views) < 256:
            self.views[(name, shape)] = v
        return v


class RenderServer:
    def __init__(self, scene: dict, opts=None, max_batch: int = 16, mem_budget: int = 6 << 30,
                 n_streams: int = 2, pairs_per_pixel: float = 20.0, device: int = 0, max_inflight: int | None = None,
                 consumer_stream=None):
        """scene: dict of device tensors (see sss.scene_struct).  At most
        `max_inflight` batches (default and at most: n_streams) are on the device at once;
        requests arriving meanwhile wait and join the next batch.
        consumer_stream: the stream results are read on (default: the
        current stream of `device` at construction)."""
        if not 1 <= max_batch <= sss.MAX_VIEWS:
            raise ValueError(f"max_batch must be in 1..{sss.MAX_VIEWS}")
        self.scene = scene
        self.n = scene["means"].shape[0]
        self.opts = sss.render_opts(opts)                 # marshalled once for every launch
        self.max_batch = max_batch
        # a stream's scratch buffers serve one batch at a time
        self.max_inflight = n_streams if max_inflight is None else max(1, min(int(max_inflight), n_streams))
        self.mem_budget = int(mem_budget)
        self.device = device
        self.consumer = consumer_stream if consumer_stream is not None else torch.cuda.current_stream(device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self._slots = [_Slot() for _ in range(n_streams)]
        self.pairs_per_pixel = float(pairs_per_pixel)   # running estimate, refined from every batch
        self.pairs_per_pixel_max = float(pairs_per_pixel)  # largest ratio seen: sizes the pair passes
        self._ws_cache = {}
        self._q = collections.deque()
        # one lock; the scheduler waits for queued requests (or room to
        # launch) on _cv_sched, the completion thread for batches in flight
        # on _cv_done, so a launch wakes only the thread that has work
        self._lock = threading.Lock()
        self._cv_sched = threading.Condition(self._lock)
        self._cv_done = threading.Condition(self._lock)
        self._inflight = collections.deque()           # (event, reqs, bytes, keepalive, stream index)
        self._mem_used = 0
        self._launching = 0                            # batches popped but not yet in flight
        self._next_stream = 0
        self._running = True
        self.batches = 0
        self.batch_sizes = []
        self._sched = threading.Thread(target=self._schedule, name="sss-sched", daemon=True)
        self._done = threading.Thread(target=self._complete, name="sss-done", daemon=True)
        self._sched.start()
        self._done.start()

    # ---------------------------------------------------------------- public
    def submit(self, cam) -> Future:
        r = _Req(cam)
        fut = r.future            # r drops it on completion, which may come before this returns
        need = self._estimate([r])
        if need > self.mem_budget:
            r.future = None
            fut.set_exception(MemoryError(f"request of {r.pixels} pixels exceeds the memory budget"))
            return fut
        with self._lock:
            if not self._running:
                raise RuntimeError("server closed")
            direct = (not self._q and not self._inflight and self._launching == 0
                      and self._mem_used + need <= self.mem_budget)
            if not direct:
                self._q.append(r)
                self._cv_sched.notify()
                return fut
            self._mem_used += need
            self._launching += 1
            k = self._take_stream()
        # the device is idle: launch from this thread, like a plain renderer
        self._run_batch([r], need, k)
        return fut

    def warmup(self, cams, fill_budget: bool = False):
        """Render the batch `cams` once on every stream before requests arrive,
        so each stream's scratch buffers and pair capacity are sized for it;
        later batches up to that size allocate nothing.  fill_budget: repeat
        the largest of `cams` up to the biggest batch the memory budget and
        max_batch admit, so no admissible batch grows a buffer later."""
        cams = list(cams)
        if fill_budget and cams:
            big = max(cams, key=lambda c: int(c["width"]) * int(c["height"]))
            batch = []
            while len(batch) < self.max_batch and self._estimate([_Req(c) for c in batch + [big]]) <= self.mem_budget:
                batch.append(big)
            cams = batch or [big]
        for stream, slot in zip(self.streams, self._slots):
            reqs = [_Req(c) for c in cams]
            keep, ev = self._launch(reqs, stream, slot)
            ev.synchronize()
            P = sum(r.pixels for r in reqs)
            if P > 0:
                self.pairs_per_pixel_max = max(self.pairs_per_pixel_max, int(keep[3][1]) / P)
            if int(keep[3][1]) > keep[1].cap():
                slot.binner.grow(int(keep[3][1]))
                keep, ev = self._launch(reqs, stream, slot)
                ev.synchronize()

    def close(self):
        with self._lock:
            self._running = False
            self._cv_sched.notify_all()
            self._cv_done.notify_all()
        self._sched.join()
        self._done.join()

    # ------------------------------------------------------------- internals
    def _estimate(self, reqs) -> int:
        """Device bytes of one batch: per-view projection + bins, the image,
        and the pair list + sort buffers from the pair estimate."""
        V = len(reqs)
        P = sum(r.pixels for r in reqs)
        E = V * self.n
        M = int(P * self.pairs_per_pixel * 1.25) + 1024
        M = ((M + (1 << 20) - 1) >> 20) << 20       # whole Mi-pairs: the workspace size cache hits
        per_entry = sss.ENTRY_BYTES + 4 + 4 + 4 + _REC
        key = (E, M)
        ws = self._ws_cache.get(key)
        if ws is None:
            ws = int(sss.lib().sss_bin_sort_workspace(E, M))
            if len(self._ws_cache) < 4096:
                self._ws_cache[key] = ws
        return E * per_entry + P * 12 + 4 * M + ws

    def _schedule(self):
        torch.cuda.set_device(self.device)
        while True:
            with self._lock:
                while self._running and not self._q:
                    self._cv_sched.wait()
                if not self._running and not self._q:
                    return
                if len(self._inflight) + self._launching >= self.max_inflight:
                    self._cv_sched.wait(timeout=0.05)        # let requests gather for the next batch
                    continue
                batch = []
                while self._q and len(batch) < self.max_batch:
                    cand = batch + [self._q[0]]
                    need = self._estimate(cand)
                    if self._mem_used + need > self.mem_budget and (batch or self._inflight):
                        break
                    batch.append(self._q.popleft())
                if not batch:                                   # memory full: wait for a completion
                    self._cv_sched.wait(timeout=0.05)
                    continue
                need = self._estimate(batch)
                self._mem_used += need
                self._launching += 1
                k = self._take_stream()
            self._run_batch(batch, need, k)

    def _take_stream(self) -> int:
        """Next stream index, round robin (called with the lock held)."""
        k = self._next_stream
        self._next_stream = (k + 1) % len(self.streams)
        return k

    def _run_batch(self, batch, need, k):
        """Launch a popped batch on stream k and put it in flight."""
        stream, slot = self.streams[k], self._slots[k]
        try:
            keep, ev = self._launch(batch, stream, slot)
        except Exception as exc:                            # pragma: no cover - surfaced to callers
            for r in batch:
                fut, r.future = r.future, None
                fut.set_exception(exc)
            with self._lock:
                self._mem_used -= need
                self._launching -= 1
                self._cv_sched.notify()
                self._cv_done.notify()
            return
        with self._lock:
            self._inflight.append((ev, batch, need, keep, k))
            self._launching -= 1
            self.batches += 1
            self.batch_sizes.append(len(batch))
            self._cv_done.notify()

    def _launch(self, batch, stream, slot):
        cams = sss.CameraBatch([r.cam for r in batch])     # marshalled once for the three calls
        dev = self.scene["means"].device
        E = len(cams) * self.n
        P = cams.n_pixels
        T = cams.n_tiles
        with torch.cuda.stream(stream):
            proj = sss.Projected(slot.take("entries", (E, sss.ENTRY_BYTES), torch.uint8, dev),
                                 slot.take("key", (E,), torch.int32, dev),
                                 slot.take("touched", (E,), torch.int32, dev))
            sss.project(self.scene, cams, self.opts, stream=stream, out=proj)
            out = sss.Binned(slot.take("order", (E,), torch.int32, dev),
                             slot.take("sorted", (E, sss.RECORD_BYTES), torch.uint8, dev),
                             slot.take("tile_start", (T + 1,), torch.int32, dev), None,
                             tile_order=slot.take("tile_order", (T,), torch.int32, dev))
            # the counts go straight to pinned host memory, written by the
            # sort's kernel and read after the batch's event (one buffer per
            # stream: a stream has one batch in flight)
            if slot.host_counts is None:
                slot.host_counts = torch.empty(2, dtype=torch.int64, pin_memory=True)
                slot.host_np = slot.host_counts.numpy()
            host_counts = slot.host_counts
            # the pair passes are sized by an estimate from the pairs per
            # pixel seen so far (a batch that needs more is rendered again)
            hint = int(self.pairs_per_pixel_max * 1.5 * P) + 8192
            bins = slot.binner(proj, cams, self.n, stream=stream, out=out, counts=host_counts, capacity=hint)
            image, _, _ = sss.render_fwd(bins, cams, self.opts, stream=stream, aux=False)
            # one event per stream: a stream has one batch in flight
            if slot.event is None:
                slot.event = torch.cuda.Event()
            ev = slot.event
            ev.record(stream)
        return (proj, bins, image, host_counts), ev

    def _complete(self):
        torch.cuda.set_device(self.device)
        while True:
            with self._lock:
                while not self._inflight:
                    if not self._running and not self._q and self._launching == 0:
                        return
                    self._cv_done.wait(timeout=0.05)
                ev, batch, need, keep, k = self._inflight[0]
            ev.synchronize()
            n_pairs = int(self._slots[k].host_np[1])
            P = sum(r.pixels for r in batch)
            if n_pairs > keep[1].cap():
                # the lists were cut short: grow this stream's buffers and
                # the estimate, and render the batch again (its stream has
                # nothing else queued: one batch per stream is in flight)
                self.pairs_per_pixel_max = max(self.pairs_per_pixel_max, n_pairs / max(P, 1))
                self._slots[k].binner.grow(n_pairs)
                keep, ev = self._launch(batch, self.streams[k], self._slots[k])
                ev.synchronize()
            t = time.perf_counter()
            image = keep[2]
            # the image was allocated on the batch's stream: tie its release
            # to the consumer stream too (see the module notes on streams)
            image.record_stream(self.consumer)
            off = 0
            for r in batch:
                H, W = int(r.cam["height"]), int(r.cam["width"])
                r.t_done = t
                # the request drops its future (future.request stays): no
                # reference cycle keeps a served image alive after the
                # caller lets go of the future
                fut, r.future = r.future, None
                fut.set_result(image[off:off + r.pixels].view(H, W, 3))
                off += r.pixels
            if P > 0:
                self.pairs_per_pixel = 0.8 * self.pairs_per_pixel + 0.2 * n_pairs / P
                self.pairs_per_pixel_max = max(self.pairs_per_pixel_max, n_pairs / P)
            with self._lock:
                self._inflight.popleft()
                self._mem_used -= need
                if self._q:
                    self._cv_sched.notify()


class PlainRenderer:
    """One request per launch sequence, FIFO, one stream."""

    def __init__(self, scene: dict, opts=None, pairs_per_pixel: float = 20.0):
        self.scene = scene
        self.n = scene["means"].shape[0]
        self.opts = sss.render_opts(opts)
        self.binner = sss.BinSorter(0, no_wait=True, work=False)
        # as the server: the pair passes are sized by the largest pairs per
        # pixel seen so far
        self.pairs_per_pixel_max = float(pairs_per_pixel)

    def warmup(self, cams):
        """Render each camera once (sizes the pair capacity and the allocator's
        cache before requests arrive)."""
        for c in cams:
            self.render(c)

    def render(self, cam):
        cams = sss.CameraBatch([cam])
        P = cams.n_pixels
        while True:
            proj = sss.project(self.scene, cams, self.opts)
            bins = self.binner(proj, cams, self.n, capacity=int(self.pairs_per_pixel_max * 1.5 * P) + 8192)
            image, _, _ = sss.render_fwd(bins, cams, self.opts, aux=False)
            torch.cuda.current_stream().synchronize()
            try:
                bins.resolve()           # counts arrived with the render
            except sss.SSSError:
                self.binner.grow(bins.n_pairs)
                continue
            finally:
                if bins.n_pairs >= 0 and P > 0:
                    self.pairs_per_pixel_max = max(self.pairs_per_pixel_max, bins.n_pairs / P)
            return image.view(int(cam["height"]), int(cam["width"]), 3)


def poisson_arrivals(rate: float, duration: float, rng):
    """Arrival times of a Poisson process of `rate` per second over `duration` s."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append(t)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def run_load(server_kind: str, scene: dict, cams, arrivals, opts=None, warm=None, fill_budget=True, **server_kw):
    """Replay `arrivals` (seconds from start) with the request cameras `cams`
    against the batched server or the plain renderer.  Latency is measured
    from the scheduled arrival to the moment the image is ready on the
    device.  `warm` (cameras, optional) is rendered before the clock starts:
    by the batched server as one batch per stream, by the plain renderer one
    by one.  Returns (latencies in s, wall time in s, server stats)."""
    lat = []
    stats = {}
    if server_kind == "batched":
        srv = RenderServer(scene, opts, **server_kw)
        if warm:
            srv.warmup(warm, fill_budget=fill_budget)
        # latencies are taken as requests complete and the futures (and with
        # them the images) are not kept: a long run at a high rate would
        # otherwise hold every image it served
        done_cv = threading.Condition()
        left = [len(arrivals)]
        errors = []

        def finished(f, ta):
            with done_cv:
                if f.exception() is None:
                    lat.append(f.request.t_done - ta)
                else:
                    errors.append(f.exception())
                left[0] -= 1
                done_cv.notify()

        t0 = time.perf_counter()
        for a, cam in zip(arrivals, cams):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            srv.submit(cam).add_done_callback(functools.partial(finished, ta=t0 + a))
        with done_cv:
            done_cv.wait_for(lambda: left[0] == 0)
        t_end = time.perf_counter()
        srv.close()
        if errors:
            raise errors[0]
        stats = dict(batches=srv.batches, mean_batch=sum(srv.batch_sizes) / max(1, len(srv.batch_sizes)))
    elif server_kind == "plain":
        pr = PlainRenderer(scene, opts)
        if warm:
            pr.warmup(warm)
        t0 = time.perf_counter()
        for a, cam in zip(arrivals, cams):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            pr.render(cam)
            lat.append(time.perf_counter() - t0 - a)
        t_end = time.perf_counter()
    else:
        raise ValueError(server_kind)
    return lat, t_end - t0, stats


def run_closed(server_kind: str, scene: dict, make_cam, n_clients: int, duration: float, opts=None, warm=None,
               fill_budget=True, **server_kw):
    """Closed loop of n_clients clients, each sending its next request
    (make_cam(k) for the k-th request overall) as soon as its previous one
    returns, for `duration` seconds.  One driver thread keeps the
    n_clients requests outstanding (client threads of their own would
    measure the interpreter's thread switching rather than the server).
    The plain renderer serves them one at a time in arrival order, so a
    request waits for the ones ahead of it.  Returns (latencies in s,
    requests completed, pixels completed, wall time in s, server stats)."""
    import concurrent.futures as cf
    lat, px, k = [], 0, 0
    stats = {}
    t0 = time.perf_counter()
    t_stop = t0 + duration
    if server_kind == "batched":
        srv = RenderServer(scene, opts, **server_kw)
        if warm:
            srv.warmup(warm, fill_budget=fill_budget)
        t0 = time.perf_counter()
        t_stop = t0 + duration
        pending = set()
        for _ in range(n_clients):
            pending.add(srv.submit(make_cam(k)))
            k += 1
        while pending:
            done, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
            now = time.perf_counter()
            for f in done:
                f.result()
                r = f.request
                lat.append(r.t_done - r.t_submit)
                px += r.pixels
                if now < t_stop:
                    pending.add(srv.submit(make_cam(k)))
                    k += 1
        t_end = time.perf_counter()
        srv.close()
        stats = dict(batches=srv.batches, mean_batch=sum(srv.batch_sizes) / max(1, len(srv.batch_sizes)))
    elif server_kind == "plain":
        pr = PlainRenderer(scene, opts)
        if warm:
            pr.warmup(warm)
        t0 = time.perf_counter()
        t_stop = t0 + duration
        queue = collections.deque()                     # (submit time, camera), FIFO
        for _ in range(n_clients):
            queue.append((t0, make_cam(k)))
            k += 1
        while queue:
            ts, cam = queue.popleft()
            pr.render(cam)
            now = time.perf_counter()
            lat.append(now - ts)
            px += int(cam["width"]) * int(cam["height"])
            if now < t_stop:
                queue.append((now, make_cam(k)))
                k += 1
        t_end = time.perf_counter()
    else:
        raise ValueError(server_kind)
    return lat, len(lat), px, t_end - t0, stats
