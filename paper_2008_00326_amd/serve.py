"""Served form of pose scoring: a request loop with continuous batching.

A request is one observed scene and its objects' candidate poses; its
answer is the minimum-cost pose of every object (Sec. IV-A "Parallel
Search").  The server

* admits requests in arrival order while the device memory they will hold
  (scene images and neighbour table, poses, cost arrays) fits a budget;
  when the next request does not fit it waits for results to free memory;
* prepares admitted requests on worker threads (one by default) -- meshes
  come from a resident cache keyed by content hash, the scene is uploaded
  and prepared on the library's own stream (or, with the optional scene
  cache, taken from the scenes already resident) -- while the device scores
  earlier requests; a preparation waits for the device (for the finished
  scene), and the wait can last as long as a scoring launch that holds
  every compute unit, so two workers keep the ready queue filled where one
  cannot;
* launches prepared requests in batches on a small set of launch slots (two
  by default): a request that becomes ready while a batch runs joins the
  next launch, which is queued behind the running one, so the device never
  waits for the host between batches (optionally a lone ready request is
  held briefly for a second to share that launch);
* returns each request's answer as soon as its batch completes and releases
  its memory.

Each request's answer is computed by the same kernels from the same device
descriptors as when it is scored alone, so it is identical whatever shares
its batch.

The executor interface (footprint / prepare / launch / done / wait /
release) separates the policy from the device; ``GpuExecutor`` drives the
library, and tests drive the policy with a fake executor on the CPU.
"""
from __future__ import annotations

import collections
import hashlib
import threading
import time
from dataclasses import dataclass, field


class OutOfMemory(Exception):
    """Preparation ran out of device memory; the request is retried later."""


@dataclass
class Request:
    """One scene to search.  ``payload`` is whatever the executor prepares
    (for ``GpuExecutor`` a generated workload: scene, meshes, objects)."""
    rid: int
    payload: object
    n_poses: int
    arrival: float | None = None
    admitted: float | None = None
    ready: float | None = None
    launched: float | None = None
    done: float | None = None
    result: list | None = None          # per object (best index, J)
    error: str | None = None
    batch: int | None = None            # sequence number of the launch that scored it
    scene_s: float | None = None        # of the preparation: time in set_scene
    upload_s: float | None = None       # and in the pose upload

    @property
    def latency(self) -> float | None:
        return None if self.done is None or self.arrival is None else self.done - self.arrival


@dataclass
class Prepared:
    req: Request
    handle: object                      # executor-specific
    n_items: int
    n_poses: int
    nbytes: int


class Server:
    """Continuous-batching request loop over an executor.

    budget_bytes:   device memory that admitted, unfinished requests may hold.
    slots:          launch slots of the executor (batches in flight at once).
    max_items, max_poses: capacity of one launch.
    prep_workers:   threads preparing admitted requests (admission stays in
                    arrival order; prepared requests are launched oldest first).
    hold_s:         while a batch runs, a lone ready request waits up to this
                    long for another to join its launch (0: launched at once).
    """

    def __init__(self, executor, *, budget_bytes: int, max_items: int, max_poses: int, clock=time.perf_counter,
                 prep_workers: int = 1, hold_s: float = 0.0):
        if prep_workers < 1:
            raise ValueError("prep_workers must be >= 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.hold_s = float(hold_s)
        self.max_items = int(max_items)
        self.max_poses = int(max_poses)
        self.clock = clock
        self.cv = threading.Condition()
        self.queue = collections.deque()     # submitted, not admitted
        self.ready = collections.deque()     # prepared, not launched
        self.inflight_bytes = 0              # held by admitted, unfinished requests
        self.peak_bytes = 0
        self.preparing = 0
        self.closed = False
        self.completed = []
        self.batches = []                    # (sequence, number of requests, poses)
        self._seq = 0
        self.n_inflight = 0                  # requests launched, not finished
        self._prep = [threading.Thread(target=self._prep_loop, name=f"perch-prep-{k}", daemon=True)
                      for k in range(prep_workers)]
        self._prep_error = None

    # -- producer side ------------------------------------------------------
    def submit(self, req: Request) -> None:
        with self.cv:
            if self.closed:
                raise RuntimeError("server is closed")
            if req.arrival is None:
                req.arrival = self.clock()
            self.queue.append(req)
            self.cv.notify_all()

    def close(self) -> None:
        """No more submissions; run() returns once everything submitted is done."""
        with self.cv:
            self.closed = True
            self.cv.notify_all()

    def cancel_pending(self) -> list:
        """Withdraw every request not yet admitted; returns them."""
        with self.cv:
            out = list(self.queue)
            self.queue.clear()
            self.cv.notify_all()
            return out

    # -- admission and preparation (worker thread) ---------------------------
    def _prep_loop(self):
        try:
            while True:
                with self.cv:
                    while True:
                        if self.queue:
                            req = self.queue[0]
                            need = self.ex.footprint(req)
                            if need > self.budget or req.n_poses > self.max_poses:
                                self.queue.popleft()
                                req.error = (f"needs {need} bytes and {req.n_poses} poses; budget {self.budget} "
                                             f"bytes, launch capacity {self.max_poses} poses")
                                req.done = self.clock()
                                self.completed.append(req)
                                self.cv.notify_all()
                                continue
                            if self.inflight_bytes + need <= self.budget:
                                self.queue.popleft()
                                self.inflight_bytes += need
                                self.peak_bytes = max(self.peak_bytes, self.inflight_bytes)
                                self.preparing += 1
                                req.admitted = self.clock()
                                break
                        elif self.closed:
                            return
                        self.cv.wait()
                try:
                    prep = self.ex.prepare(req)
                except OutOfMemory as e:
                    with self.cv:
                        self.inflight_bytes -= need
                        self.preparing -= 1
                        if not (self.ready or self.n_inflight):
                            # nothing holds memory that could come back
                            req.error = f"OutOfMemory: {e}"
                            req.done = self.clock()
                            self.completed.append(req)
                            self.cv.notify_all()
                            continue
                        # retry, first in line, once something else has finished
                        self.queue.appendleft(req)
                        req.admitted = None
                        n_done = len(self.completed)
                        while len(self.completed) == n_done:
                            self.cv.wait()
                    continue
                except Exception as e:                     # the request fails alone
                    with self.cv:
                        self.inflight_bytes -= need
                        self.preparing -= 1
                        req.error = f"{type(e).__name__}: {e}"
                        req.done = self.clock()
                        self.completed.append(req)
                        self.cv.notify_all()
                    continue
                with self.cv:
                    self.inflight_bytes += prep.nbytes - need   # the estimate becomes the real size
                    self.peak_bytes = max(self.peak_bytes, self.inflight_bytes)
                    self.preparing -= 1
                    req.ready = self.clock()
                    # oldest first: a later arrival prepared sooner by another worker waits behind it
                    k = len(self.ready)
                    while k > 0 and self.ready[k - 1].req.arrival > req.arrival:
                        k -= 1
                    self.ready.insert(k, prep)
                    self.cv.notify_all()
        except BaseException as e:                         # pragma: no cover - surfaced by run()
            with self.cv:
                self._prep_error = e
                self.cv.notify_all()

    # -- scheduling (caller's thread) -----------------------------------------
    def _take_batch(self):
        """Ready requests, oldest first, up to the launch capacity (a single
        request larger than the capacity goes alone and the executor splits
        nothing: it must fit)."""
        take, items, poses = [], 0, 0
        while self.ready:
            p = self.ready[0]
            if take and (items + p.n_items > self.max_items or poses + p.n_poses > self.max_poses):
                break
            self.ready.popleft()
            take.append(p)
            items += p.n_items
            poses += p.n_poses
        return take

    def run(self, poll_s: float = 0.0005) -> list:
        """Serve until close() and everything submitted has completed.
        Returns the completed requests in completion order."""
        free = list(range(self.ex.slots))
        self._inflight = collections.deque()          # (slot, [Prepared], seq)
        for t in self._prep:
            t.start()
        while True:
            with self.cv:
                if self._prep_error is not None:
                    raise self._prep_error
                # a lone ready request waits while a batch runs and more requests may still come
                more = not self.closed or bool(self.queue) or self.preparing > 0
                hold = (self.hold_s > 0 and len(self.ready) == 1 and len(free) < self.ex.slots and more
                        and self.clock() - self.ready[0].req.ready < self.hold_s)
                take = self._take_batch() if (self.ready and free and not hold) else []
                self.n_inflight += len(take)
                finished = (self.closed and not take and not self.queue and not self.ready and not self.preparing
                            and not self._inflight)
            if finished:
                break
            if take:
                slot = free.pop(0)
                self._seq += 1
                now = self.clock()
                for p in take:
                    p.req.launched = now
                    p.req.batch = self._seq
                try:
                    self.ex.launch(slot, [p.handle for p in take])
                except Exception as e:                   # the batch fails; its requests report it
                    self._finish(take, None, f"{type(e).__name__}: {e}")
                    free.append(slot)
                    continue
                self.batches.append((self._seq, len(take), sum(p.n_poses for p in take)))
                self._inflight.append((slot, take, self._seq))
                continue
            if self._inflight:
                slot, group, _ = self._inflight[0]
                # block on the oldest batch only when no slot is free; with a
                # free slot, poll so that work becoming ready is launched at once
                if not free or self.ex.done(slot):
                    self._inflight.popleft()
                    try:
                        results = self.ex.wait(slot)
                        self._finish(group, results, None)
                    except Exception as e:
                        self._finish(group, None, f"{type(e).__name__}: {e}")
                    free.append(slot)
                    continue
                with self.cv:
                    if not self.ready or (self.hold_s > 0 and len(self.ready) == 1):
                        self.cv.wait(timeout=poll_s)
                continue
            with self.cv:
                if not (self.ready or (self.closed and not self.queue and not self.preparing)):
                    self.cv.wait(timeout=0.05)
        for t in self._prep:
            t.join()
        return self.completed

    def _finish(self, group, results, error):
        now = self.clock()
        for k, p in enumerate(group):
            try:
                self.ex.release(p.handle)
            finally:
                with self.cv:
                    p.req.done = now
                    if error is None:
                        p.req.result = results[k]
                    else:
                        p.req.error = error
                    self.inflight_bytes -= p.nbytes
                    self.n_inflight -= 1
                    self.completed.append(p.req)
                    self.cv.notify_all()


def latency_stats(reqs, *, horizon: float | None = None) -> dict:
    """p50/p99 of arrival-to-result latency (ms).  With `horizon`, requests
    still unanswered then count with the lower bound horizon - arrival."""
    import numpy as np
    lat = [r.latency for r in reqs if r.latency is not None and r.error is None]
    cens = [horizon - r.arrival for r in reqs if r.done is None and horizon is not None and r.arrival is not None]
    allv = np.asarray(lat + cens, np.float64) * 1e3
    if allv.size == 0:
        return {"p50": None, "p99": None, "completed": 0, "unfinished": len(cens)}
    return {"p50": round(float(np.percentile(allv, 50)), 3), "p99": round(float(np.percentile(allv, 99)), 3),
            "completed": len(lat), "unfinished": len(cens)}


# ---------------------------------------------------------------- device executor

class MeshCache:
    """Resident meshes keyed by content hash, reference-counted; meshes no
    request uses are unloaded oldest first once the cache holds more than
    `max_bytes`."""

    def __init__(self, ctx, max_bytes: int = 4 << 30):
        self.ctx = ctx
        self.max_bytes = max_bytes
        self.lock = threading.Lock()
        self.entries = collections.OrderedDict()    # key -> [mesh_id, refs, bytes]
        self.bytes = 0
        self.hits = 0
        self.misses = 0
        self._seen = {}                              # id(mesh) -> (mesh, use_rgb, key): hash each object once

    @staticmethod
    def key(mesh, use_rgb: bool) -> str:
        h = hashlib.blake2b(digest_size=16)
        h.update(mesh.xyz.tobytes())
        h.update(mesh.tri.tobytes())
        if use_rgb and mesh.rgb is not None:
            h.update(mesh.rgb.tobytes())
        return h.hexdigest()

    def _key_of(self, mesh, use_rgb: bool) -> str:
        # mesh arrays are treated as immutable once submitted; the memo keeps
        # a reference, so an id is never reused while it is remembered
        m = self._seen.get(id(mesh))
        if m is not None and m[0] is mesh and m[1] == use_rgb:
            return m[2]
        k = self.key(mesh, use_rgb)
        if len(self._seen) > 4096:
            self._seen.clear()
        self._seen[id(mesh)] = (mesh, use_rgb, k)
        return k

    def acquire(self, mesh, use_rgb: bool) -> tuple:
        with self.lock:
            k = self._key_of(mesh, use_rgb)
        with self.lock:
            e = self.entries.get(k)
            if e is not None:
                e[1] += 1
                self.entries.move_to_end(k)
                self.hits += 1
                return k, e[0]
        mid = self.ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb if use_rgb else None)
        nbytes = mesh.xyz.shape[0] * (16 + (4 if use_rgb else 0)) + mesh.tri.shape[0] * 16
        with self.lock:
            e = self.entries.get(k)
            if e is not None:                         # loaded meanwhile by another thread
                e[1] += 1
                self.hits += 1
                dup = mid
                mid = e[0]
            else:
                self.entries[k] = [mid, 1, nbytes]
                self.bytes += nbytes
                self.misses += 1
                dup = None
        if dup is not None:
            self.ctx.unload_mesh(dup)
        self._evict()
        return k, mid

    def release(self, key: str) -> None:
        with self.lock:
            self.entries[key][1] -= 1
        self._evict()

    def _evict(self):
        drop = []
        with self.lock:
            for k in list(self.entries):
                if self.bytes <= self.max_bytes:
                    break
                mid, refs, nb = self.entries[k]
                if refs == 0:
                    del self.entries[k]
                    self.bytes -= nb
                    drop.append(mid)
        for mid in drop:
            self.ctx.unload_mesh(mid)


class SceneCache:
    """Resident scenes keyed by content hash (camera, images and the options
    they are prepared with), reference-counted: a request whose scene is
    already resident skips its preparation.  Scenes no request uses are
    dropped oldest first once the cache holds more than `max_bytes`, and all
    of them when a preparation runs out of device memory (then it is tried
    once more)."""

    def __init__(self, ctx, max_bytes: int = 4 << 30):
        self.ctx = ctx
        self.max_bytes = max_bytes
        self.lock = threading.Lock()
        self.entries = collections.OrderedDict()    # key -> [scene_id, refs, bytes]
        self.bytes = 0
        self.hits = 0
        self.misses = 0
        self._seen = {}                              # id(workload) -> (workload, key): hash each once

    @staticmethod
    def key(w) -> str:
        import numpy as np
        s = w.scene
        h = hashlib.blake2b(digest_size=16)
        h.update(np.asarray(s.K, np.float64).tobytes())
        h.update(np.ascontiguousarray(s.depth).tobytes())
        if w.use_rgb and s.rgb is not None:
            h.update(np.ascontiguousarray(s.rgb).tobytes())
        if w.volume == "label" and s.labels is not None:
            h.update(np.ascontiguousarray(s.labels).tobytes())
        h.update(repr((float(w.delta_mm), float(w.tau_c), bool(w.use_rgb), bool(w.mark_occluders), w.volume,
                       getattr(w, "jo", "exact"), getattr(w, "search", "table"), int(w.stride))).encode())
        return h.hexdigest()

    def _key_of(self, w) -> str:
        # workloads are treated as immutable once submitted (as meshes are)
        m = self._seen.get(id(w))
        if m is not None and m[0] is w:
            return m[1]
        k = self.key(w)
        if len(self._seen) > 4096:
            self._seen.clear()
        self._seen[id(w)] = (w, k)
        return k

    def acquire(self, w, prepare) -> tuple:
        """(key, scene_id, hit); `prepare()` makes the scene resident on a miss."""
        import paper_2008_00326_amd as pk
        with self.lock:
            k = self._key_of(w)
            e = self.entries.get(k)
            if e is not None:
                e[1] += 1
                self.entries.move_to_end(k)
                self.hits += 1
                return k, e[0], True
        try:
            sid = prepare()
        except pk.PerchError as err:
            if err.status != -2:
                raise
            self._evict(0)
            sid = prepare()
        nbytes = int(self.ctx.scene_info(sid)["device_bytes"])
        with self.lock:
            e = self.entries.get(k)
            if e is not None:                         # prepared meanwhile by another thread
                e[1] += 1
                self.hits += 1
                dup, sid = sid, e[0]
            else:
                self.entries[k] = [sid, 1, nbytes]
                self.bytes += nbytes
                self.misses += 1
                dup = None
        if dup is not None:
            self.ctx.drop_scene(dup)
        self._evict(self.max_bytes)
        return k, sid, dup is not None

    def release(self, key: str) -> None:
        with self.lock:
            self.entries[key][1] -= 1
        self._evict(self.max_bytes)

    def _evict(self, limit: int):
        drop = []
        with self.lock:
            for k in list(self.entries):
                if self.bytes <= limit:
                    break
                sid, refs, nb = self.entries[k]
                if refs == 0:
                    del self.entries[k]
                    self.bytes -= nb
                    drop.append(sid)
        for sid in drop:
            self.ctx.drop_scene(sid)

    def clear(self):
        """Drop every scene no request uses."""
        self._evict(0)


@dataclass
class _Handle:
    scene_id: int
    mesh_keys: list
    items: list                     # score_batch item dicts
    tensors: list = field(default_factory=list)
    scene_key: str | None = None    # the scene cache's key, when the scene is shared through it


class GpuExecutor:
    """Executor over a library context: ``slots`` graph-captured batches of
    capacity (max_items, max_poses) used in turn on one scoring stream.
    scene_cache_bytes > 0 keeps prepared scenes resident (SceneCache), so a
    request for a scene seen before skips its preparation; the cache's
    unused scenes are memory beyond the server's admission budget, as the
    mesh cache's are."""

    def __init__(self, ctx, *, slots: int = 2, max_items: int = 256, max_poses: int = 65536,
                 max_image_pixels: int = 640 * 480, mesh_cache_bytes: int = 4 << 30, scene_cache_bytes: int = 0):
        import torch
        self.ctx = ctx
        self.slots = slots
        self.meshes = MeshCache(ctx, mesh_cache_bytes)
        self.scenes = SceneCache(ctx, scene_cache_bytes) if scene_cache_bytes > 0 else None
        self.batches = [ctx.batch(max_items, max_poses, max_image_pixels) for _ in range(slots)]
        self.stream = torch.cuda.Stream()
        self._local = threading.local()          # a copy stream per preparation thread
        self.n_items = [0] * slots
        self.table_bytes_per_px = 400.0           # running estimate of the neighbour table size

    def footprint(self, req: Request) -> int:
        w = req.payload
        W, H = int(w.scene.K[0]), int(w.scene.K[1])
        px = W * H
        per_px = 2 + 8 + (3 + 16 if w.use_rgb else 0) + (4 if w.volume == "label" else 0) + 8 + 1
        return int(px * (per_px + self.table_bytes_per_px) + req.n_poses * (48 + 8))

    def prepare(self, req: Request) -> Prepared:
        import numpy as np
        import torch
        import paper_2008_00326_amd as pk
        w = req.payload
        keys, mids = [], []
        for o in w.objects:
            k, mid = self.meshes.acquire(w.meshes[o.mesh], w.use_rgb)
            keys.append(k)
            mids.append(mid)
        s = w.scene
        t0 = time.perf_counter()
        skey = None
        try:
            if self.scenes is not None:
                skey, sid, _ = self.scenes.acquire(w, lambda: set_scene(self.ctx, w))
            else:
                sid = set_scene(self.ctx, w)
        except pk.PerchError as e:
            for k in keys:
                self.meshes.release(k)
            if e.status == -2:
                raise OutOfMemory(str(e)) from e
            raise
        t1 = time.perf_counter()
        # every object's poses in one copy (and one allocation for the costs);
        # the items take row slices
        st = getattr(self._local, "stream", None)
        if st is None:
            st = self._local.stream = torch.cuda.Stream()
        counts = [o.poses.shape[0] for o in w.objects]
        allp = np.ascontiguousarray(np.concatenate([o.poses for o in w.objects]), dtype=np.float32)
        with torch.cuda.stream(st):
            dev = torch.from_numpy(allp).to("cuda")
            costs = torch.empty((2, allp.shape[0]), dtype=torch.int32, device="cuda")
        items, tensors = [], [dev, costs]
        k = 0
        for o, mid, n in zip(w.objects, mids, counts):
            items.append({"scene": sid, "mesh": mid, "label": o.label, "poses": dev[k:k + n],
                          "jr": costs[0, k:k + n], "jo": costs[1, k:k + n]})
            k += n
        st.synchronize()
        req.scene_s = t1 - t0
        req.upload_s = time.perf_counter() - t1
        info = self.ctx.scene_info(sid)
        W, H = int(s.K[0]), int(s.K[1])
        self.table_bytes_per_px = max(self.table_bytes_per_px, info["table_entries"] * 4.0 / (W * H))
        nbytes = int(info["device_bytes"] + req.n_poses * (48 + 8))
        return Prepared(req, _Handle(sid, keys, items, tensors, skey), len(items), req.n_poses, nbytes)

    def launch(self, slot: int, handles: list) -> None:
        items = [it for h in handles for it in h.items]
        b = self.batches[slot]
        b.set(items)
        b.launch(self.stream)
        self.n_items[slot] = [len(h.items) for h in handles]

    def done(self, slot: int) -> bool:
        return self.batches[slot].done()

    def wait(self, slot: int) -> list:
        bi, bc = self.batches[slot].wait()
        out, k = [], 0
        for n in self.n_items[slot]:
            out.append([(int(bi[k + j]), int(bc[k + j])) for j in range(n)])
            k += n
        return out

    def release(self, h: _Handle) -> None:
        if h.scene_key is not None:
            self.scenes.release(h.scene_key)
        else:
            self.ctx.drop_scene(h.scene_id)
        for k in h.mesh_keys:
            self.meshes.release(k)
        h.items.clear()
        h.tensors.clear()

    def close(self):
        for b in self.batches:
            b.close()
        self.batches = []
        if self.scenes is not None:
            self.scenes.clear()


def set_scene(ctx, w) -> int:
    """Make a workload's scene resident with the workload's own options."""
    s = w.scene
    return ctx.set_scene(s.K, s.depth, s.rgb if w.use_rgb else None, s.labels if w.volume == "label" else None,
                         delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=w.use_rgb, mark_occluders=w.mark_occluders,
                         volume=w.volume, jo=getattr(w, "jo", "exact"), search=getattr(w, "search", "table"),
                         stride=w.stride)


def plain_loop(ctx, requests, *, clock=time.perf_counter, meshes: MeshCache | None = None, stop_at=None,
               scenes: SceneCache | None = None):
    """The one-scene-per-launch reference: each request in arrival order,
    prepared and scored alone (best_poses), nothing overlapped.  With
    `scenes`, a scene seen before is taken from that cache instead of being
    prepared again.  Requests must carry their arrival times; returns them
    completed."""
    import torch
    meshes = meshes or MeshCache(ctx)
    stream = torch.cuda.current_stream()
    for r in requests:
        now = clock()
        if stop_at is not None and now > stop_at:
            break
        if r.arrival > now:
            time.sleep(r.arrival - now)
        w = r.payload
        keys_mids = [meshes.acquire(w.meshes[o.mesh], w.use_rgb) for o in w.objects]
        skey = None
        if scenes is not None:
            skey, sid, _ = scenes.acquire(w, lambda: set_scene(ctx, w))
        else:
            sid = set_scene(ctx, w)
        polys = [torch.from_numpy(o.poses).cuda() for o in w.objects]
        bi, bc = ctx.best_poses(sid, [m for _, m in keys_mids], [o.label for o in w.objects], polys, stream=stream)
        r.result = [(int(a), int(b)) for a, b in zip(bi, bc)]
        r.done = clock()
        if skey is not None:
            scenes.release(skey)
        else:
            ctx.drop_scene(sid)
        for k, _ in keys_mids:
            meshes.release(k)
    return [r for r in requests if r.done is not None]
