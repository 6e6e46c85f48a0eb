"""The serving loop's policy on the CPU: a fake executor stands in for the
device (a serial device that takes a fixed time per pose, preparation that
takes a fixed time), so admission, batching, failure isolation and latency
bookkeeping are checked without a GPU."""
import threading
import time

import pytest

from paper_2008_00326_amd.serve import OutOfMemory, Request, Server, latency_stats


class FakeExecutor:
    def __init__(self, slots=2, per_pose_s=2e-6, prep_s=0.002, fail_launch_on=None):
        self.slots = slots
        self.per_pose_s = per_pose_s
        self.prep_s = prep_s
        self.fail_launch_on = fail_launch_on or set()
        self.lock = threading.Lock()
        self.device_free_at = 0.0
        self.slot_end = {}
        self.slot_handles = {}
        self.launches = []
        self.live_bytes = 0
        self.max_live_bytes = 0
        self.released = []
        self.oom_once = set()

    def footprint(self, req):
        return req.payload["bytes"]

    def prepare(self, req):
        from paper_2008_00326_amd.serve import Prepared
        p = req.payload
        time.sleep(self.prep_s)
        if p.get("fail_prepare"):
            raise ValueError("bad scene")
        if p.get("oom_first") and req.rid not in self.oom_once:
            self.oom_once.add(req.rid)
            raise OutOfMemory("device full")
        with self.lock:
            self.live_bytes += p["bytes"]
            self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        return Prepared(req, req, len(p["answer"]), req.n_poses, p["bytes"])

    def launch(self, slot, handles):
        n = len(self.launches)
        self.launches.append([h.rid for h in handles])
        if n in self.fail_launch_on:
            raise RuntimeError("launch failed")
        now = time.perf_counter()
        start = max(now, self.device_free_at)           # a serial device: queued behind earlier launches
        end = start + self.per_pose_s * sum(h.n_poses for h in handles)
        self.device_free_at = end
        self.slot_end[slot] = end
        self.slot_handles[slot] = handles

    def done(self, slot):
        return time.perf_counter() >= self.slot_end[slot]

    def wait(self, slot):
        d = self.slot_end[slot] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        return [list(h.payload["answer"]) for h in self.slot_handles[slot]]

    def release(self, h):
        with self.lock:
            self.live_bytes -= h.payload["bytes"]
        self.released.append(h.rid)


def make_req(rid, poses=1000, nbytes=100, n_obj=3, **extra):
    payload = {"bytes": nbytes, "answer": [(rid, 10 * rid + k) for k in range(n_obj)], **extra}
    return Request(rid, payload, poses)


def serve(ex, reqs, *, budget=10_000, max_items=64, max_poses=100_000, spacing=0.0, prep_workers=1, hold_s=0.0):
    srv = Server(ex, budget_bytes=budget, max_items=max_items, max_poses=max_poses, prep_workers=prep_workers,
                 hold_s=hold_s)

    def producer():
        for r in reqs:
            srv.submit(r)
            if spacing:
                time.sleep(spacing)
        srv.close()

    t = threading.Thread(target=producer)
    t.start()
    done = srv.run()
    t.join()
    return srv, done


def test_every_request_answered_with_its_own_result():
    ex = FakeExecutor()
    reqs = [make_req(i) for i in range(40)]
    srv, done = serve(ex, reqs, spacing=0.0005)
    assert sorted(r.rid for r in done) == list(range(40))
    for r in done:
        assert r.error is None and r.result == r.payload["answer"]
        assert r.arrival <= r.admitted <= r.ready <= r.launched <= r.done
    assert sorted(ex.released) == list(range(40))
    assert srv.inflight_bytes == 0 and ex.live_bytes == 0


def test_admission_respects_budget_and_arrival_order():
    ex = FakeExecutor(per_pose_s=2e-5)
    reqs = [make_req(i, nbytes=300) for i in range(20)]
    srv, done = serve(ex, reqs, budget=1000)              # at most three in flight
    assert ex.max_live_bytes <= 1000 and srv.peak_bytes <= 1000
    adm = sorted(done, key=lambda r: r.admitted)
    assert [r.rid for r in adm] == list(range(20))        # first come, first admitted


def test_arrivals_join_later_batches():
    """With a slow device, requests arriving while a batch runs are launched
    together: fewer launches than requests, and no launch over capacity."""
    ex = FakeExecutor(per_pose_s=1e-5, prep_s=0.0005)
    reqs = [make_req(i, poses=2000) for i in range(30)]
    srv, done = serve(ex, reqs, max_poses=12_000, spacing=0.001)
    assert len(done) == 30
    assert len(ex.launches) < 30
    assert max(len(g) for g in ex.launches) > 1
    for _, n, poses in srv.batches:
        assert poses <= 12_000
    # each request is scored exactly once
    assert sorted(x for g in ex.launches for x in g) == list(range(30))


def test_two_preparation_workers():
    """Preparation-bound (preparing takes longer than scoring): a second
    worker roughly halves the time to answer everything, admission stays in
    arrival order and every launch takes its requests oldest first."""
    spans = {}
    for workers in (1, 2):
        ex = FakeExecutor(per_pose_s=1e-7, prep_s=0.01)
        reqs = [make_req(i) for i in range(24)]
        t0 = time.perf_counter()
        srv, done = serve(ex, reqs, prep_workers=workers)
        spans[workers] = time.perf_counter() - t0
        assert sorted(r.rid for r in done) == list(range(24))
        assert all(r.error is None and r.result == r.payload["answer"] for r in done)
        assert [r.rid for r in sorted(done, key=lambda r: r.admitted)] == list(range(24))
        for g in ex.launches:
            assert g == sorted(g)
        assert srv.inflight_bytes == 0 and ex.live_bytes == 0
    assert spans[2] < 0.8 * spans[1]
    with pytest.raises(ValueError):
        Server(FakeExecutor(), budget_bytes=1, max_items=1, max_poses=1, prep_workers=0)


def test_a_lone_ready_request_waits_to_be_joined():
    """While a batch runs, one ready request is held (up to hold_s) for a
    second to share its launch.  A long request runs; B arrives, then C: B
    goes alone at once without holding, and with C when held."""
    for hold, launches in ((0.0, 3), (0.03, 2)):
        ex = FakeExecutor(per_pose_s=5e-6, prep_s=0.001)
        reqs = [make_req(0, poses=10_000), make_req(1, poses=100), make_req(2, poses=100)]
        srv = Server(ex, budget_bytes=10_000, max_items=64, max_poses=100_000, hold_s=hold)

        def producer():
            srv.submit(reqs[0])
            time.sleep(0.01)                      # A is on the (serial, 50 ms) device
            srv.submit(reqs[1])
            time.sleep(0.005)
            srv.submit(reqs[2])
            srv.close()

        t = threading.Thread(target=producer)
        t.start()
        done = srv.run()
        t.join()
        assert sorted(r.rid for r in done) == [0, 1, 2]
        assert all(r.result == r.payload["answer"] for r in done)
        assert len(ex.launches) == launches, (hold, ex.launches)


def test_failures_stay_with_their_request():
    ex = FakeExecutor(fail_launch_on={2})
    reqs = [make_req(i) for i in range(12)]
    reqs[5].payload["fail_prepare"] = True
    srv, done = serve(ex, reqs, spacing=0.002)
    assert len(done) == 12
    failed_launch = set(ex.launches[2])
    for r in done:
        if r.rid == 5:
            assert r.error and "bad scene" in r.error
        elif r.rid in failed_launch:
            assert r.error and "launch failed" in r.error
        else:
            assert r.error is None and r.result == r.payload["answer"]
    assert srv.inflight_bytes == 0


def test_oversized_request_rejected_and_oom_retried():
    ex = FakeExecutor(per_pose_s=1e-5)
    reqs = [make_req(0), make_req(1, nbytes=50_000), make_req(2, oom_first=True), make_req(3, poses=10**6),
            make_req(4)]
    srv, done = serve(ex, reqs, budget=10_000, max_poses=100_000, spacing=0.003)
    by = {r.rid: r for r in done}
    assert len(by) == 5
    assert by[1].error and "budget" in by[1].error
    assert by[3].error and "capacity" in by[3].error
    for k in (0, 4):
        assert by[k].result == by[k].payload["answer"]
    # the request that hit OutOfMemory is either retried after others finished, or
    # reported when nothing in flight could free memory -- never lost
    assert by[2].result == by[2].payload["answer"] or "OutOfMemory" in (by[2].error or "")


def test_oom_with_work_in_flight_is_retried():
    ex = FakeExecutor(per_pose_s=5e-5, prep_s=0.0)
    reqs = [make_req(0, poses=4000), make_req(1, oom_first=True)]
    srv, done = serve(ex, reqs, spacing=0.002)
    by = {r.rid: r for r in done}
    assert by[1].result == by[1].payload["answer"], by[1].error


def test_latency_stats_counts_unfinished_as_lower_bounds():
    a, b, c = Request(0, None, 1, arrival=0.0), Request(1, None, 1, arrival=0.0), Request(2, None, 1, arrival=1.0)
    a.done, b.done = 0.010, 0.020
    st = latency_stats([a, b, c], horizon=3.0)
    assert st["completed"] == 2 and st["unfinished"] == 1
    assert st["p50"] == pytest.approx(20.0) and st["p99"] > 1900.0   # the unfinished one waited >= 2 s
    assert latency_stats([a, b])["p50"] == pytest.approx(15.0)


def test_closed_server_refuses_submissions():
    srv = Server(FakeExecutor(), budget_bytes=10, max_items=1, max_poses=1)
    srv.close()
    with pytest.raises(RuntimeError):
        srv.submit(make_req(0))


class FakeCtx:
    def __init__(self):
        self.next = 1
        self.loaded = {}

    def load_mesh(self, xyz, tri, rgb=None):
        mid = self.next
        self.next += 1
        self.loaded[mid] = (xyz.shape[0], tri.shape[0])
        return mid

    def unload_mesh(self, mid):
        del self.loaded[mid]


def test_mesh_cache_by_content_and_eviction():
    import numpy as np
    from types import SimpleNamespace
    from paper_2008_00326_amd.serve import MeshCache

    def mesh(seed):
        r = np.random.default_rng(seed)
        return SimpleNamespace(xyz=r.normal(size=(100, 3)).astype(np.float32),
                               tri=r.integers(0, 100, (200, 3)).astype(np.int32),
                               rgb=r.integers(0, 256, (100, 3)).astype(np.uint8))

    ctx = FakeCtx()
    one_mesh = 100 * 20 + 200 * 16
    cache = MeshCache(ctx, max_bytes=2 * one_mesh)
    a, a_copy, b, c = mesh(1), mesh(1), mesh(2), mesh(3)
    ka, ma = cache.acquire(a, True)
    kb, mb = cache.acquire(a_copy, True)              # same content, another object: a hit
    assert (ka, ma) == (kb, mb) and cache.hits == 1 and cache.misses == 1 and len(ctx.loaded) == 1
    k2, m2 = cache.acquire(b, True)
    k3, m3 = cache.acquire(c, True)                    # over budget, but everything is referenced
    assert len(ctx.loaded) == 3
    cache.release(ka)
    cache.release(kb)                                  # a unreferenced: evicted, oldest first
    assert ma not in ctx.loaded and len(ctx.loaded) == 2
    assert cache.acquire(a, True)[1] not in (ma,)      # reloaded under a new id
    assert cache.key(a, True) != cache.key(a, False)   # colours are part of the key only when used


class FakeSceneCtx:
    """set_scene / drop_scene / scene_info of a device with `capacity` bytes."""

    def __init__(self, capacity, nbytes=1000):
        self.capacity, self.nbytes = capacity, nbytes
        self.next = 1
        self.resident = {}
        self.prepared = 0

    def set_scene(self):
        import paper_2008_00326_amd as pk
        if (len(self.resident) + 1) * self.nbytes > self.capacity:
            raise pk.PerchError(-2, "out of device memory")
        sid = self.next
        self.next += 1
        self.resident[sid] = self.nbytes
        self.prepared += 1
        return sid

    def drop_scene(self, sid):
        del self.resident[sid]

    def scene_info(self, sid):
        return {"device_bytes": self.resident[sid]}


def test_scene_cache_by_content_options_and_eviction():
    import numpy as np
    from types import SimpleNamespace
    from paper_2008_00326_amd.serve import SceneCache

    def work(seed, **opts):
        r = np.random.default_rng(seed)
        sc = SimpleNamespace(K=(64, 48, 50.0, 50.0, 32.0, 24.0), depth=r.integers(0, 2000, (48, 64)).astype(np.uint16),
                             rgb=r.integers(0, 256, (48, 64, 3)).astype(np.uint8), labels=None)
        w = SimpleNamespace(scene=sc, delta_mm=10.0, tau_c=20.0, use_rgb=True, mark_occluders=True, volume="aabb",
                            jo="exact", search="table", stride=1)
        w.__dict__.update(opts)
        return w

    ctx = FakeSceneCtx(capacity=3000)
    cache = SceneCache(ctx, max_bytes=2000)
    a, a_copy, b = work(1), work(1), work(2)
    ka, sa, hit = cache.acquire(a, ctx.set_scene)
    assert not hit and ctx.prepared == 1
    kb, sb, hit = cache.acquire(a_copy, ctx.set_scene)     # same content, another object: no preparation
    assert hit and (ka, sa) == (kb, sb) and ctx.prepared == 1 and cache.hits == 1
    assert cache.key(a) != cache.key(work(1, jo="nn"))     # options are part of the key
    assert cache.key(a) != cache.key(work(1, delta_mm=12.0))
    cache.release(ka)
    cache.release(kb)
    assert sa in ctx.resident                              # unreferenced but within max_bytes: kept
    k2, s2, _ = cache.acquire(b, ctx.set_scene)
    k3, s3, _ = cache.acquire(work(3), ctx.set_scene)      # over max_bytes: a, unreferenced, dropped
    assert sa not in ctx.resident and len(ctx.resident) == 2
    cache.release(k3)
    # the device is full: the preparation runs out of memory, the cache drops
    # its unused scenes and tries once more
    ctx.capacity = 2000
    k4, s4, _ = cache.acquire(work(4), ctx.set_scene)
    assert s3 not in ctx.resident and s4 in ctx.resident and s2 in ctx.resident
    cache.release(k2)
    cache.release(k4)
    cache.clear()
    assert ctx.resident == {}
