"""Batched and graph-replayed scoring: each item's result must be bit-identical
to scoring it alone, whatever else shares the launch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd.workloads import make_config, scenes  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mixed(ctx):
    """Three different scenes (depth-only 320x240, RGB 640x480, 6-DoF RGB) and
    their objects, each with a seeded subset of its candidates."""
    rng = np.random.default_rng(5)
    items = []
    for cfg in (1, 2, 3):
        w = make_config(cfg, 0)
        sid, mids = pk.load_workload(ctx, w)
        for o in w.objects:
            sel = np.sort(rng.choice(o.poses.shape[0], min(o.poses.shape[0], 700), replace=False))
            items.append({"scene": sid, "mesh": mids[o.mesh], "label": o.label,
                          "poses": torch.from_numpy(np.ascontiguousarray(o.poses[sel])).cuda()})
    return items


def alone(ctx, it):
    jr, jo, nr, nq = ctx.score_poses(it["scene"], it["mesh"], it["poses"], label=it["label"])
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (jr, jo, nr, nq)]


def test_score_batch_equals_alone(ctx, mixed):
    say("score_batch vs alone")
    ref = [alone(ctx, it) for it in mixed]
    items = [dict(it, nr=torch.empty(it["poses"].shape[0], dtype=torch.int32, device="cuda"),
                  nq=torch.empty(it["poses"].shape[0], dtype=torch.int32, device="cuda")) for it in mixed]
    out = ctx.score_batch(items)
    torch.cuda.synchronize()
    for it, r in zip(out, ref):
        for key, a in zip(("jr", "jo", "nr", "nq"), r):
            assert np.array_equal(it[key].cpu().numpy(), a), key
    # the same items in reverse order, with an empty item in the middle
    rev = list(reversed(mixed))
    rev.insert(3, {"scene": mixed[0]["scene"], "mesh": mixed[0]["mesh"], "label": 1,
                   "poses": torch.empty((0, 12), dtype=torch.float32, device="cuda")})
    out = ctx.score_batch(rev)
    torch.cuda.synchronize()
    for it, r in zip([o for o in out if o["poses"].shape[0]], reversed(ref)):
        assert np.array_equal(it["jr"].cpu().numpy(), r[0]) and np.array_equal(it["jo"].cpu().numpy(), r[1])


def test_graph_batch_replays(ctx, mixed):
    say("graph batch")
    ref = [alone(ctx, it) for it in mixed]
    total = sum(it["poses"].shape[0] for it in mixed)
    b = ctx.batch(max_items=len(mixed) + 2, max_poses=total + 100, max_image_pixels=640 * 480)
    items = b.set(mixed)
    for rep in range(3):
        b.launch()
        bi, bc = b.wait()
        for it, r, i, c in zip(items, ref, bi, bc):
            assert np.array_equal(it["jr"].cpu().numpy(), r[0]) and np.array_equal(it["jo"].cpu().numpy(), r[1])
            J = r[0].astype(np.int64) + r[1]
            assert c == J.min() and i == int(np.flatnonzero(J == J.min())[0])
        torch.cuda.synchronize()
    # a smaller, different set in the same graph
    sub = [mixed[k] for k in (6, 2, 0)]
    items = b.set(sub)
    b.launch()
    bi, bc = b.wait()
    for it, k, i, c in zip(items, (6, 2, 0), bi, bc):
        r = ref[k]
        assert np.array_equal(it["jr"].cpu().numpy(), r[0]) and np.array_equal(it["jo"].cpu().numpy(), r[1])
        J = r[0].astype(np.int64) + r[1]
        assert c == J.min() and i == int(np.flatnonzero(J == J.min())[0])
    # capacity is enforced before anything runs
    with pytest.raises(pk.PerchError):
        b.set(mixed + mixed + mixed)
    b.close()


def test_batch_invalidated_by_dropped_scene(ctx):
    say("batch invalidation")
    w = make_config(1, 3)
    sid, mids = pk.load_workload(ctx, w)
    o = w.objects[0]
    b = ctx.batch(max_items=2, max_poses=1024, max_image_pixels=320 * 240)
    b.set([{"scene": sid, "mesh": mids[0], "label": o.label, "poses": torch.from_numpy(o.poses).cuda()}])
    b.launch()
    b.wait()
    ctx.drop_scene(sid)
    with pytest.raises(pk.PerchError):
        b.launch()
    b.close()
    ctx.unload_mesh(mids[0])


def test_cfg4_subset_batched_equals_plain(ctx):
    """Eight scenes of the uneven batched workload: one graph launch for all of
    them gives the plain per-scene path's results bit for bit."""
    say("cfg4 subset")
    lib = scenes.mesh_library(0, n=16)
    ws = scenes.config4(0, n_scenes=8, library=lib)
    mids = [ctx.load_mesh(m.xyz, m.tri, m.rgb) for m in lib]
    items, plain = [], []
    for w in ws:
        sid = ctx.set_scene(w.scene.K, w.scene.depth, w.scene.rgb, delta_mm=w.delta_mm, tau_c=w.tau_c)
        polys = [torch.from_numpy(o.poses).cuda() for o in w.objects]
        bi, bc = ctx.best_poses(sid, [mids[o.mesh] for o in w.objects], [o.label for o in w.objects], polys)
        plain += list(zip(bi, bc))
        items += [{"scene": sid, "mesh": mids[o.mesh], "label": o.label, "poses": p} for o, p in zip(w.objects, polys)]
    total = sum(it["poses"].shape[0] for it in items)
    b = ctx.batch(max_items=len(items), max_poses=total, max_image_pixels=640 * 480)
    b.set(items)
    b.launch()
    bi, bc = b.wait()
    assert list(zip(bi, bc)) == plain
    b.close()


def test_tuning_never_changes_results(ctx, mixed):
    """Every autotuner candidate (work-group size, class threshold, grids,
    work order) gives the default launch's outputs bit for bit."""
    from paper_2008_00326_amd import autotune
    say("tuning invariance")
    def with_counts():
        return [dict(it, nr=torch.empty(it["poses"].shape[0], dtype=torch.int32, device="cuda"),
                     nq=torch.empty(it["poses"].shape[0], dtype=torch.int32, device="cuda")) for it in mixed]

    ctx.set_tuning(None)
    ref = [[t.cpu().numpy() for t in (o["jr"], o["jo"], o["nr"], o["nq"])] for o in ctx.score_batch(with_counts())]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for cand in autotune.candidates(ctx.tuning(), n_cu) + [{"grid": [3, 2, 1, 1], "order": 1}]:
        ctx.set_tuning(cand)
        out = ctx.score_batch(with_counts())
        torch.cuda.synchronize()
        for o, r in zip(out, ref):
            for key, a in zip(("jr", "jo", "nr", "nq"), r):
                assert np.array_equal(o[key].cpu().numpy(), a), (cand, key)
    ctx.set_tuning(None)
    with pytest.raises(pk.PerchError):
        ctx.set_tuning({"small_block": 384})
    with pytest.raises(pk.PerchError):
        ctx.set_tuning({"order": 3})


def test_scene_prepared_while_batch_runs_and_memory_reused(ctx):
    """A scene prepared on another thread while a graph batch scores, then
    dropped and replaced without any device-wide wait: every result equals
    the one computed in isolation."""
    import threading
    say("concurrent prep / reuse")
    w2 = make_config(2, 1)
    w3 = make_config(3, 1)
    sid2, mids2 = pk.load_workload(ctx, w2)
    o = w2.objects[0]
    poses2 = torch.from_numpy(o.poses[:3000]).cuda()
    ref2 = alone(ctx, {"scene": sid2, "mesh": mids2[o.mesh], "label": o.label, "poses": poses2})
    # reference of the second scene, prepared with nothing else running
    sid3, mids3 = pk.load_workload(ctx, w3)
    objs3 = [(mids3[q.mesh], q.label, torch.from_numpy(q.poses[:256]).cuda()) for q in w3.objects]
    ref3 = ctx.best_poses(sid3, [m for m, _, _ in objs3], [l for _, l, _ in objs3], [p for _, _, p in objs3])
    ctx.drop_scene(sid3)
    b = ctx.batch(max_items=2, max_poses=4096, max_image_pixels=640 * 480)
    items = b.set([{"scene": sid2, "mesh": mids2[o.mesh], "label": o.label, "poses": poses2}])
    side = torch.cuda.Stream()
    got = {}

    def prep():
        s3 = w3.scene
        got["sid"] = ctx.set_scene(s3.K, s3.depth, s3.rgb, delta_mm=w3.delta_mm, tau_c=w3.tau_c)

    for rep in range(3):
        with torch.cuda.stream(side):
            b.launch(side)
        t = threading.Thread(target=prep)
        t.start()
        b.wait()
        t.join()
        assert np.array_equal(items[0]["jr"].cpu().numpy(), ref2[0]) and np.array_equal(items[0]["jo"].cpu().numpy(), ref2[1])
        res = ctx.best_poses(got["sid"], [m for m, _, _ in objs3], [l for _, l, _ in objs3], [p for _, _, p in objs3])
        assert [list(r) for r in res] == [list(r) for r in ref3], rep
        ctx.drop_scene(got["sid"])     # released without a wait; the next prep may reuse its memory
    b.close()
    ctx.drop_scene(sid2)


def test_scene_prepared_while_a_batch_runs(ctx):
    """A scene set while one of the context's batches runs has its neighbour
    table counted on the host (set_scene refuses it if the device's own count
    differs): the same table size, and the same scores, as the same scene set
    while the device is idle."""
    say("scene prepared while a batch runs")
    w = make_config(2, 0)
    sid, mids = pk.load_workload(ctx, w)
    items = [{"scene": sid, "mesh": mids[o.mesh], "label": o.label, "poses": torch.from_numpy(o.poses).cuda()}
             for o in w.objects]
    b = ctx.batch(64, 65536, 640 * 480)
    b.set(items + items)                                   # 64,000 poses: tens of milliseconds of work
    w2 = make_config(2, 1)
    s2 = w2.scene
    torch.cuda.synchronize()
    b.launch()
    busy = ctx.set_scene(s2.K, s2.depth, s2.rgb, delta_mm=w2.delta_mm, tau_c=w2.tau_c)
    b.wait()
    idle = ctx.set_scene(s2.K, s2.depth, s2.rgb, delta_mm=w2.delta_mm, tau_c=w2.tau_c)
    ib, ii = ctx.scene_info(busy), ctx.scene_info(idle)
    say(f"table entries {ib['table_entries']} (host count: {ib['table_counted_on_host']}) / {ii['table_entries']}")
    assert ib["table_counted_on_host"] == 1 and ii["table_counted_on_host"] == 0
    assert ib["table_entries"] == ii["table_entries"] > 0
    mids2 = [ctx.load_mesh(m.xyz, m.tri, m.rgb) for m in w2.meshes]
    for o in w2.objects:
        p = torch.from_numpy(o.poses[:2000]).cuda()
        a = ctx.score_poses(busy, mids2[o.mesh], p, label=o.label)
        c = ctx.score_poses(idle, mids2[o.mesh], p, label=o.label)
        torch.cuda.synchronize()
        for x, y in zip(a, c):
            assert torch.equal(x, y)
    b.close()
    for s_ in (sid, busy, idle):
        ctx.drop_scene(s_)
    for m in mids + mids2:
        ctx.unload_mesh(m)
