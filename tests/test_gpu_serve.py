"""The served form on the device: requests prepared while others score,
launched in shared batches, must each get exactly the answer of scoring
their scene alone -- and that answer is the oracle's minimum (Sec. IV-A,
"Parallel Search"; with the colour term, a choice that costs no more than
the oracle's optimum within the binary32 colour tolerance)."""
import dataclasses
import sys
import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd import serve  # noqa: E402
from paper_2008_00326_amd.workloads import make_config  # noqa: E402
from tiny_meshes import TMesh, TScene  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small(w, n):
    """The workload with the first n candidates of each object."""
    return dataclasses.replace(w, objects=[dataclasses.replace(o, poses=np.ascontiguousarray(o.poses[:n]))
                                           for o in w.objects])


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


def alone(ctx, w):
    sid, mids = pk.load_workload(ctx, w)
    polys = [torch.from_numpy(o.poses).cuda() for o in w.objects]
    bi, bc = ctx.best_poses(sid, [mids[o.mesh] for o in w.objects], [o.label for o in w.objects], polys)
    ctx.drop_scene(sid)
    for m in mids:
        ctx.unload_mesh(m)
    return [(int(a), int(b)) for a, b in zip(bi, bc)]


def oracle_best(w):
    """Per object: the oracle's counts of every candidate (windowed exact
    search, equal to brute force) and its minimum."""
    f = (oracle.USE_RGB if w.use_rgb else 0) | (oracle.MARK_OCCLUDERS if w.mark_occluders else 0)
    f |= {"aabb": oracle.VOL_AABB, "cyl": oracle.VOL_CYL, "label": oracle.VOL_LABEL}[w.volume]
    sc = TScene(w.scene.K, w.scene.depth, w.scene.rgb if w.use_rgb else None, w.scene.labels)
    out = []
    for o in w.objects:
        mesh = w.meshes[o.mesh]
        m = mesh if w.use_rgb else TMesh(mesh.xyz, mesh.tri, None)
        jr, jo, L, Q = oracle.score(m, sc, o.poses, delta_mm=w.delta_mm, tau_c=w.tau_c, flags=f, stride=w.stride,
                                    label=o.label, threads=0, search="window")
        out.append((jr, jo, L, Q, oracle.best(jr, jo)[:2]))
    return out


def check_against_oracle(w, answer, exp, what):
    for k, ((bi, bc), (jr, jo, L, Q, (ebi, ebc))) in enumerate(zip(answer, exp)):
        if (bi, bc) == (ebi, ebc):
            continue
        assert w.use_rgb, f"{what} object {k}: ({bi}, {bc}) against the oracle's ({ebi}, {ebc})"
        EJ = jr.astype(np.int64) + jo
        tol = np.ceil(0.001 * L) + np.ceil(0.001 * Q)
        assert abs(bc - EJ[bi]) <= tol[bi], f"{what} object {k}: cost {bc} of pose {bi}, oracle {EJ[bi]}"
        assert EJ[bi] <= ebc + tol[bi] + tol[ebi], f"{what} object {k}: pose {bi} against the oracle's {ebi}"


@pytest.fixture(scope="module")
def pool_and_ref(ctx):
    pool = [small(make_config(3, 0), 160), small(make_config(2, 1), 300), small(make_config(3, 2), 200)]
    ref = [alone(ctx, w) for w in pool]
    for k, w in enumerate(pool):
        check_against_oracle(w, ref[k], oracle_best(w), f"scene {k}")
    say("references done, equal to the oracle's minima")
    return pool, ref


@pytest.mark.parametrize("hold_s", [0.0, 0.004])
def test_served_results_equal_alone(ctx, pool_and_ref, hold_s):
    pool, ref = pool_and_ref
    ex = serve.GpuExecutor(ctx, slots=2, max_items=64, max_poses=6000)
    srv = serve.Server(ex, budget_bytes=300 << 20, max_items=64, max_poses=6000, prep_workers=2, hold_s=hold_s)
    reqs = [serve.Request(k, pool[k % 3], pool[k % 3].n_poses) for k in range(9)]

    def producer():
        for k, r in enumerate(reqs):
            srv.submit(r)
            if k % 3 == 2:
                time.sleep(0.01)
        srv.close()

    t = threading.Thread(target=producer)
    t.start()
    done = srv.run()
    t.join()
    say(f"served {len(done)} in {len(srv.batches)} launches, peak {srv.peak_bytes >> 20} MB")
    assert len(done) == 9
    for r in done:
        assert r.error is None, r.error
        assert r.result == ref[r.rid % 3], r.rid
    assert srv.peak_bytes <= 300 << 20
    assert ex.meshes.hits > 0                     # repeated scenes reuse their resident meshes
    ex.close()


def test_plain_loop_matches(ctx):
    w = small(make_config(3, 0), 128)
    ref = alone(ctx, w)
    now = time.perf_counter()
    reqs = [serve.Request(k, w, w.n_poses, arrival=now) for k in range(2)]
    done = serve.plain_loop(ctx, reqs)
    assert [r.result for r in done] == [ref, ref]


@pytest.mark.parametrize("opts", [{"jo": "nn"}, {"search": "hash"}])
def test_scene_options_follow_the_workload(ctx, opts):
    """The served form and the plain loop prepare each scene with the
    workload's own J_o rule and neighbour search, as scoring it alone does."""
    w = dataclasses.replace(small(make_config(2, 1), 96), **opts)
    ref = alone(ctx, w)
    if "jo" in opts:
        assert ref != alone(ctx, dataclasses.replace(w, jo="exact"))   # the rule changes the costs
    ex = serve.GpuExecutor(ctx, slots=2, max_items=64, max_poses=6000)
    srv = serve.Server(ex, budget_bytes=300 << 20, max_items=64, max_poses=6000)
    for k in range(3):
        srv.submit(serve.Request(k, w, w.n_poses))
    srv.close()
    done = srv.run()
    ex.close()
    assert all(r.error is None for r in done)
    assert [r.result for r in sorted(done, key=lambda r: r.rid)] == [ref] * 3
    now = time.perf_counter()
    done = serve.plain_loop(ctx, [serve.Request(k, w, w.n_poses, arrival=now) for k in range(2)])
    assert [r.result for r in done] == [ref, ref]


def test_scene_cache_serves_repeated_scenes(ctx, pool_and_ref):
    """With the scene cache a repeated scene is prepared once; every answer
    still equals scoring the scene alone, served and in the plain loop."""
    pool, ref = pool_and_ref
    ex = serve.GpuExecutor(ctx, slots=2, max_items=64, max_poses=6000, scene_cache_bytes=1 << 30)
    srv = serve.Server(ex, budget_bytes=300 << 20, max_items=64, max_poses=6000, prep_workers=2)
    for k in range(9):
        srv.submit(serve.Request(k, pool[k % 3], pool[k % 3].n_poses))
    srv.close()
    done = srv.run()
    say(f"served 9 in {len(srv.batches)} launches, scene cache {ex.scenes.misses} misses, {ex.scenes.hits} hits")
    assert len(done) == 9
    for r in done:
        assert r.error is None, r.error
        assert r.result == ref[r.rid % 3], r.rid
    assert ex.scenes.misses == 3 and ex.scenes.hits == 6
    ex.close()
    assert not ex.scenes.entries                  # closing drops the cached scenes
    cache = serve.SceneCache(ctx, 1 << 30)
    now = time.perf_counter()
    done = serve.plain_loop(ctx, [serve.Request(k, pool[k % 3], pool[k % 3].n_poses, arrival=now) for k in range(6)],
                            scenes=cache)
    assert [r.result for r in done] == [ref[k % 3] for k in range(6)]
    assert cache.misses == 3 and cache.hits == 3
    cache.clear()
    assert not cache.entries
