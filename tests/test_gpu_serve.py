"""The served form on the device: requests prepared while others score,
launched in shared batches, must each get exactly the answer of scoring
their scene alone."""
import dataclasses
import sys
import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd import serve  # noqa: E402
from paper_2008_00326_amd.workloads import make_config  # noqa: E402


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


def test_served_results_equal_alone(ctx):
    pool = [small(make_config(3, 0), 160), small(make_config(2, 1), 300), small(make_config(3, 2), 200)]
    ref = [alone(ctx, w) for w in pool]
    say("references done")
    ex = serve.GpuExecutor(ctx, slots=2, max_items=64, max_poses=6000)
    srv = serve.Server(ex, budget_bytes=300 << 20, max_items=64, max_poses=6000)
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
