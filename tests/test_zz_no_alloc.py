"""perch_score_poses_noalloc against perch_score_poses.

The allocation-free entry point scores through the same kernels with every
launch buffer in the library's per-device static scratch; its outputs must
equal perch_score_poses' bit for bit.  Two calls in a row on the same
stream, the second with fewer poses (the scratch keeps the first call's
contents), on the 640x480 RGB workload with poses of every footprint class,
including one close to the camera whose tile lies in device memory; then
the limits are refused cleanly.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd.workloads import make_config  # noqa: E402


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


def _outputs(n):
    return tuple(torch.full((n,), -7, dtype=torch.int32, device="cuda") for _ in range(4))


def _poses_every_class(ctx, sid, mid, o, rng, n_random):
    """GT pose, a pose close to the camera (large tile), one pose of each
    footprint class the plain path assigned, and n_random random candidates."""
    ctx.score_poses(sid, mid, torch.from_numpy(o.poses).cuda(), label=o.label)
    cls = ctx.last_classes(o.poses.shape[0])
    sel = [o.gt_pose[None]]
    for z in (200.0, 230.0, 260.0, 330.0, 420.0):
        near = o.gt_pose.copy()
        near[11] = z
        sel.append(near[None])
    for c in np.unique(cls):
        sel.append(o.poses[rng.choice(np.flatnonzero(cls == c), 1)])
    sel.append(o.poses[rng.choice(o.poses.shape[0], n_random, replace=False)])
    return np.ascontiguousarray(np.concatenate(sel), dtype=np.float32)


@pytest.mark.parametrize("use_rgb", [True, False])
def test_noalloc_matches_score_poses(ctx, use_rgb):
    w = make_config(2, 0)
    w.use_rgb = use_rgb
    sid, mids = pk.load_workload(ctx, w)
    rng = np.random.default_rng(77)
    stream = torch.cuda.current_stream()
    # the second call is smaller, and without key bands its large poses keep
    # their keys in the device-memory slots of class 2
    for k, n_random, bands in ((0, 3000, 2), (3, 500, 1)):
        ctx.set_tuning({"key_bands": bands})
        o = w.objects[k]
        mid = mids[o.mesh]
        poses = _poses_every_class(ctx, sid, mid, o, rng, n_random)
        n = poses.shape[0]
        say(f"noalloc rgb={use_rgb} object {o.label}: {n} poses")
        t = torch.from_numpy(poses).cuda()
        ref = ctx.score_poses(sid, mid, t, label=o.label, stream=stream)
        classes = ctx.last_classes(n, stream=stream)
        got = ctx.score_poses_noalloc(sid, mid, t, _outputs(n), label=o.label, stream=stream)
        torch.cuda.synchronize()
        for name, a, b in zip(("J_r", "J_o", "L", "Q"), got, ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(a, b), f"{name} differs at {np.flatnonzero(a != b)[:10]}"
        say(f"  bit-identical; classes {sorted(set(classes.tolist()))}")
        assert max(classes.tolist()) >= 2, "the close poses should take a device-memory class"
    ctx.set_tuning(None)
    ctx.drop_scene(sid)
    for m in mids:
        ctx.unload_mesh(m)


def test_noalloc_refuses_beyond_its_limits(ctx):
    w = make_config(1, 0)
    sid, mids = pk.load_workload(ctx, w)
    o = w.objects[0]
    big = torch.zeros((65537, 12), dtype=torch.float32, device="cuda")
    with pytest.raises(pk.PerchError, match="65536"):
        ctx.score_poses_noalloc(sid, mids[0], big, _outputs(65537), label=o.label)
    # an empty call launches nothing and succeeds
    empty = torch.zeros((0, 12), dtype=torch.float32, device="cuda")
    ctx.score_poses_noalloc(sid, mids[0], empty, _outputs(0), label=o.label)
    ctx.drop_scene(sid)
    for m in mids:
        ctx.unload_mesh(m)
