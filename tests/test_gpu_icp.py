"""GPU parity of the ICP refinement (Sec. IV-A "Parallel M2M GICP"; the
point-to-point ICP of Sec. VI-A) against the oracle.

Both sides map the source points in binary64, round them to 1/16 mm, match
in exact integers, sum exactly in int64 and update with the same sequence of
+ - * / and sqrt, so refined poses, update counts and match counts are
expected bit for bit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd.workloads import make_config  # noqa: E402
from random_cases import random_case  # noqa: E402
from tiny_meshes import TScene, box, pose_matrix, rot_x  # noqa: E402

THREADS = 16


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


def gpu_refine(ctx, sid, mid, poses, label=0, **kw):
    t = torch.from_numpy(np.ascontiguousarray(poses, np.float32)).cuda()
    r, it, mt = ctx.refine_poses(sid, mid, t, label=label, **kw)
    torch.cuda.synchronize()
    return r.cpu().numpy(), it.cpu().numpy(), mt.cpu().numpy()


def check(got, exp, what):
    r, it, mt = got
    er, eit, emt = exp
    assert np.array_equal(mt, emt), f"{what}: matches differ at {np.flatnonzero(mt != emt)[:8]}"
    assert np.array_equal(it, eit), f"{what}: updates differ at {np.flatnonzero(it != eit)[:8]}"
    assert np.array_equal(r, er), f"{what}: refined poses differ by up to {np.abs(r - er).max()}"


@pytest.mark.parametrize("seed", range(10))
def test_random_case_icp_matches_oracle(ctx, seed):
    mesh, scene, poses, p = random_case(seed)
    rng = np.random.default_rng(500 + seed)
    prm = dict(rho_mm=float(rng.choice([5.0, 15.0, 40.0])), iterations=int(rng.choice([1, 4, 12])),
               stride=int(rng.choice([1, 2, 3])), dof=int(rng.choice([3, 6])), min_points=8)
    say(f"icp case {seed}: image {scene.K[0]}x{scene.K[1]}, {mesh.tri.shape[0]} tris, {p}, {prm}")
    sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                        mark_occluders=p["occl"], stride=p["stride"])
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    poses = poses[:16]
    got = gpu_refine(ctx, sid, mid, poses, **prm)
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)
    exp = oracle.icp(mesh, scene, poses, delta_mm=p["delta"], flags=oracle.MARK_OCCLUDERS if p["occl"] else 0,
                     rho_mm=prm["rho_mm"], iterations=prm["iterations"], stride=prm["stride"], dof=prm["dof"],
                     min_points=prm["min_points"], threads=THREADS)
    check(got, exp, f"case {seed}")
    assert exp[2].sum() > 0


@pytest.mark.parametrize("dof,volume", [(3, "aabb"), (6, "aabb"), (3, "label")])
def test_cfg2_sampled_icp(ctx, dof, volume):
    """640x480 cfg2 scene: the true pose and two candidates per object,
    refined on the GPU and by the oracle; with label volumes the target is
    the object's labelled pixels."""
    w = make_config(2, 0)
    s = w.scene
    say(f"cfg2 icp sample, dof {dof}, {volume}")
    lab = s.labels if volume == "label" else None
    sid = ctx.set_scene(s.K, s.depth, s.rgb, lab, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True, volume=volume)
    oflags = oracle.MARK_OCCLUDERS | (oracle.VOL_LABEL if volume == "label" else 0)
    rng = np.random.default_rng(30 + dof)
    for o in w.objects:
        m = w.meshes[o.mesh]
        mid = ctx.load_mesh(m.xyz, m.tri, m.rgb)
        poses = np.concatenate([o.gt_pose[None], o.poses[rng.choice(o.poses.shape[0], 2, replace=False)]])
        got = gpu_refine(ctx, sid, mid, poses, label=o.label, rho_mm=20.0, iterations=8, stride=2, dof=dof)
        exp = oracle.icp(m, TScene(s.K, s.depth, None, lab), poses, delta_mm=w.delta_mm, flags=oflags,
                         label=o.label, rho_mm=20.0, iterations=8, stride=2, dof=dof, threads=THREADS)
        check(got, exp, f"cfg2 dof {dof} {volume} object {o.label}")
        ctx.unload_mesh(mid)
    ctx.drop_scene(sid)


def test_refine_then_rescore_cfg2(ctx):
    """Refine the cfg2 candidates nearest each true pose against the object's
    labelled pixels (the segmented pipeline of Sec. V-C), render and score the
    refined poses: the cost falls for most of them, and the launch is
    deterministic."""
    w = make_config(2, 0)
    w.volume = "label"
    say("cfg2 refine + rescore")
    sid, mids = pk.load_workload(ctx, w)
    for o in w.objects:
        P = o.poses.reshape(-1, 3, 4)
        near = np.argsort(np.linalg.norm(P[:, :, 3] - o.gt_pose.reshape(3, 4)[:, 3], axis=1))[:200]
        t = torch.from_numpy(np.ascontiguousarray(o.poses[near])).cuda()
        r1, it1, mt1 = ctx.refine_poses(sid, mids[o.mesh], t, label=o.label, rho_mm=30.0, iterations=10, stride=2,
                                        dof=3)
        r2, _, _ = ctx.refine_poses(sid, mids[o.mesh], t, label=o.label, rho_mm=30.0, iterations=10, stride=2, dof=3)
        jr0, jo0, _, _ = ctx.score_poses(sid, mids[o.mesh], t, label=o.label)
        jr1, jo1, _, _ = ctx.score_poses(sid, mids[o.mesh], r1, label=o.label)
        torch.cuda.synchronize()
        assert torch.equal(r1, r2)
        j0 = (jr0 + jo0).cpu().numpy()
        j1 = (jr1 + jo1).cpu().numpy()
        assert np.mean(j1 < j0) > 0.5, (o.label, np.mean(j1 < j0))
        assert np.median(j1) < np.median(j0)
        assert int(it1.cpu().numpy().max()) > 1
    ctx.drop_scene(sid)
    for mid in mids:
        ctx.unload_mesh(mid)


def test_icp_edges(ctx):
    K = (96, 72, 110.0, 110.0, 48.0, 36.0)
    cube = box((-20, -20, 0), (20, 20, 40), n=2, rgb_seed=1)
    gt = pose_matrix(rot_x(2.4), (0, 0, 500))
    d, _, c = oracle.render(cube, gt, K)
    sid = ctx.set_scene(K, d, c, delta_mm=5.0, mark_occluders=False)
    mid = ctx.load_mesh(cube.xyz, cube.tri, cube.rgb)
    # nothing within reach: unchanged, bit for bit
    far = pose_matrix(rot_x(2.4), (0, 0, 700)).astype(np.float32)[None]
    r, it, mt = gpu_refine(ctx, sid, mid, far, rho_mm=20.0, iterations=5, stride=1, dof=6)
    assert it[0] == 0 and mt[0] == 0 and np.array_equal(r, far.reshape(1, 12))
    # the true pose stays within a rounding of itself
    r, it, mt = gpu_refine(ctx, sid, mid, gt[None], rho_mm=10.0, iterations=5, stride=1, dof=3)
    assert np.abs(r - gt.reshape(1, 12)).max() < 0.05 and mt[0] > 0
    # empty input and invalid parameters
    e = torch.empty((0, 12), dtype=torch.float32, device="cuda")
    out, _, _ = ctx.refine_poses(sid, mid, e)
    assert out.shape == (0, 12)
    t = torch.from_numpy(gt[None].astype(np.float32)).cuda()
    for bad in (dict(rho_mm=0.0), dict(rho_mm=101.0), dict(dof=4), dict(iterations=0), dict(stride=0),
                dict(min_points=2)):
        with pytest.raises(pk.PerchError):
            ctx.refine_poses(sid, mid, t, **bad)
    with pytest.raises(pk.PerchError):
        ctx.refine_poses(sid + 1000, mid, t)
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)


# ------------------------------------------------------------------ GICP

@pytest.mark.parametrize("seed", range(8))
def test_random_case_gicp_matches_oracle(ctx, seed):
    """Plane-to-plane GICP: refined poses, update and match counts equal the
    oracle's (readings G1-G6: integer normals, exact fixed-point sums)."""
    mesh, scene, poses, p = random_case(seed)
    rng = np.random.default_rng(700 + seed)
    prm = dict(rho_mm=float(rng.choice([8.0, 20.0, 40.0])), iterations=int(rng.choice([1, 5, 12])),
               stride=int(rng.choice([1, 2])), min_points=8)
    say(f"gicp case {seed}: image {scene.K[0]}x{scene.K[1]}, {mesh.tri.shape[0]} tris, {p}, {prm}")
    sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                        mark_occluders=p["occl"], stride=p["stride"])
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    poses = poses[:16]
    got = gpu_refine(ctx, sid, mid, poses, dof=6, method="plane", **prm)
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)
    exp = oracle.gicp(mesh, scene, poses, delta_mm=p["delta"], flags=oracle.MARK_OCCLUDERS if p["occl"] else 0,
                      threads=THREADS, **prm)
    check(got, exp, f"gicp case {seed}")


@pytest.mark.parametrize("volume", ["aabb", "label"])
def test_cfg2_sampled_gicp(ctx, volume):
    w = make_config(2, 0)
    s = w.scene
    say(f"cfg2 gicp sample, {volume}")
    lab = s.labels if volume == "label" else None
    sid = ctx.set_scene(s.K, s.depth, s.rgb, lab, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True, volume=volume)
    oflags = oracle.MARK_OCCLUDERS | (oracle.VOL_LABEL if volume == "label" else 0)
    rng = np.random.default_rng(41)
    for o in w.objects:
        m = w.meshes[o.mesh]
        mid = ctx.load_mesh(m.xyz, m.tri, m.rgb)
        poses = np.concatenate([o.gt_pose[None], o.poses[rng.choice(o.poses.shape[0], 2, replace=False)]])
        got = gpu_refine(ctx, sid, mid, poses, label=o.label, rho_mm=20.0, iterations=8, stride=2, dof=6,
                         method="plane")
        exp = oracle.gicp(m, TScene(s.K, s.depth, None, lab), poses, delta_mm=w.delta_mm, flags=oflags,
                          label=o.label, rho_mm=20.0, iterations=8, stride=2, threads=THREADS)
        check(got, exp, f"cfg2 gicp {volume} object {o.label}")
        ctx.unload_mesh(mid)
    ctx.drop_scene(sid)


def test_gicp_needs_six_dof(ctx):
    K = (96, 72, 110.0, 110.0, 48.0, 36.0)
    cube = box((-20, -20, 0), (20, 20, 40), n=2, rgb_seed=1)
    gt = pose_matrix(rot_x(2.4), (0, 0, 500))
    d, _, c = oracle.render(cube, gt, K)
    sid = ctx.set_scene(K, d, c, delta_mm=5.0)
    mid = ctx.load_mesh(cube.xyz, cube.tri, cube.rgb)
    t = torch.from_numpy(gt[None].astype(np.float32)).cuda()
    with pytest.raises(pk.PerchError):
        ctx.refine_poses(sid, mid, t, dof=3, method="plane")
    with pytest.raises(ValueError):
        ctx.refine_poses(sid, mid, t, method="surface")
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)


@pytest.mark.parametrize("method", ["point", "plane"])
def test_device_tile_refinement_matches_oracle(ctx, method):
    """Poses 200 mm from the camera over a 320x240 image: the raster tile
    exceeds the LDS, so the ICP kernel renders into its device-memory tile;
    refined poses, update and match counts equal the oracle's."""
    from test_oracle_icp import K_HI, _scene_and_gt, _yaw_shift
    m, _, gt = _scene_and_gt(0, K_HI)
    P = gt.reshape(12).astype(np.float32).copy()
    P[11] = 200.0
    d, _, c = oracle.render(m, P, K_HI)
    scene = TScene(K_HI, d, c, None)
    starts = np.stack([_yaw_shift(P, 0.03, 2.0, -1.5), _yaw_shift(P, -0.02, -1.5, 1.0)]).astype(np.float32)
    say(f"icp device tile: {method}, {int((d > 0).sum())} observed points")
    sid = ctx.set_scene(K_HI, d, c, delta_mm=5.0, mark_occluders=False)
    mid = ctx.load_mesh(m.xyz, m.tri, m.rgb)
    prm = dict(rho_mm=10.0, iterations=5, stride=2, dof=6)
    got = gpu_refine(ctx, sid, mid, starts, method=method, **prm)
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)
    run = oracle.gicp if method == "plane" else oracle.icp
    kw = {} if method == "plane" else {"dof": 6}
    exp = run(m, scene, starts, delta_mm=5.0, flags=0, rho_mm=10.0, iterations=5, stride=2, threads=THREADS, **kw)
    check(got, exp, f"device tile {method}")
    assert exp[2].min() > 1000 and exp[1].min() >= 1
