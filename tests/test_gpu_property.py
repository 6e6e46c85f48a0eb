"""Seeded random cases against the oracle: small procedural meshes, random
intrinsics, image sizes, delta, tau_c, flags and strides, an occluded scene
with sensor noise, and candidate poses spread around the true one.  L, Q and
every depth-only count are bit-exact; counts with the colour term are within
0.1 % of the points per pose."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2008_00326_amd as pk  # noqa: E402
from paper_2008_00326_amd.workloads import meshes  # noqa: E402
from tiny_meshes import TScene, box, pose_matrix, rot_x, rot_z  # noqa: E402

CASES = 24


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


def random_case(seed):
    rng = np.random.default_rng(10_000 + seed)
    kind = meshes.SHAPES[int(rng.integers(0, len(meshes.SHAPES)))]
    mesh = meshes.make_shape(kind, int(rng.integers(60, 900)), rng).with_colours(rng, name=f"{kind}_{seed}")
    W, H = int(rng.integers(40, 200)), int(rng.integers(30, 160))
    f = float(rng.uniform(0.6, 1.6) * W)
    K = (W, H, f * float(rng.uniform(0.9, 1.1)), f, W / 2 + float(rng.uniform(-5, 5)), H / 2 + float(rng.uniform(-5, 5)))
    z = float(rng.uniform(350, 1200))
    R = rot_z(rng.uniform(0, 2 * np.pi)) @ rot_x(rng.uniform(-0.8, 0.8))
    gt = pose_matrix(R, (rng.uniform(-30, 30), rng.uniform(-30, 30), z))
    d, _, c = oracle.render(mesh, gt, K)
    # an occluding box in front of part of the object
    occ = box((-25, -25, -10), (25, 25, 10), n=1, rgb_seed=int(seed))
    od, _, oc = oracle.render(occ, pose_matrix(np.eye(3), (rng.uniform(-60, 60), rng.uniform(-60, 60), z - 150)), K)
    front = (od > 0) & ((d == 0) | (od < d))
    d = np.where(front, od, d)
    c = np.where(front[..., None], oc, c)
    # sensor noise on valid depths and on colour
    valid = d > 0
    d = np.where(valid, np.clip(np.rint(d + rng.normal(0, 2.0, d.shape)), 1, 65534), 0).astype(np.uint16)
    c = np.clip(np.rint(c + rng.normal(0, 5.0, c.shape)), 0, 255).astype(np.uint8)
    poses = []
    for _ in range(48):
        dR = rot_z(rng.normal(0, 0.3)) @ rot_x(rng.normal(0, 0.2))
        poses.append(pose_matrix(dR @ R, gt.reshape(3, 4)[:, 3] + rng.normal(0, [25, 25, 40])))
    poses = np.stack(poses).astype(np.float32)
    params = dict(delta=float(rng.uniform(3, 30)), tau=float(rng.uniform(5, 40)), rgb=bool(rng.integers(0, 2)),
                  occl=bool(rng.integers(0, 4) > 0), stride=int(rng.choice([1, 1, 2, 3])))
    return mesh, TScene(K, d, c, None), poses, params


@pytest.mark.parametrize("seed", range(CASES))
def test_random_case_matches_oracle(ctx, seed):
    mesh, scene, poses, p = random_case(seed)
    say(f"case {seed}: image {scene.K[0]}x{scene.K[1]}, {mesh.tri.shape[0]} tris, {p}")
    sid = ctx.set_scene(scene.K, scene.depth, scene.rgb, delta_mm=p["delta"], tau_c=p["tau"], use_rgb=p["rgb"],
                        mark_occluders=p["occl"], stride=p["stride"])
    mid = ctx.load_mesh(mesh.xyz, mesh.tri, mesh.rgb)
    t = torch.from_numpy(poses).cuda()
    jr, jo, nr, nq = ctx.score_poses(sid, mid, t)
    torch.cuda.synchronize()
    got = [a.cpu().numpy() for a in (jr, jo, nr, nq)]
    ctx.drop_scene(sid)
    ctx.unload_mesh(mid)
    flags = (oracle.USE_RGB if p["rgb"] else 0) | (oracle.MARK_OCCLUDERS if p["occl"] else 0)
    exp = oracle.score(mesh, scene, poses, delta_mm=p["delta"], tau_c=p["tau"], flags=flags, stride=p["stride"],
                       threads=8)
    assert np.array_equal(got[2], exp[2]), f"L differs at {np.flatnonzero(got[2] != exp[2])[:8]}"
    assert np.array_equal(got[3], exp[3]), f"Q differs at {np.flatnonzero(got[3] != exp[3])[:8]}"
    if p["rgb"]:
        assert np.all(np.abs(got[0] - exp[0]) <= np.ceil(0.001 * exp[2]))
        assert np.all(np.abs(got[1] - exp[1]) <= np.ceil(0.001 * exp[3]))
    else:
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1])
    assert exp[2].sum() > 0    # the cases render something
