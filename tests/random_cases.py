"""Seeded random scoring cases shared by the GPU property tests: a small
procedural mesh, random intrinsics and image size, an occluding box, sensor
noise on depth and colour, and candidate poses spread around the true one.
No GPU and no scoring arithmetic here."""
import numpy as np

import oracle
from paper_2008_00326_amd.workloads import meshes
from tiny_meshes import TScene, box, pose_matrix, rot_x, rot_z


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
