"""Pins for the oracle's ICP refinement (CPU only; Sec. IV-A "Parallel M2M
GICP" and the point-to-point ICP of the 3-DoF experiments, Sec. VI-A).

The update loop on fixed correspondences reaches the least-squares rigid
alignment that scipy's Rotation.align_vectors computes (6-DoF), and the
planar Procrustes solution written with atan2 (3-DoF), ignoring motion along
the axis.  On rendered scenes ICP returns perturbed poses to the true pose,
leaves the true pose where it is, matches exactly the source points that a
k-d tree finds within rho (with label volumes, among the object's labelled
points), and leaves a pose with nothing in reach unchanged.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle
from paper_2008_00326_amd.workloads import meshes
from tiny_meshes import TScene, box, pose_matrix, rot_x, rot_z

K = (120, 90, 130.0, 130.0, 60.0, 45.0)


def _cloud(rng, n=300, centre=(300.0, -200.0, 12800.0), half=800.0):
    return np.rint(np.asarray(centre) + rng.uniform(-half, half, (n, 3))).astype(np.int32)


def _axis_rotation(u, theta):
    u = np.asarray(u, np.float64)
    Kx = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return np.eye(3) + np.sin(theta) * Kx + (1 - np.cos(theta)) * (Kx @ Kx)


# ------------------------------------------------------------ fixed correspondences

@pytest.mark.parametrize("seed", range(4))
def test_pairs_6dof_reach_the_least_squares_alignment(seed):
    rng = np.random.default_rng(seed)
    src = _cloud(rng, half=4000.0)                   # a 500 mm cloud
    R = Rotation.from_rotvec(rng.normal(0, 0.12, 3)).as_matrix()
    t = rng.normal(0, 120.0, 3)
    dst = np.rint(src @ R.T + t + rng.normal(0, 2.0, src.shape)).astype(np.int32)
    A, b = oracle.icp_pairs(src, dst, dof=6, iterations=8)
    # the least-squares optimum of the same integer pairs
    ms, md = src.mean(0), dst.mean(0)
    Rs, _ = Rotation.align_vectors(dst - md, src - ms)
    Rs = Rs.as_matrix()
    ts = md - Rs @ ms
    # each update sees the mapped points rounded to 1/16 mm, which limits
    # the agreement to about that rounding over the cloud's extent
    assert np.abs(A - Rs).max() < 2e-5
    assert np.abs((A - Rs) @ ms + (b - ts)).max() < 0.5
    r_opt = np.sum((src @ Rs.T + ts - dst) ** 2)
    r_got = np.sum((src @ A.T + b - dst) ** 2)
    assert r_opt <= r_got <= r_opt * 1.001
    assert np.abs(A @ A.T - np.eye(3)).max() < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_pairs_3dof_planar_procrustes(seed):
    rng = np.random.default_rng(10 + seed)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    src = _cloud(rng)
    theta = rng.uniform(-0.5, 0.5)
    P = np.eye(3) - np.outer(u, u)
    t_plane = P @ rng.normal(0, 150.0, 3)
    R = _axis_rotation(u, theta)
    dst = np.rint(src @ R.T + t_plane + rng.normal(0, 1.5, src.shape)).astype(np.int32)
    A, b = oracle.icp_pairs(src, dst, dof=3, axis=u, iterations=1)
    # planar Procrustes with atan2: in-plane centred coordinates in a basis (e1, e2) of the plane
    e1 = np.cross(u, [1.0, 0.0, 0.0])
    if np.linalg.norm(e1) < 0.5:
        e1 = np.cross(u, [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    s2 = np.stack([(src - src.mean(0)) @ e1, (src - src.mean(0)) @ e2], 1)
    d2 = np.stack([(dst - dst.mean(0)) @ e1, (dst - dst.mean(0)) @ e2], 1)
    ang = np.arctan2(np.sum(s2[:, 0] * d2[:, 1] - s2[:, 1] * d2[:, 0]), np.sum(s2 * d2))
    Rexp = _axis_rotation(u, ang)
    assert np.abs(A - Rexp).max() < 1e-12
    assert abs(ang - theta) < 2e-3
    # the centroid moves within the plane only
    mq, mc = src.mean(0), dst.mean(0)
    moved = A @ mq + b
    assert np.abs(moved - (mq + P @ (mc - mq))).max() < 1e-6
    assert abs(np.dot(A @ mq + b - mq, u)) < 1e-6


def test_pairs_3dof_ignores_motion_along_axis():
    # an axis with an integer multiple, (3, 4, 12) / 13, so the lifted
    # matches stay exact integers
    u = np.array([3.0, 4.0, 12.0]) / 13.0
    rng = np.random.default_rng(3)
    src = _cloud(rng)
    R = _axis_rotation(u, 0.2)
    dst = np.rint(src @ R.T + rng.normal(0, 1.5, src.shape)).astype(np.int32)
    for k in (1, 7, -20):
        lift = (dst + k * np.array([3, 4, 12])).astype(np.int32)
        A, b = oracle.icp_pairs(src, dst, dof=3, axis=u, iterations=1)
        A2, b2 = oracle.icp_pairs(src, lift, dof=3, axis=u, iterations=1)
        assert np.abs(A - A2).max() < 1e-12 and np.abs(b - b2).max() < 1e-6
        # while the 6-DoF solution follows the lift
        A6, b6 = oracle.icp_pairs(src, lift, dof=6, axis=u, iterations=1)
        assert abs(np.dot(A6 @ src.mean(0) + b6 - src.mean(0) - (dst.mean(0) - src.mean(0)), u) - 13.0 * k) < 1e-6


def test_pairs_identity_when_aligned():
    rng = np.random.default_rng(5)
    src = _cloud(rng)
    for dof in (3, 6):
        A, b = oracle.icp_pairs(src, src, dof=dof, iterations=3)
        assert np.array_equal(A, np.eye(3)) and np.all(b == 0)


# ------------------------------------------------------------ rendered scenes

# Point-to-point ICP needs points several per centimetre to converge: 1.5 mm
# pixels at 600 mm.  Shapes without rotational symmetry, so yaw is observable.
K_HI = (320, 240, 400.0, 400.0, 160.0, 120.0)


def _scene_and_gt(seed, Kc=K):
    rng = np.random.default_rng(seed)
    m = meshes.make_shape(("box", "extruded_l")[seed % 2], 500, rng).with_colours(rng, name="m")
    R = rot_x(2.3) @ rot_z(rng.uniform(0, 6.28))
    gt = pose_matrix(R, (rng.uniform(-15, 15), rng.uniform(-15, 15), 600.0))
    d, _, c = oracle.render(m, gt, Kc)
    return m, TScene(Kc, d, c, None), gt


def _yaw_shift(pose, dyaw, dx, dy):
    P = pose.reshape(3, 4).astype(np.float64)
    R = P[:, :3]
    t = P[:, 3]
    # in the object's own table plane: rotate about and move normal to its z axis
    return pose_matrix(R @ rot_z(dyaw), t + R @ np.array([dx, dy, 0.0]))


def _pose_error(a, b):
    A = a.reshape(3, 4).astype(np.float64)
    B = b.reshape(3, 4).astype(np.float64)
    dR = A[:, :3] @ B[:, :3].T
    ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
    return float(np.linalg.norm(A[:, 3] - B[:, 3])), float(ang)


@pytest.mark.parametrize("seed", range(2))
def test_icp_returns_perturbed_poses_to_truth(seed):
    m, scene, gt = _scene_and_gt(seed, K_HI)
    starts = np.stack([_yaw_shift(gt, 0.05, 4.0, -3.0), _yaw_shift(gt, -0.04, -5.0, 2.0)])
    # no clutter in a self-render, and with occluder marking a hypothesis
    # behind the observed surface would lose its own points to it (I1)
    for dof in (3, 6):
        out, it, mt = oracle.icp(m, scene, starts, delta_mm=5.0, rho_mm=15.0, iterations=40, stride=1, dof=dof,
                                 flags=0, threads=8)
        for k in range(starts.shape[0]):
            e0 = _pose_error(starts[k], gt)
            e1 = _pose_error(out[k], gt)
            # point-to-point ICP slides slowly in yaw along flat faces
            assert e1[0] < 0.3 * e0[0] and e1[1] < 0.6 * e0[1], (dof, k, e0, e1)
            assert it[k] >= 5 and mt[k] > 1000


def test_icp_leaves_the_true_pose():
    m, scene, gt = _scene_and_gt(7, K_HI)
    for dof in (3, 6):
        out, it, mt = oracle.icp(m, scene, gt[None], delta_mm=5.0, rho_mm=10.0, iterations=10, stride=2, dof=dof)
        e = _pose_error(out[0], gt)
        assert e[0] < 0.1 and e[1] < 0.02, e
        assert mt[0] > 0


def test_icp_first_matches_equal_kdtree():
    m, scene, gt = _scene_and_gt(4)
    rng = np.random.default_rng(4)
    poses = np.stack([_yaw_shift(gt, rng.normal(0, 0.1), *rng.normal(0, 6.0, 2)) for _ in range(4)])
    W, H = K[0], K[1]
    obs = np.array([oracle.backproject(K, i, j, int(scene.depth[j, i]))
                    for j in range(H) for i in range(W) if scene.depth[j, i] > 0], np.float64)
    tree = cKDTree(obs)
    for rho in (3.0, 12.0):
        rq = int(np.rint(16 * rho))
        _, _, mt = oracle.icp(m, scene, poses, delta_mm=5.0, rho_mm=rho, iterations=1, stride=2, dof=3)
        for k in range(poses.shape[0]):
            d, _, _ = oracle.render(m, poses[k], K)
            src = np.array([oracle.backproject(K, i, j, int(d[j, i])) for j in range(0, H, 2) for i in range(0, W, 2)
                            if d[j, i] > 0 and not (scene.depth[j, i] > 0 and 16 * int(scene.depth[j, i]) + 80
                                                    < 16 * int(d[j, i]))], np.float64)
            dist, _ = tree.query(src, distance_upper_bound=rq + 1.0 / (4 * rq))
            assert mt[k] == int(np.isfinite(dist).sum())


def test_icp_label_target_is_the_labelled_points():
    m, scene, gt = _scene_and_gt(6)
    W, H = K[0], K[1]
    labels = np.where(np.arange(W)[None, :] < W // 2, 3, 1).astype(np.int32).repeat(H, 0)
    lscene = TScene(K, scene.depth, None, labels)
    rng = np.random.default_rng(6)
    poses = np.stack([_yaw_shift(gt, rng.normal(0, 0.1), *rng.normal(0, 6.0, 2)) for _ in range(3)])
    pts = [(oracle.backproject(K, i, j, int(scene.depth[j, i])), labels[j, i])
           for j in range(H) for i in range(W) if scene.depth[j, i] > 0]
    rq = 16 * 12
    for label in (1, 3):
        tree = cKDTree(np.array([p for p, lab in pts if lab == label], np.float64))
        _, _, mt = oracle.icp(m, lscene, poses, delta_mm=5.0, flags=oracle.VOL_LABEL, label=label, rho_mm=12.0,
                              iterations=1, stride=2, dof=3)
        for k in range(poses.shape[0]):
            d, _, _ = oracle.render(m, poses[k], K)
            src = np.array([oracle.backproject(K, i, j, int(d[j, i])) for j in range(0, H, 2) for i in range(0, W, 2)
                            if d[j, i] > 0], np.float64)
            dist, _ = tree.query(src, distance_upper_bound=rq + 1.0 / (4 * rq))
            assert mt[k] == int(np.isfinite(dist).sum())
        assert mt.sum() > 0


def test_icp_out_of_reach_is_unchanged():
    cube = box((-20, -20, 0), (20, 20, 40), n=2, rgb_seed=1)
    gt = pose_matrix(rot_x(2.4), (0, 0, 500))
    scene = TScene(K, oracle.render(cube, gt, K)[0], None, None)
    far = pose_matrix(rot_x(2.4), (0, 0, 700))      # 200 mm behind: nothing within rho
    out, it, mt = oracle.icp(cube, scene, far[None], delta_mm=5.0, rho_mm=20.0, iterations=5, stride=1, dof=6,
                             flags=0)
    assert it[0] == 0 and mt[0] == 0
    assert np.array_equal(out[0], far.astype(np.float32).reshape(12))
