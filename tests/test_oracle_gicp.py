"""Pins for the oracle's plane-to-plane GICP (CPU; Sec. IV-A "Parallel M2M
GICP"; readings G1-G6 of the oracle source).

Normals of a rendered plane are its analytic normal; pixels next to a depth
step have none.  Without normals the update is the point-to-point
Gauss-Newton step, which reaches scipy's least-squares alignment; with exact
correspondences and consistent normals it recovers the transform.  Where the
matches slide along the surfaces (the error point-to-point ICP suffers
from), the plane model still recovers the motion across them.  On rendered
scenes GICP brings perturbed poses back towards the truth, and its first
matches are ICP's.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from tiny_meshes import TScene, box, pose_matrix, rot_x, rot_z
from test_oracle_icp import K_HI, _pose_error, _scene_and_gt, _yaw_shift


def _cloud(rng, n=400, centre=(300.0, -200.0, 12800.0), half=4000.0):
    return np.rint(np.asarray(centre) + rng.uniform(-half, half, (n, 3))).astype(np.int32)


def test_normals_of_a_rendered_plane():
    K = (160, 120, 150.0, 150.0, 80.0, 60.0)
    quad = box((-200, -200, 0), (200, 200, 1), n=8)
    R = rot_x(2.6) @ rot_z(0.3)
    pose = pose_matrix(R, (10, -5, 700))
    depth, _, _ = oracle.render(quad, pose, K)
    nrm = oracle.normal_image(depth, K, 20)
    n_true = R[:, 2] / np.linalg.norm(R[:, 2])          # the quad's top face normal in the camera frame
    has = np.isfinite(nrm).all(-1)
    assert has.sum() > 1000
    cos = np.abs(nrm[has] @ n_true)
    assert np.percentile(cos, 5) > 0.995               # 1/16 mm rounding tilts a few normals slightly
    # no normal at the silhouette: a neighbour without a reading
    edge = (depth > 0) & ~has
    assert edge.sum() > 0
    rows, cols = np.nonzero(edge)
    for r, c in zip(rows[:50], cols[:50]):
        nb = [depth[r, c - 1] if c > 0 else 0, depth[r, c + 1] if c + 1 < K[0] else 0,
              depth[r - 1, c] if r > 0 else 0, depth[r + 1, c] if r + 1 < K[1] else 0]
        assert min(nb) == 0 or max(abs(int(x) - int(depth[r, c])) for x in nb) > 20


@pytest.mark.parametrize("seed", range(3))
def test_without_normals_reaches_least_squares(seed):
    rng = np.random.default_rng(seed)
    src = _cloud(rng)
    R = Rotation.from_rotvec(rng.normal(0, 0.12, 3)).as_matrix()
    t = rng.normal(0, 120.0, 3)
    dst = np.rint(src @ R.T + t + rng.normal(0, 2.0, src.shape)).astype(np.int32)
    A, b = oracle.gicp_pairs(src, dst, iterations=8)
    ms, md = src.mean(0), dst.mean(0)
    Rs, _ = Rotation.align_vectors(dst - md, src - ms)
    Rs = Rs.as_matrix()
    assert np.abs(A - Rs).max() < 2e-5
    r_opt = np.sum((src @ Rs.T + (md - Rs @ ms) - dst) ** 2)
    r_got = np.sum((src @ A.T + b - dst) ** 2)
    assert r_opt <= r_got <= r_opt * 1.001


@pytest.mark.parametrize("seed", range(3))
def test_exact_pairs_with_normals_recover_the_motion(seed):
    rng = np.random.default_rng(10 + seed)
    src = _cloud(rng)
    R = Rotation.from_rotvec(rng.normal(0, 0.15, 3)).as_matrix()
    t = rng.normal(0, 150.0, 3)
    dst = np.rint(src @ R.T + t).astype(np.int32)
    n = rng.normal(size=src.shape)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n[::7] = np.nan                                     # some points without a normal
    A, b = oracle.gicp_pairs(src, dst, n, n @ R.T, iterations=8)
    assert np.abs(A - R).max() < 2e-5 and np.abs(b - t).max() < 0.5


def test_plane_model_resists_sliding_matches():
    # two perpendicular planes (x = 0 and y = 0, 100 mm each); each match slides
    # up to 3 mm within its plane, as nearest neighbours on a moved surface do
    rng = np.random.default_rng(3)
    m = 300
    a = np.stack([np.zeros(m), rng.uniform(-800, 800, m), rng.uniform(-800, 800, m)], 1)
    c = np.stack([rng.uniform(-800, 800, m), np.zeros(m), rng.uniform(-800, 800, m)], 1)
    pts = np.concatenate([a, c]) + np.array([200.0, -100.0, 12000.0])
    nrm = np.concatenate([np.tile([1.0, 0, 0], (m, 1)), np.tile([0, 1.0, 0], (m, 1))])
    t = np.array([24.0, -40.0, 0.0])                     # 1.5 and 2.5 mm across the two planes
    slide = rng.uniform(-48, 48, pts.shape) * (1 - np.abs(nrm))
    src = np.rint(pts).astype(np.int32)
    dst = np.rint(pts + t + slide).astype(np.int32)
    _, b_plane = oracle.gicp_pairs(src, dst, nrm, nrm, iterations=6)
    _, b_point = oracle.gicp_pairs(src, dst, iterations=6)
    err_plane = np.abs(b_plane[:2] - t[:2]).max()
    err_point = np.abs(b_point[:2] - t[:2]).max()
    assert err_plane < 0.5 and err_plane < err_point / 3, (err_plane, err_point)


@pytest.mark.parametrize("seed", range(2))
def test_gicp_returns_perturbed_poses_to_truth(seed):
    m, scene, gt = _scene_and_gt(seed, K_HI)
    starts = np.stack([_yaw_shift(gt, 0.05, 4.0, -3.0), _yaw_shift(gt, -0.04, -5.0, 2.0)])
    out, it, mt = oracle.gicp(m, scene, starts, delta_mm=5.0, rho_mm=15.0, iterations=30, stride=1, flags=0,
                              threads=8)
    for k in range(starts.shape[0]):
        e0 = _pose_error(starts[k], gt)
        e1 = _pose_error(out[k], gt)
        assert e1[0] < 0.3 * e0[0] and e1[1] < 0.6 * e0[1], (k, e0, e1)
        assert it[k] >= 3 and mt[k] > 1000


def test_gicp_first_matches_are_icps():
    m, scene, gt = _scene_and_gt(4)
    rng = np.random.default_rng(5)
    poses = np.stack([_yaw_shift(gt, rng.normal(0, 0.1), *rng.normal(0, 6.0, 2)) for _ in range(4)])
    _, _, m1 = oracle.icp(m, scene, poses, delta_mm=5.0, rho_mm=12.0, iterations=1, stride=2, dof=6)
    _, _, m2 = oracle.gicp(m, scene, poses, delta_mm=5.0, rho_mm=12.0, iterations=1, stride=2)
    assert np.array_equal(m1, m2) and m1.sum() > 0
