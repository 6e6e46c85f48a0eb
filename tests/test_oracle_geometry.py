"""Pins for the oracle's rasterizer and back-projection (CPU only).

Each test checks the oracle against something fixed outside it: analytic
pixel sets of a cube, a ray-plane depth, coverage partitions and exact
rational back-projections.  The readings (fill rule, pixel centres, depth
buffer) are those listed in the oracle's header.
"""
import numpy as np
import pytest

import oracle
from tiny_meshes import TMesh, box, pose_matrix, rot_x, rot_y, rot_z

K128 = (128, 128, 500.0, 500.0, 64.0, 64.0)


def test_cube_front_face_exact_pixel_set():
    # 100 mm cube, front face at Z = 1000 mm: u spans [39, 89]; the left/top
    # edges lie on pixel centres and are inside, the right/bottom are outside.
    cube = box((-50, -50, -50), (50, 50, 50))
    depth, tri, _ = oracle.render(cube, pose_matrix(np.eye(3), (0, 0, 1050)), K128)
    expect = np.zeros((128, 128), bool)
    expect[39:89, 39:89] = True
    assert np.array_equal(depth > 0, expect)
    assert (depth > 0).sum() == 2500
    assert np.all(depth[expect] == 1000)
    assert np.all(tri[~expect] == -1)


def test_cube_rotated_about_optical_axis_same_set():
    cube = box((-50, -50, -50), (50, 50, 50))
    R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    depth, _, _ = oracle.render(cube, pose_matrix(R, (0, 0, 1050)), K128)
    expect = np.zeros((128, 128), bool)
    expect[39:89, 39:89] = True
    assert np.array_equal(depth > 0, expect)
    assert np.all(depth[expect] == 1000)


@pytest.mark.parametrize("half", [50.3, 49.7, 37.1, 12.45])
def test_cube_non_integer_edges_count_strict_interior(half):
    cube = box((-half, -half, -half), (half, half, half))
    depth, _, _ = oracle.render(cube, pose_matrix(np.eye(3), (0, 0, 1000 + half)), K128)
    h32 = float(np.float32(half))
    z = float(np.float32(1000 + half)) - h32
    lo, hi = 64 - 500 * h32 / z, 64 + 500 * h32 / z
    cols = [i for i in range(128) if lo < i < hi]
    assert (depth > 0).sum() == len(cols) ** 2
    ys, xs = np.nonzero(depth)
    assert xs.min() == cols[0] and xs.max() == cols[-1]


def test_back_faces_and_behind_camera_are_culled():
    cube = box((-50, -50, -50), (50, 50, 50))
    # camera inside the cube: every face is seen from behind
    depth, _, _ = oracle.render(cube, pose_matrix(np.eye(3), (0, 0, 0)), K128)
    assert depth.sum() == 0
    # whole object behind the near plane
    depth, _, _ = oracle.render(cube, pose_matrix(np.eye(3), (0, 0, -500)), K128)
    assert depth.sum() == 0


def _single(tri_xyz):
    return TMesh(np.asarray(tri_xyz, np.float32).reshape(-1, 3), np.arange(len(tri_xyz), dtype=np.int32).reshape(-1, 3))


def test_top_left_rule_on_pixel_centre_edges():
    # Right triangle with a horizontal top edge and a vertical left edge that
    # both run through pixel centres (Z = 1000, f = 500, so 2 mm = 1 px).
    # Screen corners (40, 40), (40, 60), (60, 40): top and left edges inside,
    # hypotenuse through centres excluded (it is a right/bottom edge).
    def P(u, v):
        return ((u - 64) * 2.0, (v - 64) * 2.0, 0.0)
    m = TMesh(np.array([P(40, 40), P(40, 60), P(60, 40)], np.float32), np.array([[0, 1, 2]], np.int32))
    A = oracle.render(m, pose_matrix(np.eye(3), (0, 0, 1000)), K128)[0] > 0
    if A.sum() == 0:  # winding seen from the camera is clockwise: flip it
        m = TMesh(m.xyz, np.array([[0, 2, 1]], np.int32))
        A = oracle.render(m, pose_matrix(np.eye(3), (0, 0, 1000)), K128)[0] > 0
    expect = np.zeros_like(A)
    for j in range(40, 61):
        for i in range(40, 61):
            if (i - 40) + (j - 40) < 20:
                expect[j, i] = True
    assert np.array_equal(A, expect)


def _random_quad(rng):
    # convex quad in the plane Z = 900..1100, well inside the view
    c = rng.uniform(-80, 80, size=2)
    ang = np.sort(rng.uniform(0, 2 * np.pi, size=4))
    r = rng.uniform(20, 60, size=4)
    pts = [(c[0] + r[k] * np.cos(ang[k]), c[1] + r[k] * np.sin(ang[k]), rng.uniform(900, 1100)) for k in range(4)]
    return np.asarray(pts, np.float32)


@pytest.mark.parametrize("seed", range(12))
def test_shared_edge_watertight(seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        q = _random_quad(rng)
        # try both windings; keep the front-facing one
        for order in ([0, 1, 2, 0, 2, 3], [0, 2, 1, 0, 3, 2]):
            t = np.asarray(order, np.int32).reshape(2, 3)
            full = TMesh(q, t)
            d, tri, _ = oracle.render(full, pose_matrix(np.eye(3), (0, 0, 0)), K128)
            if (d > 0).sum() > 0:
                break
        a = oracle.render(TMesh(q, t[:1]), pose_matrix(np.eye(3), (0, 0, 0)), K128)[0] > 0
        b = oracle.render(TMesh(q, t[1:]), pose_matrix(np.eye(3), (0, 0, 0)), K128)[0] > 0
        assert not np.any(a & b), "pixel covered by both triangles"
        assert np.array_equal(a | b, d > 0), "gap or extra pixel along the shared diagonal"


@pytest.mark.parametrize("seed", range(4))
def test_convex_mesh_front_faces_cover_each_pixel_once(seed):
    rng = np.random.default_rng(100 + seed)
    cube = box((-40, -30, -20), (40, 30, 20), n=3)
    R = rot_z(rng.uniform(0, 6.3)) @ rot_x(rng.uniform(0, 6.3)) @ rot_y(rng.uniform(0, 6.3))
    pose = pose_matrix(R, (rng.uniform(-40, 40), rng.uniform(-40, 40), rng.uniform(700, 900)))
    K = (96, 96, 300.0, 300.0, 48.0, 47.5)
    d, _, _ = oracle.render(cube, pose, K)
    count = np.zeros((96, 96), int)
    for t in range(cube.tri.shape[0]):
        dt = oracle.render(TMesh(cube.xyz, cube.tri[t:t + 1]), pose, K)[0]
        count += dt > 0
    assert count.max() == 1
    assert np.array_equal(count == 1, d > 0)


@pytest.mark.parametrize("seed", range(4))
def test_depth_invariant_under_triangle_permutation(seed):
    rng = np.random.default_rng(seed)
    a = box((-40, -30, 0), (40, 30, 90), n=4)
    b = box((-20, -60, 10), (30, 10, 60), n=3)
    xyz = np.concatenate([a.xyz, b.xyz])
    tri = np.concatenate([a.tri, b.tri + len(a.xyz)])
    R = rot_x(0.7) @ rot_z(rng.uniform(0, 6.3))
    pose = pose_matrix(R, (rng.uniform(-20, 20), rng.uniform(-20, 20), 800))
    d0, t0, _ = oracle.render(TMesh(xyz, tri), pose, K128)
    perm = rng.permutation(len(tri))
    d1, t1, _ = oracle.render(TMesh(xyz, tri[perm]), pose, K128)
    assert np.array_equal(d0, d1)
    # the winning fragment has the smallest (depth, index): mapping back the
    # permuted winner must give a triangle whose own depth equals d0 there
    assert np.array_equal(t0 >= 0, t1 >= 0)


def test_tilted_plane_depth_matches_ray_plane_intersection():
    # large quad in a tilted plane; depth must be rint(analytic) except near ties
    R = rot_x(0.6) @ rot_y(-0.35)
    half = 150.0
    q = np.array([[-half, -half, 0], [half, -half, 0], [half, half, 0], [-half, half, 0]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    pose = pose_matrix(R, (5, -7, 1000))
    d, _, _ = oracle.render(TMesh(q, t), pose, K128)
    if (d > 0).sum() == 0:
        t = t[:, ::-1].copy()
        d, _, _ = oracle.render(TMesh(q, t), pose, K128)
    P = pose.reshape(3, 4).astype(np.float64)
    n = P[:, :3] @ np.array([0, 0, 1.0])
    c = float(n @ P[:, 3])
    checked = 0
    for j in range(128):
        for i in range(128):
            if d[j, i] == 0:
                continue
            ray = np.array([(i - 64) / 500.0, (j - 64) / 500.0, 1.0])
            z = c / float(n @ ray)
            frac = z - np.floor(z)
            assert abs(d[j, i] - z) <= 0.52
            if abs(frac - 0.5) > 0.05:
                assert d[j, i] == int(np.rint(z)), (i, j, z)
                checked += 1
    assert checked > 5000


def test_backprojection_exact_rationals_and_half_even():
    K = (640, 480, 500.0, 500.0, 320.0, 240.0)
    # 16 (i - cx) d / fx = 16 * 25 * 1000 / 500 = 800 exactly
    assert oracle.backproject(K, 345, 240, 1000) == (800, 0, 16000)
    assert oracle.backproject(K, 295, 215, 1000) == (-800, -800, 16000)
    # fx = 256, i - cx = 1: kx = 1/16, d = 8 -> 0.5 -> 0 (even); d = 24 -> 1.5 -> 2
    K2 = (64, 64, 256.0, 256.0, 10.0, 10.0)
    assert oracle.backproject(K2, 11, 10, 8)[0] == 0
    assert oracle.backproject(K2, 11, 10, 24)[0] == 2
    assert oracle.backproject(K2, 11, 10, 40)[0] == 2
    assert oracle.backproject(K2, 9, 10, 24)[0] == -2


def test_backprojection_within_half_unit_of_real_point():
    rng = np.random.default_rng(7)
    K = (320, 240, 262.5, 262.5, 160.0, 120.0)
    for _ in range(500):
        i, j, d = int(rng.integers(0, 320)), int(rng.integers(0, 240)), int(rng.integers(1, 65535))
        x, y, z = oracle.backproject(K, i, j, d)
        assert z == 16 * d
        assert abs(x - 16 * (i - 160) * d / 262.5) <= 0.5 + 1e-6
        assert abs(y - 16 * (j - 120) * d / 262.5) <= 0.5 + 1e-6
