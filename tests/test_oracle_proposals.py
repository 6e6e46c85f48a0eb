"""Pins for the oracle's 6-DoF pose proposals (CPU; Sec. V-B "Pose Proposal
Generation"): properties a proposal set must have, checked without the
oracle's formulas.  Rotations are proper; the viewpoints (the object-frame
direction of the camera) cover the sphere evenly; the in-plane proposals of a
viewpoint are turns about the optical axis by 2 pi k / N; every translation
projects onto the centre of the label's pixel box; the depths start at the
nearest labelled reading, step as asked and stay within the farthest, or are
spread over exactly that range when capped; all of that for the object's
centre, the centre of its mesh's box."""
import numpy as np
import pytest

import oracle
from tiny_meshes import TScene, box

MESH = box((-10, -20, 0), (30, 40, 90), n=1)       # AABB centre (10, 10, 45), off the origin

K = (160, 120, 150.0, 152.0, 79.5, 61.0)


def _scene(seed=0):
    rng = np.random.default_rng(seed)
    W, H = K[0], K[1]
    labels = np.zeros((H, W), np.int32)
    depth = rng.integers(900, 1000, (H, W)).astype(np.uint16)
    labels[30:71, 40:95] = 4                        # box x 40..94, y 30..70
    depth[30:71, 40:95] = rng.integers(612, 688, (41, 55))
    depth[35, 50] = 0                               # a missing reading under the label
    labels[100:110, 5:9] = 7
    depth[100:110, 5:9] = 0                         # label 7 has no reading at all
    return TScene(K, depth, None, labels)


def _split(P, M, N, T):
    return P.reshape(M, N, T, 3, 4).astype(np.float64)


@pytest.mark.parametrize("M,N", [(1, 1), (7, 3), (64, 12), (200, 4)])
def test_rotations_proper_and_viewpoints_cover_the_sphere(M, N):
    s = _scene()
    P = oracle.propose(s, MESH, 4, viewpoints=M, inplane=N, z_step_mm=20.0, max_depths=3)
    T = P.shape[0] // (M * N)
    assert P.shape[0] == M * N * T
    A = _split(P, M, N, T)
    R = A[..., :3]
    I = np.einsum("...ij,...kj->...ik", R, R)
    assert np.abs(I - np.eye(3)).max() < 2e-6
    assert np.abs(np.linalg.det(R) - 1).max() < 2e-6
    # the camera direction in the object frame: R^T (0, 0, -1)
    v = -R[:, 0, 0, 2, :]
    assert np.abs(np.linalg.norm(v, axis=1) - 1).max() < 2e-6
    for i in range(M):                               # the same viewpoint for every angle and depth
        assert np.abs(-R[i, :, :, 2, :] - v[i]).max() < 2e-6
    if M >= 7:
        assert np.linalg.norm(v.mean(0)) < 1.5 / M + 1e-6
        dots = np.clip(v @ v.T, -1, 1)
        np.fill_diagonal(dots, -1)
        nearest = np.arccos(dots.max(1))
        spacing = np.sqrt(4 * np.pi / M)
        assert nearest.min() > 0.5 * spacing and nearest.max() < 1.5 * spacing


def test_inplane_turns_about_the_optical_axis():
    s = _scene()
    M, N = 9, 8
    P = oracle.propose(s, MESH, 4, viewpoints=M, inplane=N, z_step_mm=30.0, max_depths=2)
    R = _split(P, M, N, P.shape[0] // (M * N))[..., :3]
    for i in range(M):
        for k in range(N):
            D = R[i, k, 0] @ R[i, 0, 0].T                # camera-frame turn from angle 0 to angle k
            assert abs(D[2, 2] - 1) < 2e-6
            ang = np.arctan2(D[1, 0], D[0, 0]) % (2 * np.pi)
            assert abs(((ang - 2 * np.pi * k / N) + np.pi) % (2 * np.pi) - np.pi) < 4e-6


@pytest.mark.parametrize("step,cap", [(10.0, 100), (7.5, 100), (10.0, 4), (1000.0, 5)])
def test_translations_on_the_box_centre_ray_over_the_depth_range(step, cap):
    s = _scene()
    P = oracle.propose(s, MESH, 4, viewpoints=3, inplane=2, z_step_mm=step, max_depths=cap)
    m = s.labels == 4
    d = s.depth[m]
    d = d[d > 0]
    zmin, zmax = float(d.min()), float(d.max())
    ys, xs = np.nonzero(m)
    uc, vc = (xs.min() + xs.max()) / 2.0, (ys.min() + ys.max()) / 2.0
    # where the object's centre lands: t + R c
    A = P.reshape(-1, 3, 4).astype(np.float64)
    t = A[:, :, 3] + A[:, :, :3] @ np.array([10.0, 10.0, 45.0])
    u = K[2] * t[:, 0] / t[:, 2] + K[4]
    v = K[3] * t[:, 1] / t[:, 2] + K[5]
    assert np.abs(u - uc).max() < 1e-3 and np.abs(v - vc).max() < 1e-3
    z = np.unique(np.round(t[:, 2], 2))            # binary32 poses: the centre depth to 0.01 mm
    assert abs(z[0] - zmin) < 1e-3 and z[-1] <= zmax + 1e-3
    n_full = int(np.floor((zmax - zmin) / step)) + 1
    if n_full <= cap:
        assert z.size == n_full and np.allclose(np.diff(z), step, atol=1e-3)
        assert zmax - z[-1] < step
    else:
        assert z.size == cap and abs(z[-1] - zmax) < 1e-3 and np.allclose(np.diff(z), (zmax - zmin) / (cap - 1), atol=1e-3)
    assert P.shape[0] == 3 * 2 * z.size


def test_no_reading_or_no_pixel_gives_nothing():
    s = _scene()
    assert oracle.propose(s, MESH, 7, viewpoints=4, inplane=4, z_step_mm=10.0, max_depths=8).shape == (0, 12)
    assert oracle.propose(s, MESH, 99, viewpoints=4, inplane=4, z_step_mm=10.0, max_depths=8).shape == (0, 12)
