"""Pin of the oracle's rendered colours (its reading R5, perspective-correct
vertex colour rounded to sRGB8; Sec. IV-B renders colour alongside depth)
against an independent renderer: the binary64 ray caster of the workload
generator, which intersects the ray through each pixel centre with every
triangle (Moller-Trumbore) and interpolates the vertex colours with the
barycentric coordinates of the 3-D hit point.  At pixels inside a triangle
the two must agree to the rounding of the colour (plus the 1/256-pixel
snapping of the rasterizer's vertices).

Two negative controls, computed here from the projected vertices, show that
the comparison has the power to catch the plausible mistakes: screen-space
(affine) interpolation and a weight paired with the wrong vertex both miss
the ray caster by tens of levels on the same pixels.
"""
import numpy as np
import pytest

import oracle
from paper_2008_00326_amd.workloads import sensor
from tiny_meshes import TMesh, box, pose_matrix, rot_x, rot_z

K = (320, 240, 262.5, 262.5, 160.0, 120.0)


def _quad(a, b, c, d, colours):
    """Two triangles (a, b, c), (a, c, d) of a planar quad, wound so that
    they face the camera (positive signed area on the y-down screen)."""
    xyz = np.array([a, b, c, d], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    u = K[2] * xyz[:, 0] / xyz[:, 2]
    v = K[3] * xyz[:, 1] / xyz[:, 2]
    # E_01(v2) = (v1 - v0)(u2 - u0) - (u1 - u0)(v2 - v0) > 0 faces the camera
    area = (v[1] - v[0]) * (u[2] - u[0]) - (u[1] - u[0]) * (v[2] - v[0])
    if area <= 0:
        tri = tri[:, ::-1].copy()
    return TMesh(xyz, tri, np.asarray(colours, np.uint8))


# a quad receding from 420 mm to 1100 mm, and a fronto-parallel one
TILTED = _quad((-160, -110, 420), (160, -110, 420), (160, 110, 1100), (-160, 110, 1100),
               [(255, 0, 0), (0, 255, 0), (0, 0, 255), (255, 255, 255)])
TILTED_SIDE = _quad((-200, -90, 500), (40, -90, 1200), (40, 90, 1200), (-200, 90, 500),
                    [(20, 200, 90), (250, 10, 30), (0, 90, 255), (128, 255, 0)])
FRONTAL = _quad((-100, -80, 700), (100, -80, 700), (100, 80, 700), (-100, 80, 700),
                [(10, 20, 30), (240, 40, 200), (90, 250, 60), (200, 200, 10)])
IDENTITY = pose_matrix(np.eye(3), (0.0, 0.0, 0.0))


def _interior(tri):
    """Pixels whose 3x3 neighbourhood all shows the same triangle."""
    t = tri
    ok = t >= 0
    inner = ok.copy()
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            s = np.roll(np.roll(t, dj, axis=0), di, axis=1)
            inner &= s == t
    inner[0, :] = inner[-1, :] = inner[:, 0] = inner[:, -1] = False
    return inner


def _raycast_rgb(mesh, pose):
    z, rgb, lab = sensor.cast(K, [(mesh, np.asarray(pose, np.float64).reshape(3, 4), 1)])
    return z, rgb


def _controls(mesh, pose, tri, pix):
    """Colours at pixels `pix` of the oracle's triangles by screen-space
    (affine) weights, and by perspective weights paired with the wrong
    vertices (rotated by one)."""
    P = np.asarray(pose, np.float64).reshape(3, 4)
    X = (P[:, :3] @ mesh.xyz.astype(np.float64).T).T + P[:, 3]
    u = K[2] * X[:, 0] / X[:, 2] + K[4]
    v = K[3] * X[:, 1] / X[:, 2] + K[5]
    jj, ii = pix
    t = tri[jj, ii]
    ix = mesh.tri[t]
    ua, ub, uc = u[ix[:, 0]], u[ix[:, 1]], u[ix[:, 2]]
    va, vb, vc = v[ix[:, 0]], v[ix[:, 1]], v[ix[:, 2]]
    px, py = ii.astype(np.float64), jj.astype(np.float64)
    area = (ub - ua) * (vc - va) - (uc - ua) * (vb - va)
    w0 = ((ub - px) * (vc - py) - (uc - px) * (vb - py)) / area
    w1 = ((uc - px) * (va - py) - (ua - px) * (vc - py)) / area
    w2 = 1.0 - w0 - w1
    c = mesh.rgb.astype(np.float64)
    ca, cb, cc = c[ix[:, 0]], c[ix[:, 1]], c[ix[:, 2]]
    affine = w0[:, None] * ca + w1[:, None] * cb + w2[:, None] * cc
    iz = 1.0 / X[:, 2]
    t0, t1, t2 = w0 * iz[ix[:, 0]], w1 * iz[ix[:, 1]], w2 * iz[ix[:, 2]]
    s = t0 + t1 + t2
    swapped = (t0[:, None] * cb + t1[:, None] * cc + t2[:, None] * ca) / s[:, None]
    return affine, swapped


@pytest.mark.parametrize("mesh,name,tilted", [(TILTED, "tilted", True), (TILTED_SIDE, "tilted sideways", True),
                                              (FRONTAL, "fronto-parallel", False)])
def test_rendered_colour_matches_ray_caster(mesh, name, tilted):
    depth, tri, rgb = oracle.render(mesh, IDENTITY, K)
    z, rc = _raycast_rgb(mesh, IDENTITY)
    inner = _interior(tri) & (z > 0)
    assert inner.sum() > 2000, name
    diff = np.abs(rgb[inner].astype(np.float64) - rc[inner].astype(np.float64))
    assert diff.max() <= 1.0, f"{name}: rendered colour off by {diff.max():.2f} levels"
    affine, swapped = _controls(mesh, IDENTITY, tri, np.nonzero(inner))
    err_aff = np.abs(affine - rc[inner]).max()
    err_swp = np.abs(swapped - rc[inner]).max()
    assert err_swp > 30.0, f"{name}: swapped pairing is not told apart ({err_swp:.1f})"
    if tilted:
        assert err_aff > 10.0, f"{name}: affine interpolation is not told apart ({err_aff:.1f})"
    else:
        assert err_aff <= 1.0       # on a fronto-parallel face the two interpolations agree


def test_rendered_colour_matches_ray_caster_many_small_triangles():
    mesh = box((-60, -45, -70), (60, 45, 70), n=4, rgb_seed=5)
    pose = pose_matrix(rot_z(0.7) @ rot_x(1.1), (15.0, -10.0, 650.0))
    depth, tri, rgb = oracle.render(mesh, pose, K)
    z, rc = _raycast_rgb(mesh, pose)
    inner = _interior(tri) & (z > 0)
    assert inner.sum() > 500
    diff = np.abs(rgb[inner].astype(np.float64) - rc[inner].astype(np.float64))
    assert diff.max() <= 1.0, f"rendered colour off by {diff.max():.2f} levels"
    # depth agrees with the ray caster to the millimetre rounding as well
    assert np.abs(depth[inner].astype(np.float64) - z[inner]).max() <= 0.5 + 1e-3
