"""Pins for the oracle's windowed exact search and for the pixel-window bound
(CPU only).

The windowed search (each point compared only with the other cloud's pixels
inside a window derived from delta and depth) must reproduce the brute-force
counts of Eq. 3 / Eq. 4 exactly: on every pose of the 320x240 depth-only
workload, on seeded subsets of the 640x480 RGB and 6-DoF workloads, and on
seeded random cases in every scoring mode.

The bound behind every window in this repository (oracle and HIP path alike)
is checked separately by enumerating neighbour pairs: two back-projected pixel
centres whose 1/16 mm points lie within delta are at most
floor(f e sqrt(1 + ((i - c)/f)^2) / (Z - e)) pixels apart along each axis,
with e = delta + 1/4 mm, (i, Z) the pixel and depth of either point.  The
HIP path's marking also cuts each row of a window to the joint bound
(di/fx)^2 + (dj/fy)^2 <= (1 + xh^2 + yh^2) e^2 / (Z - e)^2, with
(xh, yh) = ((i - cx)/fx, (j - cy)/fy): checked on the same pairs.
"""
import numpy as np
import pytest

import oracle
from paper_2008_00326_amd.workloads import make_config
from random_cases import random_case


def _both(mesh, scene, poses, **kw):
    b = oracle.score(mesh, scene, poses, search="brute", **kw)
    w = oracle.score(mesh, scene, poses, search="window", **kw)
    return b, w


def _assert_same(b, w, what):
    for name, x, y in zip(("J_r", "J_o", "L", "Q"), b, w):
        bad = np.flatnonzero(x != y)
        assert bad.size == 0, f"{what}: windowed {name} differs from brute force at poses {bad[:8]}"


def _flags(w):
    f = (oracle.MARK_OCCLUDERS if w.mark_occluders else 0) | (oracle.USE_RGB if w.use_rgb else 0)
    return f | {"aabb": oracle.VOL_AABB, "cyl": oracle.VOL_CYL, "label": oracle.VOL_LABEL}[w.volume]


def _near_and_random(o, rng, n_near, n_rand):
    """Indices of the candidates nearest the true pose (so that counts are
    far from trivial) plus seeded random ones."""
    d = np.abs(o.poses - o.gt_pose[None, :]).sum(axis=1)
    near = np.argsort(d, kind="stable")[:n_near]
    rand = rng.choice(o.poses.shape[0], size=n_rand, replace=False)
    return np.unique(np.concatenate([near, rand]))


def test_windowed_equals_brute_force_cfg1_every_pose():
    w = make_config(1, 0)
    o = w.objects[0]
    b, v = _both(w.meshes[o.mesh], w.scene, o.poses, delta_mm=w.delta_mm, tau_c=w.tau_c, flags=_flags(w),
                 label=o.label)
    _assert_same(b, v, "cfg1")
    assert b[0].min() < b[2].max()        # some poses explain part of the scene


@pytest.mark.parametrize("cfg", [2, 3])
def test_windowed_equals_brute_force_sampled(cfg):
    w = make_config(cfg, 0)
    rng = np.random.default_rng(77 + cfg)
    for o in w.objects:
        idx = _near_and_random(o, rng, 2, 1)
        b, v = _both(w.meshes[o.mesh], w.scene, o.poses[idx], delta_mm=w.delta_mm, tau_c=w.tau_c,
                     flags=_flags(w), label=o.label)
        _assert_same(b, v, f"cfg{cfg} object {o.label} poses {idx}")
        assert (b[2] - b[0]).max() > 0    # at least one rendered inlier


@pytest.mark.parametrize("seed", range(10))
def test_windowed_equals_brute_force_random_modes(seed):
    mesh, scene, poses, p = random_case(seed)
    flags = (oracle.MARK_OCCLUDERS if p["occl"] else 0) | (oracle.USE_RGB if p["rgb"] else 0)
    flags |= [oracle.VOL_AABB, oracle.VOL_CYL, oracle.VOL_AABB][seed % 3]
    if seed % 4 == 3:
        flags |= oracle.JO_NN
    b, v = _both(mesh, scene, poses[:24], delta_mm=p["delta"], tau_c=p["tau"], flags=flags, stride=p["stride"])
    _assert_same(b, v, f"random case {seed}")


def test_windowed_equals_brute_force_near_camera():
    # objects 150-250 mm from the camera: windows of tens of pixels, and
    # some of them the whole image
    mesh, scene, poses, p = random_case(3)
    P = poses[:16].copy()
    P[:, 11] = np.linspace(150.0, 250.0, P.shape[0])
    d, _, c = oracle.render(mesh, P[5], scene.K)
    from tiny_meshes import TScene
    sc = TScene(scene.K, d, c, None)
    b, v = _both(mesh, sc, P, delta_mm=25.0, tau_c=10.0, flags=oracle.MARK_OCCLUDERS | oracle.USE_RGB)
    _assert_same(b, v, "near camera")
    assert b[0][5] == 0 and b[1][5] == 0     # the self-render


# ---------------------------------------------------------------- the bound


def _points(K, depth):
    """1/16 mm points of a depth image (reading R7 of the oracle)."""
    W, H, fx, fy, cx, cy = K
    kx = ((np.arange(W, dtype=np.float64) - cx) * 16.0) / fx
    ky = ((np.arange(H, dtype=np.float64) - cy) * 16.0) / fy
    d = depth.astype(np.float64)
    X = np.rint(kx[None, :] * d).astype(np.int64)
    Y = np.rint(ky[:, None] * d).astype(np.int64)
    Z = 16 * depth.astype(np.int64)
    return X, Y, Z


def _surfaces(rng, K, n):
    """Depth images that put many neighbour pairs at the edge of the bound:
    planes from fronto-parallel to grazing, near and far, with noise and
    steps."""
    W, H, fx, fy, cx, cy = K
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    rx, ry = (ii - cx) / fx, (jj - cy) / fy
    out = []
    for _ in range(n):
        z0 = rng.uniform(150.0, 1500.0)
        nrm = rng.normal(size=3)
        nrm[2] = abs(nrm[2]) + rng.uniform(0.02, 1.0)
        nrm /= np.linalg.norm(nrm)
        # plane n . X = n_z z0 along each ray (X = z (rx, ry, 1))
        den = nrm[0] * rx + nrm[1] * ry + nrm[2]
        z = np.where(den > 0.05, nrm[2] * z0 / np.maximum(den, 0.05), 0.0)
        z = z + rng.normal(0, rng.uniform(0, 6), z.shape)
        step = rng.random(z.shape) < 0.05
        z = np.where(step, z + rng.uniform(-40, 40), z)
        d = np.where((z >= 1) & (z <= 65534), np.rint(z), 0).astype(np.uint16)
        d[rng.random(d.shape) < 0.03] = 0
        out.append(d)
    return out


@pytest.mark.parametrize("K,delta", [((160, 120, 131.25, 131.25, 80.0, 60.0), 10.0),
                                     ((160, 120, 300.0, 280.0, 70.5, 64.25), 7.5),
                                     ((120, 90, 90.0, 90.0, 60.0, 45.0), 25.0)])
def test_window_bound_holds_for_every_neighbour_pair(K, delta):
    W, H, fx, fy, cx, cy = K
    rng = np.random.default_rng(int(fx * 7 + delta))
    dq = int(np.rint(16.0 * delta))
    e = delta + 0.25
    checked = edge = ell_edge = 0
    for depth in _surfaces(rng, K, 6):
        X, Y, Z = _points(K, depth)
        valid = depth > 0
        zmm = depth.astype(np.float64)
        den = zmm - e
        ok = valid & (den > 1.0)
        jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
        bu = np.where(ok, fx * e * np.sqrt(1.0 + ((ii - cx) / fx) ** 2) / np.where(ok, den, 1.0), np.inf)
        bv = np.where(ok, fy * e * np.sqrt(1.0 + ((jj - cy) / fy) ** 2) / np.where(ok, den, 1.0), np.inf)
        fu, fv = np.floor(bu), np.floor(bv)
        # joint (ellipse) bound: squared normalised radius of every neighbour
        r2 = np.where(ok, (1.0 + ((ii - cx) / fx) ** 2 + ((jj - cy) / fy) ** 2) * e * e
                      / np.where(ok, den, 1.0) ** 2, np.inf)
        R = int(min(np.nanmax(np.where(ok, fu, 0)), W - 1)) + 3
        Rv = int(min(np.nanmax(np.where(ok, fv, 0)), H - 1)) + 3
        for dj in range(-Rv, Rv + 1):
            for di in range(-R, R + 1):
                # pairs (r at (i, j), p at (i + di, j + dj))
                a0, a1 = max(0, -dj), min(H, H - dj)
                b0, b1 = max(0, -di), min(W, W - di)
                if a0 >= a1 or b0 >= b1:
                    continue
                sr = (slice(a0, a1), slice(b0, b1))
                sp = (slice(a0 + dj, a1 + dj), slice(b0 + di, b1 + di))
                both = valid[sr] & valid[sp]
                dz = Z[sp] - Z[sr]
                near = both & (np.abs(dz) <= dq)
                if not near.any():
                    continue
                dx = X[sp] - X[sr]
                dy = Y[sp] - Y[sr]
                pair = near & (dx * dx + dy * dy + dz * dz <= dq * dq)
                if not pair.any():
                    continue
                n = int(pair.sum())
                checked += n
                # the bound from r's side and from p's side
                q = (di / fx) ** 2 + (dj / fy) ** 2
                for f_u, f_v, s in ((fu, fv, sr), (fu, fv, sp)):
                    assert np.all(abs(di) <= f_u[s][pair]), f"column offset {di} beyond the bound"
                    assert np.all(abs(dj) <= f_v[s][pair]), f"row offset {dj} beyond the bound"
                    assert np.all(q <= r2[s][pair]), f"offset ({di}, {dj}) beyond the joint bound"
                edge += int((pair & ((abs(di) == fu[sr]) | (abs(dj) == fv[sr]))).sum())
                ell_edge += int((pair & (q > 0.8 * r2[sr])).sum())
    assert checked > 10**6
    assert edge > 100                       # the bound is met with equality: no slack to spare
    assert ell_edge > 100                   # and pairs come near the joint bound
