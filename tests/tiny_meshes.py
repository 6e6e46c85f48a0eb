"""Small hand-built meshes and scenes for the oracle's pin tests."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class TMesh:
    xyz: np.ndarray
    tri: np.ndarray
    rgb: np.ndarray | None = None


@dataclass
class TScene:
    K: tuple
    depth: np.ndarray
    rgb: np.ndarray | None = None
    labels: np.ndarray | None = None


def box(lo, hi, n=1, rgb_seed=None):
    """Closed box with each face split into n x n quads, CCW about the outward normal."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    verts = {}
    xyz = []
    tris = []

    def vid(p):
        key = tuple(np.round(p, 9))
        if key not in verts:
            verts[key] = len(xyz)
            xyz.append(p)
        return verts[key]

    # each face: origin corner, two in-plane axes (a, b) with a x b = outward normal
    c = (lo + hi) / 2
    for axis in range(3):
        for side in (0, 1):
            nrm = np.zeros(3)
            nrm[axis] = 1.0 if side else -1.0
            u_ax, v_ax = [a for a in range(3) if a != axis]
            eu = np.zeros(3); eu[u_ax] = 1.0
            ev = np.zeros(3); ev[v_ax] = 1.0
            if np.dot(np.cross(eu, ev), nrm) < 0:
                eu, ev = ev, eu
                u_ax, v_ax = v_ax, u_ax
            for a in range(n):
                for b in range(n):
                    def P(sa, sb):
                        p = c.copy()
                        p[axis] = hi[axis] if side else lo[axis]
                        p[u_ax] = lo[u_ax] + (hi[u_ax] - lo[u_ax]) * sa / n
                        p[v_ax] = lo[v_ax] + (hi[v_ax] - lo[v_ax]) * sb / n
                        return p
                    p00, p10, p11, p01 = P(a, b), P(a + 1, b), P(a + 1, b + 1), P(a, b + 1)
                    i00, i10, i11, i01 = vid(p00), vid(p10), vid(p11), vid(p01)
                    tris.append((i00, i10, i11))
                    tris.append((i00, i11, i01))
    xyz = np.asarray(xyz, np.float32)
    tri = np.asarray(tris, np.int32)
    rgb = None
    if rgb_seed is not None:
        rgb = np.random.default_rng(rgb_seed).integers(0, 256, size=(len(xyz), 3), dtype=np.uint8)
    return TMesh(xyz, tri, rgb)


def pose_matrix(R, t):
    P = np.zeros((3, 4), np.float32)
    P[:, :3] = np.asarray(R, np.float32)
    P[:, 3] = np.asarray(t, np.float32)
    return P.reshape(12)


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0, 0], [0, c, -s], [0, s, c]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1.0, 0], [-s, 0, c]])
