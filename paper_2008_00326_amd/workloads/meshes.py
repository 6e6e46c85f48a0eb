"""Procedural closed meshes (box, cylinder, cone, torus, extruded L).

Every mesh is watertight (vertices shared along seams), counter-clockwise
about the outward normal, in millimetres, with its origin at the centre of
its base so that it rests on a table plane z = 0.  Triangle counts are set
through a target; the achieved count is reported by ``Mesh.n_tris``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    xyz: np.ndarray            # V x 3 float32, mm
    tri: np.ndarray            # T x 3 int32
    rgb: np.ndarray | None     # V x 3 uint8, or None
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def n_verts(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tri.shape[0])

    def with_colours(self, rng: np.random.Generator, name: str | None = None) -> "Mesh":
        rgb = rng.integers(0, 256, size=(self.n_verts, 3), dtype=np.uint8)
        return Mesh(self.xyz, self.tri, rgb, name or self.name, dict(self.params))


class _Builder:
    def __init__(self):
        self.index = {}
        self.xyz = []
        self.tri = []

    def v(self, p):
        key = tuple(int(round(c * 1e6)) for c in p)
        k = self.index.get(key)
        if k is None:
            k = len(self.xyz)
            self.index[key] = k
            self.xyz.append(tuple(float(c) for c in p))
        return k

    def quad(self, a, b, c, d):
        """a, b, c, d counter-clockwise about the outward normal"""
        ia, ib, ic, id_ = self.v(a), self.v(b), self.v(c), self.v(d)
        if ia != ib and ib != ic and ia != ic:
            self.tri.append((ia, ib, ic))
        if ia != ic and ic != id_ and ia != id_:
            self.tri.append((ia, ic, id_))

    def triangle(self, a, b, c):
        ia, ib, ic = self.v(a), self.v(b), self.v(c)
        if len({ia, ib, ic}) == 3:
            self.tri.append((ia, ib, ic))

    def mesh(self, name, **params):
        return Mesh(np.asarray(self.xyz, np.float32), np.asarray(self.tri, np.int32), None, name, params)


def _grid_face(b: _Builder, origin, eu, ev, nu, nv):
    o, eu, ev = (np.asarray(x, float) for x in (origin, eu, ev))
    for a in range(nu):
        for c in range(nv):
            p00 = o + eu * a / nu + ev * c / nv
            p10 = o + eu * (a + 1) / nu + ev * c / nv
            p11 = o + eu * (a + 1) / nu + ev * (c + 1) / nv
            p01 = o + eu * a / nu + ev * (c + 1) / nv
            b.quad(p00, p10, p11, p01)


def box(sx: float, sy: float, sz: float, target_tris: int) -> Mesh:
    """Box sx x sy x sz mm, base centred on the origin, faces split into near-square quads."""
    area = 2 * (sx * sy + sx * sz + sy * sz)
    h = np.sqrt(area / max(target_tris / 2, 6))
    nx, ny, nz = (max(1, int(round(s / h))) for s in (sx, sy, sz))
    b = _Builder()
    x0, y0 = -sx / 2, -sy / 2
    X, Y, Z = np.array([sx, 0, 0.0]), np.array([0, sy, 0.0]), np.array([0, 0, sz])
    o = np.array([x0, y0, 0.0])
    _grid_face(b, o, Y, X, ny, nx)               # bottom, normal -z
    _grid_face(b, o + Z, X, Y, nx, ny)           # top, +z
    _grid_face(b, o, X, Z, nx, nz)               # front y0, normal -y
    _grid_face(b, o + Y, Z, X, nz, nx)           # back, +y
    _grid_face(b, o, Z, Y, nz, ny)               # left x0, normal -x
    _grid_face(b, o + X, Y, Z, ny, nz)           # right, +x
    return b.mesh("box", sx=sx, sy=sy, sz=sz)


def _revolve(profile, n_seg: int, name: str, **params) -> Mesh:
    """Surface of revolution about z of a polyline profile [(r, z), ...] that
    runs from the axis at the bottom, outwards, up, and back to the axis at
    the top (so the result is closed)."""
    b = _Builder()
    ang = np.linspace(0, 2 * np.pi, n_seg + 1)[:-1]
    cs, sn = np.cos(ang), np.sin(ang)

    def P(k, r, z):
        k %= n_seg
        return (r * cs[k], r * sn[k], z) if r > 0 else (0.0, 0.0, z)

    for s in range(len(profile) - 1):
        (r0, z0), (r1, z1) = profile[s], profile[s + 1]
        for k in range(n_seg):
            # angle first, then along the profile: outward normal
            b.quad(P(k, r0, z0), P(k + 1, r0, z0), P(k + 1, r1, z1), P(k, r1, z1))
    return b.mesh(name, **params)


def _profile_counts(lengths, n_total):
    lengths = np.asarray(lengths, float)
    w = lengths / lengths.sum()
    return [max(1, int(round(n_total * x))) for x in w]


def cylinder(radius: float, height: float, target_tris: int) -> Mesh:
    # tris ~= 2 * n_seg * (rings);  rings = cap rings * 2 + side rings
    circ = 2 * np.pi * radius
    path = 2 * radius + height
    n_seg = max(8, int(round(np.sqrt(target_tris / 2 * circ / path))))
    n_prof = max(3, int(round(target_tris / 2 / n_seg)))
    nc, nh, _ = _profile_counts([radius, height, radius], n_prof)
    prof = [(radius * i / nc, 0.0) for i in range(nc + 1)]
    prof += [(radius, height * i / nh) for i in range(1, nh + 1)]
    prof += [(radius * (nc - i) / nc, height) for i in range(1, nc + 1)]
    return _revolve(prof, n_seg, "cylinder", radius=radius, height=height)


def cone(radius: float, height: float, target_tris: int) -> Mesh:
    slant = float(np.hypot(radius, height))
    circ = 2 * np.pi * radius
    path = radius + slant
    n_seg = max(8, int(round(np.sqrt(target_tris / 2 * circ / path))))
    n_prof = max(2, int(round(target_tris / 2 / n_seg)))
    nb, ns = _profile_counts([radius, slant], n_prof)
    prof = [(radius * i / nb, 0.0) for i in range(nb + 1)]
    prof += [(radius * (ns - i) / ns, height * i / ns) for i in range(1, ns + 1)]
    return _revolve(prof, n_seg, "cone", radius=radius, height=height)


def torus(major: float, minor: float, target_tris: int) -> Mesh:
    """Torus lying flat on the table (axis z, resting at z = 0)."""
    ratio = major / minor
    n_v = max(6, int(round(np.sqrt(target_tris / 2 / ratio))))
    n_u = max(8, int(round(target_tris / 2 / n_v)))
    b = _Builder()
    U = np.linspace(0, 2 * np.pi, n_u + 1)[:-1]
    V = np.linspace(0, 2 * np.pi, n_v + 1)[:-1]

    def P(a, c):
        u, v = U[a % n_u], V[c % n_v]
        r = major + minor * np.cos(v)
        return (r * np.cos(u), r * np.sin(u), minor + minor * np.sin(v))

    for a in range(n_u):
        for c in range(n_v):
            b.quad(P(a, c), P(a + 1, c), P(a + 1, c + 1), P(a, c + 1))
    return b.mesh("torus", major=major, minor=minor)


def extruded_l(arm_x: float, arm_y: float, width: float, height: float, target_tris: int) -> Mesh:
    """An L-shaped prism: the union of [0, arm_x] x [0, width] and
    [0, width] x [0, arm_y], extruded to `height`, re-centred on its base."""
    area_cap = width * (arm_x + arm_y - width)
    perim = 2 * (arm_x + arm_y)
    area = 2 * area_cap + perim * height
    h = np.sqrt(area / max(target_tris / 2, 8))
    n = max(2, int(round(width / h)))
    cell = width / n
    gx = max(n + 1, int(round(arm_x / cell)))
    gy = max(n + 1, int(round(arm_y / cell)))
    cx_, cy_ = arm_x / gx, arm_y / gy
    inside = np.zeros((gx, gy), bool)
    for a in range(gx):
        for c in range(gy):
            x, y = (a + 0.5) * cx_, (c + 0.5) * cy_
            inside[a, c] = (y < width) or (x < width)
    nz = max(1, int(round(height / h)))
    b = _Builder()
    ox, oy = arm_x / 2, arm_y / 2

    def p(a, c, z):
        return (a * cx_ - ox, c * cy_ - oy, z)

    for a in range(gx):
        for c in range(gy):
            if not inside[a, c]:
                continue
            b.quad(p(a, c, height), p(a + 1, c, height), p(a + 1, c + 1, height), p(a, c + 1, height))
            b.quad(p(a, c, 0), p(a, c + 1, 0), p(a + 1, c + 1, 0), p(a + 1, c, 0))

            def out(aa, cc):
                return not (0 <= aa < gx and 0 <= cc < gy and inside[aa, cc])
            for k in range(nz):
                z0, z1 = height * k / nz, height * (k + 1) / nz
                if out(a, c - 1):   # wall facing -y
                    b.quad(p(a, c, z0), p(a + 1, c, z0), p(a + 1, c, z1), p(a, c, z1))
                if out(a, c + 1):   # +y
                    b.quad(p(a + 1, c + 1, z0), p(a, c + 1, z0), p(a, c + 1, z1), p(a + 1, c + 1, z1))
                if out(a - 1, c):   # -x
                    b.quad(p(a, c + 1, z0), p(a, c, z0), p(a, c, z1), p(a, c + 1, z1))
                if out(a + 1, c):   # +x
                    b.quad(p(a + 1, c, z0), p(a + 1, c + 1, z0), p(a + 1, c + 1, z1), p(a + 1, c, z1))
    return b.mesh("extruded_l", arm_x=arm_x, arm_y=arm_y, width=width, height=height)


SHAPES = ("box", "cylinder", "cone", "torus", "extruded_l")


def make_shape(kind: str, target_tris: int, rng: np.random.Generator | None = None) -> Mesh:
    """A shape of table-top size; `rng` jitters its dimensions by up to 15%."""
    j = (lambda: 1.0) if rng is None else (lambda: float(rng.uniform(0.85, 1.15)))
    if kind == "box":
        return box(80 * j(), 60 * j(), 120 * j(), target_tris)
    if kind == "cylinder":
        return cylinder(38 * j(), 120 * j(), target_tris)
    if kind == "cone":
        return cone(50 * j(), 110 * j(), target_tris)
    if kind == "torus":
        return torus(50 * j(), 18 * j(), target_tris)
    if kind == "extruded_l":
        return extruded_l(110 * j(), 90 * j(), 40 * j(), 70 * j(), target_tris)
    raise ValueError(kind)
