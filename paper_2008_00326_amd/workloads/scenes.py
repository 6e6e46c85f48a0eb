"""Seeded synthetic workloads for PERCH 2.0 pose scoring.

The paper evaluates on 75 photo-realistic table-top scenes with 3-DoF object
poses (Sec. VI-A) and on YCB-Video with 6-DoF poses (Sec. VI-B); neither
dataset is available, so these procedural scenes stand in for them, with the
paper's parameters where they apply (delta, tau_c, the 22.5 degree yaw step).

Geometry: world z is up and the table top is the plane z = 0.  The camera
sits 0.8 m from the world origin, 45 degrees above the table, looking at the
origin, with OpenCV axes (x right, y down, z forward).  A table-top pose
(x, y, yaw) is the object->camera transform T_cam<-world * [Rz(yaw) | (x,y,0)].

The observed RGB-D image comes from the sensor simulator (a ray caster),
with Gaussian depth noise rounded to millimetres and Gaussian colour noise
rounded to 8 bits.  Candidate poses are produced here in binary64 and handed
to every consumer as binary32 3x4 row-major [R|t] in millimetres.

Seeds: ``numpy.random.default_rng(1000 * config + scene)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes as M
from . import sensor


@dataclass
class Scene:
    K: tuple                       # (width, height, fx, fy, cx, cy)
    depth: np.ndarray              # H x W uint16 mm, 0 = no reading
    rgb: np.ndarray | None         # H x W x 3 uint8
    labels: np.ndarray             # H x W int32 (0 table, k >= 1 object k, 255 occluder, -1 nothing)


@dataclass
class ObjectQuery:
    mesh: int                      # index into Workload.meshes
    label: int                     # object label in Scene.labels
    poses: np.ndarray              # n x 12 float32 candidates
    gt_pose: np.ndarray            # 12 float32


@dataclass
class Workload:
    name: str
    config: int
    seed: int
    scene: Scene
    meshes: list
    objects: list
    delta_mm: float = 10.0
    tau_c: float = 20.0
    use_rgb: bool = True
    mark_occluders: bool = True
    volume: str = "aabb"           # "aabb" | "cyl" | "label"
    jo: str = "exact"              # "exact" (Eq. 3) | "nn" (nearest-neighbour marking)
    search: str = "table"          # "table" | "hash" (voxel hash) | "knn2" (the paper's scan of the whole cloud)
    stride: int = 1
    info: dict = field(default_factory=dict)

    @property
    def n_poses(self) -> int:
        return int(sum(o.poses.shape[0] for o in self.objects))


# ---------------------------------------------------------------- rig / poses

def camera_rig(distance_mm: float = 800.0, elevation_deg: float = 45.0):
    e = np.radians(elevation_deg)
    c = distance_mm * np.array([0.0, -np.cos(e), np.sin(e)])
    f = -c / np.linalg.norm(c)
    right = np.cross(f, [0.0, 0.0, 1.0])
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f]), c


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def exp_so3(w):
    th = float(np.linalg.norm(w))
    if th < 1e-12:
        return np.eye(3)
    k = np.asarray(w) / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx


def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def world_to_cam(rig, R_wo, t_wo):
    R_cw, c = rig
    P = np.zeros((3, 4))
    P[:, :3] = R_cw @ R_wo
    P[:, 3] = R_cw @ (np.asarray(t_wo, float) - c)
    return P


def table_pose(rig, x, y, yaw):
    return world_to_cam(rig, rot_z(yaw), (x, y, 0.0))


def grid_poses(rig, xs, ys, yaws):
    out = [table_pose(rig, x, y, a).reshape(12) for x in xs for y in ys for a in yaws]
    return np.asarray(out, np.float64).astype(np.float32)


def perturbed_poses(rig, R_seeds, t_seeds, n_per_seed, rng, sigma_t=15.0, sigma_r_deg=10.0):
    """6-DoF samples around seed poses: R = R_s exp([w]x), w ~ N(0, s_r^2 I);
    t = t_s + N(0, s_t^2 I) (world frame, mm)."""
    out = []
    sr = np.radians(sigma_r_deg)
    for R_s, t_s in zip(R_seeds, t_seeds):
        for _ in range(n_per_seed):
            R = R_s @ exp_so3(rng.normal(0, sr, 3))
            t = np.asarray(t_s) + rng.normal(0, sigma_t, 3)
            out.append(world_to_cam(rig, R, t).reshape(12))
    return np.asarray(out, np.float64).astype(np.float32)


# ---------------------------------------------------------------- scene parts

def _table_mesh(size=1600.0, thickness=20.0):
    t = M.box(size, size, thickness, 12)
    xyz = t.xyz.copy()
    xyz[:, 2] -= thickness
    return M.Mesh(xyz, t.tri, np.full((t.n_verts, 3), 128, np.uint8), "table")


def _observe(K, parts, rng, sigma_d=2.0, sigma_c=5.0):
    z, c, lab = sensor.cast(K, parts)
    valid = z > 0
    d = np.rint(z + rng.normal(0.0, sigma_d, z.shape))
    d = np.clip(d, 1, 65534).astype(np.uint16)
    d[~valid] = 0
    rgb = np.clip(np.rint(c + rng.normal(0.0, sigma_c, c.shape)), 0, 255).astype(np.uint8)
    rgb[~valid] = 0
    return d, rgb, lab


def _rest_pose(mesh, R_rest):
    """Translation offset that puts the rotated mesh's lowest point on z = 0."""
    z = (mesh.xyz.astype(np.float64) @ R_rest.T)[:, 2]
    return -float(z.min())


def _footprint_radius(mesh):
    return float(np.max(np.linalg.norm(mesh.xyz[:, :2].astype(np.float64), axis=1)))


def _place_non_overlapping(rng, radii, half_extent, gap=10.0, tries=2000):
    pos = []
    for r in radii:
        for _ in range(tries):
            p = rng.uniform(-half_extent + r, half_extent - r, 2)
            if all(np.linalg.norm(p - q) >= r + s + gap for q, s in zip(pos, radii)):
                pos.append(p)
                break
        else:
            raise RuntimeError("could not place objects without overlap")
    return pos


# ---------------------------------------------------------------- configs

def config1(seed: int = 0) -> Workload:
    """3-DoF, one 8x6x12 cm box (~1.2k triangles), 320x240 depth, 512 poses,
    20% of the object hidden by a random occluding box, delta 10 mm."""
    rng = np.random.default_rng(1000 * 1 + seed)
    K = (320, 240, 262.5, 262.5, 160.0, 120.0)
    rig = camera_rig()
    box = M.box(80.0, 60.0, 120.0, 1260)
    box = M.Mesh(box.xyz, box.tri, None, "box")
    table = _table_mesh()
    gt = (rng.uniform(-70, 70), rng.uniform(-70, 70), rng.uniform(0, 2 * np.pi))
    P_gt = table_pose(rig, *gt)
    P_table = table_pose(rig, 0, 0, 0)
    z_alone, _, lab_alone = sensor.cast(K, [(table, P_table, 0), (box, P_gt, 1)])
    n_vis = int((lab_alone == 1).sum())

    # occluder: a box standing between camera and object; its sideways offset
    # is bisected until 20 +- 2 % of the object's visible pixels are hidden
    R_cw, c = rig
    to_cam = np.array([c[0] - gt[0], c[1] - gt[1]])
    to_cam /= np.linalg.norm(to_cam)
    side = np.array([-to_cam[1], to_cam[0]])
    if rng.uniform() < 0.5:
        side = -side
    dims = (rng.uniform(50, 80), rng.uniform(30, 50), rng.uniform(140, 200))
    occ = M.box(*dims, 12)
    occ = M.Mesh(occ.xyz, occ.tri, None, "occluder")
    dist = rng.uniform(110, 160)
    yaw_o = np.arctan2(to_cam[1], to_cam[0]) + np.pi / 2

    def hidden(off):
        p = np.array(gt[:2]) + to_cam * dist + side * off
        P_o = table_pose(rig, p[0], p[1], yaw_o)
        _, _, lab = sensor.cast(K, [(table, P_table, 0), (box, P_gt, 1), (occ, P_o, 255)])
        return 1.0 - (lab == 1).sum() / max(n_vis, 1), P_o

    lo, hi = 0.0, 200.0
    frac, P_occ = hidden(hi)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        frac, P_occ = hidden(mid)
        if abs(frac - 0.20) <= 0.02:
            break
        if frac > 0.20:
            lo = mid
        else:
            hi = mid
    depth, _, labels = _observe(K, [(table, P_table, 0), (box, P_gt, 1), (occ, P_occ, 255)], rng)
    xs = np.arange(-70.0, 70.1, 20.0)
    yaws = np.radians(np.arange(0, 360, 45.0))
    poses = grid_poses(rig, xs, xs, yaws)
    obj = ObjectQuery(0, 1, poses, P_gt.reshape(12).astype(np.float32))
    return Workload("cfg1-3dof-depth", 1, seed, Scene(K, depth, None, labels), [box], [obj],
                    delta_mm=10.0, tau_c=0.0, use_rgb=False, mark_occluders=True, volume="aabb",
                    info={"occluded_fraction": float(frac), "gt": gt, "n_tris": box.n_tris})


def config2(seed: int = 0) -> Workload:
    """3-DoF with the RGB term: 5 objects of 2k-8k triangles with random
    per-vertex colours, two of them the same shape in different colours;
    640x480; 20x20 grid at 3 cm x 16 yaws = 6400 poses per object."""
    rng = np.random.default_rng(1000 * 2 + seed)
    K = (640, 480, 525.0, 525.0, 320.0, 240.0)
    rig = camera_rig()
    kinds = list(rng.permutation(M.SHAPES)[:4])
    kinds.append(kinds[0])                    # the colour twin of object 1
    meshes = []
    for k, kind in enumerate(kinds):
        if k == 4:
            base = meshes[0]
            meshes.append(M.Mesh(base.xyz, base.tri, None, base.name + "_twin", dict(base.params)))
        else:
            meshes.append(M.make_shape(str(kind), int(rng.integers(2000, 8001)), rng))
    meshes = [m.with_colours(rng) for m in meshes]
    radii = [_footprint_radius(m) for m in meshes]
    pos = _place_non_overlapping(rng, radii, 300.0)
    table = _table_mesh()
    parts = [(table, table_pose(rig, 0, 0, 0), 0)]
    objs = []
    xs = -285.0 + 30.0 * np.arange(20)
    yaws = np.radians(np.arange(16) * 22.5)
    grid = grid_poses(rig, xs, xs, yaws)
    for k, m in enumerate(meshes):
        yaw = rng.uniform(0, 2 * np.pi)
        P = table_pose(rig, pos[k][0], pos[k][1], yaw)
        parts.append((m, P, k + 1))
        objs.append(ObjectQuery(k, k + 1, grid, P.reshape(12).astype(np.float32)))
    depth, rgb, labels = _observe(K, parts, rng)
    return Workload("cfg2-3dof-rgb", 2, seed, Scene(K, depth, rgb, labels), meshes, objs,
                    delta_mm=10.0, tau_c=20.0, use_rgb=True, mark_occluders=True, volume="aabb",
                    info={"kinds": [str(k) for k in kinds], "n_tris": [m.n_tris for m in meshes]})


def config3(seed: int = 0, tris: int = 20000, samples_per_seed: int = 256) -> Workload:
    """6-DoF refinement: 8 objects of ~20k triangles in a jittered 3x3 layout
    with inter-object occlusion; per object 4 seed poses (ground truth with
    noise, and three random rotations at the ground-truth translation) x 256
    samples with sigma_t = 15 mm, sigma_r = 10 degrees."""
    rng = np.random.default_rng(1000 * 3 + seed)
    K = (640, 480, 525.0, 525.0, 320.0, 240.0)
    rig = camera_rig()
    kinds = [M.SHAPES[k % len(M.SHAPES)] for k in range(8)]
    meshes = [M.make_shape(k, tris, rng).with_colours(rng) for k in kinds]
    cells = [(i, j) for i in range(3) for j in range(3)]
    skip = int(rng.integers(0, 9))
    cells = [c for k, c in enumerate(cells) if k != skip]
    table = _table_mesh()
    parts = [(table, table_pose(rig, 0, 0, 0), 0)]
    rests = [np.eye(3), rot_x(np.pi / 2), rot_y(np.pi / 2)]
    objs = []
    for k, m in enumerate(meshes):
        R_rest = rests[int(rng.integers(0, 3))]
        R_wo = rot_z(rng.uniform(0, 2 * np.pi)) @ R_rest
        ci, cj = cells[k]
        xy = np.array([(ci - 1) * 150.0, (cj - 1) * 150.0]) + rng.uniform(-25, 25, 2)
        t_wo = np.array([xy[0], xy[1], _rest_pose(m, R_wo)])
        P = world_to_cam(rig, R_wo, t_wo)
        parts.append((m, P, k + 1))
        sr = np.radians(10.0)
        R_seeds = [R_wo @ exp_so3(rng.normal(0, sr, 3))] + [random_rotation(rng) for _ in range(3)]
        t_seeds = [t_wo + rng.normal(0, 15.0, 3)] + [t_wo] * 3
        poses = perturbed_poses(rig, R_seeds, t_seeds, samples_per_seed, rng)
        objs.append(ObjectQuery(k, k + 1, poses, P.reshape(12).astype(np.float32)))
    depth, rgb, labels = _observe(K, parts, rng)
    return Workload("cfg3-6dof-rgb", 3, seed, Scene(K, depth, rgb, labels), meshes, objs,
                    delta_mm=10.0, tau_c=20.0, use_rgb=True, mark_occluders=True, volume="aabb",
                    info={"kinds": kinds, "n_tris": [m.n_tris for m in meshes]})


def mesh_library(seed: int = 0, n: int = 64, lo: int = 500, hi: int = 50000):
    """n seeded meshes of the five procedural shapes with log-uniform
    triangle counts in [lo, hi] and random per-vertex colours."""
    rng = np.random.default_rng(1000 * 4 + 500 + seed)
    lib = []
    for k in range(n):
        kind = M.SHAPES[k % len(M.SHAPES)]
        tris = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        lib.append(M.make_shape(kind, tris, rng).with_colours(rng, name=f"{kind}_{k}"))
    return lib


def _cells(rng, n, spacing=140.0, grid=4, jitter=20.0):
    cells = [(i, j) for i in range(grid) for j in range(grid)]
    pick = rng.permutation(len(cells))[:n]
    off = (grid - 1) / 2.0
    return [np.array([(cells[c][0] - off) * spacing, (cells[c][1] - off) * spacing]) + rng.uniform(-jitter, jitter, 2)
            for c in pick]


def config4(seed: int = 0, n_scenes: int = 64, library=None):
    """Batched uneven workload: n_scenes 640x480 RGB-D scenes, each with 1-10
    objects drawn from a 64-mesh library (500-50k triangles, log-uniform),
    200-8000 candidate poses per object (log-uniform), 3-DoF or 6-DoF by a
    coin flip per scene.  Returns one Workload per scene; the meshes are
    shared objects of the library (index = position in the library)."""
    lib = mesh_library(seed) if library is None else library
    K = (640, 480, 525.0, 525.0, 320.0, 240.0)
    rig = camera_rig()
    table = _table_mesh()
    out = []
    for sc in range(n_scenes):
        rng = np.random.default_rng(1000 * 4 + 64 * seed + sc)
        six = bool(rng.uniform() < 0.5)
        n_obj = int(rng.integers(1, 11))
        mesh_idx = [int(x) for x in rng.integers(0, len(lib), n_obj)]
        pos = _cells(rng, n_obj)
        parts = [(table, table_pose(rig, 0, 0, 0), 0)]
        objs = []
        rests = [np.eye(3), rot_x(np.pi / 2), rot_y(np.pi / 2)]
        for k, (mi, xy) in enumerate(zip(mesh_idx, pos)):
            m = lib[mi]
            n_p = int(np.exp(rng.uniform(np.log(200), np.log(8000))))
            if six:
                R_wo = rot_z(rng.uniform(0, 2 * np.pi)) @ rests[int(rng.integers(0, 3))]
                t_wo = np.array([xy[0], xy[1], _rest_pose(m, R_wo)])
                sr = np.radians(10.0)
                R_seeds = [R_wo @ exp_so3(rng.normal(0, sr, 3))] + [random_rotation(rng) for _ in range(3)]
                t_seeds = [t_wo + rng.normal(0, 15.0, 3)] + [t_wo] * 3
                per = [n_p // 4 + (1 if q < n_p % 4 else 0) for q in range(4)]
                poses = np.concatenate([perturbed_poses(rig, [R_seeds[q]], [t_seeds[q]], per[q], rng)
                                        for q in range(4) if per[q] > 0])
            else:
                yaw = rng.uniform(0, 2 * np.pi)
                R_wo = rot_z(yaw)
                t_wo = np.array([xy[0], xy[1], 0.0])
                cand = [table_pose(rig, x, y, a).reshape(12) for x, y, a in
                        zip(rng.uniform(-280, 280, n_p), rng.uniform(-280, 280, n_p), rng.uniform(0, 2 * np.pi, n_p))]
                poses = np.asarray(cand, np.float64).astype(np.float32)
            P = world_to_cam(rig, R_wo, t_wo)
            parts.append((m, P, k + 1))
            objs.append(ObjectQuery(mi, k + 1, poses, P.reshape(12).astype(np.float32)))
        depth, rgb, labels = _observe(K, parts, rng)
        out.append(Workload(f"cfg4-scene{sc}-{'6dof' if six else '3dof'}", 4, sc, Scene(K, depth, rgb, labels), lib,
                            objs, delta_mm=10.0, tau_c=20.0, use_rgb=True, mark_occluders=True, volume="aabb",
                            info={"six_dof": six, "n_objects": n_obj}))
    return out


def make_config(k: int, seed: int = 0, **kw):
    """Configs 1-3 return one Workload; config 4 a list of per-scene Workloads."""
    return {1: config1, 2: config2, 3: config3, 4: config4}[k](seed, **kw)
