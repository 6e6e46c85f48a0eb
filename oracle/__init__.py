"""CPU oracle for PERCH 2.0 pose scoring -- test infrastructure only.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``liboracle.so`` (built from
``perch_oracle.c`` by ``oracle.build.build()``) with ctypes; the arithmetic
lives in the C file, whose header lists the paper passages it follows and the
readings it takes where the paper is silent.

Meshes are any object with ``xyz`` (V x 3 float32, mm), ``tri`` (T x 3 int32)
and ``rgb`` (V x 3 uint8 or None).  Scenes are any object with ``K`` (a
``(width, height, fx, fy, cx, cy)`` tuple), ``depth`` (H x W uint16 mm),
``rgb`` (H x W x 3 uint8 or None) and ``labels`` (H x W int32 or None).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

USE_RGB = 1
MARK_OCCLUDERS = 2
VOL_AABB = 0 << 4
VOL_CYL = 1 << 4
VOL_LABEL = 2 << 4
JO_NN = 1 << 6

_HERE = os.path.dirname(os.path.abspath(__file__))
# PERCH_ORACLE_LIBRARY selects another build of the same source (the
# sanitizer test loads an AddressSanitizer / UBSan build this way)
_LIB_PATH = os.environ.get("PERCH_ORACLE_LIBRARY", os.path.join(_HERE, "liboracle.so"))


class _Intrinsics(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class _Mesh(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("n_verts", ctypes.c_int32),
                ("tri", ctypes.c_void_p), ("n_tris", ctypes.c_int32),
                ("rgb", ctypes.c_void_p)]


class _Scene(ctypes.Structure):
    _fields_ = [("K", _Intrinsics), ("depth", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("labels", ctypes.c_void_p), ("delta_mm", ctypes.c_float),
                ("tau_c", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("stride", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_render.argtypes = [P, P, P, P, P, P]
        lib.oracle_render.restype = ctypes.c_int
        lib.oracle_backproject.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]
        lib.oracle_backproject.restype = None
        lib.oracle_srgb_to_lab64.argtypes = [P, P]
        lib.oracle_srgb_to_lab32.argtypes = [P, P]
        lib.oracle_ciede2000_64.argtypes = [P, P]
        lib.oracle_ciede2000_64.restype = ctypes.c_double
        lib.oracle_ciede2000_32.argtypes = [P, P]
        lib.oracle_ciede2000_32.restype = ctypes.c_float
        lib.oracle_score.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, P, P, P, P, ctypes.c_int32]
        lib.oracle_score.restype = ctypes.c_int
        lib.oracle_score_windowed.argtypes = lib.oracle_score.argtypes
        lib.oracle_score_windowed.restype = ctypes.c_int
        lib.oracle_score_detail.argtypes = [P, P, ctypes.c_int32, P, P, P, P]
        lib.oracle_score_detail.restype = ctypes.c_int
        lib.oracle_score_detail_windowed.argtypes = lib.oracle_score_detail.argtypes
        lib.oracle_score_detail_windowed.restype = ctypes.c_int
        lib.oracle_best.argtypes = [P, P, ctypes.c_int32, P, P, P]
        lib.oracle_icp.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int32]
        lib.oracle_icp_pairs.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P, P]
        lib.oracle_gicp.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int32]
        lib.oracle_gicp_pairs.argtypes = [P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, P]
        lib.oracle_normal_image.argtypes = [P, P, ctypes.c_int32, P]
        lib.oracle_msg_expand.argtypes = [P, P, P, P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32,
                                          P, P, P, P, P, ctypes.c_int32]
        lib.oracle_msg_expand.restype = ctypes.c_int
        lib.oracle_best.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _intr(K):
    w, h, fx, fy, cx, cy = K
    return _Intrinsics(int(w), int(h), float(fx), float(fy), float(cx), float(cy))


class _MeshArgs:
    def __init__(self, mesh):
        self.xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float32)
        self.tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        rgb = getattr(mesh, "rgb", None)
        self.rgb = None if rgb is None else np.ascontiguousarray(rgb, dtype=np.uint8)
        self.s = _Mesh(_ptr(self.xyz), self.xyz.shape[0], _ptr(self.tri), self.tri.shape[0],
                       _ptr(self.rgb))


class _SceneArgs:
    def __init__(self, scene, delta_mm, tau_c, flags, stride):
        self.depth = np.ascontiguousarray(scene.depth, dtype=np.uint16)
        rgb = getattr(scene, "rgb", None)
        lab = getattr(scene, "labels", None)
        self.rgb = None if rgb is None else np.ascontiguousarray(rgb, dtype=np.uint8)
        self.labels = None if lab is None else np.ascontiguousarray(lab, dtype=np.int32)
        self.s = _Scene(_intr(scene.K), _ptr(self.depth), _ptr(self.rgb), _ptr(self.labels),
                        float(delta_mm), float(tau_c), int(flags), int(stride))


def render(mesh, pose, K):
    """Full-image render of one pose (Sec. IV-A "Parallel Rendering").

    Returns (depth uint16 H x W, tri_id int32 H x W (-1 empty), rgb uint8 H x W x 3).
    """
    lib = _load()
    m = _MeshArgs(mesh)
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    k = _intr(K)
    depth = np.zeros((k.height, k.width), np.uint16)
    tri = np.zeros((k.height, k.width), np.int32)
    rgb = np.zeros((k.height, k.width, 3), np.uint8)
    rc = lib.oracle_render(ctypes.byref(m.s), _ptr(pose), ctypes.byref(k), _ptr(depth), _ptr(tri),
                           _ptr(rgb))
    if rc != 0:
        raise ValueError(f"oracle_render failed ({rc})")
    return depth, tri, rgb


def backproject(K, i, j, d):
    """Pixel (i, j) at depth d mm -> (Xq, Yq, Zq) in 1/16 mm (Sec. IV-A)."""
    lib = _load()
    out = np.zeros(3, np.int32)
    k = _intr(K)
    lib.oracle_backproject(ctypes.byref(k), int(i), int(j), int(d), _ptr(out))
    return tuple(int(v) for v in out)


def srgb_to_lab64(rgb):
    lib = _load()
    a = np.ascontiguousarray(rgb, dtype=np.uint8).reshape(3)
    out = np.zeros(3, np.float64)
    lib.oracle_srgb_to_lab64(_ptr(a), _ptr(out))
    return out


def srgb_to_lab32(rgb):
    lib = _load()
    a = np.ascontiguousarray(rgb, dtype=np.uint8).reshape(3)
    out = np.zeros(3, np.float32)
    lib.oracle_srgb_to_lab32(_ptr(a), _ptr(out))
    return out


def ciede2000_64(lab1, lab2):
    """CIEDE2000 colour difference in binary64 (Sec. IV-B, Eq. 4)."""
    lib = _load()
    a = np.ascontiguousarray(lab1, dtype=np.float64).reshape(3)
    b = np.ascontiguousarray(lab2, dtype=np.float64).reshape(3)
    return float(lib.oracle_ciede2000_64(_ptr(a), _ptr(b)))


def ciede2000_32(lab1, lab2):
    """CIEDE2000 in binary32, the precision of the colour decision."""
    lib = _load()
    a = np.ascontiguousarray(lab1, dtype=np.float32).reshape(3)
    b = np.ascontiguousarray(lab2, dtype=np.float32).reshape(3)
    return float(lib.oracle_ciede2000_32(_ptr(a), _ptr(b)))


def threads():
    """Threads the oracle's OpenMP loops use when none is asked for."""
    return int(_load().oracle_threads())


def score(mesh, scene, poses, *, delta_mm, tau_c=0.0, flags=MARK_OCCLUDERS, stride=1, label=0,
          threads=0, search="brute"):
    """J_r, J_o, L, Q for every pose (Eq. 3, Eq. 4).

    poses: n x 12 float32 row-major [R|t], object -> camera, mm.
    search: "brute" compares every point with the whole other cloud (the
    definition); "window" only with the pixels of the window that provably
    holds all its neighbours (same result, for large workloads).
    Returns four int32 arrays (jr, jo, nr, nq).
    """
    lib = _load()
    if search not in ("brute", "window"):
        raise ValueError(f"unknown search {search!r}")
    fn = lib.oracle_score if search == "brute" else lib.oracle_score_windowed
    m = _MeshArgs(mesh)
    s = _SceneArgs(scene, delta_mm, tau_c, flags, stride)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    n = poses.shape[0]
    jr = np.zeros(n, np.int32)
    jo = np.zeros(n, np.int32)
    nr = np.zeros(n, np.int32)
    nq = np.zeros(n, np.int32)
    rc = fn(ctypes.byref(m.s), ctypes.byref(s.s), int(label), _ptr(poses), n,
            _ptr(jr), _ptr(jo), _ptr(nr), _ptr(nq), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_score failed ({rc})")
    return jr, jo, nr, nq


def score_detail(mesh, scene, pose, *, delta_mm, tau_c=0.0, flags=MARK_OCCLUDERS, stride=1,
                 label=0, search="brute"):
    """One pose with per-pixel classes.

    Returns ((jr, jo, L, Q), r_flag, o_flag) where r_flag is 0 not rendered,
    1 inlier, 2 distance outlier, 3 colour outlier, 4 occluded; o_flag is 0
    outside V, 1 explained, 2 distance outlier, 3 colour outlier.  search:
    "brute" or "window", as for score().
    """
    lib = _load()
    if search not in ("brute", "window"):
        raise ValueError(f"unknown search {search!r}")
    fn = lib.oracle_score_detail if search == "brute" else lib.oracle_score_detail_windowed
    m = _MeshArgs(mesh)
    s = _SceneArgs(scene, delta_mm, tau_c, flags, stride)
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    W, H = int(scene.K[0]), int(scene.K[1])
    out = np.zeros(4, np.int32)
    rf = np.zeros((H, W), np.uint8)
    of = np.zeros((H, W), np.uint8)
    rc = fn(ctypes.byref(m.s), ctypes.byref(s.s), int(label), _ptr(pose), _ptr(out), _ptr(rf), _ptr(of))
    if rc != 0:
        raise ValueError(f"oracle_score_detail failed ({rc})")
    return tuple(int(v) for v in out), rf, of


def best(jr, jo):
    """argmin of J = J_r + J_o, lowest index among ties (Sec. IV-A)."""
    lib = _load()
    jr = np.ascontiguousarray(jr, dtype=np.int32)
    jo = np.ascontiguousarray(jo, dtype=np.int32)
    bi = np.zeros(1, np.int32)
    bc = np.zeros(1, np.int32)
    nt = np.zeros(1, np.int32)
    rc = lib.oracle_best(_ptr(jr), _ptr(jo), jr.shape[0], _ptr(bi), _ptr(bc), _ptr(nt))
    if rc != 0:
        raise ValueError("oracle_best: empty input")
    return int(bi[0]), int(bc[0]), int(nt[0])


def icp(mesh, scene, poses, *, delta_mm, flags=MARK_OCCLUDERS, label=0, rho_mm=20.0, iterations=10, stride=2,
        dof=3, min_points=16, threads=0):
    """ICP refinement of every pose against the observed cloud (readings
    I1-I8 of the oracle source; Sec. IV-A "Parallel M2M GICP").

    Returns (refined n x 12 float32, updates applied int32, matches of the
    last iteration examined int32)."""
    lib = _load()
    m = _MeshArgs(mesh)
    s = _SceneArgs(scene, delta_mm, 0.0, flags & ~USE_RGB, 1)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    n = poses.shape[0]
    out = np.zeros((n, 12), np.float32)
    it = np.zeros(n, np.int32)
    mt = np.zeros(n, np.int32)
    rc = lib.oracle_icp(ctypes.byref(m.s), ctypes.byref(s.s), int(label), _ptr(poses), n, float(rho_mm),
                        int(iterations), int(stride), int(dof), int(min_points), _ptr(out), _ptr(it), _ptr(mt),
                        int(threads))
    if rc != 0:
        raise ValueError(f"oracle_icp failed ({rc})")
    return out, it, mt


def icp_pairs(src, dst, *, dof=6, axis=(0.0, 0.0, 1.0), iterations=1):
    """The ICP update loop on fixed correspondences (dst[i] matches src[i],
    int32 1/16 mm).  Returns (A 3x3, b 3) with dst ~ A src + b."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32).reshape(-1, 3)
    dst = np.ascontiguousarray(dst, dtype=np.int32).reshape(-1, 3)
    u = np.ascontiguousarray(axis, dtype=np.float64)
    A = np.zeros(9, np.float64)
    b = np.zeros(3, np.float64)
    rc = lib.oracle_icp_pairs(_ptr(src), _ptr(dst), src.shape[0], int(dof), _ptr(u), int(iterations), _ptr(A),
                              _ptr(b))
    if rc != 0:
        raise ValueError(f"oracle_icp_pairs failed ({rc})")
    return A.reshape(3, 3), b


def propose(scene, mesh, label, *, viewpoints, inplane, z_step_mm, max_depths):
    """6-DoF pose proposals of one labelled object (Sec. V-B "Pose Proposal
    Generation"), in plain binary64 numpy.  Readings of the paper:

    P1 Rotations: M viewpoints "equidistant" on the unit sphere, taken as the
       Fibonacci lattice, z_i = 1 - (2i + 1)/M at longitude i pi (3 - sqrt 5);
       the camera sits in direction v_i from the object, so the rotation maps
       v_i to the camera's -z axis: rows b1, b2, b3 with b3 = -v_i,
       b1 = a x b3 / |a x b3| (a = object z axis, or object y axis when
       |z_i| > 0.999), b2 = b3 x b1.
    P2 In-plane angles 2 pi k / N: the rotation above, turned about the
       optical axis, rows (cos b1 - sin b2, sin b1 + cos b2, b3).
    P3 Translations: the object's centre c (the centre of the mesh's
       object-frame AABB) on the ray through the centre of the label's pixel
       box (the visible box; the labels stand in for the segmentation masks),
       u_c = x0 + (w - 1)/2, so t = z_t ((u_c - cx)/fx, (v_c - cy)/fy, 1) - R c,
       at depths z_t = z_min +
       t step, t = 0 .. floor((z_max - z_min)/step), [z_min, z_max] the range
       of valid observed depths under the label; when that is more than
       max_depths depths, max_depths of them spread evenly from z_min to
       z_max.
    P4 Order: pose p = (i N + k) T + t; binary32 [R|t] rows.

    Returns an (M N T, 12) float32 array (empty when the label has no pixel
    with a depth reading)."""
    labels = np.asarray(scene.labels)
    depth = np.asarray(scene.depth)
    mask = labels == label
    ys, xs = np.nonzero(mask)
    d = depth[mask]
    d = d[d > 0]
    if xs.size == 0 or d.size == 0:
        return np.zeros((0, 12), np.float32)
    x0, x1, y0, y1 = int(xs.min()), int(xs.max()), int(ys.min()), int(ys.max())
    zmin, zmax = float(d.min()), float(d.max())
    T = int(np.floor((zmax - zmin) / float(np.float32(z_step_mm)))) + 1
    if T > max_depths:
        T = max_depths
        step = (zmax - zmin) / (T - 1) if T > 1 else 0.0
    else:
        step = float(np.float32(z_step_mm))
    _, _, fx, fy, cx, cy = [float(np.float32(v)) for v in scene.K]
    xyz = np.asarray(mesh.xyz, np.float32).astype(np.float64)
    centre = (xyz.min(0) + xyz.max(0)) / 2.0
    uc = x0 + (x1 - x0) / 2.0
    vc = y0 + (y1 - y0) / 2.0
    out = np.zeros((viewpoints, inplane, T, 12), np.float64)
    golden = np.pi * (3.0 - np.sqrt(5.0))
    for i in range(viewpoints):
        vz = 1.0 - (2 * i + 1) / viewpoints
        r = np.sqrt(max(0.0, 1.0 - vz * vz))
        v = np.array([r * np.cos(i * golden), r * np.sin(i * golden), vz])
        b3 = -v
        a = np.array([0.0, 1.0, 0.0]) if abs(vz) > 0.999 else np.array([0.0, 0.0, 1.0])
        b1 = np.cross(a, b3)
        b1 = b1 / np.linalg.norm(b1)
        b2 = np.cross(b3, b1)
        for k in range(inplane):
            th = 2.0 * np.pi * k / inplane
            R = np.stack([np.cos(th) * b1 - np.sin(th) * b2, np.sin(th) * b1 + np.cos(th) * b2, b3])
            for t in range(T):
                z = zmin + t * step
                ray = np.array([z * ((uc - cx) / fx), z * ((vc - cy) / fy), z])
                tr = np.array([ray[r] - ((R[r, 0] * centre[0] + R[r, 1] * centre[1]) + R[r, 2] * centre[2])
                               for r in range(3)])
                out[i, k, t] = np.concatenate([R, tr[:, None]], axis=1).reshape(12)
    return out.reshape(-1, 12).astype(np.float32)


def gicp(mesh, scene, poses, *, delta_mm, flags=MARK_OCCLUDERS, label=0, rho_mm=20.0, iterations=10, stride=2,
         min_points=16, threads=0):
    """Plane-to-plane GICP refinement (readings G1-G6 of the oracle source;
    Sec. IV-A "Parallel M2M GICP"), 6-DoF.  Returns as `icp`."""
    lib = _load()
    m = _MeshArgs(mesh)
    s = _SceneArgs(scene, delta_mm, 0.0, flags & ~USE_RGB, 1)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    n = poses.shape[0]
    out = np.zeros((n, 12), np.float32)
    it = np.zeros(n, np.int32)
    mt = np.zeros(n, np.int32)
    rc = lib.oracle_gicp(ctypes.byref(m.s), ctypes.byref(s.s), int(label), _ptr(poses), n, float(rho_mm),
                         int(iterations), int(stride), int(min_points), _ptr(out), _ptr(it), _ptr(mt), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_gicp failed ({rc})")
    return out, it, mt


def gicp_pairs(src, dst, src_normals=None, dst_normals=None, *, iterations=1):
    """GICP updates on fixed correspondences (dst[i] matches src[i], int32
    1/16 mm) with unit normals per point (rows of NaN or None: no normal).
    Returns (A 3x3, b 3)."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32).reshape(-1, 3)
    dst = np.ascontiguousarray(dst, dtype=np.int32).reshape(-1, 3)
    n = src.shape[0]

    def norms(x):
        if x is None:
            return np.zeros((n, 3)), np.zeros(n, np.uint8)
        x = np.asarray(x, np.float64).reshape(n, 3)
        has = np.isfinite(x).all(1)
        return np.ascontiguousarray(np.where(has[:, None], x, 0.0)), has.astype(np.uint8)
    sn, sh = norms(src_normals)
    dn, dh = norms(dst_normals)
    A = np.zeros(9, np.float64)
    b = np.zeros(3, np.float64)
    rc = lib.oracle_gicp_pairs(_ptr(src), _ptr(dst), _ptr(sn), _ptr(sh), _ptr(dn), _ptr(dh), n, int(iterations),
                               _ptr(A), _ptr(b))
    if rc != 0:
        raise ValueError(f"oracle_gicp_pairs failed ({rc})")
    return A.reshape(3, 3), b


def normal_image(depth, K, gap_mm):
    """G1 normals of a depth image: H x W x 3 unit vectors, NaN where none."""
    lib = _load()
    depth = np.ascontiguousarray(depth, dtype=np.uint16)
    k = _intr(K)
    out = np.zeros(depth.shape + (3,), np.float64)
    lib.oracle_normal_image(_ptr(depth), ctypes.byref(k), int(gap_mm), _ptr(out))
    return out


def msg_expand(scene, state, mesh, poses, *, delta_mm, tau_c=0.0, flags=MARK_OCCLUDERS, stride=1, label=0,
               threads=0):
    """Edges of the Monotone Scene Generation tree (readings M1-M3) from one
    state to one object at each of its candidate poses.

    state: a sequence of (mesh, label, pose) already placed, in order.
    Returns five int32 arrays (valid, jr, jo, nr, nq); a successor that
    would occlude a placed object has valid 0 and zero costs."""
    lib = _load()
    s = _SceneArgs(scene, delta_mm, tau_c, flags, stride)
    m = _MeshArgs(mesh)
    sm = [_MeshArgs(x[0]) for x in state]
    arr = (ctypes.POINTER(_Mesh) * max(1, len(sm)))(*[ctypes.pointer(a.s) for a in sm])
    sl = np.array([int(x[1]) for x in state] or [0], np.int32)
    sp = np.ascontiguousarray(np.array([np.asarray(x[2], np.float32).reshape(12) for x in state]
                                       or [np.zeros(12, np.float32)]), dtype=np.float32)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    n = poses.shape[0]
    out = [np.zeros(n, np.int32) for _ in range(5)]
    rc = lib.oracle_msg_expand(ctypes.byref(s.s), ctypes.cast(arr, ctypes.c_void_p), _ptr(sl), _ptr(sp),
                               len(state), ctypes.byref(m.s), int(label), _ptr(poses), n,
                               *[_ptr(a) for a in out], int(threads))
    if rc != 0:
        raise ValueError(f"oracle_msg_expand failed ({rc})")
    return tuple(out)


def msg_search(scene, objects, *, beam, delta_mm, tau_c=0.0, flags=MARK_OCCLUDERS, stride=1, threads=0):
    """Beam search over the Monotone Scene Generation tree (reading M4).

    objects: a sequence of (mesh, label, poses (n_k x 12)).  beam: states kept
    per level (0 = all, an exhaustive search).  Returns (cost, sequence) of
    the goal of least (cost, sequence), the sequence a tuple of
    (object, pose index) pairs in placement order, or None when no monotone
    goal exists; also the number of successors scored."""
    level = [(0, ())]
    scored = 0
    for _ in range(len(objects)):
        cand = []
        for cost, seq in level:
            placed = {o for o, _ in seq}
            state = [(objects[o][0], objects[o][1], objects[o][2][k]) for o, k in seq]
            for o, (mesh, label, poses) in enumerate(objects):
                if o in placed:
                    continue
                valid, jr, jo, _, _ = msg_expand(scene, state, mesh, poses, delta_mm=delta_mm, tau_c=tau_c,
                                                 flags=flags, stride=stride, label=label, threads=threads)
                scored += len(valid)
                for k in np.flatnonzero(valid):
                    cand.append((cost + int(jr[k]) + int(jo[k]), seq + ((o, int(k)),)))
        cand.sort()
        level = cand if beam <= 0 else cand[:beam]
        if not level:
            return None, scored
    return level[0], scored
