"""ctypes wrapper of the sensor simulator (``sensor.c``), built with gcc."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sensor.c")
_LIB = os.path.join(_HERE, "libperch_sensor.so")
_lib = None


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


def build(verbose: bool = False) -> str:
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.ss_cast.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P]
        lib.ss_cast.restype = ctypes.c_int
        _lib = lib
    return _lib


def cast(K, objects):
    """Ray-cast a scene.

    K: (width, height, fx, fy, cx, cy).  objects: list of (mesh, pose 3x4
    float64 object->camera mm, label).  Returns (z float64 H x W, 0 = no hit;
    rgb float32 H x W x 3; labels int32 H x W, -1 = no hit).
    """
    lib = _load()
    W, H = int(K[0]), int(K[1])
    cam = _Camera(W, H, float(K[2]), float(K[3]), float(K[4]), float(K[5]))
    n = len(objects)
    keep = []
    xyz_p = (ctypes.c_void_p * n)()
    tri_p = (ctypes.c_void_p * n)()
    rgb_p = (ctypes.c_void_p * n)()
    nv = np.zeros(n, np.int32)
    nt = np.zeros(n, np.int32)
    poses = np.zeros((n, 12), np.float64)
    labels = np.zeros(n, np.int32)
    for k, (mesh, pose, label) in enumerate(objects):
        x = np.ascontiguousarray(mesh.xyz, np.float32)
        t = np.ascontiguousarray(mesh.tri, np.int32)
        c = None if mesh.rgb is None else np.ascontiguousarray(mesh.rgb, np.uint8)
        keep += [x, t, c]
        xyz_p[k] = x.ctypes.data
        tri_p[k] = t.ctypes.data
        rgb_p[k] = None if c is None else c.ctypes.data
        nv[k], nt[k] = x.shape[0], t.shape[0]
        poses[k] = np.asarray(pose, np.float64).reshape(12)
        labels[k] = label
    z = np.zeros((H, W), np.float64)
    rgb = np.zeros((H, W, 3), np.float32)
    lab = np.zeros((H, W), np.int32)
    rc = lib.ss_cast(ctypes.byref(cam), n, xyz_p, nv.ctypes.data, tri_p, nt.ctypes.data, rgb_p,
                     poses.ctypes.data, labels.ctypes.data, z.ctypes.data, rgb.ctypes.data,
                     lab.ctypes.data)
    if rc != 0:
        raise RuntimeError("sensor simulator failed")
    return z, rgb, lab
