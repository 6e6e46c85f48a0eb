"""MI355X-native PERCH 2.0 pose scoring: Python binding of libperch.so.

The binding only marshals arguments to the C ABI declared in
``include/perch.h``; every step of rendering and scoring runs in the HIP
kernels of the library.  Torch tensors provide device memory and streams.
There is no fallback: if the library is missing, importing the binding's
entry points raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Context", "PerchError", "load_library", "library_path", "USE_RGB", "MARK_OCCLUDERS",
           "VOL_AABB", "VOL_CYL", "VOL_LABEL", "JO_NN", "KNN2", "KNN1", "HASH"]

USE_RGB = 1
MARK_OCCLUDERS = 2
VOL_AABB = 0 << 4
VOL_CYL = 1 << 4
VOL_LABEL = 2 << 4
JO_NN = 1 << 6
KNN2 = 1 << 7
KNN1 = 1 << 8
HASH = 1 << 9
_VOLUMES = {"aabb": VOL_AABB, "cyl": VOL_CYL, "label": VOL_LABEL}
_JO_MODES = {"exact": 0, "nn": JO_NN}
_SEARCHES = {"table": 0, "knn2": KNN2, "knn1": KNN1, "hash": HASH}

_HERE = os.path.dirname(os.path.abspath(__file__))
_STATUS = {0: "PERCH_OK", -1: "PERCH_EINVAL", -2: "PERCH_ENOMEM", -3: "PERCH_EDEVICE",
           -4: "PERCH_ENOTFOUND", -5: "PERCH_EBUSY"}


class PerchError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class _Intrinsics(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class _SceneInfo(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_size_t), ("table_entries", ctypes.c_int64),
                ("window_x", ctypes.c_int32), ("window_y", ctypes.c_int32),
                ("tile_cap_small", ctypes.c_int32), ("tile_cap_large", ctypes.c_int32),
                ("table_counted_on_host", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Work(ctypes.Structure):
    _fields_ = [("scene_id", ctypes.c_int32), ("mesh_id", ctypes.c_int32), ("label", ctypes.c_int32),
                ("n_poses", ctypes.c_int32), ("poses_dev", ctypes.c_void_p), ("jr_dev", ctypes.c_void_p),
                ("jo_dev", ctypes.c_void_p), ("nr_dev", ctypes.c_void_p), ("nq_dev", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("small_block", ctypes.c_int32), ("small_words", ctypes.c_int32), ("grid", ctypes.c_int32 * 4),
                ("order", ctypes.c_int32), ("key_bands", ctypes.c_int32)]


class _IcpParams(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("max_corr_mm", ctypes.c_float), ("stride", ctypes.c_int32),
                ("dof", ctypes.c_int32), ("min_points", ctypes.c_int32), ("method", ctypes.c_int32)]


class _ProposalParams(ctypes.Structure):
    _fields_ = [("viewpoints", ctypes.c_int32), ("inplane", ctypes.c_int32), ("z_step_mm", ctypes.c_float),
                ("max_depths", ctypes.c_int32)]


class _Placed(ctypes.Structure):
    _fields_ = [("mesh_id", ctypes.c_int32), ("label", ctypes.c_int32), ("pose", ctypes.c_float * 12)]


class _MsgObject(ctypes.Structure):
    _fields_ = [("mesh_id", ctypes.c_int32), ("label", ctypes.c_int32), ("n_poses", ctypes.c_int32),
                ("poses_dev", ctypes.c_void_p)]


class _SceneDesc(ctypes.Structure):
    _fields_ = [("K", _Intrinsics), ("depth_mm", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("labels", ctypes.c_void_p), ("delta_mm", ctypes.c_float), ("tau_c", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("stride", ctypes.c_int32)]


def library_path() -> str:
    return os.environ.get("PERCH_LIBRARY", os.path.join(_HERE, "libperch.so"))


_lib = None


def load_library():
    """Load libperch.so (built by ``paper_2008_00326_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"libperch.so not built ({path}); run paper_2008_00326_amd.build.build()")
    lib = ctypes.CDLL(path)
    P, I32, VP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p
    sig = {
        "perch_create": ([ctypes.c_int, ctypes.c_size_t, P], ctypes.c_int),
        "perch_destroy": ([P], ctypes.c_int),
        "perch_load_mesh": ([P, P, I32, P, I32, P, P], ctypes.c_int),
        "perch_unload_mesh": ([P, I32], ctypes.c_int),
        "perch_set_scene": ([P, P, P], ctypes.c_int),
        "perch_drop_scene": ([P, I32], ctypes.c_int),
        "perch_score_poses": ([P, I32, I32, I32, VP, I32, VP, VP, VP, VP, VP], ctypes.c_int),
        "perch_score_detail": ([P, I32, I32, I32, VP, I32, VP, VP, VP, VP, VP, VP, VP], ctypes.c_int),
        "perch_score_poses_noalloc": ([P, I32, I32, I32, VP, I32, VP, VP, VP, VP, VP], ctypes.c_int),
        "perch_best_poses": ([P, I32, I32, P, P, P, P, P, P, VP], ctypes.c_int),
        "perch_render": ([P, I32, I32, VP, I32, VP, VP, VP, VP], ctypes.c_int),
        "perch_refine_poses": ([P, I32, I32, I32, VP, I32, P, VP, VP, VP, VP], ctypes.c_int),
        "perch_propose_poses": ([P, I32, I32, I32, P, VP, I32, P, VP], ctypes.c_int),
        "perch_msg_expand": ([P, I32, P, I32, I32, I32, VP, I32, VP, VP, VP, VP, VP, VP], ctypes.c_int),
        "perch_msg_search": ([P, I32, P, I32, I32, P, P, P, P, VP], ctypes.c_int),
        "perch_scene_info_get": ([P, I32, P], ctypes.c_int),
        "perch_table_entries": ([P, I32, I32, I32, I32, I32, P], ctypes.c_int),
        "perch_profile_enable": ([P, I32], ctypes.c_int),
        "perch_profile_read": ([P, I32, P, P], ctypes.c_int),
        "perch_last_classes": ([P, VP, I32, P], ctypes.c_int),
        "perch_score_batch": ([P, P, I32, VP], ctypes.c_int),
        "perch_batch_create": ([P, I32, I32, I32, P], ctypes.c_int),
        "perch_batch_set": ([P, P, I32], ctypes.c_int),
        "perch_batch_launch": ([P, VP], ctypes.c_int),
        "perch_batch_wait": ([P, P, P], ctypes.c_int),
        "perch_batch_destroy": ([P], ctypes.c_int),
        "perch_batch_query": ([P], ctypes.c_int),
        "perch_set_tuning": ([P, P], ctypes.c_int),
        "perch_get_tuning": ([P, P], ctypes.c_int),
        "perch_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().perch_last_error().decode(errors="replace")
        raise PerchError(status, msg)


def _np_ptr(a):
    return None if a is None else a.ctypes.data


def _dev_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def table_entries(depth, wx: int, wy: int, dzmm: int) -> int:
    """Entries of the neighbour table of a uint16 mm depth image with pixel
    half-windows (wx, wy) and depth reach dzmm, counted on the host as
    set_scene counts them while the device is busy (-1: windows too wide)."""
    lib = load_library()
    d = np.ascontiguousarray(depth, np.uint16)
    out = ctypes.c_int64()
    _check(lib.perch_table_entries(_np_ptr(d), d.shape[1], d.shape[0], int(wx), int(wy), int(dzmm),
                                   ctypes.byref(out)))
    return int(out.value)


class Context:
    """One device context: resident meshes and scenes, scoring entry points."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.perch_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = device
        self._scene_size = {}

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.perch_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- resident objects -------------------------------------------------
    def load_mesh(self, xyz, tri, rgb=None) -> int:
        xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
        tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
        rgb = None if rgb is None else np.ascontiguousarray(rgb, np.uint8).reshape(-1, 3)
        mid = ctypes.c_int32()
        _check(self._lib.perch_load_mesh(self._h, _np_ptr(xyz), xyz.shape[0], _np_ptr(tri), tri.shape[0],
                                         _np_ptr(rgb), ctypes.byref(mid)))
        return mid.value

    def unload_mesh(self, mesh_id: int):
        _check(self._lib.perch_unload_mesh(self._h, int(mesh_id)))

    def set_scene(self, K, depth, rgb=None, labels=None, *, delta_mm=10.0, tau_c=20.0, flags=None,
                  use_rgb=None, mark_occluders=True, volume="aabb", jo="exact", search="table",
                  stride=1) -> int:
        """Upload an observed scene.  volume: "aabb", "cyl" or "label" (V(O));
        jo: "exact" (any rendered point within delta explains an observed
        point) or "nn" (only the points that are some inlier's nearest
        neighbour are explained); search: "table" (the scene's neighbour
        table), "hash" (a uniform-grid voxel hash of the observed cloud:
        the same results, a fraction of the scene memory), "knn2" (the
        paper's scan of the whole cloud, a slow baseline with the same
        results) or "knn1" (the paper's full distance array, one pose at a
        time, scored by score_poses only).  `flags`, when given, overrides
        use_rgb, mark_occluders, volume, jo and search."""
        depth = np.ascontiguousarray(depth, np.uint16)
        rgb = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        labels = None if labels is None else np.ascontiguousarray(labels, np.int32)
        if flags is None:
            if use_rgb is None:
                use_rgb = rgb is not None
            flags = (USE_RGB if use_rgb else 0) | (MARK_OCCLUDERS if mark_occluders else 0)
            if volume not in _VOLUMES or jo not in _JO_MODES or search not in _SEARCHES:
                raise ValueError(f"volume must be one of {sorted(_VOLUMES)}, jo one of {sorted(_JO_MODES)}, "
                                 f"search one of {sorted(_SEARCHES)}")
            flags |= _VOLUMES[volume] | _JO_MODES[jo] | _SEARCHES[search]
        w, h, fx, fy, cx, cy = K
        desc = _SceneDesc(_Intrinsics(int(w), int(h), float(fx), float(fy), float(cx), float(cy)),
                          _np_ptr(depth), _np_ptr(rgb), _np_ptr(labels), float(delta_mm), float(tau_c),
                          int(flags), int(stride))
        sid = ctypes.c_int32()
        _check(self._lib.perch_set_scene(self._h, ctypes.byref(desc), ctypes.byref(sid)))
        self._scene_size[sid.value] = (int(w), int(h))
        return sid.value

    def drop_scene(self, scene_id: int):
        _check(self._lib.perch_drop_scene(self._h, int(scene_id)))
        self._scene_size.pop(int(scene_id), None)

    def scene_info(self, scene_id: int) -> dict:
        """HBM footprint, neighbour-table size, search windows and tile classes of a scene."""
        info = _SceneInfo()
        _check(self._lib.perch_scene_info_get(self._h, int(scene_id), ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in _SceneInfo._fields_}

    # -- scoring -----------------------------------------------------------
    def score_poses(self, scene_id, mesh_id, poses, *, label=0, out=None, counts=True, stream=None):
        """Score a (n, 12) float32 CUDA tensor of poses.  Returns (jr, jo, nr, nq)
        int32 CUDA tensors (nr, nq None when counts=False).  Asynchronous."""
        import torch
        if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()):
            raise ValueError("poses must be a contiguous float32 CUDA tensor")
        n = poses.numel() // 12
        if out is None:
            jr = torch.empty(n, dtype=torch.int32, device=poses.device)
            jo = torch.empty_like(jr)
            nr = torch.empty_like(jr) if counts else None
            nq = torch.empty_like(jr) if counts else None
        else:
            jr, jo, nr, nq = out
        if stream is None:
            stream = torch.cuda.current_stream(poses.device)
        _check(self._lib.perch_score_poses(self._h, int(scene_id), int(mesh_id), int(label), _dev_ptr(poses), n,
                                           _dev_ptr(jr), _dev_ptr(jo), _dev_ptr(nr), _dev_ptr(nq),
                                           _stream_ptr(stream)))
        return jr, jo, nr, nq

    def score_poses_noalloc(self, scene_id, mesh_id, poses, out, *, label=0, stream=None):
        """perch_score_poses_noalloc: score_poses into caller-provided outputs
        out = (jr, jo, nr, nq) (int32 CUDA tensors; nr, nq may be None) with
        no allocation by the library.  Asynchronous."""
        import torch
        if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()):
            raise ValueError("poses must be a contiguous float32 CUDA tensor")
        n = poses.numel() // 12
        jr, jo, nr, nq = out
        if stream is None:
            stream = torch.cuda.current_stream(poses.device)
        _check(self._lib.perch_score_poses_noalloc(self._h, int(scene_id), int(mesh_id), int(label), _dev_ptr(poses),
                                                   n, _dev_ptr(jr), _dev_ptr(jo), _dev_ptr(nr), _dev_ptr(nq),
                                                   _stream_ptr(stream)))
        return jr, jo, nr, nq

    def score_detail(self, scene_id, mesh_id, poses, *, label=0, stream=None):
        """perch_score_detail: scores and per-pixel classes of up to 256 poses.
        Returns (jr, jo, nr, nq, rflag, oflag) CUDA tensors; rflag / oflag are
        (n, H, W) uint8.  Asynchronous."""
        import torch
        if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()):
            raise ValueError("poses must be a contiguous float32 CUDA tensor")
        n = poses.numel() // 12
        W, H = self._scene_size[int(scene_id)]
        jr = torch.empty(n, dtype=torch.int32, device=poses.device)
        jo, nr, nq = torch.empty_like(jr), torch.empty_like(jr), torch.empty_like(jr)
        rflag = torch.empty((n, H, W), dtype=torch.uint8, device=poses.device)
        oflag = torch.empty_like(rflag)
        if stream is None:
            stream = torch.cuda.current_stream(poses.device)
        _check(self._lib.perch_score_detail(self._h, int(scene_id), int(mesh_id), int(label), _dev_ptr(poses), n,
                                            _dev_ptr(jr), _dev_ptr(jo), _dev_ptr(nr), _dev_ptr(nq), _dev_ptr(rflag),
                                            _dev_ptr(oflag), _stream_ptr(stream)))
        return jr, jo, nr, nq, rflag, oflag

    def best_poses(self, scene_id, mesh_ids, labels, poses_list, stream=None):
        """Per object (mesh_ids[k], labels[k], poses_list[k] CUDA tensor): the
        index and cost of the minimum-cost pose.  Blocks."""
        import torch
        k = len(mesh_ids)
        mids = np.ascontiguousarray(mesh_ids, np.int32)
        labs = np.ascontiguousarray(labels, np.int32)
        ptrs = (ctypes.c_void_p * k)(*[p.data_ptr() for p in poses_list])
        ns = np.ascontiguousarray([p.numel() // 12 for p in poses_list], np.int32)
        bi = np.zeros(k, np.int32)
        bc = np.zeros(k, np.int32)
        if stream is None:
            stream = torch.cuda.current_stream(poses_list[0].device)
        _check(self._lib.perch_best_poses(self._h, int(scene_id), k, _np_ptr(mids), _np_ptr(labs), ptrs, _np_ptr(ns),
                                          _np_ptr(bi), _np_ptr(bc), _stream_ptr(stream)))
        return bi, bc

    def set_tuning(self, tuning=None):
        """Set the launch tuning from a dict with any of small_block,
        small_words, grid (4 ints), order; None restores the defaults.
        Results never depend on it."""
        if tuning is None:
            _check(self._lib.perch_set_tuning(self._h, None))
            return
        t = _Tuning()
        t.small_block = int(tuning.get("small_block", 0))
        t.small_words = int(tuning.get("small_words", 0))
        for k, g in enumerate(tuning.get("grid", (0, 0, 0, 0))):
            t.grid[k] = int(g)
        t.order = int(tuning.get("order", 0))
        t.key_bands = int(tuning.get("key_bands", 0))
        _check(self._lib.perch_set_tuning(self._h, ctypes.byref(t)))

    def tuning(self) -> dict:
        """The launch tuning in force, defaults resolved."""
        t = _Tuning()
        _check(self._lib.perch_get_tuning(self._h, ctypes.byref(t)))
        return {"small_block": t.small_block, "small_words": t.small_words, "grid": list(t.grid), "order": t.order,
                "key_bands": t.key_bands}

    PROFILE_SLOTS = ("setup", "score_lds_small", "score_lds_large", "score_lds_tile", "score_device", "argmin",
                     "scene_prep", "render", "icp", "msg", "knn1", "batch_graph")

    def profile(self, enable: bool = True):
        """Start (clearing the record) or stop bracketing kernel launches with HIP events."""
        _check(self._lib.perch_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{slot name: (total ms, launches)} since the last profile(True)."""
        n = len(self.PROFILE_SLOTS)
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int32)
        _check(self._lib.perch_profile_read(self._h, n, _np_ptr(ms), _np_ptr(cnt)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.PROFILE_SLOTS)}

    def score_batch(self, items, stream=None):
        """Score a list of work items in one launch.  Each item is a dict with
        scene, mesh, label, poses (CUDA tensor) and optionally jr, jo, nr, nq
        output tensors (allocated when absent).  Returns the items with their
        outputs filled in (asynchronously)."""
        import torch
        arr, items = _work_array(items)
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(self._lib.perch_score_batch(self._h, ctypes.byref(arr) if len(items) else None, len(items),
                                           _stream_ptr(stream)))
        return items

    def batch(self, max_items: int, max_poses: int, max_image_pixels: int) -> "Batch":
        """A prepared, graph-captured batch of the given capacity."""
        return Batch(self, max_items, max_poses, max_image_pixels)

    def last_classes(self, n: int, stream=None):
        """Footprint class (0..3) of each pose of the last score_poses call on the stream."""
        import torch
        out = np.zeros(n, np.int32)
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(self._lib.perch_last_classes(self._h, _stream_ptr(stream), int(n), _np_ptr(out)))
        return out

    def refine_poses(self, scene_id, mesh_id, poses, *, label=0, rho_mm=20.0, iterations=10, stride=2, dof=3,
                     min_points=16, method="point", out=None, stream=None):
        """ICP refinement of a (n, 12) float32 CUDA tensor of poses against the
        scene; method "point" (point-to-point) or "plane" (GICP, dof 6).
        Returns (refined (n, 12) float32, updates applied int32, matches of
        the last iteration int32) CUDA tensors.  Asynchronous."""
        import torch
        if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()):
            raise ValueError("poses must be a contiguous float32 CUDA tensor")
        n = poses.numel() // 12
        refined = out if out is not None else torch.empty((n, 12), dtype=torch.float32, device=poses.device)
        iters = torch.empty(n, dtype=torch.int32, device=poses.device)
        matched = torch.empty(n, dtype=torch.int32, device=poses.device)
        if method not in ("point", "plane"):
            raise ValueError('method must be "point" or "plane"')
        prm = _IcpParams(int(iterations), float(rho_mm), int(stride), int(dof), int(min_points),
                         1 if method == "plane" else 0)
        if stream is None:
            stream = torch.cuda.current_stream(poses.device)
        _check(self._lib.perch_refine_poses(self._h, int(scene_id), int(mesh_id), int(label), _dev_ptr(poses), n,
                                            ctypes.byref(prm), _dev_ptr(refined), _dev_ptr(iters), _dev_ptr(matched),
                                            _stream_ptr(stream)))
        return refined, iters, matched

    def propose_poses(self, scene_id, mesh_id, label, *, viewpoints=64, inplane=12, z_step_mm=10.0, max_depths=16,
                      stream=None):
        """6-DoF proposals of one labelled object: a (M*N*T, 12) float32 CUDA
        tensor (asynchronous; the count is known at return)."""
        import torch
        prm = _ProposalParams(int(viewpoints), int(inplane), float(z_step_mm), int(max_depths))
        n = ctypes.c_int32()
        _check(self._lib.perch_propose_poses(self._h, int(scene_id), int(mesh_id), int(label), ctypes.byref(prm), None,
                                             0, ctypes.byref(n), None))
        out = torch.empty((n.value, 12), dtype=torch.float32, device=f"cuda:{self.device}")
        if n.value == 0:
            return out
        if stream is None:
            stream = torch.cuda.current_stream(out.device)
        _check(self._lib.perch_propose_poses(self._h, int(scene_id), int(mesh_id), int(label), ctypes.byref(prm),
                                             _dev_ptr(out), n.value, ctypes.byref(n), _stream_ptr(stream)))
        return out

    def msg_expand(self, scene_id, state, mesh_id, poses, *, label=0, stream=None):
        """Edges of the Monotone Scene Generation tree from one state to one
        object at each of its (n, 12) float32 CUDA poses.  state: a sequence
        of (mesh_id, label, pose (12 floats)) already placed, in order.
        Returns (valid, jr, jo, nr, nq) int32 CUDA tensors; blocks while a
        non-empty state is composed and checked."""
        import torch
        if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()):
            raise ValueError("poses must be a contiguous float32 CUDA tensor")
        n = poses.numel() // 12
        arr = (_Placed * max(1, len(state)))()
        for k, (mid, lab, pose) in enumerate(state):
            arr[k].mesh_id = int(mid)
            arr[k].label = int(lab)
            arr[k].pose[:] = [float(x) for x in np.asarray(pose, np.float32).reshape(12)]
        out = [torch.empty(n, dtype=torch.int32, device=poses.device) for _ in range(5)]
        if stream is None:
            stream = torch.cuda.current_stream(poses.device)
        _check(self._lib.perch_msg_expand(self._h, int(scene_id), arr, len(state), int(mesh_id), int(label),
                                          _dev_ptr(poses), n, *[_dev_ptr(t) for t in out], _stream_ptr(stream)))
        return tuple(out)

    def msg_search(self, scene_id, objects, *, beam, stream=None):
        """Beam search over the Monotone Scene Generation tree.  objects: a
        sequence of (mesh_id, label, poses (n, 12) float32 CUDA tensor);
        beam: states kept per level (0 = all).  Returns ((cost, sequence) or
        None, successors scored), the sequence a tuple of (object, pose
        index) pairs in placement order.  Synchronous."""
        import torch
        k = len(objects)
        arr = (_MsgObject * max(1, k))()
        for o, (mid, lab, poses) in enumerate(objects):
            if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()):
                raise ValueError("poses must be contiguous float32 CUDA tensors")
            arr[o].mesh_id = int(mid)
            arr[o].label = int(lab)
            arr[o].n_poses = poses.numel() // 12
            arr[o].poses_dev = _dev_ptr(poses)
        order = (ctypes.c_int32 * max(1, k))()
        pose = (ctypes.c_int32 * max(1, k))()
        cost = ctypes.c_int64()
        scored = ctypes.c_int64()
        dev = objects[0][2].device if k else torch.device("cuda", self.device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(self._lib.perch_msg_search(self._h, int(scene_id), arr, k, int(beam), order, pose,
                                          ctypes.byref(cost), ctypes.byref(scored), _stream_ptr(stream)))
        if cost.value < 0:
            return None, scored.value
        return (cost.value, tuple((order[q], pose[q]) for q in range(k))), scored.value

    def render(self, scene_id, mesh_id, poses, K, *, rgb=False, tri=False, stream=None):
        """Full-image renders of (n, 12) poses: (depth u16, rgb u8 or None, tri i32 or None) tensors."""
        import torch
        n = poses.numel() // 12
        W, H = int(K[0]), int(K[1])
        depth = torch.empty((n, H, W), dtype=torch.int16, device=poses.device)
        col = torch.empty((n, H, W, 3), dtype=torch.uint8, device=poses.device) if rgb else None
        tid = torch.empty((n, H, W), dtype=torch.int32, device=poses.device) if tri else None
        if stream is None:
            stream = torch.cuda.current_stream(poses.device)
        _check(self._lib.perch_render(self._h, int(scene_id), int(mesh_id), _dev_ptr(poses), n, _dev_ptr(depth),
                                      _dev_ptr(col), _dev_ptr(tid), _stream_ptr(stream)))
        return depth, col, tid


def _work_array(items):
    import torch
    out = []
    arr = (_Work * max(len(items), 1))()
    for k, it in enumerate(items):
        poses = it["poses"]
        n = poses.numel() // 12
        it = dict(it)
        for key in ("jr", "jo"):
            if it.get(key) is None:
                it[key] = torch.empty(n, dtype=torch.int32, device=poses.device)
        for key in ("nr", "nq"):
            it.setdefault(key, None)
        arr[k] = _Work(int(it["scene"]), int(it["mesh"]), int(it.get("label", 0)), n, poses.data_ptr(),
                       it["jr"].data_ptr(), it["jo"].data_ptr(),
                       None if it["nr"] is None else it["nr"].data_ptr(),
                       None if it["nq"] is None else it["nq"].data_ptr())
        out.append(it)
    return arr, out


class Batch:
    """A prepared batch: fixed capacity, work descriptors rewritten per set(),
    the launch replayed as one captured HIP graph."""

    def __init__(self, ctx: Context, max_items: int, max_poses: int, max_image_pixels: int):
        self.ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        _check(self._lib.perch_batch_create(ctx._h, int(max_items), int(max_poses), int(max_image_pixels),
                                            ctypes.byref(h)))
        self._h = h
        self.items = []
        self._arr = None

    def set(self, items):
        arr, self.items = _work_array(items)
        self._arr = arr
        _check(self._lib.perch_batch_set(self._h, ctypes.byref(arr), len(self.items)))
        return self.items

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(self._lib.perch_batch_launch(self._h, _stream_ptr(stream)))

    def wait(self):
        """Per item: (index of the minimum-cost pose, its J)."""
        n = len(self.items)
        bi = np.zeros(max(n, 1), np.int32)
        bc = np.zeros(max(n, 1), np.int32)
        _check(self._lib.perch_batch_wait(self._h, _np_ptr(bi), _np_ptr(bc)))
        return bi[:n], bc[:n]

    def done(self) -> bool:
        """True once the last launch has finished (non-blocking)."""
        st = self._lib.perch_batch_query(self._h)
        if st == -5:
            return False
        _check(st)
        return True

    def close(self):
        if getattr(self, "_h", None) and getattr(self.ctx, "_h", None):
            _check(self._lib.perch_batch_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load_workload(ctx: Context, w, *, flags=None):
    """Make a generated workload resident: returns (scene_id, [mesh_id per mesh])."""
    s = w.scene
    sid = ctx.set_scene(s.K, s.depth, s.rgb if w.use_rgb else None,
                        s.labels if w.volume == "label" else None,
                        delta_mm=w.delta_mm, tau_c=w.tau_c, flags=flags, use_rgb=w.use_rgb,
                        mark_occluders=w.mark_occluders, volume=w.volume, jo=getattr(w, "jo", "exact"),
                        search=getattr(w, "search", "table"), stride=w.stride)
    mids = [ctx.load_mesh(m.xyz, m.tri, m.rgb if w.use_rgb else None) for m in w.meshes]
    return sid, mids
