"""Python binding of the C ABI in include/ar.h (argument marshalling only).

Every step of the abstract render runs in the HIP library (libabstract_render.so);
this module converts NumPy / dict inputs to the C structures, uses PyTorch only to
allocate device memory and to name the current HIP stream, and raises if the library
is missing or a call fails.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabstract_render.so")

AR_OK, AR_E_INVALID, AR_E_OOM, AR_E_DEVICE, AR_E_UNSUPPORTED, AR_E_BUDGET = 0, -1, -2, -3, -4, -5
AR_PENDING = 1
AR_POSE_CAMERA6, AR_POSE_ORBIT = 0, 1


class ARError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"abstract-render error {code}: {msg}")
        self.code = code


class SceneDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("cov_factor", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("scale", ctypes.c_void_p)]


class SceneSet(ctypes.Structure):
    _fields_ = [("nvar", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("lo", ctypes.c_double * 6), ("hi", ctypes.c_double * 6),
                ("rgb_hi", ctypes.c_void_p), ("opacity_lo", ctypes.c_void_p),
                ("mean_var", ctypes.c_void_p), ("mean_dir", ctypes.c_void_p)]


# keys of a scene dict that make it a set of scenes (see SceneSet)
SET_KEYS = ("rgb_hi", "opacity_lo", "set_lo", "set_hi", "mean_var", "mean_dir")


class Intrinsics(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class PoseBox(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("R0", ctypes.c_double * 9), ("t0", ctypes.c_double * 3),
                ("pivot", ctypes.c_double * 3), ("lo", ctypes.c_double * 6), ("hi", ctypes.c_double * 6)]


class Options(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("ind_window", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("taylor_k", ctypes.c_int32), ("cull_budget", ctypes.c_double),
                ("z_near", ctypes.c_double), ("t_min", ctypes.c_double),
                ("cells_per_launch", ctypes.c_int32), ("prefix_entries", ctypes.c_int32),
                ("abs_sums", ctypes.c_int32), ("ind_copy", ctypes.c_int32), ("ind_masks", ctypes.c_int32),
                ("group_entries", ctypes.c_int32), ("inverse", ctypes.c_int32), ("group_runs", ctypes.c_int32),
                ("ind_quick", ctypes.c_int32)]


# ar_options.inverse: the covariance inverse of Step 3
INVERSE = {"matrixinv": 0, "matrixinv_backward": 1, "adjugate": 2}


class Stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("tile_pairs", ctypes.c_int64),
                ("n_fallback", ctypes.c_int32), ("n_wild", ctypes.c_int32), ("n_dropped", ctypes.c_int32),
                ("P", ctypes.c_int32), ("max_window", ctypes.c_int32), ("segment_length", ctypes.c_int32),
                ("raster_ms", ctypes.c_double), ("total_ms", ctypes.c_double), ("runs", ctypes.c_int64),
                ("cycles_a", ctypes.c_int64), ("cycles_b", ctypes.c_int64), ("ind_tests", ctypes.c_int64),
                ("ind_borderline", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_int32), ("overlap_queue", ctypes.c_int32),
                ("batch_max", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class QueryResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("stats", Stats), ("est_bytes", ctypes.c_uint64),
                ("ws_bytes", ctypes.c_uint64), ("batched", ctypes.c_int32), ("error", ctypes.c_char * 256)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("slots", ctypes.c_int32), ("peak_inflight", ctypes.c_int32),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("hbm_budget", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("pairs", ctypes.c_int64), ("releases", ctypes.c_int64),
                ("shared_launches", ctypes.c_int64), ("shared_queries", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# the exported C symbols and their signatures (the same list as include/ar.h)
SYMBOLS = {
    "ar_scene_create": (ctypes.c_int, [ctypes.POINTER(SceneDesc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ar_scene_create_set": (ctypes.c_int, [ctypes.POINTER(SceneDesc), ctypes.POINTER(SceneSet), ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "ar_scene_destroy": (None, [ctypes.c_void_p]),
    "ar_scene_size": (ctypes.c_int32, [ctypes.c_void_p]),
    "ar_render_bounds": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                        ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ar_render_bounds_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                                ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ar_render_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                       ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ar_render_batch_scenes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Intrinsics),
                                              ctypes.POINTER(PoseBox), ctypes.c_int32, ctypes.POINTER(Options),
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(Stats)]),
    "ar_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                      ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ar_plan_set_cells": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PoseBox)]),
    "ar_plan_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Stats),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "ar_plan_destroy": (None, [ctypes.c_void_p]),
    "ar_render_partitioned": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Options), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ar_classify_cells": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                         ctypes.c_int32, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_void_p]),
    "ar_count_ind_uncertain": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                              ctypes.c_int32, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int64),
                                              ctypes.c_void_p]),
    "ar_render_refined": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox),
                                         ctypes.POINTER(Options), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(PoseBox),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Stats)]),
    "ar_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Intrinsics), ctypes.POINTER(PoseBox), ctypes.c_int32,
                                   ctypes.POINTER(Options), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.POINTER(Options), ctypes.POINTER(Stats)]),
    "ar_last_error": (ctypes.c_char_p, []),
    "ar_version": (ctypes.c_char_p, []),
    "ar_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "ar_server_destroy": (None, [ctypes.c_void_p]),
    "ar_server_add_scene": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "ar_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Intrinsics),
                                        ctypes.POINTER(PoseBox), ctypes.POINTER(Options), ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "ar_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(QueryResult)]),
    "ar_server_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ARError(AR_E_UNSUPPORTED, f"HIP library not built: {path} (run paper_2503_00308_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != AR_OK:
        raise ARError(code, load().ar_last_error().decode())


def intrinsics(d) -> Intrinsics:
    return Intrinsics(int(d["width"]), int(d["height"]), float(d["fx"]), float(d["fy"]),
                      float(d["cx"]), float(d["cy"]))


def pose_box(d) -> PoseBox:
    b = PoseBox()
    b.model = int(d.get("model", AR_POSE_CAMERA6))
    b.R0[:] = [float(v) for v in np.asarray(d.get("R0", np.eye(3)), np.float64).reshape(9)]
    b.t0[:] = [float(v) for v in np.asarray(d.get("t0", np.zeros(3)), np.float64).reshape(3)]
    b.pivot[:] = [float(v) for v in np.asarray(d.get("pivot", np.zeros(3)), np.float64).reshape(3)]
    b.lo[:] = [float(v) for v in np.asarray(d["lo"], np.float64).reshape(6)]
    b.hi[:] = [float(v) for v in np.asarray(d["hi"], np.float64).reshape(6)]
    return b


def options(d=None) -> Options:
    d = d or {}
    return Options(int(d.get("tile", 0)), int(d.get("ind_window", 0)), int(d.get("chunk", 0)),
                   int(d.get("taylor_k", 0)), float(d.get("cull_budget", 0.0)),
                   float(d.get("z_near", 0.0)), float(d.get("t_min", 0.0)),
                   int(d.get("cells_per_launch", 0)), int(d.get("prefix_entries", 0)),
                   int(d.get("abs_sums", 0)), int(d.get("ind_copy", 0)), int(d.get("ind_masks", 0)),
                   int(d.get("group_entries", 0)),
                   INVERSE.get(d.get("inverse", 0), d.get("inverse", 0)), int(d.get("group_runs", 0)),
                   int(d.get("ind_quick", 0)))


class Scene:
    """A device-resident scene (ar_scene handle) built from a dict of arrays:
    mean (N,3), cov_factor (N,3,3) or quat (N,4, w x y z) and scale (N,3), opacity (N,),
    rgb (N,3); with any of the keys rgb_hi (N,3), opacity_lo (N,), set_lo / set_hi
    (nvar,), mean_var (N,), mean_dir (N,3) a set of scenes (ar_scene_create_set)."""

    def __init__(self, scene, stream=None):
        lib = load()
        n = len(scene["mean"])
        # structure-of-arrays, float32, contiguous (the layout include/ar.h specifies)
        self._mean = np.ascontiguousarray(np.asarray(scene["mean"], np.float32).T)
        self._op = np.ascontiguousarray(np.asarray(scene["opacity"], np.float32))
        self._rgb = np.ascontiguousarray(np.asarray(scene["rgb"], np.float32).T)
        self._cov = self._quat = self._scale = None
        if "cov_factor" in scene:
            self._cov = np.ascontiguousarray(np.asarray(scene["cov_factor"], np.float32).reshape(n, 9).T)
        else:
            self._quat = np.ascontiguousarray(np.asarray(scene["quat"], np.float32).reshape(n, 4).T)
            self._scale = np.ascontiguousarray(np.asarray(scene["scale"], np.float32).reshape(n, 3).T)
        ptr = lambda a: a.ctypes.data if a is not None else None
        desc = SceneDesc(n, 0, self._mean.ctypes.data, ptr(self._cov), self._op.ctypes.data, self._rgb.ctypes.data,
                         ptr(self._quat), ptr(self._scale))
        h = ctypes.c_void_p()
        if any(k in scene for k in SET_KEYS):
            st = SceneSet()
            lo = np.asarray(scene.get("set_lo", []), np.float64).reshape(-1)
            hi = np.asarray(scene.get("set_hi", []), np.float64).reshape(-1)
            st.nvar = len(lo)
            st.lo[:len(lo)] = [float(v) for v in lo]
            st.hi[:len(hi)] = [float(v) for v in hi]
            self._keep = []
            if "rgb_hi" in scene:
                self._keep.append(np.ascontiguousarray(np.asarray(scene["rgb_hi"], np.float32).T))
                st.rgb_hi = self._keep[-1].ctypes.data
            if "opacity_lo" in scene:
                self._keep.append(np.ascontiguousarray(np.asarray(scene["opacity_lo"], np.float32)))
                st.opacity_lo = self._keep[-1].ctypes.data
            if "mean_var" in scene:
                self._keep.append(np.ascontiguousarray(np.asarray(scene["mean_var"], np.int32)))
                st.mean_var = self._keep[-1].ctypes.data
            if "mean_dir" in scene:
                self._keep.append(np.ascontiguousarray(np.asarray(scene["mean_dir"], np.float32).T))
                st.mean_dir = self._keep[-1].ctypes.data
            _check(lib.ar_scene_create_set(ctypes.byref(desc), ctypes.byref(st), _stream_ptr(stream), ctypes.byref(h)))
        else:
            _check(lib.ar_scene_create(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.n = n

    def close(self):
        if self.handle:
            load().ar_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def render_bounds(scene: Scene, intr, box, opts=None, stream=None, out=None):
    """Lower / upper images (torch float32 tensors (H, W, 3) on the GPU) and stats.
    out = (lo, hi) may give the output tensors (float32, contiguous; GPU or CPU: host
    outputs are copied back by the library)."""
    import torch
    lib = load()
    ci = intrinsics(intr)
    H, W = ci.height, ci.width
    if out is None:
        lo = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        hi = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    else:
        lo, hi = out
    st = Stats()
    cb = pose_box(box)
    co = options(opts)
    _check(lib.ar_render_bounds(scene.handle, ctypes.byref(ci), ctypes.byref(cb), ctypes.byref(co),
                                ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                _stream_ptr(stream), ctypes.byref(st)))
    return lo, hi, st.as_dict()


def render_bounds_noalloc(scene: Scene, intr, box, out, opts=None, stream=None):
    """ar_render_bounds_noalloc into the caller's output tensors out = (lo, hi) (device,
    float32 (H, W, 3)); returns the stats.  Translation boxes only; the library's static
    scratch array holds every buffer, so the call allocates nothing."""
    lib = load()
    ci = intrinsics(intr)
    lo, hi = out
    st = Stats()
    cb = pose_box(box)
    co = options(opts)
    _check(lib.ar_render_bounds_noalloc(scene.handle, ctypes.byref(ci), ctypes.byref(cb), ctypes.byref(co),
                                        ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                        _stream_ptr(stream), ctypes.byref(st)))
    return st.as_dict()


class Plan:
    """A planned batched render (ar_plan_*): the batch's launch sequence captured once in a
    HIP graph.  Holds its output tensors lo, hi (ncells, H, W, 3), which hold the cells'
    bounds after creation and after every launch()."""

    def __init__(self, scene: Scene, intr, cells, opts=None, stream=None):
        import torch
        lib = load()
        ci = intrinsics(intr)
        m = len(cells)
        arr = (PoseBox * m)(*[pose_box(c) for c in cells])
        self.lo = torch.empty((m, ci.height, ci.width, 3), dtype=torch.float32, device="cuda")
        self.hi = torch.empty_like(self.lo)
        self.ncells = m
        self.scene = scene
        h = ctypes.c_void_p()
        _check(lib.ar_plan_create(scene.handle, ctypes.byref(ci), arr, m, ctypes.byref(options(opts)),
                                  ctypes.c_void_p(self.lo.data_ptr()), ctypes.c_void_p(self.hi.data_ptr()),
                                  _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def set_cells(self, cells):
        if len(cells) != self.ncells:
            raise ValueError(f"the plan holds {self.ncells} cells")
        arr = (PoseBox * self.ncells)(*[pose_box(c) for c in cells])
        _check(load().ar_plan_set_cells(self.handle, arr))

    def launch(self, stream=None):
        """Replay; returns (stats, replanned)."""
        st = Stats()
        rp = ctypes.c_int32(0)
        _check(load().ar_plan_launch(self.handle, _stream_ptr(stream), ctypes.byref(st), ctypes.byref(rp)))
        return st.as_dict(), bool(rp.value)

    def close(self):
        if getattr(self, "handle", None):
            load().ar_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render_batch(scene: Scene, intr, cells, opts=None, stream=None, out=None):
    """Bounds for a list of pose boxes: tensors (ncells, H, W, 3) and accumulated stats.
    out = (lo, hi) may give the output tensors (float32, contiguous; GPU or CPU: host
    outputs are copied back by the library)."""
    import torch
    lib = load()
    ci = intrinsics(intr)
    H, W = ci.height, ci.width
    m = len(cells)
    arr = (PoseBox * m)(*[pose_box(c) for c in cells])
    if out is None:
        lo = torch.empty((m, H, W, 3), dtype=torch.float32, device="cuda")
        hi = torch.empty((m, H, W, 3), dtype=torch.float32, device="cuda")
    else:
        lo, hi = out
    st = Stats()
    co = options(opts)
    _check(lib.ar_render_batch(scene.handle, ctypes.byref(ci), arr, m, ctypes.byref(co),
                               ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                               _stream_ptr(stream), ctypes.byref(st)))
    return lo, hi, st.as_dict()


def render_batch_scenes(scenes, intr, cells, opts=None, stream=None, out=None):
    """Bounds for a list of pose boxes, cell c rendering scenes[c] (Scene handles, one per
    cell): tensors (ncells, H, W, 3) and accumulated stats (ar_render_batch_scenes)."""
    import torch
    lib = load()
    ci = intrinsics(intr)
    H, W = ci.height, ci.width
    m = len(cells)
    if len(scenes) != m:
        raise ValueError(f"{len(scenes)} scenes for {m} cells")
    arr = (PoseBox * m)(*[pose_box(c) for c in cells])
    handles = (ctypes.c_void_p * m)(*[sc.handle.value if isinstance(sc.handle, ctypes.c_void_p) else sc.handle
                                       for sc in scenes])
    if out is None:
        lo = torch.empty((m, H, W, 3), dtype=torch.float32, device="cuda")
        hi = torch.empty((m, H, W, 3), dtype=torch.float32, device="cuda")
    else:
        lo, hi = out
    st = Stats()
    co = options(opts)
    _check(lib.ar_render_batch_scenes(handles, ctypes.byref(ci), arr, m, ctypes.byref(co),
                                      ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                      _stream_ptr(stream), ctypes.byref(st)))
    return lo, hi, st.as_dict()


def render_partitioned(scene: Scene, intr, box, splits, opts=None, stream=None, out=None):
    """Bounds over a pose box cut into a grid of cells (splits: cuts per axis, up to 6),
    the union of the cells' bounds: tensors (H, W, 3) and the cells' accumulated stats."""
    import torch
    lib = load()
    ci = intrinsics(intr)
    H, W = ci.height, ci.width
    if out is None:
        lo = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        hi = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    else:
        lo, hi = out
    sp = list(splits) + [1] * (6 - len(splits))
    arr = (ctypes.c_int32 * 6)(*[int(v) for v in sp[:6]])
    st = Stats()
    cb = pose_box(box)
    co = options(opts)
    _check(lib.ar_render_partitioned(scene.handle, ctypes.byref(ci), ctypes.byref(cb), arr, ctypes.byref(co),
                                     ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                     _stream_ptr(stream), ctypes.byref(st)))
    return lo, hi, st.as_dict()


REFINE_MATINV = 1
REFINE_NEAR = 2
REFINE_IND = 4


def classify_cells(scene: Scene, intr, cells, opts=None, stream=None):
    """Per pose cell: (MatrixInv failures kept somewhere in the image, near-plane
    straddlers), an int64 array (ncells, 2)."""
    lib = load()
    ci = intrinsics(intr)
    arr = (PoseBox * len(cells))(*[pose_box(c) for c in cells])
    out = (ctypes.c_int64 * (2 * len(cells)))()
    co = options(opts)
    _check(lib.ar_classify_cells(scene.handle, ctypes.byref(ci), arr, len(cells), ctypes.byref(co), out,
                                 _stream_ptr(stream)))
    return np.array(out[:], dtype=np.int64).reshape(len(cells), 2)


def count_ind_uncertain(scene: Scene, intr, cells, opts=None, stream=None):
    """Per pose cell: the ordered pairs of Gaussians sharing a tile list whose depth-order
    test Ind stays undecided (summed over the tile lists), an int64 array (ncells,)."""
    lib = load()
    ci = intrinsics(intr)
    arr = (PoseBox * len(cells))(*[pose_box(c) for c in cells])
    out = (ctypes.c_int64 * len(cells))()
    co = options(opts)
    _check(lib.ar_count_ind_uncertain(scene.handle, ctypes.byref(ci), arr, len(cells), ctypes.byref(co), out,
                                      _stream_ptr(stream)))
    return np.array(out[:], dtype=np.int64)


def _box_dict(b: PoseBox) -> dict:
    return {"model": b.model, "R0": np.array(b.R0[:], np.float64).reshape(3, 3), "t0": np.array(b.t0[:], np.float64),
            "pivot": np.array(b.pivot[:], np.float64), "lo": np.array(b.lo[:], np.float64),
            "hi": np.array(b.hi[:], np.float64)}


def render_refined(scene: Scene, intr, box, max_cells=64, criteria=REFINE_MATINV, opts=None, stream=None, out=None):
    """Bounds over a pose box refined where the criteria flag a cell (REFINE_MATINV,
    REFINE_NEAR, REFINE_IND; cells bisected level by level, united): tensors (H, W, 3),
    the leaf cells (pose-box dicts, in the order they were settled) and the leaves'
    accumulated stats."""
    import torch
    lib = load()
    ci = intrinsics(intr)
    H, W = ci.height, ci.width
    if out is None:
        lo = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        hi = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    else:
        lo, hi = out
    cells = (PoseBox * int(max_cells))()
    n = ctypes.c_int32(0)
    st = Stats()
    cb = pose_box(box)
    co = options(opts)
    _check(lib.ar_render_refined(scene.handle, ctypes.byref(ci), ctypes.byref(cb), ctypes.byref(co), int(max_cells),
                                 int(criteria), ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                 _stream_ptr(stream), cells, ctypes.byref(n), ctypes.byref(st)))
    return lo, hi, [_box_dict(cells[i]) for i in range(n.value)], st.as_dict()


def options_dict(o: Options) -> dict:
    return {f: getattr(o, f) for f, _ in o._fields_}


def autotune(scene: Scene, intr, cells, opts=None, reps: int = 2, stream=None):
    """Binning tile, segment length of the pixel loop and cells per launch tuned on a
    workload (a pose box or a list of cells, as render_batch); returns the tuned options
    (a dict for render_bounds / render_batch), the bounds rendered with them and their
    stats."""
    import torch
    lib = load()
    if isinstance(cells, dict):
        cells = [cells]
    ci = intrinsics(intr)
    H, W = ci.height, ci.width
    m = len(cells)
    arr = (PoseBox * m)(*[pose_box(c) for c in cells])
    lo = torch.empty((m, H, W, 3), dtype=torch.float32, device="cuda")
    hi = torch.empty((m, H, W, 3), dtype=torch.float32, device="cuda")
    st = Stats()
    co = options(opts)
    tuned = Options()
    _check(lib.ar_autotune(scene.handle, ctypes.byref(ci), arr, m, ctypes.byref(co), int(reps),
                           ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()), _stream_ptr(stream),
                           ctypes.byref(tuned), ctypes.byref(st)))
    return options_dict(tuned), lo, hi, st.as_dict()


class Server:
    """Query server over resident scenes (continuous batching; see include/ar.h).

    submit() allocates the two output tensors with torch and keeps them until wait()
    returns them; the server writes them from its own streams."""

    def __init__(self, slots: int = 0, hbm_budget: int = 0, overlap_queue: int = 0, batch_max: int = 0):
        lib = load()
        self.handle = ctypes.c_void_p()
        cfg = ServerConfig(int(hbm_budget), int(slots), int(overlap_queue), int(batch_max), 0)
        _check(lib.ar_server_create(ctypes.byref(cfg), ctypes.byref(self.handle)))
        self._scenes = []
        self._out = {}

    def add_scene(self, scene: "Scene") -> int:
        sid = ctypes.c_int32()
        _check(load().ar_server_add_scene(self.handle, scene.handle, ctypes.byref(sid)))
        self._scenes.append(scene)
        return sid.value

    def submit(self, scene_id: int, intr, box, opts=None) -> int:
        import torch
        ci = intrinsics(intr)
        lo = torch.empty((ci.height, ci.width, 3), dtype=torch.float32, device="cuda")
        hi = torch.empty_like(lo)
        # pending work of torch's stream on this memory finishes before the server's
        # streams write it (waits for torch's stream only, not for queries in flight)
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_int64()
        b = pose_box(box)
        co = options(opts)
        _check(load().ar_server_submit(self.handle, int(scene_id), ctypes.byref(ci), ctypes.byref(b),
                                       ctypes.byref(co), ctypes.c_void_p(lo.data_ptr()),
                                       ctypes.c_void_p(hi.data_ptr()), ctypes.byref(t)))
        self._out[t.value] = (lo, hi)
        return t.value

    def wait(self, ticket: int, block: bool = True):
        """(lo, hi, result dict) of a finished query, or None while it runs (block=False)."""
        r = QueryResult()
        code = load().ar_server_wait(self.handle, int(ticket), 1 if block else 0, ctypes.byref(r))
        if code == AR_PENDING:
            return None
        bufs = self._out.pop(ticket, None)
        _check(code)
        lo, hi = bufs
        res = {"status": r.status, "slot": r.slot, "queue_ms": r.queue_ms, "latency_ms": r.latency_ms,
               "stats": r.stats.as_dict(), "est_bytes": r.est_bytes, "ws_bytes": r.ws_bytes, "batched": r.batched}
        return lo, hi, res

    def report(self) -> dict:
        st = ServerStats()
        _check(load().ar_server_report(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.handle:
            load().ar_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self._out.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
