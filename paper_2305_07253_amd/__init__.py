"""Combined BVH + distance-field ray queries on AMD Instinct MI355X.

Thin Python binding over the C ABI of libhyb.so (include/hyb.h): argument
checks and marshalling only.  Every step of a query runs in the library's HIP
kernels; PyTorch provides device memory and streams.  There is no CPU
fallback: if libhyb.so is missing the calls raise.

    import paper_2305_07253_amd as hyb
    bvh = hyb.build_bvh(verts, tris)                 # host numpy arrays
    sdf = hyb.build_sdf(bvh, 128, grid4)             # exact signed distance grid
    t, prim, u, v = hyb.trace(bvh, sdf, rays, tmax=0.5, threshold=1.0)

Rays are a (6, n) float32 CUDA tensor with rows ox, oy, oz, dx, dy, dz (unit
directions); hits come back as float32 t, int32 prim (>= 0 triangle, -2
distance-field hit, -1 miss), float32 u, v.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyb.so")

HYB_MISS = -1
HYB_DF_HIT = -2
EXTERIOR_SOLID = 1
LIPSCHITZ_SAMPLES = 2
UPDATE_DEFERRED = 4
SDF_F32, SDF_F16, SDF_I8_BRICK = 0, 1, 2
MODE_COMBINED, MODE_BVH, MODE_DF, MODE_SHADOW = 0, 1, 2, 3

_STATUS = {0: "HYB_OK", 1: "HYB_ERR_INVALID_ARG", 2: "HYB_ERR_OOM", 3: "HYB_ERR_HIP", 4: "HYB_ERR_UNSUPPORTED"}


class HybError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__("%s failed: %s" % (fn, _STATUS.get(status, status)))


class _Rays(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("ox", "oy", "oz", "dx", "dy", "dz", "tmin", "tmax")]


class _Hits(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("t", "prim", "u", "v")]


class _BatchItem(ctypes.Structure):
    _fields_ = [("bvh", ctypes.c_void_p), ("sdf", ctypes.c_void_p), ("rays", _Rays), ("hits", _Hits),
                ("n", ctypes.c_int64), ("tmax", ctypes.c_float), ("threshold", ctypes.c_float)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("lds_depth", ctypes.c_int32), ("rays_per_item", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class _TuneOpts(ctypes.Structure):
    _fields_ = [("thresholds", ctypes.c_void_p), ("n_thresholds", ctypes.c_int32), ("max_error_rate", ctypes.c_float),
                ("reps", ctypes.c_int32), ("flags", ctypes.c_uint32)]


TUNE_THRESHOLD, TUNE_LAUNCH = 1, 2


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libhyb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhyb.so is not built (run `python -m paper_2305_07253_amd.build`); "
                              "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint32
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "hyb_build_bvh": [P, i64, P, i64, P, PP],
            "hyb_bvh_info": [P, P, P, P],
            "hyb_build_sdf": [P, i32, P, u32, i32, P, PP],
            "hyb_sdf_from_grid": [P, i32, P, u32, i32, P, PP],
            "hyb_sdf_update": [P, P, u32, P],
            "hyb_sdf_info": [P, P, P, P],
            "hyb_sdf_voxel_size": [P, P],
            "hyb_sdf_check": [P, P],
            "hyb_sdf_read": [P, P, P],
            "hyb_trace": [P, P, P, i64, f32, f32, P, P],
            "hyb_trace_bvh": [P, P, i64, f32, P, P],
            "hyb_trace_df": [P, P, i64, f32, P, P],
            "hyb_trace_counters": [P, P, P, i64, f32, f32, i32, P, P, P],
            "hyb_trace_shadow": [P, P, P, i64, f32, f32, f32, P, P],
            "hyb_df_backward": [P, P, i64, f32, P, P, P, P],
            "hyb_bvh_destroy": [P],
            "hyb_sdf_destroy": [P],
            "hyb_batch_create": [P, i32, P, PP],
            "hyb_batch_set_config": [P, P],
            "hyb_batch_get_config": [P, P],
            "hyb_batch_set_threshold": [P, i32, f32],
            "hyb_batch_get_threshold": [P, i32, P],
            "hyb_batch_launch": [P, P],
            "hyb_batch_launch_eager": [P, P],
            "hyb_batch_tune": [P, P, P, P, P],
            "hyb_batch_destroy": [P],
            "hyb_batch_launch_static": [P, i32, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.hyb_status_str.argtypes = [ctypes.c_int]
        L.hyb_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(fn, status):
    if status != 0:
        raise HybError(fn, status)


def _torch():
    import torch
    return torch


def _stream(stream, current=True):
    """hipStream_t of a torch stream; None means torch's current stream for
    trace calls and the default (NULL) stream for the synchronous builds."""
    if stream is None:
        if not current:
            return ctypes.c_void_p(None)
        stream = _torch().cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Bvh:
    """Library-owned triangle BVH (device memory)."""

    def __init__(self, handle):
        self._h = handle
        self._L = lib()
        n_nodes, n_tris, depth = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check("hyb_bvh_info", lib().hyb_bvh_info(handle, ctypes.byref(n_nodes), ctypes.byref(n_tris),
                                                  ctypes.byref(depth)))
        self.n_nodes, self.n_tris, self.depth = n_nodes.value, n_tris.value, depth.value

    @property
    def handle(self):
        return self._h

    def __del__(self):
        # destroyed by the library that made the handle
        L = getattr(self, "_L", None)
        if getattr(self, "_h", None) and L is not None:
            L.hyb_bvh_destroy(self._h)
            self._h = None


class Sdf:
    """Library-owned distance-field grid (device memory)."""

    def __init__(self, handle):
        self._h = handle
        self._L = lib()
        g4 = (ctypes.c_float * 4)()
        n = ctypes.c_int32()
        _check("hyb_sdf_info", lib().hyb_sdf_info(handle, g4, ctypes.byref(n), None))
        self.grid4 = np.array(list(g4), dtype=np.float32)
        self.n = n.value

    @property
    def lipschitz(self) -> float:
        """Lipschitz bound of the stored samples' interpolant (hyb_sdf_info;
        waits for the device after a deferred update)."""
        L = ctypes.c_float()
        _check("hyb_sdf_info", lib().hyb_sdf_info(self._h, None, None, ctypes.byref(L)))
        return L.value

    def check(self, stream=None):
        """Raises HybError if the last deferred update had a sample that is
        not finite (hyb_sdf_check; waits for the stream)."""
        _check("hyb_sdf_check", lib().hyb_sdf_check(self._h, _stream(stream)))

    @property
    def h(self) -> float:
        """Voxel size (hyb_sdf_voxel_size): the unit of the switch thresholds."""
        h = ctypes.c_float()
        _check("hyb_sdf_voxel_size", lib().hyb_sdf_voxel_size(self._h, ctypes.byref(h)))
        return h.value

    @property
    def handle(self):
        return self._h

    def __del__(self):
        # destroyed by the library that made the handle
        L = getattr(self, "_L", None)
        if getattr(self, "_h", None) and L is not None:
            L.hyb_sdf_destroy(self._h)
            self._h = None


def build_bvh(verts, tris, stream=None) -> Bvh:
    """BVH over host arrays verts (V,3) float32 and tris (T,3) int32."""
    v = np.ascontiguousarray(verts, dtype=np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    out = ctypes.c_void_p()
    _check("hyb_build_bvh", lib().hyb_build_bvh(v.ctypes.data_as(ctypes.c_void_p), v.shape[0],
                                                t.ctypes.data_as(ctypes.c_void_p), t.shape[0],
                                                _stream(stream, False), ctypes.byref(out)))
    return Bvh(out)


def build_sdf(bvh: Bvh, n: int, grid4=None, exterior_solid: bool = True, fmt: int = SDF_F32, stream=None) -> Sdf:
    """Exact n^3 signed distance grid of the BVH's mesh; grid4 = [lo_x, lo_y,
    lo_z, h] (float32) or None for the padded mesh bounds."""
    g = None if grid4 is None else np.ascontiguousarray(grid4, dtype=np.float32)
    out = ctypes.c_void_p()
    _check("hyb_build_sdf", lib().hyb_build_sdf(bvh.handle, int(n), None if g is None else g.ctypes.data_as(
        ctypes.c_void_p), EXTERIOR_SOLID if exterior_solid else 0, fmt, _stream(stream, False), ctypes.byref(out)))
    return Sdf(out)


def sdf_from_grid(values, grid4, lipschitz_samples: bool = False, fmt: int = SDF_F32, stream=None) -> Sdf:
    """Wrap a CUDA float32 tensor of n^3 samples (x fastest) as a grid.
    lipschitz_samples certifies the samples are FP32 roundings of a
    1-Lipschitz function (exact distances), which allows longer steps."""
    torch = _torch()
    if not (values.is_cuda and values.dtype == torch.float32 and values.is_contiguous()):
        raise ValueError("values must be a contiguous float32 CUDA tensor")
    n = round(values.numel() ** (1.0 / 3.0))
    if n ** 3 != values.numel():
        raise ValueError("values must hold n^3 samples")
    g = np.ascontiguousarray(grid4, dtype=np.float32)
    out = ctypes.c_void_p()
    _check("hyb_sdf_from_grid", lib().hyb_sdf_from_grid(
        _ptr(values), n, g.ctypes.data_as(ctypes.c_void_p), LIPSCHITZ_SAMPLES if lipschitz_samples else 0, fmt,
        _stream(stream), ctypes.byref(out)))
    return Sdf(out)


def sdf_update(sdf: Sdf, values, lipschitz_samples: bool = False, stream=None, deferred: bool = False) -> Sdf:
    """Replace the samples of `sdf` in place by a CUDA float32 tensor of its
    n^3 samples (x fastest), reusing its device memory; returns sdf.
    deferred: queue the work on the stream without waiting for the device
    (HYB_SDF_UPDATE_DEFERRED; non-finite samples then show as NaN hits and
    through sdf.check())."""
    torch = _torch()
    if not (values.is_cuda and values.dtype == torch.float32 and values.is_contiguous()):
        raise ValueError("values must be a contiguous float32 CUDA tensor")
    if values.numel() != sdf.n ** 3:
        raise ValueError("values must hold the grid's n^3 samples")
    flags = (LIPSCHITZ_SAMPLES if lipschitz_samples else 0) | (UPDATE_DEFERRED if deferred else 0)
    _check("hyb_sdf_update", lib().hyb_sdf_update(sdf.handle, _ptr(values), flags, _stream(stream)))
    return sdf


def sdf_read(sdf: Sdf, stream=None):
    """The samples as the kernels see them: CUDA float32 tensor (n,n,n), [k,j,i]."""
    torch = _torch()
    out = torch.empty((sdf.n, sdf.n, sdf.n), dtype=torch.float32, device="cuda")
    _check("hyb_sdf_read", lib().hyb_sdf_read(sdf.handle, _ptr(out), _stream(stream)))
    return out


def _rays_struct(rays, tmin, tmax_ray=None):
    torch = _torch()
    if not (rays.is_cuda and rays.dtype == torch.float32 and rays.dim() == 2 and rays.shape[0] == 6
            and rays.is_contiguous()):
        raise ValueError("rays must be a contiguous (6, n) float32 CUDA tensor")
    n = rays.shape[1]
    base, step = rays.data_ptr(), 4 * n
    r = _Rays(*[base + k * step for k in range(6)], None, None)
    for name, x in (("tmin", tmin), ("tmax", tmax_ray)):
        if x is not None:
            if not (x.is_cuda and x.dtype == torch.float32 and x.numel() == n and x.is_contiguous()):
                raise ValueError("%s must be a contiguous float32 CUDA tensor of n entries" % name)
            setattr(r, name, x.data_ptr())
    return r, n


def alloc_hits(n: int, device="cuda"):
    torch = _torch()
    return (torch.empty(n, dtype=torch.float32, device=device), torch.empty(n, dtype=torch.int32, device=device),
            torch.empty(n, dtype=torch.float32, device=device), torch.empty(n, dtype=torch.float32, device=device))


def _hits_struct(out, n):
    torch = _torch()
    t, p, u, v = out
    for x, dt in ((t, torch.float32), (p, torch.int32), (u, torch.float32), (v, torch.float32)):
        if not (x.is_cuda and x.dtype == dt and x.numel() >= n and x.is_contiguous()):
            raise ValueError("hit buffers must be contiguous CUDA tensors (f32, i32, f32, f32) of n entries")
    return _Hits(t.data_ptr(), p.data_ptr(), u.data_ptr(), v.data_ptr())


def _query_args(tmax, threshold):
    if not (tmax >= 0.0) or math.isnan(tmax):
        raise ValueError("tmax must be >= 0")
    if threshold is not None and (not (threshold >= 0.0) or math.isnan(threshold)):
        raise ValueError("threshold must be >= 0")


def trace(bvh: Bvh, sdf: Sdf, rays, tmax: float, threshold: float, tmin=None, out=None, stream=None, tmax_ray=None):
    """Combined first-hit query: triangles on [tmin, t1], distance field on
    [t1, tmax], t1 = min(tmin + threshold*h, tmax).  Returns (t, prim, u, v).
    tmax_ray: optional per-ray end (min with tmax)."""
    _query_args(tmax, threshold)
    r, n = _rays_struct(rays, tmin, tmax_ray)
    out = alloc_hits(n) if out is None else out
    h = _hits_struct(out, n)
    _check("hyb_trace", lib().hyb_trace(bvh.handle, sdf.handle, ctypes.byref(r), n, tmax, threshold,
                                        ctypes.byref(h), _stream(stream)))
    return out


def trace_bvh(bvh: Bvh, rays, tmax: float, tmin=None, out=None, stream=None, tmax_ray=None):
    """Pure triangle tracing on [tmin, tmax]."""
    _query_args(tmax, None)
    r, n = _rays_struct(rays, tmin, tmax_ray)
    out = alloc_hits(n) if out is None else out
    h = _hits_struct(out, n)
    _check("hyb_trace_bvh", lib().hyb_trace_bvh(bvh.handle, ctypes.byref(r), n, tmax, ctypes.byref(h),
                                                _stream(stream)))
    return out


def trace_df(sdf: Sdf, rays, tmax: float, tmin=None, out=None, stream=None, tmax_ray=None):
    """Pure distance-field tracing on [tmin, tmax]."""
    _query_args(tmax, None)
    r, n = _rays_struct(rays, tmin, tmax_ray)
    out = alloc_hits(n) if out is None else out
    h = _hits_struct(out, n)
    _check("hyb_trace_df", lib().hyb_trace_df(sdf.handle, ctypes.byref(r), n, tmax, ctypes.byref(h),
                                              _stream(stream)))
    return out


def trace_shadow(bvh: Bvh, sdf: Sdf, rays, tmax: float, threshold_start: float, threshold_end: float, tmin=None,
                 tmax_ray=None, out=None, stream=None):
    """Any-hit shadow query: triangles on [tmin, t1] and [t2, tmax], the
    distance field on [t1, t2] (traced first).  prim -1 unoccluded, -2 DF
    occluder, >= 0 a triangle occluder."""
    _query_args(tmax, threshold_start)
    _query_args(tmax, threshold_end)
    r, n = _rays_struct(rays, tmin, tmax_ray)
    out = alloc_hits(n) if out is None else out
    h = _hits_struct(out, n)
    _check("hyb_trace_shadow", lib().hyb_trace_shadow(bvh.handle, sdf.handle, ctypes.byref(r), n, tmax,
                                                      threshold_start, threshold_end, ctypes.byref(h),
                                                      _stream(stream)))
    return out


def df_backward(sdf: Sdf, rays, tmax: float, t_hit, grad_t, grad_grid, tmin=None, tmax_ray=None, stream=None):
    """grad_grid += d loss / d samples for the DF hits t_hit of hyb_trace_df on
    the same rays and segment (implicit differentiation at the hit)."""
    torch = _torch()
    _query_args(tmax, None)
    r, n = _rays_struct(rays, tmin, tmax_ray)
    for x, m in ((t_hit, n), (grad_t, n), (grad_grid, sdf.n ** 3)):
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.numel() == m):
            raise ValueError("t_hit, grad_t (n) and grad_grid (n_grid^3) must be contiguous float32 CUDA tensors")
    _check("hyb_df_backward", lib().hyb_df_backward(sdf.handle, ctypes.byref(r), n, tmax, _ptr(t_hit), _ptr(grad_t),
                                                    _ptr(grad_grid), _stream(stream)))
    return grad_grid


def trace_counters(bvh, sdf, rays, tmax: float, threshold: float, mode: int = MODE_COMBINED, tmin=None,
                   stream=None, tmax_ray=None):
    """The same query with per-ray work counters: returns (t, prim, u, v) and
    an int32 (n, 3) tensor of [BVH nodes, triangles tested, DF sample fetches]."""
    torch = _torch()
    _query_args(tmax, threshold)
    r, n = _rays_struct(rays, tmin, tmax_ray)
    out = alloc_hits(n)
    h = _hits_struct(out, n)
    counts = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    _check("hyb_trace_counters", lib().hyb_trace_counters(
        None if bvh is None else bvh.handle, None if sdf is None else sdf.handle, ctypes.byref(r), n, tmax,
        threshold, mode, ctypes.byref(h), _ptr(counts), _stream(stream)))
    return out, counts


def _batch_items(items):
    """The hyb_batch_item array of a sequence of item dicts (see Batch), the
    objects it points at, and each item's hit buffers."""
    items = list(items)
    arr = (_BatchItem * len(items))()
    keep, outs = [], []
    for k, it in enumerate(items):
        thr = float(it["threshold"])
        _query_args(float(it["tmax"]), thr)
        r, n = _rays_struct(it["rays"], it.get("tmin"), it.get("tmax_ray"))
        out = it.get("out") or alloc_hits(n)
        arr[k].bvh = None if it.get("bvh") is None else it["bvh"].handle
        arr[k].sdf = None if it.get("sdf") is None else it["sdf"].handle
        arr[k].rays = r
        arr[k].hits = _hits_struct(out, n)
        arr[k].n = n
        arr[k].tmax = float(it["tmax"])
        arr[k].threshold = thr
        keep.append((it.get("bvh"), it.get("sdf"), it["rays"], it.get("tmin"), it.get("tmax_ray"), out))
        outs.append(out)
    return arr, keep, outs


STATIC_BATCH_MAX_ITEMS = 256


def batch_launch_static(items, config=None, stream=None):
    """One launch of the batch kernels over `items` (dicts as for Batch) with
    no allocation in the library (hyb_batch_launch_static): the work counter
    and descriptors live in the library's fixed device array.  Returns each
    item's hit buffers.  Launches on one device must not overlap."""
    arr, keep, outs = _batch_items(items)
    cfg = None
    if config is not None:
        cfg = _BatchConfig(int(config["lds_depth"]), int(config["rays_per_item"]), int(config["blocks_per_cu"]))
    _check("hyb_batch_launch_static", lib().hyb_batch_launch_static(
        arr, len(keep), None if cfg is None else ctypes.byref(cfg), _stream(stream)))
    return outs


class Batch:
    """Many independent combined queries run by one persistent kernel (one HIP
    graph launch).  `items` is a sequence of dicts with keys bvh, sdf, rays,
    tmax, threshold and optionally out (hit buffers), tmin, tmax_ray; bvh may
    be None for threshold 0, sdf None for threshold +inf.  The batch keeps
    references to every tensor and handle it points at."""

    def __init__(self, items, stream=None):
        arr, self._keep, self.outs = _batch_items(items)
        h = ctypes.c_void_p()
        _check("hyb_batch_create", lib().hyb_batch_create(arr, len(items), _stream(stream), ctypes.byref(h)))
        self._h = h
        self._L = lib()
        self.n_items = len(items)

    @property
    def handle(self):
        return self._h

    def launch(self, stream=None, graph: bool = True):
        fn = "hyb_batch_launch" if graph else "hyb_batch_launch_eager"
        _check(fn, getattr(lib(), fn)(self._h, _stream(stream)))
        return self.outs

    @property
    def config(self):
        c = _BatchConfig()
        _check("hyb_batch_get_config", lib().hyb_batch_get_config(self._h, ctypes.byref(c)))
        return dict(lds_depth=c.lds_depth, rays_per_item=c.rays_per_item, blocks_per_cu=c.blocks_per_cu)

    @config.setter
    def config(self, cfg):
        c = _BatchConfig(int(cfg["lds_depth"]), int(cfg["rays_per_item"]), int(cfg["blocks_per_cu"]))
        _check("hyb_batch_set_config", lib().hyb_batch_set_config(self._h, ctypes.byref(c)))

    def threshold(self, item: int) -> float:
        v = ctypes.c_float()
        _check("hyb_batch_get_threshold", lib().hyb_batch_get_threshold(self._h, int(item), ctypes.byref(v)))
        return v.value

    def set_threshold(self, item: int, threshold: float):
        _check("hyb_batch_set_threshold", lib().hyb_batch_set_threshold(self._h, int(item), float(threshold)))

    def tune(self, max_error_rate: float, thresholds=None, reps: int = 3, threshold: bool = True,
             launch: bool = True, stream=None):
        """Autotune (synchronous; overwrites the hit buffers).  Returns
        (per-item error rates at the chosen thresholds, fastest batch ms)."""
        cands = None if thresholds is None else np.ascontiguousarray(thresholds, dtype=np.float32)
        o = _TuneOpts(None if cands is None else cands.ctypes.data, 0 if cands is None else len(cands),
                      float(max_error_rate), int(reps),
                      (TUNE_THRESHOLD if threshold else 0) | (TUNE_LAUNCH if launch else 0))
        err = np.zeros(self.n_items, dtype=np.float32)
        ms = ctypes.c_float()
        _check("hyb_batch_tune", lib().hyb_batch_tune(self._h, ctypes.byref(o), err.ctypes.data_as(ctypes.c_void_p),
                                                      ctypes.byref(ms), _stream(stream)))
        return err, ms.value

    def __del__(self):
        # destroyed by the library that made the handle
        L = getattr(self, "_L", None)
        if getattr(self, "_h", None) and L is not None:
            L.hyb_batch_destroy(self._h)
            self._h = None
