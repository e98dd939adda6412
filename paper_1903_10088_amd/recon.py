"""Python binding of librecon.so (ctypes).

Argument marshalling only: every step of the reconstruction runs in the
library's HIP kernels.  Device buffers are torch CUDA tensors (float32,
contiguous); the library is handed their data pointers and torch's current
stream.  There is no fallback: if librecon.so is missing or fails to load,
importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librecon.so")

RECON_OK, RECON_INVALID_ARG, RECON_DEVICE, RECON_NUMERIC, RECON_OOM = range(5)


class ReconError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class Geometry_c(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("sad_mm", ctypes.c_double), ("sdd_mm", ctypes.c_double),
                ("fan_half_angle_rad", ctypes.c_double), ("start_angle_rad", ctypes.c_double),
                ("scan_arc_rad", ctypes.c_double)]


class Params_c(ctypes.Structure):
    _fields_ = [("lambda0", ctypes.c_double), ("lambda_inc", ctypes.c_double), ("lambda_dec", ctypes.c_double),
                ("lambda_min", ctypes.c_double), ("mu0_per_mm", ctypes.c_double),
                ("tv_eps_per_mm", ctypes.c_double), ("lambda_compare", ctypes.c_int32),
                ("keep_best", ctypes.c_int32)]


class State_c(ctypes.Structure):
    _fields_ = [("n_done", ctypes.c_int32), ("flags", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("f_prev", ctypes.c_double), ("best_f", ctypes.c_double), ("epoch_sum", ctypes.c_double),
                ("best_n", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTS = ["recon_default_params", "recon_status_string", "recon_last_error", "recon_create", "recon_destroy",
           "recon_project", "recon_backproject", "recon_tv_grad", "recon_os_iterate", "recon_os_iterate_ex",
           "recon_initial_image",
           "recon_subset_size", "recon_set_launch", "recon_check_tables", "recon_count_pairs",
           "recon_time_kernels", "recon_batch_create", "recon_batch_destroy", "recon_batch_initial_images",
           "recon_batch_run", "recon_batch_tune", "recon_batch_set_launch", "recon_batch",
           "recon_cnn_param_count", "recon_cnn_create", "recon_cnn_destroy", "recon_cnn_get_state",
           "recon_cnn_set_state", "recon_cnn_save", "recon_cnn_load", "recon_cnn_forward", "recon_cnn_loss_grad",
           "recon_cnn_adam_step", "recon_cnn_train_step", "recon_cnn_tensor", "recon_cnn_time_kernels",
           "recon_data_residual", "recon_warm_start", "recon_warm_start_noalloc", "recon_warm_start_async",
           "recon_batch_wait", "recon_fbp",
           "recon_rebin_helical", "recon_read_bandwidth", "recon_valu_rate", "recon_batch_check_work"]

_lib = None


def lib():
    """Loads librecon.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1903_10088_amd/build.py (or "
                              "__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, vp = ctypes.POINTER, ctypes.c_void_p
        i32, i64, d, f = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
        L.recon_default_params.argtypes = [P(Params_c)]
        L.recon_default_params.restype = None
        L.recon_status_string.argtypes = [ctypes.c_int]
        L.recon_status_string.restype = ctypes.c_char_p
        L.recon_last_error.restype = ctypes.c_char_p
        L.recon_create.argtypes = [P(Geometry_c), i32, d, P(Params_c), P(vp)]
        L.recon_destroy.argtypes = [vp]
        L.recon_project.argtypes = [vp, vp, vp, i32, vp]
        L.recon_backproject.argtypes = [vp, vp, vp, i32, vp]
        L.recon_tv_grad.argtypes = [vp, vp, vp, vp]
        L.recon_os_iterate.argtypes = [vp, vp, f, vp, i32, P(State_c), vp, vp, vp]
        L.recon_os_iterate_ex.argtypes = [vp, vp, f, vp, i32, P(State_c), vp, vp, vp, vp, vp]
        L.recon_fbp.argtypes = [vp, vp, f, vp, vp]
        L.recon_rebin_helical.argtypes = [P(Geometry_c), i32, d, d, vp, f, P(d), i32, vp, vp]
        L.recon_initial_image.argtypes = [vp, vp, vp]
        L.recon_subset_size.argtypes = [vp, i32, P(i32)]
        L.recon_set_launch.argtypes = [vp, i32, i32]
        L.recon_read_bandwidth.argtypes = [i64, i32, P(d), vp]
        L.recon_valu_rate.argtypes = [i32, i32, P(d), vp]
        L.recon_batch_check_work.argtypes = [P(Geometry_c), i32, i32, i32, P(i64), P(i64)]
        L.recon_check_tables.argtypes = [P(Geometry_c), i32, i32, P(i64), P(i64), P(i64)]
        L.recon_count_pairs.argtypes = [vp, i32, i32, P(i64)]
        L.recon_time_kernels.argtypes = [vp, vp, f, vp, i32, P(d), vp]
        PP = P(vp)
        L.recon_batch_create.argtypes = [P(Geometry_c), i32, i32, d, P(Params_c), P(vp)]
        L.recon_batch_destroy.argtypes = [vp]
        L.recon_batch_initial_images.argtypes = [vp, PP, vp]
        L.recon_batch_run.argtypes = [vp, PP, P(f), PP, i32, PP, vp]
        L.recon_batch_tune.argtypes = [vp, PP, P(f), PP, i32, P(i32), P(i32), vp]
        L.recon_batch_set_launch.argtypes = [vp, i32, i32]
        L.recon_batch.argtypes = [P(Geometry_c), i32, i32, d, P(Params_c), PP, P(f), PP, i32, vp]
        L.recon_data_residual.argtypes = [vp, vp, f, vp, i32, vp, vp]
        L.recon_warm_start.argtypes = [vp, vp, PP, P(f), PP, i32, i32, i32, d, i32, P(d), P(d), P(i32), vp]
        L.recon_warm_start_noalloc.argtypes = [vp, vp, PP, P(f), PP, i32, i32, i32, d, i32, P(d), P(d), P(i32), vp]
        L.recon_warm_start_async.argtypes = [vp, vp, PP, P(f), PP, i32, i32, i32, d, i32, P(d), P(d), P(i32), vp]
        L.recon_batch_wait.argtypes = [vp]
        L.recon_cnn_param_count.argtypes = []
        L.recon_cnn_param_count.restype = i64
        L.recon_cnn_create.argtypes = [P(f), i32, i32, f, P(vp)]
        L.recon_cnn_destroy.argtypes = [vp]
        L.recon_cnn_get_state.argtypes = [vp, P(f), P(f), P(f), P(i32)]
        L.recon_cnn_set_state.argtypes = [vp, P(f), P(f), P(f), i32]
        L.recon_cnn_save.argtypes = [vp, ctypes.c_char_p]
        L.recon_cnn_load.argtypes = [vp, ctypes.c_char_p]
        L.recon_cnn_forward.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.recon_cnn_loss_grad.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
        L.recon_cnn_adam_step.argtypes = [vp, f, vp]
        L.recon_cnn_train_step.argtypes = [vp, vp, vp, i32, i32, f, vp, vp]
        L.recon_cnn_tensor.argtypes = [vp, i32, i32, vp, i64, vp]
        L.recon_cnn_time_kernels.argtypes = [vp, vp, vp, i32, i32, i32, P(d), vp]
        for name in EXPORTS:
            getattr(L, name)
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != RECON_OK:
        msg = lib().recon_last_error().decode(errors="replace")
        raise ReconError(rc, where, msg)


def geometry_c(g) -> Geometry_c:
    """From a phantom.Geometry-like object (n, pixel_mm, n_views, n_channels, sad_mm, sdd_mm, ...)."""
    return Geometry_c(int(g.n), 0, float(g.pixel_mm), int(g.n_views), int(g.n_channels), float(g.sad_mm),
                      float(g.sdd_mm), float(g.fan_half_angle_rad), float(g.start_angle_rad),
                      float(getattr(g, "scan_arc_rad", 0.0)))


def default_params() -> dict:
    p = Params_c()
    lib().recon_default_params(ctypes.byref(p))
    return {name: getattr(p, name) for name, _ in Params_c._fields_}


def batch_check_work(geometries, subsets: int, fp_segments: int = 4):
    """Host-only check of a batch's work tables: (errors, blocks)."""
    n = len(geometries)
    garr = (Geometry_c * max(1, n))(*[geometry_c(g) for g in geometries])
    e, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().recon_batch_check_work(garr, n, subsets, fp_segments, ctypes.byref(e), ctypes.byref(b)),
           "recon_batch_check_work")
    return int(e.value), int(b.value)


def read_bandwidth(nbytes: int = 2 << 20, reps: int = 10) -> float:
    """recon_read_bandwidth: GB/s that 2048 blocks reading an L2-resident buffer of nbytes achieve."""
    out = ctypes.c_double()
    _check(lib().recon_read_bandwidth(int(nbytes), int(reps), ctypes.byref(out), _stream()), "recon_read_bandwidth")
    return float(out.value)


VALU_OPS = ("v_fmac_f32", "v_add_f32", "v_add_u32", "v_cvt_f32_i32", "v_lshl_add_u64", "v_dot2c_f32_bf16")


def valu_rate(op: int, reps: int = 5) -> float:
    """recon_valu_rate: lane operations per second of one VALU instruction (VALU_OPS[op])."""
    out = ctypes.c_double()
    _check(lib().recon_valu_rate(int(op), int(reps), ctypes.byref(out), _stream()), "recon_valu_rate")
    return float(out.value)


def check_tables(g, subsets: int, view_stride: int = 1):
    """Host-only check of the gather's candidate windows: (missed, candidates, pairs)."""
    m, c, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().recon_check_tables(ctypes.byref(geometry_c(g)), subsets, view_stride, ctypes.byref(m),
                                    ctypes.byref(c), ctypes.byref(p)), "recon_check_tables")
    return int(m.value), int(c.value), int(p.value)


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor"):
    torch = _torch()
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class State:
    """Resumable iteration state (mirrors recon_state)."""

    def __init__(self, n_done: int = 0, lam: float = 0.0, f_prev: float = 0.0, flags: int = 0):
        self.c = State_c(n_done, flags, lam, f_prev, 0.0, 0.0, 0, 0)

    n_done = property(lambda self: self.c.n_done)
    lam = property(lambda self: self.c.lambda_)
    f_prev = property(lambda self: self.c.f_prev)
    flags = property(lambda self: self.c.flags)
    best_f = property(lambda self: self.c.best_f)
    best_n = property(lambda self: self.c.best_n)
    epoch_sum = property(lambda self: self.c.epoch_sum)


class Recon:
    """One geometry, M subsets and TV weight beta on the current HIP device."""

    def __init__(self, geometry, subsets: int, beta: float, params: dict | None = None):
        self.geometry = geometry
        self.subsets = int(subsets)
        self.beta = float(beta)
        p = default_params()
        if params:
            p.update(params)
        self.params = p
        pc = Params_c(**p)
        h = ctypes.c_void_p()
        _check(lib().recon_create(ctypes.byref(geometry_c(geometry)), self.subsets, self.beta, ctypes.byref(pc),
                                  ctypes.byref(h)), "recon_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().recon_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ----------------------------------------------------------
    @property
    def n(self):
        return self.geometry.n

    def subset_size(self, subset: int) -> int:
        out = ctypes.c_int32()
        _check(lib().recon_subset_size(self._h, subset, ctypes.byref(out)), "recon_subset_size")
        return int(out.value)

    def count_pairs(self, subset: int = -1, disc_only: bool = False) -> int:
        out = ctypes.c_int64()
        _check(lib().recon_count_pairs(self._h, subset, int(bool(disc_only)), ctypes.byref(out)),
               "recon_count_pairs")
        return int(out.value)

    def data_residual(self, counts, i0: float, img, subset_stride: int = 1):
        """(mean (l - p)^2, mean 1 / max(y, 1)) over the rays of every subset_stride-th subset (1: all
        rays) as a float64 CUDA tensor [2]."""
        torch = _torch()
        g = self.geometry
        out = torch.empty(2, dtype=torch.float64, device=img.device)
        _check(lib().recon_data_residual(self._h, _ptr(counts, torch.float32, (g.n_views, g.n_channels), "counts"),
                                         float(i0), _ptr(img, torch.float32, (g.n, g.n), "img"), int(subset_stride),
                                         _ptr(out, torch.float64, (2,), "out"), _stream()), "recon_data_residual")
        return out

    def fbp(self, counts, i0: float, out=None):
        """recon_fbp: filtered backprojection of the counts, a float32 CUDA tensor [n][n] in 1/mm."""
        torch = _torch()
        g = self.geometry
        if out is None:
            out = torch.empty((g.n, g.n), dtype=torch.float32, device=counts.device)
        _check(lib().recon_fbp(self._h, _ptr(counts, torch.float32, (g.n_views, g.n_channels), "counts"), float(i0),
                               _ptr(out, torch.float32, (g.n, g.n), "img"), _stream()), "recon_fbp")
        return out

    def time_kernels(self, counts, i0: float, img, n_iter: int):
        """Mean kernel durations (ms): (fp, 0, bp_update) over n_iter back-to-back launches of each,
        then (bp_update, fp) over launches in sub-iteration order, each between events of its own."""
        torch = _torch()
        g = self.geometry
        out = (ctypes.c_double * 5)()
        _check(lib().recon_time_kernels(self._h, _ptr(counts, torch.float32, (g.n_views, g.n_channels), "counts"),
                                        float(i0), _ptr(img, torch.float32, (g.n, g.n), "img"), int(n_iter), out,
                                        _stream()), "recon_time_kernels")
        return tuple(out)

    def set_launch(self, fp_segments: int = 0, bp_variant: int = 0):
        """fp_segments in {1,2,4,8,16}; bp_variant 1-6 as recon_set_launch numbers them; 0 keeps."""
        _check(lib().recon_set_launch(self._h, fp_segments, bp_variant), "recon_set_launch")

    # -- operators ---------------------------------------------------------
    def project(self, img, subset: int = -1, out=None):
        torch = _torch()
        g = self.geometry
        rows = self.subset_size(subset)
        if out is None:
            out = torch.empty((rows, g.n_channels), dtype=torch.float32, device=img.device)
        _check(lib().recon_project(self._h, _ptr(img, torch.float32, (g.n, g.n), "img"),
                                   _ptr(out, torch.float32, (rows, g.n_channels), "sino"), subset, _stream()),
               "recon_project")
        return out

    def backproject(self, sino, subset: int = -1, out=None):
        torch = _torch()
        g = self.geometry
        rows = self.subset_size(subset)
        if out is None:
            out = torch.empty((g.n, g.n), dtype=torch.float32, device=sino.device)
        _check(lib().recon_backproject(self._h, _ptr(sino, torch.float32, (rows, g.n_channels), "sino"),
                                       _ptr(out, torch.float32, (g.n, g.n), "img"), subset, _stream()),
               "recon_backproject")
        return out

    def tv_grad(self, img, out=None):
        torch = _torch()
        g = self.geometry
        if out is None:
            out = torch.empty_like(img)
        _check(lib().recon_tv_grad(self._h, _ptr(img, torch.float32, (g.n, g.n), "img"),
                                   _ptr(out, torch.float32, (g.n, g.n), "grad"), _stream()), "recon_tv_grad")
        return out

    def initial_image(self, device="cuda"):
        torch = _torch()
        out = torch.empty((self.n, self.n), dtype=torch.float32, device=device)
        return self.initial_image_(out)

    def initial_image_(self, out):
        """Writes the homogeneous start image into `out` ([n][n] float32) and returns it."""
        torch = _torch()
        _check(lib().recon_initial_image(self._h, _ptr(out, torch.float32, (self.n, self.n), "img"), _stream()),
               "recon_initial_image")
        return out

    def os_iterate(self, counts, i0: float, img=None, n_iter: int = 1, state: State | None = None,
                   trace: bool = False, lambda_schedule=None, f_hist=None, best=None):
        """Runs n_iter sub-iterations in place on img (created from the homogeneous start if None).

        f_hist: None or a float64 CUDA tensor [M], the per-subset history that params lambda_compare
        reads (pass the same tensor again to resume).  best: float32 CUDA tensor [n][n] receiving the
        kept iterate; required exactly when params keep_best is set (recon_os_iterate_ex).
        Returns (img, trace) with trace a float64 CUDA tensor [n_iter][2] of (f_n, lambda_n) or None."""
        torch = _torch()
        g = self.geometry
        if img is None:
            img = self.initial_image(counts.device)
        tr = torch.empty((n_iter, 2), dtype=torch.float64, device=counts.device) if trace else None
        sched = None
        if lambda_schedule is not None:
            sched = torch.as_tensor(np.asarray(lambda_schedule, dtype=np.float64)).to(counts.device)
            if sched.numel() < n_iter:
                raise ValueError("lambda_schedule shorter than n_iter")
        _check(lib().recon_os_iterate_ex(self._h, _ptr(counts, torch.float32, (g.n_views, g.n_channels), "counts"),
                                         float(i0), _ptr(img, torch.float32, (g.n, g.n), "img"), int(n_iter),
                                         ctypes.byref(state.c) if state is not None else None,
                                         _ptr(tr, torch.float64, None, "trace"),
                                         _ptr(sched, torch.float64, None, "lambda_schedule"),
                                         _ptr(f_hist, torch.float64, (self.subsets,), "f_hist"),
                                         _ptr(best, torch.float32, (g.n, g.n), "best"), _stream()),
               "recon_os_iterate_ex")
        return img, tr


def rebin_helical(geometry, counts, i0: float, pitch_mm: float, z0_mm: float, z_slices, out=None):
    """recon_rebin_helical: helical single-row counts [n_helical][n_channels] (float32 CUDA tensor;
    view h at the angle of view h mod n_views of `geometry`, source z0 + pitch h / n_views) ->
    per-slice full-turn counts [len(z_slices)][n_views][n_channels] by 360-degree linear
    interpolation along z."""
    torch = _torch()
    g = geometry
    nh = int(counts.shape[0])
    zs = [float(z) for z in z_slices]
    if out is None:
        out = torch.empty((len(zs), g.n_views, g.n_channels), dtype=torch.float32, device=counts.device)
    za = (ctypes.c_double * max(1, len(zs)))(*zs)
    gc = geometry_c(g)
    _check(lib().recon_rebin_helical(ctypes.byref(gc), nh, float(pitch_mm), float(z0_mm),
                                     _ptr(counts, torch.float32, (nh, g.n_channels), "counts"), float(i0), za, len(zs),
                                     _ptr(out, torch.float32, (len(zs), g.n_views, g.n_channels), "out"), _stream()),
           "recon_rebin_helical")
    return out


def _ptr_array(tensors, dtype, shapes, name):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, (t, shp) in enumerate(zip(tensors, shapes)):
        arr[i] = _ptr(t, dtype, shp, f"{name}[{i}]")
    return arr


class Batch:
    """Many slices of different geometry reconstructed together (one launch per kernel per sub-iteration)."""

    def __init__(self, geometries, subsets: int, beta: float, params: dict | None = None):
        self.geometries = list(geometries)
        self.subsets = int(subsets)
        self.beta = float(beta)
        p = default_params()
        if params:
            p.update(params)
        self.params = p
        n = len(self.geometries)
        garr = (Geometry_c * n)(*[geometry_c(g) for g in self.geometries])
        h = ctypes.c_void_p()
        _check(lib().recon_batch_create(garr, n, self.subsets, self.beta, ctypes.byref(Params_c(**p)),
                                        ctypes.byref(h)), "recon_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().recon_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.geometries)

    def _img_shapes(self):
        return [(g.n, g.n) for g in self.geometries]

    def _count_shapes(self):
        return [(g.n_views, g.n_channels) for g in self.geometries]

    def initial_images(self, device="cuda"):
        torch = _torch()
        imgs = [torch.empty((g.n, g.n), dtype=torch.float32, device=device) for g in self.geometries]
        _check(lib().recon_batch_initial_images(self._h, _ptr_array(imgs, torch.float32, self._img_shapes(), "img"),
                                                _stream()), "recon_batch_initial_images")
        return imgs

    def initial_images_into(self, imgs):
        """Writes every slice's homogeneous start image into the given [n][n] tensors."""
        torch = _torch()
        _check(lib().recon_batch_initial_images(self._h, _ptr_array(imgs, torch.float32, self._img_shapes(), "img"),
                                                _stream()), "recon_batch_initial_images")
        return imgs

    def run(self, counts, i0s, imgs=None, n_iter: int = 1, trace: bool = False):
        """Runs n_iter sub-iterations of every slice (fresh state); imgs updated in place.

        Returns (imgs, traces) with traces a list of float64 [n_iter][2] tensors or None."""
        torch = _torch()
        if imgs is None:
            imgs = self.initial_images(counts[0].device)
        traces = None
        tarr = None
        if trace:
            traces = [torch.empty((n_iter, 2), dtype=torch.float64, device=counts[0].device) for _ in counts]
            tarr = _ptr_array(traces, torch.float64, [None] * len(traces), "trace")
        i0 = (ctypes.c_float * len(i0s))(*[float(x) for x in i0s])
        _check(lib().recon_batch_run(self._h, _ptr_array(counts, torch.float32, self._count_shapes(), "counts"), i0,
                                     _ptr_array(imgs, torch.float32, self._img_shapes(), "img"), int(n_iter), tarr,
                                     _stream()), "recon_batch_run")
        return imgs, traces

    def tune(self, counts, i0s, imgs, reps: int = 20):
        """Autotunes launch shapes on this batch's data; returns (fp_segments, bp_variant)."""
        torch = _torch()
        i0 = (ctypes.c_float * len(i0s))(*[float(x) for x in i0s])
        fs, bv = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().recon_batch_tune(self._h, _ptr_array(counts, torch.float32, self._count_shapes(), "counts"), i0,
                                      _ptr_array(imgs, torch.float32, self._img_shapes(), "img"), int(reps),
                                      ctypes.byref(fs), ctypes.byref(bv), _stream()), "recon_batch_tune")
        return int(fs.value), int(bv.value)

    def set_launch(self, fp_segments: int = 0, bp_variant: int = 0):
        _check(lib().recon_batch_set_launch(self._h, fp_segments, bp_variant), "recon_batch_set_launch")

    def warm_start(self, net, counts, i0s, imgs=None, n_pre: int = 10, n_refine: int = 40, n_cold: int = 500,
                   residual_ratio: float = 1.0, noalloc: bool = False, check_stride: int = 1,
                   async_fallback: bool = False):
        """recon_warm_start (noalloc: recon_warm_start_noalloc, the entry point that allocates no device
        memory; async_fallback: recon_warm_start_async, whose fallback cold starts are final only after
        wait()): returns (imgs, residual, floor, fallback) with numpy per-slice arrays."""
        if noalloc and async_fallback:
            raise ValueError("noalloc and async_fallback are separate entry points")
        torch = _torch()
        n = len(self.geometries)
        if imgs is None:
            imgs = [torch.empty((g.n, g.n), dtype=torch.float32, device=counts[0].device) for g in self.geometries]
        i0 = (ctypes.c_float * n)(*[float(x) for x in i0s])
        res, flo = np.zeros(n), np.zeros(n)
        fb = np.zeros(n, dtype=np.int32)
        name = ("recon_warm_start_noalloc" if noalloc else
                "recon_warm_start_async" if async_fallback else "recon_warm_start")
        _check(getattr(lib(), name)(self._h, net._h, _ptr_array(counts, torch.float32, self._count_shapes(), "counts"),
                                    i0, _ptr_array(imgs, torch.float32, self._img_shapes(), "img"), int(n_pre),
                                    int(n_refine), int(n_cold), float(residual_ratio), int(check_stride),
                                    res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    flo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream()), name)
        return imgs, res, flo, fb

    def wait(self):
        """recon_batch_wait: blocks until the cold starts of warm_start(async_fallback=True) are done."""
        _check(lib().recon_batch_wait(self._h), "recon_batch_wait")


def _fptr(a):
    """Host float32 numpy array -> ctypes float pointer (None passes NULL)."""
    if a is None:
        return None
    if a.dtype != np.float32 or not a.flags["C_CONTIGUOUS"]:
        raise ValueError("host arrays must be contiguous float32")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Cnn:
    """The warm-start network (recon_cnn.h) on the current HIP device."""

    def __init__(self, params=None, max_batch: int = 8, max_n: int = 512, mu_scale: float = 0.0049):
        self.max_batch, self.max_n, self.mu_scale = int(max_batch), int(max_n), float(mu_scale)
        p = None
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.size != self.param_count():
                raise ValueError(f"params must have {self.param_count()} floats")
        h = ctypes.c_void_p()
        _check(lib().recon_cnn_create(_fptr(p), self.max_batch, self.max_n, self.mu_scale, ctypes.byref(h)),
               "recon_cnn_create")
        self._h = h

    @staticmethod
    def param_count() -> int:
        return int(lib().recon_cnn_param_count())

    def close(self):
        if getattr(self, "_h", None):
            lib().recon_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_state(self):
        """(params, adam_m, adam_v, step) as host float32 arrays."""
        n = self.param_count()
        th, m, v = (np.empty(n, np.float32) for _ in range(3))
        st = ctypes.c_int32()
        _check(lib().recon_cnn_get_state(self._h, _fptr(th), _fptr(m), _fptr(v), ctypes.byref(st)),
               "recon_cnn_get_state")
        return th, m, v, int(st.value)

    def set_state(self, params=None, adam_m=None, adam_v=None, step: int = 0):
        conv = [None if a is None else np.ascontiguousarray(a, dtype=np.float32) for a in (params, adam_m, adam_v)]
        _check(lib().recon_cnn_set_state(self._h, *[_fptr(a) for a in conv], int(step)), "recon_cnn_set_state")

    def save(self, path: str):
        _check(lib().recon_cnn_save(self._h, os.fsencode(path)), "recon_cnn_save")

    def load(self, path: str):
        _check(lib().recon_cnn_load(self._h, os.fsencode(path)), "recon_cnn_load")

    def forward(self, mu, out=None, project: bool = False):
        """mu: float32 CUDA tensor [B][n][n] (1/mm); returns mu_scale * y (in place if out is mu)."""
        torch = _torch()
        B, n, _ = mu.shape
        if out is None:
            out = torch.empty_like(mu)
        _check(lib().recon_cnn_forward(self._h, _ptr(mu, torch.float32, (B, n, n), "mu"),
                                       _ptr(out, torch.float32, (B, n, n), "out"), B, n, int(bool(project)),
                                       _stream()), "recon_cnn_forward")
        return out

    def loss_grad(self, mu, target, grad=None, loss=None):
        """Loss and gradient at the current parameters; grad (float32 [P]) and loss (float64 [1])
        are optional CUDA tensors that receive them."""
        torch = _torch()
        B, n, _ = mu.shape
        _check(lib().recon_cnn_loss_grad(self._h, _ptr(mu, torch.float32, (B, n, n), "mu"),
                                         _ptr(target, torch.float32, (B, n, n), "target"), B, n,
                                         _ptr(grad, torch.float32, (self.param_count(),), "grad"),
                                         _ptr(loss, torch.float64, (1,), "loss"), _stream()), "recon_cnn_loss_grad")
        return grad, loss

    def adam_step(self, lr: float):
        _check(lib().recon_cnn_adam_step(self._h, float(lr), _stream()), "recon_cnn_adam_step")

    def train_step(self, mu, target, lr: float, loss=None):
        torch = _torch()
        B, n, _ = mu.shape
        _check(lib().recon_cnn_train_step(self._h, _ptr(mu, torch.float32, (B, n, n), "mu"),
                                          _ptr(target, torch.float32, (B, n, n), "target"), B, n, float(lr),
                                          _ptr(loss, torch.float64, (1,), "loss"), _stream()),
               "recon_cnn_train_step")
        return loss

    def tensor(self, kind: int, layer: int, batch: int, n: int):
        """Internal tensor of the last call (recon_cnn_tensor): bf16 kinds come back as float32."""
        torch = _torch()
        if kind in (0, 1):
            shape = (batch, n, n) if (kind == 0 and layer == 0) else (batch, n, n, 32)
            raw = torch.empty(shape, dtype=torch.int16, device="cuda")
        else:
            raw = torch.empty((batch, n, n), dtype=torch.float32, device="cuda")
        _check(lib().recon_cnn_tensor(self._h, int(kind), int(layer), ctypes.c_void_p(raw.data_ptr()),
                                      raw.numel() * raw.element_size(), _stream()), "recon_cnn_tensor")
        if kind in (0, 1):
            return raw.view(torch.bfloat16).float()
        return raw

    def time_kernels(self, mu, target, reps: int = 20):
        """Mean ms per launch: (conv32 forward, conv32 dgrad, wgrad32, forward pass, loss_grad)."""
        torch = _torch()
        B, n, _ = mu.shape
        out = (ctypes.c_double * 5)()
        _check(lib().recon_cnn_time_kernels(self._h, _ptr(mu, torch.float32, (B, n, n), "mu"),
                                            _ptr(target, torch.float32, (B, n, n), "target"), B, n, int(reps), out,
                                            _stream()), "recon_cnn_time_kernels")
        return tuple(out)
