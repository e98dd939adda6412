"""FP64 CPU oracle (ctypes wrapper around oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports or links it.

Every function takes geometry in mm and images in 1/mm, as numpy float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, OpenMP).  Returns the library path."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-std=c11",
                        "-Wall", "-shared", "-fPIC", "-o", tmp, SRC_PATH, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pad0", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("sad_mm", ctypes.c_double), ("sdd_mm", ctypes.c_double),
                ("fan_half_angle_rad", ctypes.c_double), ("start_angle_rad", ctypes.c_double),
                ("scan_arc_rad", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("lambda0", ctypes.c_double), ("lambda_inc", ctypes.c_double),
                ("lambda_dec", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("mu0_per_mm", ctypes.c_double), ("tv_eps_per_mm", ctypes.c_double),
                ("lambda_compare", ctypes.c_int32), ("keep_best", ctypes.c_int32)]


class _State(ctypes.Structure):
    _fields_ = [("n_done", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("f_prev", ctypes.c_double),
                ("best_f", ctypes.c_double), ("epoch_sum", ctypes.c_double),
                ("best_n", ctypes.c_int32), ("pad", ctypes.c_int32)]


DEFAULT_PARAMS = dict(lambda0=0.01, lambda_inc=1e-4, lambda_dec=2e-4, lambda_min=1e-4,
                      mu0_per_mm=0.005, tv_eps_per_mm=1e-5, lambda_compare=0, keep_best=0)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        L.oracle_project.argtypes = [P(_Geom), P(d), P(d), P(i32), i32]
        L.oracle_backproject.argtypes = [P(_Geom), P(d), P(d), P(i32), i32]
        L.oracle_fbp.argtypes = [P(_Geom), P(d), P(d)]
        L.oracle_count_pairs.argtypes = [P(_Geom), P(i32), i32, P(i64)]
        L.oracle_ray_major.argtypes = [P(_Geom), P(i32)]
        L.oracle_tv.argtypes = [i32, d, P(d), P(d), P(d)]
        L.oracle_loglik.argtypes = [i64, P(d), P(d)]
        L.oracle_loglik.restype = d
        L.oracle_lambda_next.argtypes = [P(_Params), i32, d, d, d]
        L.oracle_lambda_next.restype = d
        L.oracle_initial_image.argtypes = [P(_Geom), d, P(d)]
        L.oracle_os_iterate.argtypes = [P(_Geom), i32, d, P(_Params), P(d), d, P(d), i32, P(_State),
                                        P(d), P(d), P(d), P(d)]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _g(geom) -> _Geom:
    n, px, nv, nc, sad, sdd, fan, start, arc = geom.as_tuple()
    return _Geom(n, 0, px, nv, nc, sad, sdd, fan, start, arc)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _views(views):
    if views is None:
        return None, 0
    v = np.ascontiguousarray(views, dtype=np.int32)
    return v, len(v)


def subset_views(n_views: int, subsets: int, s: int) -> np.ndarray:
    """Views of subset s: every M-th view starting at s (equal-interval thinning)."""
    return np.arange(s, n_views, subsets, dtype=np.int32)


def project(geom, img, views=None) -> np.ndarray:
    """Joseph line integrals of img (1/mm) for the listed views (default all): [n_sel][n_ch]."""
    img = np.ascontiguousarray(img, dtype=np.float64).reshape(geom.n, geom.n)
    v, nv = _views(views)
    nsel = geom.n_views if v is None else nv
    out = np.zeros((nsel, geom.n_channels), np.float64)
    _check(lib().oracle_project(ctypes.byref(_g(geom)), _dp(img), _dp(out), None if v is None else _ip(v), nv),
           "project")
    return out


def fbp(geom, sino) -> np.ndarray:
    """Fan-beam filtered backprojection of line integrals [n_views][n_ch] over the full turn: [N][N] in
    1/mm (oracle_fbp)."""
    sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(geom.n_views, geom.n_channels)
    out = np.zeros((geom.n, geom.n), np.float64)
    _check(lib().oracle_fbp(ctypes.byref(_g(geom)), _dp(sino), _dp(out)), "fbp")
    return out


def line_integrals(counts, i0: float) -> np.ndarray:
    """p = ln(I0 / max(y, 1)), the measured line integrals the methods use (section 3.C.2)."""
    return np.log(i0 / np.maximum(np.asarray(counts, np.float64), 1.0))


def rebin_helical(geom, counts, i0: float, pitch_mm: float, z0_mm: float, z_slices) -> np.ndarray:
    """Helical single-row fan data -> one full-turn fan sinogram per slice position, by 360-degree
    linear interpolation along z (360LI, Kalender et al. 1990): for view v of a turn and slice z,
    the two helical views at that angle whose source z brackets z are interpolated linearly in z.
    Helical view h has angle start + 2 pi h / n_views and source z0 + pitch h / n_views.  The
    interpolation runs on the measured line integrals ln(I0 / max(y, 1)); the result is returned
    as counts I0 exp(-l), [n_slices][n_views][n_channels] float64, ready for the iterative method.
    Raises ValueError when a slice lacks helical views on either side.  (The paper reconstructs
    helical MVCT slices but does not state its rebinning; this is the textbook method.)"""
    nv, nch = geom.n_views, geom.n_channels
    ell = line_integrals(counts, i0).reshape(-1, nch)
    nh = ell.shape[0]
    v = np.arange(nv)
    out = np.empty((len(z_slices), nv, nch))
    for s, z in enumerate(z_slices):
        q = (float(z) - z0_mm) / pitch_mm - v / nv  # turns since the first view at this angle
        m = np.floor(q)
        w = q - m  # (z - z_lower) / pitch
        h = v + m.astype(np.int64) * nv
        if h.min() < 0 or (h + nv).max() >= nh:
            raise ValueError(f"slice z = {z} mm is not bracketed by the helical views")
        out[s] = i0 * np.exp(-((1.0 - w)[:, None] * ell[h] + w[:, None] * ell[h + nv]))
    return out


def backproject(geom, sino, views=None) -> np.ndarray:
    """Exact transpose of project (weights in mm): [N][N]."""
    v, nv = _views(views)
    nsel = geom.n_views if v is None else nv
    sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(nsel, geom.n_channels)
    out = np.zeros((geom.n, geom.n), np.float64)
    _check(lib().oracle_backproject(ctypes.byref(_g(geom)), _dp(sino), _dp(out),
                                    None if v is None else _ip(v), nv), "backproject")
    return out


def count_pairs(geom, views=None) -> int:
    """Number of (ray, in-image pixel) interpolation pairs over the listed views."""
    v, nv = _views(views)
    out = ctypes.c_int64(0)
    _check(lib().oracle_count_pairs(ctypes.byref(_g(geom)), None if v is None else _ip(v), nv,
                                    ctypes.byref(out)), "count_pairs")
    return int(out.value)


def ray_major(geom) -> np.ndarray:
    """0 = x-major, 1 = y-major, [n_views][n_ch]."""
    out = np.zeros((geom.n_views, geom.n_channels), np.int32)
    _check(lib().oracle_ray_major(ctypes.byref(_g(geom)), _ip(out)), "ray_major")
    return out


def tv(img, eps: float):
    """(TV value, g_R = -dTV/dmu) of an N x N image."""
    img = np.ascontiguousarray(img, dtype=np.float64)
    n = img.shape[0]
    val = ctypes.c_double(0)
    grad = np.zeros_like(img)
    _check(lib().oracle_tv(n, eps, _dp(img), ctypes.byref(val), _dp(grad)), "tv")
    return float(val.value), grad


def loglik(ell, ytilde) -> float:
    ell = np.ascontiguousarray(ell, dtype=np.float64).ravel()
    yt = np.ascontiguousarray(ytilde, dtype=np.float64).ravel()
    return float(lib().oracle_loglik(ell.size, _dp(ell), _dp(yt)))


def lambda_next(first: bool, lam_prev: float, f_n: float, f_prev: float, params=None) -> float:
    p = _Params(**(params or DEFAULT_PARAMS))
    return float(lib().oracle_lambda_next(ctypes.byref(p), int(first), lam_prev, f_n, f_prev))


def initial_image(geom, mu0_per_mm: float = 0.005) -> np.ndarray:
    out = np.zeros((geom.n, geom.n), np.float64)
    _check(lib().oracle_initial_image(ctypes.byref(_g(geom)), mu0_per_mm, _dp(out)), "initial_image")
    return out


class State:
    """Resumable iteration state (sub-iterations done, lambda, previous f, flags)."""

    def __init__(self):
        self._s = _State(0, 0, 0.0, 0.0, 0.0, 0.0, 0, 0)

    @property
    def best_f(self):
        return self._s.best_f

    @property
    def best_n(self):
        return self._s.best_n

    @property
    def n_done(self):
        return self._s.n_done

    @property
    def lam(self):
        return self._s.lambda_

    @property
    def f_prev(self):
        return self._s.f_prev

    @property
    def flags(self):
        return self._s.flags


def os_iterate(geom, subsets: int, beta: float, counts, i0: float, img=None, n_iter: int = 1,
               state: State | None = None, lambda_schedule=None, params=None, want_trace=True,
               allow_numeric=False, f_hist=None, best=None):
    """Ordered-subset TV gradient iteration (Eq. 3 with Eqs. 4-5).  Returns (img, trace[n_iter][2]).

    f_hist: None or float64 [M] in/out (per-subset f, read by lambda_compare = 1); best: None or
    float64 [n][n] receiving the kept iterate when params['keep_best'] is 1."""
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    cp = _Params(**p)
    counts = np.ascontiguousarray(counts, dtype=np.float64).reshape(geom.n_views, geom.n_channels)
    if img is None:
        img = initial_image(geom, p["mu0_per_mm"])
    img = np.array(img, dtype=np.float64, order="C").reshape(geom.n, geom.n)
    trace = np.zeros((n_iter, 2), np.float64) if want_trace else None
    sched = None
    if lambda_schedule is not None:
        sched = np.ascontiguousarray(lambda_schedule, dtype=np.float64)
        assert sched.size >= n_iter
    if f_hist is not None:
        assert f_hist.dtype == np.float64 and f_hist.size == subsets and f_hist.flags["C_CONTIGUOUS"]
    if best is not None:
        assert best.dtype == np.float64 and best.shape == (geom.n, geom.n) and best.flags["C_CONTIGUOUS"]
    rc = lib().oracle_os_iterate(ctypes.byref(_g(geom)), subsets, beta, ctypes.byref(cp), _dp(counts), i0,
                                 _dp(img), n_iter, ctypes.byref(state._s) if state else None,
                                 _dp(trace) if trace is not None else None,
                                 _dp(sched) if sched is not None else None,
                                 _dp(f_hist) if f_hist is not None else None,
                                 _dp(best) if best is not None else None)
    if rc == 3 and allow_numeric:
        return img, trace
    _check(rc, "os_iterate")
    return img, trace


def set_threads(n: int):
    lib().oracle_set_num_threads(n)


def num_threads() -> int:
    return int(lib().oracle_num_threads())
