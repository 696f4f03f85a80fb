"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct implementation of what the GPU path computes, used only by
the tests, the smoke check and the bench's CPU-baseline leg.  It shares no code with the HIP
library and never imports it.  The arithmetic lives in oracle.c (ray-disk geometry, bounce
recursion, the Eq. (14) field sum); this module is ctypes marshalling plus the RCS definition.

Pins (tests/test_oracle_*.py, run with -m "not gpu"):
  - flat-plate broadside RCS 4 pi A^2 / lambda^2 and its sinc^2 pattern (closed form);
  - dihedral double-bounce peak 8 pi a^2 b^2 / lambda^2 and aperture 2 b sin(alpha);
  - large PEC sphere pi a^2 [1 - sin(2ka)/ka + sin^2(ka)/(ka)^2];
  - Eq. (2)-(3) decomposition == vector reflection, norms preserved;
  - monostatic reciprocity, zero single-bounce cross-polarisation;
  - frequency independence of the trace;
  - hand-derived hits on 1-3 disks; grid-culled first hit == brute force, bitwise.
Eq. (23) overlap refinement and normal blending (set_blend) is pinned in
tests/test_oracle_blend.py; the K-point heap of Algorithm 1 (render_tube_topk) by brute force in
tests/test_oracle_pins.py.  GFB edge filtering and fusion live in oracle/fuse.py and the
densifier's FP64 layers in oracle/nn.py, each with their own pins.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

C0 = 299_792_458.0
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    lib.or_scene_new.restype = ctypes.c_void_p
    lib.or_scene_new.argtypes = [ctypes.c_int64, _d, _d, _d, _u8, ctypes.POINTER(ctypes.c_int)]
    lib.or_scene_free.argtypes = [ctypes.c_void_p]
    lib.or_scene_frame.argtypes = [ctypes.c_void_p, _d, _d]
    lib.or_scene_build_grid.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_screen.argtypes = [ctypes.c_void_p, _d, ctypes.c_int, ctypes.c_int, _d, _d, _d]
    lib.or_first_hit.restype = ctypes.c_int64
    lib.or_first_hit.argtypes = [ctypes.c_void_p, _d, _d, ctypes.c_double, ctypes.c_int, _d]
    lib.or_render_disk.argtypes = [ctypes.c_void_p, _d, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   _d, _i64, _d, _u8]
    lib.or_render_tube.argtypes = [ctypes.c_void_p, _d, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, _d, _i64]
    lib.or_trace_pixels.argtypes = [ctypes.c_void_p, _d, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int64, _i64, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, _i32, _d, _i64]
    lib.or_solve.argtypes = [ctypes.c_void_p, ctypes.c_int, _d, ctypes.c_int, _d, ctypes.c_int,
                             _d, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, _d, _d]
    lib.or_render_tube_topk.argtypes = [ctypes.c_void_p, _d, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int, _d, _i64]
    lib.or_scene_set_views.argtypes = [ctypes.c_void_p, ctypes.c_int, _d, ctypes.c_int,
                                       ctypes.c_int]
    lib.or_first_hit_views.restype = ctypes.c_int64
    lib.or_first_hit_views.argtypes = [ctypes.c_void_p, _d, _d, ctypes.c_double, _d]
    lib.or_admissible.argtypes = [ctypes.c_void_p, ctypes.c_int64, _d]
    lib.or_reflect_field_decomposed.argtypes = [_d, _d, _d, _d, _d]
    lib.or_reflect_field_vector.argtypes = [_d, _d, _d, _d, _d]
    lib.or_pol_basis.argtypes = [_d, _d, _d]
    lib.or_scene_set_blend.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.or_blend_hit.restype = ctypes.c_int64
    lib.or_blend_hit.argtypes = [ctypes.c_void_p, _d, _d, ctypes.c_int64, _d, _d, _d]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(n: int) -> None:
    _load().or_set_num_threads(int(n))


class OracleScene:
    """Disks built from a scenes.Scene (or raw arrays).  grid=G builds the culled-exact grid."""

    def __init__(self, xyz, nrm=None, radius=None, material=None, grid: int | None = None):
        if nrm is None:  # a scenes.Scene
            sc = xyz
            xyz, nrm, radius, material = sc.xyz, sc.nrm, sc.radius_array(), sc.material
        lib = _load()
        self.xyz = _f64(xyz).reshape(-1, 3)
        n = self.xyz.shape[0]
        self.nrm = _f64(nrm).reshape(-1, 3)
        r = np.asarray(radius, dtype=np.float64)
        self.rad = _f64(np.full(n, float(r)) if r.ndim == 0 else r)
        self.mat = np.ascontiguousarray(np.zeros(n, np.uint8) if material is None else material,
                                        dtype=np.uint8)
        err = ctypes.c_int(0)
        self._h = lib.or_scene_new(n, _p(self.xyz), _p(self.nrm), _p(self.rad), _p(self.mat, _u8),
                                   ctypes.byref(err))
        if err.value or not self._h:
            raise ValueError("invalid scene (non-finite position, zero normal, bad radius or material)")
        self.n = n
        self.use_grid = 0
        if grid:
            lib.or_scene_build_grid(self._h, int(grid))
            self.use_grid = 1

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_scene_free(self._h)
            self._h = None

    def frame(self):
        c = np.zeros(3)
        R = np.zeros(1)
        _load().or_scene_frame(self._h, _p(c), _p(R))
        return c, float(R[0])

    def screen(self, k, W, H):
        o = np.zeros(3); du = np.zeros(3); dv = np.zeros(3)
        _load().or_screen(self._h, _p(_f64(k)), W, H, _p(o), _p(du), _p(dv))
        return o, du, dv

    def first_hit(self, o, k, tmin=0.0, grid=None):
        t = np.zeros(1)
        g = self.use_grid if grid is None else int(grid)
        i = _load().or_first_hit(self._h, _p(_f64(o)), _p(_f64(k)), tmin, g, _p(t))
        return int(i), float(t[0])

    def render_disk(self, k, W, H, grid=None):
        depth = np.zeros(W * H); idx = np.zeros(W * H, np.int64)
        nrm = np.zeros(W * H * 3); mask = np.zeros(W * H, np.uint8)
        g = self.use_grid if grid is None else int(grid)
        _load().or_render_disk(self._h, _p(_f64(k)), W, H, g, _p(depth), _p(idx, _i64), _p(nrm),
                               _p(mask, _u8))
        return (depth.reshape(H, W), idx.reshape(H, W), nrm.reshape(H, W, 3),
                mask.reshape(H, W))

    def render_tube(self, k, W, H, delta):
        depth = np.zeros(W * H); idx = np.zeros(W * H, np.int64)
        _load().or_render_tube(self._h, _p(_f64(k)), W, H, float(delta), _p(depth), _p(idx, _i64))
        return depth.reshape(H, W), idx.reshape(H, W)

    AXIS_VIEWS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                          dtype=np.float64)

    def set_blend(self, r):
        """Eq. (23) overlap refinement and normal blending of every hit within r (0 = off)."""
        _load().or_scene_set_blend(self._h, float(r))

    def blend_hit(self, x, k, h0):
        """Refinement of one hit at x on disk h0 along k: (disk, point, normal, offset)."""
        xo = np.zeros(3); no = np.zeros(3); so = np.zeros(1)
        h = _load().or_blend_hit(self._h, _p(_f64(x)), _p(_f64(k)), int(h0), _p(xo), _p(no),
                                 _p(so))
        return int(h), xo, no, float(so[0])

    def set_views(self, res, dirs=None):
        """Aggregation views of the method's secondary-hit rule (default: the six axis
        directions) as first-hit index maps at res x res."""
        d = _f64(self.AXIS_VIEWS if dirs is None else dirs).reshape(-1, 3)
        if _load().or_scene_set_views(self._h, d.shape[0], _p(d), int(res), self.use_grid):
            raise ValueError("bad views")
        self.views = (d, int(res))

    def first_hit_views(self, o, k, tmin):
        t = np.zeros(1)
        i = _load().or_first_hit_views(self._h, _p(_f64(o)), _p(_f64(k)), float(tmin), _p(t))
        if i == -2:
            raise ValueError("set_views first")
        return int(i), float(t[0])

    def admissible(self, i, pt):
        r = _load().or_admissible(self._h, int(i), _p(_f64(pt)))
        if r < 0:
            raise ValueError("set_views first")
        return bool(r)

    def render_tube_topk(self, k, W, H, delta, K):
        """Algorithm 1 with a K-point heap: Euclidean depth |p - o| of the chosen point."""
        depth = np.zeros(W * H); idx = np.zeros(W * H, np.int64)
        _load().or_render_tube_topk(self._h, _p(_f64(k)), W, H, float(delta), int(K), _p(depth),
                                    _p(idx, _i64))
        return depth.reshape(H, W), idx.reshape(H, W)

    def trace_pixels(self, k, W, H, pix, max_bounces, eps, grid=None, restricted=False):
        """Per pixel: number of bounces M and the per-bounce records (see oracle.c)."""
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        m = pix.size
        nb = np.zeros(m, np.int32)
        rec = np.zeros((m, max_bounces, 22))
        hidx = np.full((m, max_bounces), -1, np.int64)
        g = self.use_grid if grid is None else int(grid)
        if _load().or_trace_pixels(self._h, _p(_f64(k)), W, H, m, _p(pix, _i64), max_bounces,
                                   float(eps), g, int(restricted), _p(nb, _i32), _p(rec),
                                   _p(hidx, _i64)):
            raise ValueError("restricted tracing needs set_views")
        return nb, rec, hidx

    def solve(self, inc_dir, freq_hz, W, H, max_bounces, eps, obs_dir=None, contrib="last",
              grid=None, restricted=False):
        """Complex field E[inc][obs][freq][rx][tx] (rx, tx in (theta, phi)) and stats.
        restricted=True applies the method's secondary-hit and visibility rules (set_views)."""
        inc = _f64(inc_dir).reshape(-1, 3)
        fr = _f64(freq_hz).ravel()
        no = 1 if obs_dir is None else _f64(obs_dir).reshape(-1, 3).shape[0]
        out = np.zeros((inc.shape[0], no, fr.size, 2, 2, 2))
        stats = np.zeros(3)
        obs = None if obs_dir is None else _f64(obs_dir).reshape(-1, 3)
        g = self.use_grid if grid is None else int(grid)
        if _load().or_solve(self._h, inc.shape[0], _p(inc), no, None if obs is None else _p(obs),
                            fr.size, _p(fr), W, H, max_bounces, float(eps),
                            1 if contrib == "every" else 0, g, int(restricted), _p(out),
                            _p(stats)):
            raise ValueError("restricted solve needs set_views")
        E = out[..., 0] + 1j * out[..., 1]
        return E, dict(disk_tests=stats[0], queries=stats[1], facets=stats[2])


def rcs_m2(E):
    """sigma = 4 pi |E_s|^2 for |E_i| = 1 with the far-field factor removed."""
    return 4 * math.pi * np.abs(E) ** 2


def rcs_dbsm(E):
    with np.errstate(divide="ignore"):
        return 10 * np.log10(rcs_m2(E))


def reflect_decomposed(k, n, E):
    Eo = np.zeros(3); ko = np.zeros(3)
    _load().or_reflect_field_decomposed(_p(_f64(k)), _p(_f64(n)), _p(_f64(E)), _p(Eo), _p(ko))
    return Eo, ko


def reflect_vector(k, n, E):
    Eo = np.zeros(3); ko = np.zeros(3)
    _load().or_reflect_field_vector(_p(_f64(k)), _p(_f64(n)), _p(_f64(E)), _p(Eo), _p(ko))
    return Eo, ko


def pol_basis(s):
    th = np.zeros(3); ph = np.zeros(3)
    _load().or_pol_basis(_p(_f64(s)), _p(th), _p(ph))
    return th, ph
