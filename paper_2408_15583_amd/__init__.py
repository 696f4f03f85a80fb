"""MI355X point-cloud SBR library: Python binding of the C ABI (include/pointemray.h).

The binding only marshals arguments: every step of splatting, bouncing and the PO sum runs in
the HIP library (libpointemray.so).  PyTorch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import (PE_CONTRIB_EVERY, PE_CONTRIB_LAST, PE_F32, PE_F64, PE_GEOM_DENSIFIED,
                      PE_GEOM_PLAIN, PE_MEM_DEVICE, PE_MEM_HOST, PE_PREC_FP32,
                      PE_PREC_FP64PHASE, PE_SPLAT_DISK, PE_SPLAT_TUBE, PEError, check, lib)

__all__ = ["Context", "Scene", "solve", "render_gfb", "trace_pixels", "PEError", "lib", "check"]


def _torch():
    import torch
    return torch


def current_stream():
    """hipStream_t of torch's current stream (as an int), or None on the null stream."""
    torch = _torch()
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


def _dptr(a):
    return ctypes.c_void_p(a.data_ptr()) if a is not None else None


class Context:
    """A pe_ctx bound to one HIP device with an HBM budget (0 = 90% of free memory)."""

    def __init__(self, device: int = 0, budget: int = 0):
        self.h = _native.pe_ctx()
        check(lib().pe_ctx_create(device, budget, ctypes.byref(self.h)))

    def footprint(self):
        used = ctypes.c_uint64()
        bud = ctypes.c_uint64()
        check(lib().pe_ctx_footprint(self.h, ctypes.byref(used), ctypes.byref(bud)))
        return used.value, bud.value

    def set_profiling(self, enable: bool = True):
        check(lib().pe_ctx_set_profiling(self.h, 1 if enable else 0))

    def kernel_stats(self, reset: bool = False):
        """{kernel: (total_ms, launches)} recorded with HIP events while profiling is on."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int32()
        check(lib().pe_ctx_kernel_stats(self.h, cap, names, ms, cnt, ctypes.byref(n),
                                        1 if reset else 0))
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(n.value, cap))}

    def close(self):
        if self.h:
            check(lib().pe_ctx_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Scene:
    """A resident scene (pe_scene).  xyz (n,3) f32/f64, nrm (n,3) f32; numpy arrays are read
    from host memory, torch CUDA tensors from device memory."""

    def __init__(self, ctx: Context, xyz, nrm, radius, material=None, view_dirs=None,
                 view_res: int = 256, stream=None):
        torch = _torch()
        self.ctx = ctx
        d = _native.pe_scene_desc()
        keep = []
        is_dev = isinstance(xyz, torch.Tensor) and xyz.is_cuda
        if is_dev:
            xyz_t = xyz.contiguous()
            nrm_t = nrm.to(torch.float32).contiguous()
            keep += [xyz_t, nrm_t]
            d.n = xyz_t.shape[0]
            d.xyz = xyz_t.data_ptr()
            d.xyz_type = PE_F64 if xyz_t.dtype == torch.float64 else PE_F32
            d.nrm = ctypes.cast(nrm_t.data_ptr(), _native.c_float_p)
            d.mem_kind = PE_MEM_DEVICE
            if material is not None:
                m = material.to(torch.uint8).contiguous()
                keep.append(m)
                d.material = ctypes.cast(m.data_ptr(), _native.c_u8_p)
            if radius is not None and not np.isscalar(radius) and getattr(radius, "ndim", 0) > 0:
                r = radius.to(torch.float32).contiguous()
                keep.append(r)
                d.radius = ctypes.cast(r.data_ptr(), _native.c_float_p)
            else:
                d.radius_scalar = float(radius)
        else:
            xyz_a = np.ascontiguousarray(xyz)
            if xyz_a.dtype not in (np.float32, np.float64):
                xyz_a = xyz_a.astype(np.float64)
            nrm_a = np.ascontiguousarray(nrm, dtype=np.float32)
            keep += [xyz_a, nrm_a]
            d.n = xyz_a.shape[0]
            d.xyz = xyz_a.ctypes.data
            d.xyz_type = PE_F64 if xyz_a.dtype == np.float64 else PE_F32
            d.nrm = nrm_a.ctypes.data_as(_native.c_float_p)
            d.mem_kind = PE_MEM_HOST
            if material is not None:
                m = np.ascontiguousarray(material, dtype=np.uint8)
                keep.append(m)
                d.material = m.ctypes.data_as(_native.c_u8_p)
            if radius is not None and np.ndim(radius) > 0:
                r = np.ascontiguousarray(radius, dtype=np.float32)
                keep.append(r)
                d.radius = r.ctypes.data_as(_native.c_float_p)
            else:
                d.radius_scalar = float(radius)
        if view_dirs is not None:
            vd = np.ascontiguousarray(view_dirs, dtype=np.float64).reshape(-1, 3)
            keep.append(vd)
            d.n_views = vd.shape[0]
            d.view_dirs = vd.ctypes.data_as(_native.c_double_p)
        d.view_res = int(view_res)
        self.h = _native.pe_scene()
        st = current_stream() if stream is None else stream
        check(lib().pe_scene_create(ctx.h, ctypes.byref(d), st, ctypes.byref(self.h)))
        del keep

    @classmethod
    def from_scene(cls, ctx, sc, view_res=256, view_dirs=None, device=True):
        """Builds from a scenes.Scene; device=True uploads through torch first."""
        torch = _torch()
        if device and torch.cuda.is_available():
            xyz = torch.from_numpy(np.ascontiguousarray(sc.xyz)).cuda()
            nrm = torch.from_numpy(np.ascontiguousarray(sc.nrm, dtype=np.float32)).cuda()
            mat = torch.from_numpy(np.ascontiguousarray(sc.material)).cuda()
            rad = sc.radius if np.isscalar(sc.radius) else torch.from_numpy(
                np.asarray(sc.radius, np.float32)).cuda()
            return cls(ctx, xyz, nrm, rad, mat, view_dirs=view_dirs, view_res=view_res)
        return cls(ctx, sc.xyz, sc.nrm, sc.radius, sc.material, view_dirs=view_dirs,
                   view_res=view_res)

    def info(self):
        c = (ctypes.c_double * 3)()
        R = ctypes.c_double()
        rm = ctypes.c_double()
        b = ctypes.c_uint64()
        check(lib().pe_scene_info(self.h, c, ctypes.byref(R), ctypes.byref(rm), ctypes.byref(b)))
        return dict(centre=np.array(list(c)), R=R.value, r_max=rm.value, bytes=b.value)

    def close(self):
        if self.h:
            check(lib().pe_scene_destroy(self.h))
            self.h = None


_CONTRIB = {"last": PE_CONTRIB_LAST, "every": PE_CONTRIB_EVERY}
_PREC = {"fp64phase": PE_PREC_FP64PHASE, "fp32": PE_PREC_FP32}


def make_solve_desc(inc_dir, freq_hz, screen, max_bounces=1, eps=0.0, obs_dir=None,
                    contrib="last", precision="fp64phase", densifier=None):
    inc = np.ascontiguousarray(inc_dir, dtype=np.float64).reshape(-1, 3)
    fr = np.ascontiguousarray(freq_hz, dtype=np.float64).ravel()
    d = _native.pe_solve_desc()
    d.n_inc = inc.shape[0]
    d.inc_dir = inc.ctypes.data_as(_native.c_double_p)
    keep = [inc, fr]
    if obs_dir is not None:
        ob = np.ascontiguousarray(obs_dir, dtype=np.float64).reshape(-1, 3)
        keep.append(ob)
        d.n_obs = ob.shape[0]
        d.obs_dir = ob.ctypes.data_as(_native.c_double_p)
    d.n_freq = fr.size
    d.freq_hz = fr.ctypes.data_as(_native.c_double_p)
    w, h = (screen, screen) if np.isscalar(screen) else screen
    d.screen_w, d.screen_h = int(w), int(h)
    d.max_bounces = int(max_bounces)
    d.eps = float(eps)
    d.contrib = _CONTRIB[contrib]
    d.precision = _PREC[precision]
    if densifier is not None:
        d.geometry = PE_GEOM_DENSIFIED
        d.densifier = densifier.h if hasattr(densifier, "h") else densifier
    return d, keep


def solve(ctx: Context, scene: Scene, inc_dir, freq_hz, screen, max_bounces=1, eps=0.0,
          obs_dir=None, contrib="last", precision="fp64phase", densifier=None, stream=None):
    """Synchronous pe_solve.  Returns (E complex [inc, obs, freq, rx, tx], rcs_dbsm, stats)."""
    d, keep = make_solve_desc(inc_dir, freq_hz, screen, max_bounces, eps, obs_dir, contrib,
                              precision, densifier)
    no = 1 if obs_dir is None else d.n_obs
    E = np.zeros((d.n_inc, no, d.n_freq, 2, 2, 2))
    rcs = np.zeros((d.n_inc, no, d.n_freq, 2, 2))
    st = _native.pe_stats()
    res = _native.pe_result(E.ctypes.data_as(_native.c_double_p),
                            rcs.ctypes.data_as(_native.c_double_p), ctypes.pointer(st))
    s = current_stream() if stream is None else stream
    check(lib().pe_solve(ctx.h, scene.h, ctypes.byref(d), ctypes.byref(res), s))
    del keep
    stats = {f: getattr(st, f) for f, _ in _native.pe_stats._fields_}
    return E[..., 0] + 1j * E[..., 1], rcs, stats


def render_gfb(ctx: Context, scene: Scene, direction, w, h, mode="disk", tube_radius=0.0,
               stream=None):
    """Geometric frame buffer of one view as torch CUDA tensors (depth, nrm, idx, mask)."""
    torch = _torch()
    dev = torch.device("cuda")
    depth = torch.empty((h, w), dtype=torch.float32, device=dev)
    nrm = torch.empty((h, w, 3), dtype=torch.float32, device=dev)
    idx = torch.empty((h, w), dtype=torch.int32, device=dev)
    mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    dr = (ctypes.c_double * 3)(*[float(x) for x in direction])
    s = current_stream() if stream is None else stream
    check(lib().pe_render_gfb(ctx.h, scene.h, dr, w, h,
                              PE_SPLAT_TUBE if mode == "tube" else PE_SPLAT_DISK,
                              float(tube_radius), _dptr(depth), _dptr(nrm), _dptr(idx),
                              _dptr(mask), s))
    return dict(depth=depth, nrm=nrm, idx=idx, mask=mask)


def trace_pixels(ctx: Context, scene: Scene, inc_dir, w, h, max_bounces, eps, stream=None):
    """Per-pixel last bounce records of one incidence as torch CUDA tensors."""
    torch = _torch()
    dev = torch.device("cuda")
    nb = torch.empty((h, w), dtype=torch.int32, device=dev)
    lx = torch.empty((h, w, 3), dtype=torch.float32, device=dev)
    ln = torch.empty((h, w, 3), dtype=torch.float32, device=dev)
    path = torch.empty((h, w), dtype=torch.float64, device=dev)
    li = torch.empty((h, w), dtype=torch.int32, device=dev)
    dr = (ctypes.c_double * 3)(*[float(x) for x in inc_dir])
    s = current_stream() if stream is None else stream
    check(lib().pe_trace_pixels(ctx.h, scene.h, dr, w, h, int(max_bounces), float(eps),
                                _dptr(nb), _dptr(lx), _dptr(ln), _dptr(path), _dptr(li), s))
    return dict(n_bounce=nb, last_x=lx, last_n=ln, path=path, last_idx=li)
