"""MI355X point-cloud SBR library: Python binding of the C ABI (include/pointemray.h).

The binding only marshals arguments: every step of splatting, bouncing and the PO sum runs in
the HIP library (libpointemray.so).  PyTorch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import (PE_CONTRIB_EVERY, PE_CONTRIB_LAST, PE_F32, PE_F64, PE_GEOM_COARSE,
                      PE_GEOM_DENSIFIED, PE_GEOM_PLAIN, PE_MEM_DEVICE, PE_MEM_HOST, PE_PREC_FP32,
                      PE_PREC_FP64PHASE, PE_SECONDARY_SPLATS, PE_SECONDARY_VIEWS, PE_SPLAT_DISK,
                      PE_SPLAT_TUBE, PEError, check, lib)

__all__ = ["Context", "Scene", "Densifier", "Ticket", "solve", "solve_noalloc", "submit",
           "server_stats",
           "render_gfb", "render_tube_topk", "trace_pixels", "make_pair", "fuse_gfbs",
           "estimate_normals",
           "PEError", "lib", "check"]


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
                 view_res: int = 256, stream=None, blend_radius: float = 0.0):
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
        d.blend_radius = float(blend_radius)
        self.h = _native.pe_scene()
        st = current_stream() if stream is None else stream
        check(lib().pe_scene_create(ctx.h, ctypes.byref(d), st, ctypes.byref(self.h)))
        del keep

    @classmethod
    def from_scene(cls, ctx, sc, view_res=256, view_dirs=None, device=True, blend_radius=0.0):
        """Builds from a scenes.Scene; device=True uploads through torch first."""
        torch = _torch()
        if device and torch.cuda.is_available():
            xyz = torch.from_numpy(np.ascontiguousarray(sc.xyz)).cuda()
            nrm = torch.from_numpy(np.ascontiguousarray(sc.nrm, dtype=np.float32)).cuda()
            mat = torch.from_numpy(np.ascontiguousarray(sc.material)).cuda()
            rad = sc.radius if np.isscalar(sc.radius) else torch.from_numpy(
                np.asarray(sc.radius, np.float32)).cuda()
            return cls(ctx, xyz, nrm, rad, mat, view_dirs=view_dirs, view_res=view_res,
                       blend_radius=blend_radius)
        return cls(ctx, sc.xyz, sc.nrm, sc.radius, sc.material, view_dirs=view_dirs,
                   view_res=view_res, blend_radius=blend_radius)

    def info(self):
        c = (ctypes.c_double * 3)()
        R = ctypes.c_double()
        rm = ctypes.c_double()
        b = ctypes.c_uint64()
        check(lib().pe_scene_info(self.h, c, ctypes.byref(R), ctypes.byref(rm), ctypes.byref(b)))
        return dict(centre=np.array(list(c)), R=R.value, r_max=rm.value, bytes=b.value)

    def close(self):
        """Frees the scene; raises PEError (PE_EBUSY) while submitted requests still use it."""
        if self.h:
            check(lib().pe_scene_destroy(self.h))
            self.h = None


_CONTRIB = {"last": PE_CONTRIB_LAST, "every": PE_CONTRIB_EVERY}
_PREC = {"fp64phase": PE_PREC_FP64PHASE, "fp32": PE_PREC_FP32, "fp64acc": _native.PE_PREC_FP64ACC}
_SECONDARY = {"views": PE_SECONDARY_VIEWS, "splats": PE_SECONDARY_SPLATS}


def make_solve_desc(inc_dir, freq_hz, screen, max_bounces=1, eps=0.0, obs_dir=None,
                    contrib="last", precision="fp64phase", densifier=None, geometry=None,
                    tube_px=0.0, max_uncertain=0.0, tube_k=0, secondary="views"):
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
    if geometry is None:
        geometry = "densified" if densifier is not None else "plain"
    d.geometry = {"plain": PE_GEOM_PLAIN, "densified": PE_GEOM_DENSIFIED,
                  "coarse": PE_GEOM_COARSE}[geometry]
    if densifier is not None:
        d.densifier = densifier.h if hasattr(densifier, "h") else densifier
    d.tube_px = float(tube_px)
    d.max_uncertain = float(max_uncertain)
    d.tube_k = int(tube_k)
    d.secondary = _SECONDARY[secondary]
    return d, keep


def solve(ctx: Context, scene: Scene, inc_dir, freq_hz, screen, max_bounces=1, eps=0.0,
          obs_dir=None, contrib="last", precision="fp64phase", densifier=None, stream=None,
          geometry=None, tube_px=0.0, max_uncertain=0.0, tube_k=0, secondary="views"):
    """Synchronous pe_solve.  Returns (E complex [inc, obs, freq, rx, tx], rcs_dbsm, stats).
    geometry: "plain" (default), "densified" (needs densifier) or "coarse"; tube_k: heap size
    of the coarse buffer (0 = unbounded); secondary: "views" (what the aggregation views
    retain) or "splats" (every splat, through the object-space hierarchy)."""
    d, keep = make_solve_desc(inc_dir, freq_hz, screen, max_bounces, eps, obs_dir, contrib,
                              precision, densifier, geometry, tube_px, max_uncertain, tube_k,
                              secondary)
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


def solve_noalloc(ctx: Context, scene: Scene, inc_dir, freq_hz, screen, max_bounces=1, eps=0.0,
                  obs_dir=None, contrib="last", precision="fp64phase", stream=None,
                  secondary="views"):
    """pe_solve_noalloc: the plain solve with every transient buffer in the library's fixed
    per-device scratch array (no device allocation).  Same returns as solve()."""
    d, keep = make_solve_desc(inc_dir, freq_hz, screen, max_bounces, eps, obs_dir, contrib,
                              precision, secondary=secondary)
    no = 1 if obs_dir is None else d.n_obs
    E = np.zeros((d.n_inc, no, d.n_freq, 2, 2, 2))
    rcs = np.zeros((d.n_inc, no, d.n_freq, 2, 2))
    st = _native.pe_stats()
    res = _native.pe_result(E.ctypes.data_as(_native.c_double_p),
                            rcs.ctypes.data_as(_native.c_double_p), ctypes.pointer(st))
    s = current_stream() if stream is None else stream
    check(lib().pe_solve_noalloc(ctx.h, scene.h, ctypes.byref(d), ctypes.byref(res), s))
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


def render_tube_topk(ctx: Context, scene: Scene, direction, w, h, tube_radius, K, stream=None):
    """Coarse buffer of Algorithm 1 with a K-point heap (torch CUDA tensors depth, nrm, idx,
    mask); depth is the Euclidean distance from the pixel centre."""
    torch = _torch()
    dev = torch.device("cuda")
    depth = torch.empty((h, w), dtype=torch.float32, device=dev)
    nrm = torch.empty((h, w, 3), dtype=torch.float32, device=dev)
    idx = torch.empty((h, w), dtype=torch.int32, device=dev)
    mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    dr = (ctypes.c_double * 3)(*[float(x) for x in direction])
    s = current_stream() if stream is None else stream
    check(lib().pe_render_tube_topk(ctx.h, scene.h, dr, w, h, float(tube_radius), int(K),
                                    _dptr(depth), _dptr(nrm), _dptr(idx), _dptr(mask), s))
    return dict(depth=depth, nrm=nrm, idx=idx, mask=mask)


def trace_pixels(ctx: Context, scene: Scene, inc_dir, w, h, max_bounces, eps, stream=None,
                 secondary="views"):
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
                                _SECONDARY[secondary], _dptr(nb), _dptr(lx), _dptr(ln),
                                _dptr(path), _dptr(li), s))
    return dict(n_bounce=nb, last_x=lx, last_n=ln, path=path, last_idx=li)


class Densifier:
    """pe_densifier: the U-Net of Sec. III-A on the device (bf16 weights, fp32 masters, AdamW)."""

    def __init__(self, ctx: Context, base: int = 32, seed: int = 0):
        self.ctx = ctx
        h = _native.pe_densifier()
        check(lib().pe_densifier_create(ctx.h, int(base), int(seed), ctypes.byref(h)))
        self.h = h
        n = ctypes.c_uint64()
        check(lib().pe_densifier_num_params(self.h, ctypes.byref(n)))
        self.n_params = n.value

    def tensors(self):
        """[(name, offset, shape)] of the flat parameter vector."""
        n = ctypes.c_int32()
        check(lib().pe_densifier_tensors(self.h, 0, None, None, None, ctypes.byref(n)))
        names = (ctypes.c_char_p * n.value)()
        offs = (ctypes.c_uint64 * n.value)()
        shp = (ctypes.c_int32 * (4 * n.value))()
        check(lib().pe_densifier_tensors(self.h, n.value, names, offs, shp, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            shape = tuple(d for d in shp[4 * i:4 * i + 4] if d > 0)
            out.append((names[i].decode(), offs[i], shape))
        return out

    def get(self, which="params"):
        which = {"params": 0, "grads": 1, "m": 2, "v": 3}[which]
        a = np.empty(self.n_params, dtype=np.float32)
        check(lib().pe_densifier_get(self.h, which, a.ctypes.data_as(_native.c_float_p),
                                     self.n_params))
        return a

    def set(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        check(lib().pe_densifier_set(self.h, a.ctypes.data_as(_native.c_float_p), a.size))

    def get_dict(self, which="params"):
        flat = self.get(which)
        return {n: flat[o:o + int(np.prod(s))].reshape(s) for n, o, s in self.tensors()}

    def train_step(self, coarse, depth_gt, nrm_gt, mask_gt, lr, weight_decay=0.0, stream=None):
        """One AdamW step on torch CUDA float32 tensors [b,h,w], [b,2h,2w], [b,2h,2w,3],
        [b,2h,2w].  Returns the losses (total, L1, L2, L3, L4)."""
        b, h, w = coarse.shape
        out = (ctypes.c_double * 5)()
        s = current_stream() if stream is None else stream
        check(lib().pe_densifier_train_step(self.h, b, h, w, _dptr(coarse), _dptr(depth_gt),
                                            _dptr(nrm_gt), _dptr(mask_gt), float(lr),
                                            float(weight_decay), out, s))
        return tuple(out)

    def infer(self, coarse, stream=None):
        """(depth, unit normal, hit probability) torch tensors at twice the input size."""
        torch = _torch()
        b, h, w = coarse.shape
        dev = coarse.device
        depth = torch.empty((b, 2 * h, 2 * w), dtype=torch.float32, device=dev)
        nrm = torch.empty((b, 2 * h, 2 * w, 3), dtype=torch.float32, device=dev)
        prob = torch.empty((b, 2 * h, 2 * w), dtype=torch.float32, device=dev)
        s = current_stream() if stream is None else stream
        check(lib().pe_densifier_infer(self.h, b, h, w, _dptr(coarse), _dptr(depth), _dptr(nrm),
                                       _dptr(prob), s))
        return depth, nrm, prob

    def save(self, path):
        check(lib().pe_densifier_save(self.h, str(path).encode()))

    def load(self, path):
        check(lib().pe_densifier_load(self.h, str(path).encode()))

    def close(self):
        if self.h:
            check(lib().pe_densifier_destroy(self.h))
            self.h = None


def make_pair(ctx: Context, scene: Scene, dirs, h, w, tube_px=2.0, tube_k=0, stream=None):
    """Network input and targets for each propagation direction (torch CUDA tensors):
    coarse [n,h,w], depth_gt [n,2h,2w], nrm_gt [n,2h,2w,3], mask_gt [n,2h,2w]."""
    torch = _torch()
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = d.shape[0]
    dev = torch.device("cuda")
    coarse = torch.empty((n, h, w), dtype=torch.float32, device=dev)
    dg = torch.empty((n, 2 * h, 2 * w), dtype=torch.float32, device=dev)
    ng = torch.empty((n, 2 * h, 2 * w, 3), dtype=torch.float32, device=dev)
    mg = torch.empty((n, 2 * h, 2 * w), dtype=torch.float32, device=dev)
    s = current_stream() if stream is None else stream
    check(lib().pe_densifier_make_pair(ctx.h, scene.h, n, d.ctypes.data_as(_native.c_double_p),
                                       int(h), int(w), float(tube_px), int(tube_k),
                                       _dptr(coarse), _dptr(dg),
                                       _dptr(ng), _dptr(mg), s))
    return coarse, dg, ng, mg


def estimate_normals(ctx: Context, xyz, k=16, stream=None):
    """PCA normals of the k nearest neighbours (pe_estimate_normals).  xyz: numpy (n,3) f32/f64
    (returns numpy) or a torch CUDA tensor (returns a torch CUDA tensor)."""
    torch = _torch()
    s = current_stream() if stream is None else stream
    if isinstance(xyz, torch.Tensor) and xyz.is_cuda:
        x = xyz.contiguous()
        if x.dtype not in (torch.float32, torch.float64):
            x = x.to(torch.float64)
        out = torch.empty((x.shape[0], 3), dtype=torch.float32, device=x.device)
        check(lib().pe_estimate_normals(ctx.h, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                        PE_F64 if x.dtype == torch.float64 else PE_F32,
                                        PE_MEM_DEVICE, int(k), ctypes.c_void_p(out.data_ptr()), s))
        return out
    x = np.ascontiguousarray(xyz)
    if x.dtype not in (np.float32, np.float64):
        x = x.astype(np.float64)
    out = np.empty((x.shape[0], 3), np.float32)
    check(lib().pe_estimate_normals(ctx.h, x.shape[0], ctypes.c_void_p(x.ctypes.data),
                                    PE_F64 if x.dtype == np.float64 else PE_F32, PE_MEM_HOST,
                                    int(k), ctypes.c_void_p(out.ctypes.data), s))
    return out


def fuse_gfbs(ctx: Context, view_dirs, depth, nrm, hit, centre, R, grid=256, grid_side=0.0,
              edge_lo=0.0, edge_hi=0.0, edge_dilate=-1, stream=None):
    """Edge filtering and grid fusion of GFBs into splats (pe_fuse_gfbs).  depth [n,h,w] (t/D),
    nrm [n,h,w,3] (view frame), hit [n,h,w] float torch CUDA tensors; returns torch CUDA
    tensors xyz [m,3] f64 (world), nrm [m,3], radius [m], count [m] and edge [n,h,w] u8."""
    torch = _torch()
    vd = np.ascontiguousarray(view_dirs, dtype=np.float64).reshape(-1, 3)
    dev = depth.device
    depth = depth.to(torch.float32).contiguous()
    nrm = nrm.to(torch.float32).contiguous()
    hit = hit.to(torch.float32).contiguous()
    n, h, w = depth.shape
    g = _native.pe_gfb_set()
    g.n_views = n
    g.view_dirs = vd.ctypes.data_as(_native.c_double_p)
    g.w, g.h = w, h
    for k in range(3):
        g.centre[k] = float(centre[k])
    g.R = float(R)
    g.depth, g.nrm, g.hit = depth.data_ptr(), nrm.data_ptr(), hit.data_ptr()
    f = _native.pe_fuse_desc(int(grid), float(grid_side), float(edge_lo), float(edge_hi),
                             int(edge_dilate))
    cap = n * h * w
    xyz = torch.empty((cap, 3), dtype=torch.float64, device=dev)
    nr = torch.empty((cap, 3), dtype=torch.float32, device=dev)
    rad = torch.empty((cap,), dtype=torch.float32, device=dev)
    cnt = torch.empty((cap,), dtype=torch.int32, device=dev)
    edge = torch.empty((n, h, w), dtype=torch.uint8, device=dev)
    m = ctypes.c_uint64()
    s = current_stream() if stream is None else stream
    check(lib().pe_fuse_gfbs(ctx.h, ctypes.byref(g), ctypes.byref(f), _dptr(xyz), _dptr(nr),
                             _dptr(rad), _dptr(cnt), _dptr(edge), cap, ctypes.byref(m), s))
    k = m.value
    return dict(xyz=xyz[:k], nrm=nr[:k], radius=rad[:k], count=cnt[:k], edge=edge)


class Ticket:
    """A request submitted to the context's continuous-batching server.

    The server writes the request's result into buffers this object owns, so they must outlive
    the request: a Ticket dropped before its request finished cancels it and waits for the
    server to let go of the buffers (finalizer)."""

    def __init__(self, ctx, ticket, E, rcs, st, res, keep):
        self.ctx, self.id, self._E, self._rcs, self._st = ctx, ticket, E, rcs, st
        self._res, self._keep = res, keep
        self._final = False  # pe_wait returned the request's final status

    def wait(self, timeout_s=None):
        """Blocks until the request finishes; returns (E complex, rcs_dbsm, stats).  Raises
        PEError (PE_ECANCELED, a failure) or TimeoutError (still pending)."""
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        s = lib().pe_wait(self.ctx.h, self.id, us)
        if s == _native.PE_ETIMEOUT:
            raise TimeoutError(f"request {self.id} still pending")
        self._final = True
        check(s)
        stats = {f: getattr(self._st, f) for f, _ in _native.pe_stats._fields_}
        return self._E[..., 0] + 1j * self._E[..., 1], self._rcs, stats

    def cancel(self):
        check(lib().pe_cancel(self.ctx.h, self.id))

    def __del__(self):
        # A closed context has already finished (cancelled) every request of its server.
        if getattr(self, "_final", True) or not getattr(self.ctx, "h", None):
            return
        try:
            lib().pe_cancel(self.ctx.h, self.id)
            lib().pe_wait(self.ctx.h, self.id, -1)
        except Exception:
            pass


def submit(ctx: Context, scene: Scene, inc_dir, freq_hz, screen, max_bounces=1, eps=0.0,
           obs_dir=None, contrib="last", precision="fp64phase", secondary="views"):
    """Asynchronous solve through the server (pe_submit); returns a Ticket."""
    d, keep = make_solve_desc(inc_dir, freq_hz, screen, max_bounces, eps, obs_dir, contrib,
                              precision, secondary=secondary)
    no = 1 if obs_dir is None else d.n_obs
    E = np.zeros((d.n_inc, no, d.n_freq, 2, 2, 2))
    rcs = np.zeros((d.n_inc, no, d.n_freq, 2, 2))
    st = _native.pe_stats()
    res = _native.pe_result(E.ctypes.data_as(_native.c_double_p),
                            rcs.ctypes.data_as(_native.c_double_p), ctypes.pointer(st))
    t = _native.pe_ticket()
    check(lib().pe_submit(ctx.h, scene.h, ctypes.byref(d), ctypes.byref(res), ctypes.byref(t)))
    return Ticket(ctx, t.value, E, rcs, st, res, keep)


def server_stats(ctx: Context, reset=False):
    """Server counters: completed, p50/p99/mean latency (ms), max concurrent requests, mean
    requests per shared launch batch."""
    out = (ctypes.c_double * 6)()
    check(lib().pe_server_stats(ctx.h, out, int(bool(reset))))
    keys = ("completed", "p50_ms", "p99_ms", "mean_ms", "max_concurrent", "reqs_per_batch")
    return dict(zip(keys, list(out)))


def request_footprint(inc_dir, freq_hz, screen, max_bounces=1, eps=0.0, obs_dir=None,
                      contrib="last", precision="fp64phase", secondary="views"):
    """HBM bytes the server charges a request for admission."""
    d, keep = make_solve_desc(inc_dir, freq_hz, screen, max_bounces, eps, obs_dir, contrib,
                              precision, secondary=secondary)
    b = ctypes.c_uint64()
    check(lib().pe_request_footprint(ctypes.byref(d), ctypes.byref(b)))
    del keep
    return b.value
