"""ctypes binding of the C ABI in include/pointemray.h (argument marshalling only).

Every function keeps the C name and signature.  Loading fails loudly when the HIP library has
not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpointemray.so")

PE_OK = 0
PE_EINVAL = -1
PE_ENOMEM = -2
PE_EDEVICE = -3
PE_EUNSUPPORTED = -4
PE_EBUSY = -5
PE_ECANCELED = -6
PE_ETIMEOUT = -7
STATUS_NAMES = {0: "PE_OK", -1: "PE_EINVAL", -2: "PE_ENOMEM", -3: "PE_EDEVICE",
                -4: "PE_EUNSUPPORTED", -5: "PE_EBUSY", -6: "PE_ECANCELED", -7: "PE_ETIMEOUT"}

PE_MEM_HOST, PE_MEM_DEVICE = 0, 1
PE_F32, PE_F64 = 0, 1
PE_MAT_PEC, PE_MAT_ABSORBER = 0, 1
PE_CONTRIB_LAST, PE_CONTRIB_EVERY = 0, 1
PE_PREC_FP64PHASE, PE_PREC_FP32, PE_PREC_FP64ACC = 0, 1, 2
PE_GEOM_PLAIN, PE_GEOM_DENSIFIED, PE_GEOM_COARSE = 0, 1, 2
PE_SPLAT_DISK, PE_SPLAT_TUBE = 0, 1
PE_SECONDARY_VIEWS, PE_SECONDARY_SPLATS = 0, 1

c_double_p = ctypes.POINTER(ctypes.c_double)
c_float_p = ctypes.POINTER(ctypes.c_float)
c_u8_p = ctypes.POINTER(ctypes.c_uint8)
c_u32_p = ctypes.POINTER(ctypes.c_uint32)
c_i32_p = ctypes.POINTER(ctypes.c_int32)
c_u64_p = ctypes.POINTER(ctypes.c_uint64)
pe_ctx = ctypes.c_void_p
pe_scene = ctypes.c_void_p
pe_densifier = ctypes.c_void_p
pe_ticket = ctypes.c_uint64


class pe_scene_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("xyz", ctypes.c_void_p), ("xyz_type", ctypes.c_int32),
                ("nrm", c_float_p), ("material", c_u8_p), ("radius", c_float_p),
                ("radius_scalar", ctypes.c_float), ("mem_kind", ctypes.c_int32),
                ("n_views", ctypes.c_int32), ("view_dirs", c_double_p),
                ("view_res", ctypes.c_int32), ("blend_radius", ctypes.c_double)]


class pe_solve_desc(ctypes.Structure):
    _fields_ = [("n_inc", ctypes.c_int32), ("inc_dir", c_double_p), ("n_obs", ctypes.c_int32),
                ("obs_dir", c_double_p), ("n_freq", ctypes.c_int32), ("freq_hz", c_double_p),
                ("screen_w", ctypes.c_int32), ("screen_h", ctypes.c_int32),
                ("max_bounces", ctypes.c_int32), ("eps", ctypes.c_double),
                ("contrib", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("geometry", ctypes.c_int32), ("densifier", pe_densifier),
                ("seed", ctypes.c_uint64), ("tube_px", ctypes.c_double),
                ("max_uncertain", ctypes.c_double), ("tube_k", ctypes.c_int32),
                ("secondary", ctypes.c_int32)]


class pe_stats(ctypes.Structure):
    _fields_ = [("ray_queries", ctypes.c_double), ("exit_records", ctypes.c_double),
                ("po_terms", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("march_cap_hits", ctypes.c_double), ("densifier_fallbacks", ctypes.c_double),
                ("march_rays", ctypes.c_double), ("march_hits", ctypes.c_double)]


class pe_gfb_set(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("view_dirs", c_double_p), ("w", ctypes.c_int32),
                ("h", ctypes.c_int32), ("centre", ctypes.c_double * 3), ("R", ctypes.c_double),
                ("depth", ctypes.c_void_p), ("nrm", ctypes.c_void_p), ("hit", ctypes.c_void_p)]


class pe_fuse_desc(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("grid_side", ctypes.c_double),
                ("edge_lo", ctypes.c_double), ("edge_hi", ctypes.c_double),
                ("edge_dilate", ctypes.c_int32)]


class pe_result(ctypes.Structure):
    _fields_ = [("E", c_double_p), ("rcs_dbsm", c_double_p),
                ("stats", ctypes.POINTER(pe_stats))]


_SIGS = {
    "pe_ctx_create": [ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(pe_ctx)],
    "pe_ctx_destroy": [pe_ctx],
    "pe_ctx_footprint": [pe_ctx, c_u64_p, c_u64_p],
    "pe_ctx_set_profiling": [pe_ctx, ctypes.c_int32],
    "pe_ctx_kernel_stats": [pe_ctx, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p), c_double_p,
                            c_u64_p, c_i32_p, ctypes.c_int32],
    "pe_scene_create": [pe_ctx, ctypes.POINTER(pe_scene_desc), ctypes.c_void_p,
                        ctypes.POINTER(pe_scene)],
    "pe_scene_destroy": [pe_scene],
    "pe_scene_info": [pe_scene, c_double_p, c_double_p, c_double_p, c_u64_p],
    "pe_solve": [pe_ctx, pe_scene, ctypes.POINTER(pe_solve_desc), ctypes.POINTER(pe_result),
                 ctypes.c_void_p],
    "pe_solve_noalloc": [pe_ctx, pe_scene, ctypes.POINTER(pe_solve_desc),
                         ctypes.POINTER(pe_result), ctypes.c_void_p],
    "pe_submit": [pe_ctx, pe_scene, ctypes.POINTER(pe_solve_desc), ctypes.POINTER(pe_result),
                  ctypes.POINTER(pe_ticket)],
    "pe_wait": [pe_ctx, pe_ticket, ctypes.c_int64],
    "pe_cancel": [pe_ctx, pe_ticket],
    "pe_server_stats": [pe_ctx, c_double_p, ctypes.c_int32],
    "pe_request_footprint": [ctypes.POINTER(pe_solve_desc), c_u64_p],
    "pe_render_gfb": [pe_ctx, pe_scene, c_double_p, ctypes.c_int32, ctypes.c_int32,
                      ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "pe_render_tube_topk": [pe_ctx, pe_scene, c_double_p, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "pe_trace_pixels": [pe_ctx, pe_scene, c_double_p, ctypes.c_int32, ctypes.c_int32,
                        ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p],
    "pe_estimate_normals": [pe_ctx, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int32,
                            ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "pe_fuse_gfbs": [pe_ctx, ctypes.POINTER(pe_gfb_set), ctypes.POINTER(pe_fuse_desc),
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_uint64, c_u64_p, ctypes.c_void_p],
    "pe_densifier_create": [pe_ctx, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(pe_densifier)],
    "pe_densifier_destroy": [pe_densifier],
    "pe_densifier_save": [pe_densifier, ctypes.c_char_p],
    "pe_densifier_load": [pe_densifier, ctypes.c_char_p],
    "pe_densifier_num_params": [pe_densifier, c_u64_p],
    "pe_densifier_train_step": [pe_densifier, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_float, ctypes.c_float, c_double_p,
                                ctypes.c_void_p],
    "pe_densifier_infer": [pe_densifier, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p],
    "pe_densifier_tensors": [pe_densifier, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p),
                             c_u64_p, c_i32_p, c_i32_p],
    "pe_densifier_get": [pe_densifier, ctypes.c_int32, c_float_p, ctypes.c_uint64],
    "pe_densifier_set": [pe_densifier, c_float_p, ctypes.c_uint64],
    "pe_densifier_make_pair": [pe_ctx, pe_scene, ctypes.c_int32, c_double_p, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p],
}

_lib = None


class PEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded HIP library.  Raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or paper_2408_15583_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.pe_last_error.argtypes = []
        L.pe_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status: int) -> int:
    if status != PE_OK:
        msg = lib().pe_last_error()
        raise PEError(status, msg.decode() if msg else "")
    return status


def __getattr__(name):
    if name.startswith("pe_"):
        return getattr(lib(), name)
    raise AttributeError(name)
