"""ctypes declarations of the libvbm C ABI (include/vbm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvbm.so")

VBM_TF_MAX_POINTS = 16
VBM_IMAGE_LOSS_STATIC_SCRATCH_BYTES = 64 << 20
VBM_BANK_FLOATS = 12
VBM_WS_REGIONS = 24
MODE_BATCHED, MODE_EXACT = 0, 1
WAVELETS = {"haar": 0, "bior4.4": 1}
REGION = dict(counters=0, item_depth=1, item_rect=2, item_ntiles=3, item_rec=4, item_blue=5, pair_tile=6,
              pair_item=7, ranges=8, grad2d=9, item_coef=19)
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "workspace too small", -4: "HIP error",
          -5: "capacity exceeded"}


class vbm_tf(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("x", C.c_float * VBM_TF_MAX_POINTS),
                ("rgba", (C.c_float * 4) * VBM_TF_MAX_POINTS)]


class vbm_bank_entry(C.Structure):
    _fields_ = [("j", C.c_int32), ("o", C.c_int32), ("roi_size", C.c_int32), ("pad", C.c_int32),
                ("w", C.c_double), ("u", C.c_double * 3), ("sigma", C.c_double * 6), ("scale", C.c_double * 3),
                ("quat", C.c_double * 4)]


class vbm_gaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacity", C.c_void_p),
                ("rgb", C.c_void_p), ("stride", C.c_int64)]


vbm_gaussians_c = vbm_gaussians  # identical layout; const-ness is only a C-side promise


class vbm_build_opts(C.Structure):
    _fields_ = [("s_mode", C.c_int32), ("delta", C.c_float), ("opacity_min", C.c_float),
                ("opacity_max", C.c_float), ("isotropic", C.c_int32), ("unit_weight", C.c_int32)]


class vbm_adaptive_opts(C.Structure):
    _fields_ = [("K_tot", C.c_int64), ("alpha", C.c_double), ("beta", C.c_double), ("lam", C.c_float),
                ("ref_channel", C.c_int32), ("min_band", C.c_int64)]


VBM_ADAPTIVE_STATS = 12
ADAPTIVE_STATS = ("E", "N", "quotient", "K_band", "median", "mad", "sigma", "T", "C", "K", "vK", "kept")


class vbm_view(C.Structure):
    _fields_ = [("scene", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("near_plane", C.c_float), ("viewmat", C.c_float * 12), ("bg", C.c_float * 3)]


class vbm_schedule(C.Structure):
    _fields_ = [("tile", C.c_int32), ("sort_bits", C.c_int32), ("pair_capacity", C.c_int64), ("mode", C.c_int32),
                ("lds_batch", C.c_int32), ("lds_batch_bwd", C.c_int32), ("pad0", C.c_int32)]


class vbm_plan(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("n_scenes", C.c_int32), ("tile", C.c_int32), ("mode", C.c_int32),
                ("sort_bits", C.c_int32), ("tile_key_bits", C.c_int32), ("lds_batch", C.c_int32),
                ("lds_batch_bwd", C.c_int32),
                ("n_gaussians", C.c_int64), ("n_items", C.c_int64), ("n_tiles", C.c_int64), ("n_pixels", C.c_int64),
                ("pair_capacity", C.c_int64), ("view_table_bytes", C.c_size_t), ("ws_bytes", C.c_size_t),
                ("region_offset", C.c_size_t * VBM_WS_REGIONS), ("region_bytes", C.c_size_t * VBM_WS_REGIONS)]


class vbm_adam_opts(C.Structure):
    _fields_ = [("lr", C.c_float * 5), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32), ("pad", C.c_int32)]


_SIGS = {
    "vbm_version": (C.c_char_p, []),
    "vbm_last_error": (C.c_char_p, []),
    "vbm_dwt3d_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32]),
    "vbm_dwt3d": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vbm_tf), C.c_void_p, C.c_void_p,
                              C.c_size_t, C.c_void_p]),
    "vbm_bank_size": (C.c_int32, [C.c_int32]),
    "vbm_bank_build": (C.c_int32, [C.c_int32, C.c_int32, C.c_double, C.c_double, C.POINTER(vbm_bank_entry)]),
    "vbm_bank_pack": (C.c_int32, [C.POINTER(vbm_bank_entry), C.c_int32, C.POINTER(C.c_float)]),
    "vbm_build_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32]),
    "vbm_build_gaussians": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                        C.POINTER(vbm_build_opts), vbm_gaussians, C.c_void_p, C.c_void_p,
                                        C.c_size_t, C.c_void_p]),
    "vbm_adaptive_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32]),
    "vbm_adaptive_select": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(vbm_adaptive_opts), C.c_int64,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "vbm_construct_gaussians": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                            C.POINTER(vbm_build_opts), vbm_gaussians, C.c_void_p]),
    "vbm_plan_make": (C.c_int32, [C.POINTER(vbm_view), C.c_int32, C.POINTER(C.c_int64), C.c_int32,
                                  C.POINTER(vbm_schedule), C.POINTER(vbm_plan), C.c_void_p]),
    "vbm_render_fwd": (C.c_int32, [C.POINTER(vbm_plan), C.c_void_p, vbm_gaussians_c, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "vbm_render_bwd": (C.c_int32, [C.POINTER(vbm_plan), C.c_void_p, vbm_gaussians_c, C.c_void_p, C.c_void_p,
                                   C.c_void_p, vbm_gaussians, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "vbm_image_loss_workspace_size": (C.c_size_t, [C.POINTER(C.c_int32), C.c_int32, C.c_int32]),
    "vbm_image_loss": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.c_float,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "vbm_image_loss_static": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                          C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vbm_adam_step": (C.c_int32, [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, vbm_gaussians_c,
                                  vbm_gaussians, C.POINTER(vbm_adam_opts), C.c_void_p, C.c_void_p]),
    "vbm_adam_init": (C.c_int32, [C.c_int64, C.c_int64, vbm_gaussians_c, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "vbm_dvr_render": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(vbm_tf), C.POINTER(vbm_view), C.c_int32,
                                   C.c_float, C.c_void_p, C.c_void_p]),
    "vbm_profile_events": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vbm_profile_counters": (C.c_int32, [C.c_void_p]),
}

EXPORTS = tuple(_SIGS)

_lib = None


class VBMError(RuntimeError):
    pass


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads libvbm.so (built in-tree by __graft_entry__.build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise VBMError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                       "(the HIP library is required; there is no fallback path)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str) -> None:
    if status != 0:
        msg = load().vbm_last_error().decode(errors="replace")
        raise VBMError(f"{what} failed ({STATUS.get(status, status)}): {msg}")
