"""ctypes mirror of include/gbb.h and loader of the in-tree libgbb.so.

Argument marshalling only: every step of the rasterizer runs in the HIP library. Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgbb.so")

GB_OK, GB_ERR_ARG, GB_ERR_HIP, GB_ERR_CAPACITY, GB_ERR_UNSUPPORTED = 0, 1, 2, 3, 4
GB_F32, GB_BF16 = 0, 1

EXPORTS = (
    "gb_workspace_layout", "gb_count_pairs", "gb_render_fwd", "gb_render_bwd",
    "gb_read_status", "gb_blend_stats", "gb_timing_enable", "gb_timing_read",
    "gb_timing_stage_name", "gb_default_options", "gb_status_string", "gb_last_error",
    "gb_activate_fwd", "gb_activate_bwd", "gb_l1_loss", "gb_adam_step", "gb_to_bf16",
    "gb_mse_loss", "gb_box_filter_textures", "gb_rotz_only",
    "gb_densify_stats", "gb_densify_work_bytes", "gb_densify_plan", "gb_densify_apply",
    "gb_densify_noalloc", "gb_render_fwd_zeroing",
)

# most splats gb_densify_noalloc takes (GB_DENSIFY_NOALLOC_MAX_P)
DENSIFY_NOALLOC_MAX_P = 1 << 20


class GbView(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("R", c_float * 9), ("t", c_float * 3),
                ("z_near", c_float)]


class GbSplats(ctypes.Structure):
    _fields_ = [("P", c_int32), ("N", c_int32), ("tex_dtype", c_int32), ("means", c_void_p),
                ("tan_u", c_void_p), ("tan_v", c_void_p), ("scales", c_void_p),
                ("opacity", c_void_p), ("textures", c_void_p), ("sh_degree", c_int32),
                ("sh", c_void_p), ("tex_side", c_void_p), ("tex_offset", c_void_p),
                ("n_texels", c_int64)]


class GbOptions(ctypes.Structure):
    _fields_ = [("sigma", c_float), ("alpha_min", c_float), ("alpha_max", c_float),
                ("t_min", c_float), ("lowpass_var", c_float), ("bg", c_float * 3),
                ("tile_w", c_int32), ("tile_h", c_int32), ("batch", c_int32),
                ("batch_bwd", c_int32), ("prefix_pairs_per_tile", c_int32),
                ("tile_order", c_int32)]


class GbGrads(ctypes.Structure):
    _fields_ = [("d_means", c_void_p), ("d_tan_u", c_void_p), ("d_tan_v", c_void_p),
                ("d_scales", c_void_p), ("d_opacity", c_void_p), ("d_textures", c_void_p),
                ("d_sh", c_void_p)]


class GbLayout(ctypes.Structure):
    _fields_ = [("total_bytes", c_size_t), ("status", c_size_t), ("depth_key", c_size_t),
                ("tile_count", c_size_t), ("records", c_size_t), ("order", c_size_t),
                ("pair_keys", c_size_t), ("pair_vals", c_size_t), ("ranges", c_size_t),
                ("n_last", c_size_t), ("pair_capacity", c_int64), ("total_tiles", c_int64),
                ("prefix_capacity", c_int64), ("pair_keys_rest", c_size_t),
                ("pair_vals_rest", c_size_t), ("ranges_rest", c_size_t),
                ("n_last_rest", c_size_t), ("open_tiles", c_size_t), ("tile_order", c_size_t),
                ("tile_work", c_size_t)]


class GbDensifyOptions(ctypes.Structure):
    _fields_ = [("grad_threshold", c_float), ("dense_scale", c_float), ("min_opacity", c_float),
                ("max_scale", c_float), ("split_shrink", c_float)]


class GbRawSplats(ctypes.Structure):
    _fields_ = [("P", c_int32), ("N", c_int32), ("sh_coef", c_int32), ("means", c_void_p),
                ("quats", c_void_p), ("log_scales", c_void_p), ("opacity_logits", c_void_p),
                ("textures", c_void_p), ("sh", c_void_p)]


class GbRowState(ctypes.Structure):
    _fields_ = [("src", c_void_p), ("dst", c_void_p), ("width", c_int32)]


class GbbError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libgbb.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2412_12734_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.gb_workspace_layout.argtypes = [c_int32, c_int32, POINTER(GbView), c_int32,
                                        POINTER(GbOptions), c_int64, POINTER(GbLayout)]
    lib.gb_count_pairs.argtypes = [POINTER(GbSplats), POINTER(GbView), c_int32,
                                   POINTER(GbOptions), c_void_p, c_size_t, c_int64,
                                   POINTER(c_int64), c_void_p]
    lib.gb_render_fwd.argtypes = [POINTER(GbSplats), POINTER(GbView), c_int32,
                                  POINTER(GbOptions), c_void_p, c_size_t, c_int64, c_void_p,
                                  c_void_p, c_void_p]
    lib.gb_render_fwd_zeroing.argtypes = [POINTER(GbSplats), POINTER(GbView), c_int32,
                                          POINTER(GbOptions), c_void_p, c_size_t, c_int64,
                                          c_void_p, c_void_p, c_void_p, c_void_p]
    lib.gb_render_bwd.argtypes = [POINTER(GbSplats), POINTER(GbView), c_int32,
                                  POINTER(GbOptions), c_void_p, c_size_t, c_int64, c_void_p,
                                  c_void_p, POINTER(GbGrads), c_void_p]
    lib.gb_read_status.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int32),
                                   POINTER(c_int64), c_int32, c_void_p]
    lib.gb_blend_stats.argtypes = [POINTER(GbSplats), POINTER(GbView), c_int32,
                                   POINTER(GbOptions), c_void_p, c_size_t, c_int64, c_void_p,
                                   c_void_p, POINTER(c_int64), c_void_p]
    lib.gb_timing_enable.argtypes = [c_int32]
    lib.gb_timing_read.argtypes = [POINTER(c_float), c_int32, POINTER(c_int32)]
    lib.gb_timing_stage_name.argtypes = [c_int32]
    lib.gb_timing_stage_name.restype = c_char_p
    lib.gb_default_options.argtypes = [POINTER(GbOptions)]
    lib.gb_default_options.restype = None
    lib.gb_status_string.argtypes = [c_int32]
    lib.gb_status_string.restype = c_char_p
    lib.gb_last_error.argtypes = []
    lib.gb_last_error.restype = c_char_p
    lib.gb_activate_fwd.argtypes = [c_int32] + [c_void_p] * 7 + [c_void_p]
    lib.gb_activate_bwd.argtypes = [c_int32] + [c_void_p] * 10 + [c_void_p]
    lib.gb_l1_loss.argtypes = [c_int64, c_void_p, c_void_p, c_float, c_void_p, c_void_p, c_void_p]
    lib.gb_adam_step.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                 c_float, c_float, c_float, c_float, c_void_p, c_void_p]
    lib.gb_to_bf16.argtypes = [c_int64, c_void_p, c_void_p, c_void_p]
    lib.gb_mse_loss.argtypes = [c_int64, c_void_p, c_void_p, c_float, c_void_p, c_void_p, c_void_p]
    lib.gb_box_filter_textures.argtypes = [c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                           c_void_p]
    lib.gb_rotz_only.argtypes = [c_int32, c_void_p, c_void_p]
    lib.gb_densify_stats.argtypes = [POINTER(GbSplats), POINTER(GbView), c_int32,
                                     POINTER(GbOptions), c_void_p, c_size_t, c_int64, c_void_p,
                                     c_void_p, c_void_p]
    lib.gb_densify_work_bytes.argtypes = [c_int32]
    lib.gb_densify_work_bytes.restype = c_size_t
    lib.gb_densify_plan.argtypes = [POINTER(GbRawSplats), c_void_p, c_void_p,
                                    POINTER(GbDensifyOptions), c_void_p, c_size_t,
                                    POINTER(c_int64), c_void_p]
    lib.gb_densify_apply.argtypes = [POINTER(GbRawSplats), c_void_p, c_void_p, c_float,
                                     POINTER(GbDensifyOptions), POINTER(GbRawSplats),
                                     POINTER(GbRowState), c_int32, c_void_p]
    lib.gb_densify_noalloc.argtypes = [POINTER(GbRawSplats), c_void_p, c_void_p,
                                       POINTER(GbDensifyOptions), c_void_p, c_float,
                                       POINTER(GbRawSplats), POINTER(GbRowState), c_int32,
                                       POINTER(c_int64), c_void_p]
    for name in ("gb_workspace_layout", "gb_count_pairs", "gb_render_fwd", "gb_render_bwd",
                 "gb_render_fwd_zeroing",
                 "gb_read_status", "gb_blend_stats", "gb_timing_enable", "gb_timing_read",
                 "gb_activate_fwd", "gb_activate_bwd", "gb_l1_loss", "gb_adam_step",
                 "gb_to_bf16", "gb_mse_loss", "gb_box_filter_textures", "gb_rotz_only",
                 "gb_densify_stats", "gb_densify_plan",
                 "gb_densify_apply", "gb_densify_noalloc"):
        getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != GB_OK:
        lib = load()
        detail = lib.gb_last_error().decode() or lib.gb_status_string(status).decode()
        raise GbbError(status, where, detail)


def make_views(views) -> ctypes.Array:
    """Array of GbView from objects with width, height, fx, fy, cx, cy, R, t, z_near."""
    arr = (GbView * len(views))()
    for i, v in enumerate(views):
        R = [float(x) for x in np.asarray(v.R, dtype=np.float32).reshape(-1)]
        t = [float(x) for x in np.asarray(v.t, dtype=np.float32).reshape(-1)]
        arr[i] = GbView(int(v.width), int(v.height), float(v.fx), float(v.fy), float(v.cx),
                        float(v.cy), (c_float * 9)(*R), (c_float * 3)(*t), float(v.z_near))
    return arr


def make_options(sigma=0.5, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4,
                 lowpass_var=0.5, bg=(0.0, 0.0, 0.0), tile_w=16, tile_h=16, batch=0,
                 batch_bwd=0, prefix_pairs_per_tile=0, tile_order=0) -> GbOptions:
    return GbOptions(sigma, alpha_min, alpha_max, t_min, lowpass_var, (c_float * 3)(*bg),
                     tile_w, tile_h, batch, batch_bwd, prefix_pairs_per_tile, tile_order)
