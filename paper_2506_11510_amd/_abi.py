"""ctypes binding of libtetvol.so (include/tetvol.h).  Argument marshalling
only: every step of the method runs in the library's HIP kernels.  Device
buffers are torch tensors (memory and streams); torch does no compute here."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libtetvol.so")

TET_OK, TET_ERR_INVALID_ARG, TET_ERR_OUT_OF_MEMORY, TET_ERR_CAPACITY = 0, -1, -2, -3
TET_ERR_DEVICE, TET_ERR_NUMERIC, TET_ERR_UNSUPPORTED, TET_ERR_INTERNAL = -4, -5, -6, -7

_lib = None


class TetError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class TetDensity(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("density_scale", ctypes.c_float)]


class TetSparseDensity(ctypes.Structure):
    _fields_ = [("brick_coords", ctypes.c_void_p), ("brick_values", ctypes.c_void_p), ("num_bricks", ctypes.c_int64),
                ("n", ctypes.c_int32), ("on_device", ctypes.c_int32), ("density_scale", ctypes.c_float)]


class TetCamera(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("look_at", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y_deg", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class TetMedium(ctypes.Structure):
    _fields_ = [("albedo", ctypes.c_float), ("g", ctypes.c_float)]


class TetLight(ctypes.Structure):
    _fields_ = [("sun_dir", ctypes.c_float * 3), ("sun_irradiance", ctypes.c_float * 3),
                ("env_radiance", ctypes.c_float * 3)]


class TetBuildOpts(ctypes.Structure):
    _fields_ = [("want_mode", ctypes.c_int32), ("uniform_depth", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("majorant_mode", ctypes.c_int32), ("variation_tau", ctypes.c_double), ("max_tets", ctypes.c_int64),
                ("rand_seed", ctypes.c_uint64), ("rand_thresh", ctypes.c_int32), ("host_rounds", ctypes.c_int32)]


class TetRenderOpts(ctypes.Structure):
    _fields_ = [("max_bounces", ctypes.c_int32), ("transmittance", ctypes.c_int32),
                ("max_steps_per_path", ctypes.c_int64), ("sample_offset", ctypes.c_int32),
                ("samples_per_item", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("record_layout", ctypes.c_int32), ("batch_items", ctypes.c_int32), ("event_wait", ctypes.c_int32),
                ("nrc", ctypes.c_void_p), ("nrc_train", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("emission", ctypes.c_float * 3)]


class TetChannels(ctypes.Structure):
    _fields_ = [("temperature", ctypes.c_void_p), ("albedo", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("on_device", ctypes.c_int32)]


class TetRenderStats(ctypes.Structure):
    _fields_ = [("tet_steps", ctypes.c_int64), ("null_collisions", ctypes.c_int64),
                ("real_collisions", ctypes.c_int64), ("escapes", ctypes.c_int64), ("truncated", ctypes.c_int64),
                ("ms", ctypes.c_double), ("trace_ms", ctypes.c_double), ("cache_ms", ctypes.c_double),
                ("cache_queries", ctypes.c_int64), ("cache_records", ctypes.c_int64), ("cache_loss", ctypes.c_double),
                ("light_rays_queued", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TetNrcOpts(ctypes.Structure):
    _fields_ = [("truncate_bounce", ctypes.c_int32), ("train_paths", ctypes.c_int32),
                ("train_vertices", ctypes.c_int32), ("train_steps", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("sigma_ref", ctypes.c_float), ("ema", ctypes.c_float), ("seed", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TetNrcStats(ctypes.Structure):
    _fields_ = [("records", ctypes.c_int64), ("loss", ctypes.c_double), ("ms", ctypes.c_double),
                ("trace_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TetAutotuneOpts(ctypes.Structure):
    _fields_ = [("probe_spp", ctypes.c_int32), ("probe_repeats", ctypes.c_int32), ("cache_path", ctypes.c_char_p)]


class TetBuildStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("max_depth", ctypes.c_int32), ("num_tets", ctypes.c_int64),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes) for every entry point of include/tetvol.h
VP = ctypes.c_void_p
SIGNATURES = {
    "tet_build_opts_defaults": (None, [ctypes.POINTER(TetBuildOpts)]),
    "tet_render_opts_defaults": (None, [ctypes.POINTER(TetRenderOpts)]),
    "leb_build": (ctypes.c_int, [ctypes.POINTER(TetDensity), ctypes.POINTER(TetCamera), ctypes.c_float,
                                 ctypes.POINTER(TetBuildOpts), VP, ctypes.POINTER(VP)]),
    "leb_build_sparse": (ctypes.c_int, [ctypes.POINTER(TetSparseDensity), ctypes.POINTER(TetCamera), ctypes.c_float,
                                        ctypes.POINTER(TetBuildOpts), VP, ctypes.POINTER(VP)]),
    "leb_update": (ctypes.c_int, [VP, ctypes.POINTER(TetDensity), ctypes.POINTER(TetCamera), ctypes.c_float,
                                  ctypes.POINTER(TetBuildOpts), VP]),
    "leb_update_sparse": (ctypes.c_int, [VP, ctypes.POINTER(TetSparseDensity), ctypes.POINTER(TetCamera),
                                         ctypes.c_float, ctypes.POINTER(TetBuildOpts), VP]),
    "tet_grid_info": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(TetBuildStats)]),
    "tet_grid_export": (ctypes.c_int, [VP, VP, VP, VP, VP, VP, ctypes.c_int32, VP]),
    "tet_grid_export_faces": (ctypes.c_int, [VP, ctypes.c_int32, VP, VP, VP, ctypes.c_int32, VP]),
    "tet_grid_set_channels": (ctypes.c_int, [VP, ctypes.POINTER(TetChannels), VP]),
    "tet_grid_export_channels": (ctypes.c_int, [VP, VP, VP, VP, ctypes.c_int32]),
    "tet_grid_set_density_model": (ctypes.c_int, [VP, ctypes.POINTER(TetDensity), ctypes.c_int32, VP]),
    "tet_grid_export_density_model": (ctypes.c_int, [VP, VP, VP, ctypes.c_int32]),
    "tet_render": (ctypes.c_int, [VP, ctypes.POINTER(TetCamera), ctypes.POINTER(TetMedium), ctypes.POINTER(TetLight),
                                  ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(TetRenderOpts), VP, ctypes.c_int32,
                                  VP, ctypes.POINTER(TetRenderStats)]),
    "tet_render_noalloc": (ctypes.c_int, [VP, ctypes.POINTER(TetCamera), ctypes.POINTER(TetMedium),
                                          ctypes.POINTER(TetLight), ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.POINTER(TetRenderOpts), VP, VP]),
    "tet_locate": (ctypes.c_int, [VP, VP, ctypes.c_int64, VP, ctypes.c_int32, VP]),
    "tet_eval_functions": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, VP, VP, VP, ctypes.c_int32, VP]),
    "dda_render": (ctypes.c_int, [ctypes.POINTER(TetDensity), ctypes.POINTER(TetCamera), ctypes.POINTER(TetMedium),
                                  ctypes.POINTER(TetLight), ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.POINTER(TetRenderOpts), VP, ctypes.c_int32, VP,
                                  ctypes.POINTER(TetRenderStats)]),
    "tet_grid_free": (None, [VP]),
    "tet_autotune_opts_defaults": (None, [ctypes.POINTER(TetAutotuneOpts)]),
    "tet_autotune": (ctypes.c_int, [VP, ctypes.POINTER(TetCamera), ctypes.POINTER(TetMedium), ctypes.POINTER(TetLight),
                                    ctypes.POINTER(TetAutotuneOpts), ctypes.POINTER(TetRenderOpts), VP,
                                    ctypes.POINTER(ctypes.c_double)]),
    "tet_render_batch": (ctypes.c_int, [ctypes.c_int32, VP, VP, VP, VP, VP, VP, ctypes.POINTER(TetRenderOpts), VP,
                                        VP, ctypes.POINTER(TetRenderStats)]),
    "tet_batch_create": (ctypes.c_int, [ctypes.c_int32, VP, VP, VP, VP, VP, ctypes.POINTER(TetRenderOpts), VP,
                                        ctypes.POINTER(VP)]),
    "tet_batch_render": (ctypes.c_int, [VP, VP, VP, ctypes.POINTER(TetRenderStats)]),
    "tet_batch_free": (None, [VP]),
    "tet_nrc_opts_defaults": (None, [ctypes.POINTER(TetNrcOpts)]),
    "tet_nrc_create": (ctypes.c_int, [ctypes.POINTER(TetNrcOpts), ctypes.POINTER(VP)]),
    "tet_nrc_free": (None, [VP]),
    "tet_nrc_info": (ctypes.c_int, [VP, ctypes.POINTER(TetNrcOpts), ctypes.POINTER(ctypes.c_int64)]),
    "tet_nrc_export": (ctypes.c_int, [VP, VP, ctypes.c_int32, VP]),
    "tet_nrc_export_inference": (ctypes.c_int, [VP, VP, ctypes.c_int32, VP]),
    "tet_nrc_import": (ctypes.c_int, [VP, VP, ctypes.c_int32, VP]),
    "tet_nrc_infer": (ctypes.c_int, [VP, ctypes.c_int64, VP, VP, VP, VP, ctypes.c_int32, VP]),
    "tet_nrc_forward_backward": (ctypes.c_int, [VP, ctypes.c_int32, VP, VP, VP, VP, ctypes.c_int32, VP]),
    "tet_nrc_train_batch": (ctypes.c_int, [VP, ctypes.c_int32, VP, VP, VP, VP, VP, ctypes.c_int32, VP]),
    "tet_nrc_collect": (ctypes.c_int, [VP, VP, ctypes.POINTER(TetCamera), ctypes.POINTER(TetMedium),
                                       ctypes.POINTER(TetLight), ctypes.c_uint64, ctypes.POINTER(TetRenderOpts),
                                       VP, VP, VP, VP, VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.c_int32, VP]),
    "tet_nrc_train_frame": (ctypes.c_int, [VP, VP, ctypes.POINTER(TetCamera), ctypes.POINTER(TetMedium),
                                           ctypes.POINTER(TetLight), ctypes.c_uint64, ctypes.POINTER(TetRenderOpts),
                                           VP, ctypes.POINTER(TetNrcStats)]),
    "tet_release_cache": (None, []),
    "tet_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library; raises if it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with __graft_entry__.build() "
                               "(python paper_2506_11510_amd/build.py)")
        L = ctypes.CDLL(SO_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, what: str):
    if rc != TET_OK:
        msg = lib().tet_last_error()
        raise TetError(rc, f"{what}: {msg.decode() if msg else ''}")


def make_camera(c: dict) -> TetCamera:
    k = TetCamera()
    k.pos[:] = [float(x) for x in c["pos"]]
    k.look_at[:] = [float(x) for x in c["look_at"]]
    k.up[:] = [float(x) for x in c["up"]]
    k.fov_y_deg = float(c["fov_y_deg"])
    k.width = int(c["width"])
    k.height = int(c["height"])
    return k


def make_medium(m: dict) -> TetMedium:
    return TetMedium(float(m["albedo"]), float(m["g"]))


def make_light(l: dict) -> TetLight:
    o = TetLight()
    o.sun_dir[:] = [float(x) for x in l["sun_dir"]]
    o.sun_irradiance[:] = [float(x) for x in l["sun_irradiance"]]
    o.env_radiance[:] = [float(x) for x in l["env_radiance"]]
    return o


def make_build_opts(b: dict | None) -> TetBuildOpts:
    o = TetBuildOpts()
    lib().tet_build_opts_defaults(ctypes.byref(o))
    for k, v in (b or {}).items():
        if hasattr(o, k):
            setattr(o, k, type(getattr(o, k))(v))
    return o


def make_render_opts(r: dict | None) -> TetRenderOpts:
    """Render options from a dict; "nrc" takes a cache object (with a
    `handle`) or None."""
    o = TetRenderOpts()
    lib().tet_render_opts_defaults(ctypes.byref(o))
    for k, v in (r or {}).items():
        if k == "nrc":
            o.nrc = v.handle if v is not None else None
        elif k == "emission":
            o.emission[:] = [float(x) for x in v]
        elif hasattr(o, k):
            setattr(o, k, type(getattr(o, k))(v))
    return o


def make_nrc_opts(d: dict | None) -> TetNrcOpts:
    o = TetNrcOpts()
    lib().tet_nrc_opts_defaults(ctypes.byref(o))
    for k, v in (d or {}).items():
        if not hasattr(o, k):
            raise KeyError(f"unknown radiance-cache option {k}")
        setattr(o, k, type(getattr(o, k))(v))
    return o
