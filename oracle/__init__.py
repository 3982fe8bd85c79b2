"""Python access to the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product package never imports it.  The oracle
is a plain, slow C statement of the method (see oracle.h for the section map
and the readings of what the paper leaves open).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = ["leb.c", "transport.c", "mlp.c"]
_lib = None

N_PARAMS = 17603
N_FEATS = 76


def build() -> None:
    """Compile liboracle.so: plain C11, IEEE arithmetic, no contraction."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wno-unknown-pragmas"]
    cmd += [os.path.join(_HERE, s) for s in _SRC] + ["-o", _SO + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)


class OCam(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("look_at", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y_deg", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class OMedium(ctypes.Structure):
    _fields_ = [("albedo", ctypes.c_float), ("g", ctypes.c_float)]


class OLight(ctypes.Structure):
    _fields_ = [("sun_dir", ctypes.c_float * 3), ("sun_irradiance", ctypes.c_float * 3),
                ("env_radiance", ctypes.c_float * 3)]


class OBuildOpts(ctypes.Structure):
    _fields_ = [("want_mode", ctypes.c_int32), ("uniform_depth", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("majorant_mode", ctypes.c_int32), ("variation_tau", ctypes.c_double),
                ("target_px", ctypes.c_float), ("density_scale", ctypes.c_float), ("max_tets", ctypes.c_int64),
                ("rand_seed", ctypes.c_uint64), ("rand_thresh", ctypes.c_int32), ("shuffle_seed", ctypes.c_uint64)]


class ORenderOpts(ctypes.Structure):
    _fields_ = [("max_bounces", ctypes.c_int32), ("transmittance", ctypes.c_int32),
                ("max_steps_per_path", ctypes.c_int64), ("sample_offset", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("emission", ctypes.c_float * 3)]


class ORenderStats(ctypes.Structure):
    _fields_ = [("tet_steps", ctypes.c_int64), ("null_collisions", ctypes.c_int64),
                ("real_collisions", ctypes.c_int64), ("escapes", ctypes.c_int64), ("truncated", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class OracleError(RuntimeError):
    pass


def _p(a, t):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp = ctypes.c_void_p
        L.oracle_leb_build.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(OCam), ctypes.POINTER(OBuildOpts),
                                       ctypes.POINTER(vp)]
        L.oracle_grid_num_tets.argtypes = [vp]
        L.oracle_grid_num_tets.restype = ctypes.c_int64
        L.oracle_grid_max_depth.argtypes = [vp]
        L.oracle_grid_export.argtypes = [vp] * 8
        L.oracle_grid_set_channels.argtypes = [vp, vp, vp, vp, ctypes.c_int32]
        L.oracle_grid_export_channels.argtypes = [vp, vp, vp, vp]
        L.oracle_grid_set_density_model.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_int32]
        L.oracle_grid_export_density_model.argtypes = [vp, vp, vp]
        L.oracle_grid_free.argtypes = [vp]
        L.oracle_grid_free.restype = None
        L.oracle_box_stats.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
        L.oracle_want.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(OCam), ctypes.POINTER(OBuildOpts),
                                  ctypes.c_int64, vp, vp, vp, vp]
        L.oracle_locate.argtypes = [vp, ctypes.c_int64, vp, vp]
        L.oracle_walk.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp]
        L.oracle_tet_render.argtypes = [vp, ctypes.POINTER(OCam), ctypes.POINTER(OMedium), ctypes.POINTER(OLight),
                                        ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(ORenderOpts), vp,
                                        ctypes.c_int64, vp, ctypes.POINTER(ORenderStats), ctypes.c_int32]
        L.oracle_dda_render.argtypes = [vp, ctypes.c_int32, ctypes.c_float, ctypes.POINTER(OCam),
                                        ctypes.POINTER(OMedium), ctypes.POINTER(OLight), ctypes.c_int32,
                                        ctypes.c_uint64, ctypes.POINTER(ORenderOpts), vp, ctypes.c_int64, vp,
                                        ctypes.POINTER(ORenderStats), ctypes.c_int32]
        L.oracle_philox4x32_10.argtypes = [vp, vp, vp]
        L.oracle_philox4x32_10.restype = None
        L.oracle_uniform.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 5
        L.oracle_uniform.restype = ctypes.c_float
        L.oracle_hg_sample_mu.argtypes = [ctypes.c_float, ctypes.c_float]
        L.oracle_hg_sample_mu.restype = ctypes.c_float
        L.oracle_neglog1m.argtypes = [ctypes.c_float]
        L.oracle_neglog1m.restype = ctypes.c_float
        L.oracle_expneg.argtypes = [ctypes.c_float]
        L.oracle_expneg.restype = ctypes.c_float
        L.oracle_sincos2pi.argtypes = [ctypes.c_float, vp, vp]
        L.oracle_sincos2pi.restype = None
        L.oracle_hg_eval.argtypes = [ctypes.c_float, ctypes.c_float]
        L.oracle_hg_eval.restype = ctypes.c_float
        L.oracle_hg_direction.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.oracle_hg_direction.restype = None
        L.oracle_camera_ray.argtypes = [ctypes.POINTER(OCam), ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                        ctypes.c_float, vp, vp]
        L.oracle_camera_ray.restype = None
        L.oracle_bf16_round.argtypes = [ctypes.c_float]
        L.oracle_bf16_round.restype = ctypes.c_float
        L.oracle_nrc_encode.argtypes = [ctypes.c_int64, vp, vp, vp, ctypes.c_float, vp]
        L.oracle_mlp_forward.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_int32]
        L.oracle_mlp_backward.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int32]
        L.oracle_ema_step.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_double, ctypes.c_int64, vp]
        L.oracle_nrc_eval_point.argtypes = [vp, ctypes.c_int32, ctypes.c_float, vp, vp, ctypes.c_float, vp]
        L.oracle_nrc_eval_point.restype = None
        L.oracle_nrc_render.argtypes = [vp, ctypes.POINTER(OCam), ctypes.POINTER(OMedium), ctypes.POINTER(OLight),
                                        ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(ORenderOpts), vp,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_float, vp, ctypes.c_int64, vp,
                                        ctypes.POINTER(ORenderStats), ctypes.c_int32]
        L.oracle_train_pixel.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64]
        L.oracle_train_pixel.restype = ctypes.c_int32
        L.oracle_nrc_collect.argtypes = [vp, ctypes.POINTER(OCam), ctypes.POINTER(OMedium), ctypes.POINTER(OLight),
                                         ctypes.c_uint64, ctypes.POINTER(ORenderOpts), ctypes.c_int32,
                                         ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32]
        L.oracle_nrc_loss_grad.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
        L.oracle_adam_step.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


def _vp(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def make_cam(c: dict) -> OCam:
    k = OCam()
    k.pos[:] = [float(x) for x in c["pos"]]
    k.look_at[:] = [float(x) for x in c["look_at"]]
    k.up[:] = [float(x) for x in c["up"]]
    k.fov_y_deg = float(c["fov_y_deg"])
    k.width = int(c["width"])
    k.height = int(c["height"])
    return k


def make_medium(m: dict) -> OMedium:
    return OMedium(float(m["albedo"]), float(m["g"]))


def make_light(l: dict) -> OLight:
    o = OLight()
    o.sun_dir[:] = [float(x) for x in l["sun_dir"]]
    o.sun_irradiance[:] = [float(x) for x in l["sun_irradiance"]]
    o.env_radiance[:] = [float(x) for x in l["env_radiance"]]
    return o


def make_build_opts(b: dict) -> OBuildOpts:
    o = OBuildOpts()
    o.want_mode = int(b.get("want_mode", 0))
    o.uniform_depth = int(b.get("uniform_depth", 0))
    o.max_depth = int(b.get("max_depth", 24))
    o.majorant_mode = int(b.get("majorant_mode", 0))
    o.variation_tau = float(b.get("variation_tau", 0.0))
    o.target_px = float(b.get("target_px", 1.0))
    o.density_scale = float(b.get("density_scale", 1.0))
    o.max_tets = int(b.get("max_tets", 1 << 26))
    o.rand_seed = int(b.get("rand_seed", 0))
    o.rand_thresh = int(b.get("rand_thresh", 0))
    o.shuffle_seed = int(b.get("shuffle_seed", 0))
    return o


def make_render_opts(r: dict) -> ORenderOpts:
    o = ORenderOpts(int(r.get("max_bounces", 8)), int(r.get("transmittance", 0)),
                    int(r.get("max_steps_per_path", (1 << 31) - 1)), int(r.get("sample_offset", 0)),
                    int(r.get("channels", 0)))
    o.emission[:] = [float(x) for x in r.get("emission", (0.0, 0.0, 0.0))]
    return o


class Grid:
    """A grid built by the oracle (owns the C handle)."""

    def __init__(self, handle):
        self._h = handle

    def __del__(self):
        if getattr(self, "_h", None):
            lib().oracle_grid_free(self._h)
            self._h = None

    @property
    def num_tets(self) -> int:
        return int(lib().oracle_grid_num_tets(self._h))

    @property
    def max_depth(self) -> int:
        return int(lib().oracle_grid_max_depth(self._h))

    def export(self) -> dict:
        n = self.num_tets
        out = dict(ids=np.empty(n, np.uint64), verts=np.empty((n, 4, 3), np.int32), nbr=np.empty((n, 4), np.uint32),
                   sigma=np.empty(n, np.float32), majorant=np.empty(n, np.float32), codes=np.empty((n, 4), np.uint8),
                   offsets=np.empty((n, 4), np.int32))
        _check(lib().oracle_grid_export(self._h, _vp(out["ids"]), _vp(out["verts"]), _vp(out["nbr"]),
                                        _vp(out["sigma"]), _vp(out["majorant"]), _vp(out["codes"]),
                                        _vp(out["offsets"])), "oracle_grid_export")
        return out

    def set_channels(self, n: int, temperature=None, albedo=None, g=None):
        """Per-tet means of extra channel grids (n^3 FP32 each, x fastest;
        None = absent), leb.c item 8."""
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32).reshape(-1) for a in (temperature, albedo, g)]
        for a in arrs:
            assert a is None or a.size == n ** 3
        _check(lib().oracle_grid_set_channels(self._h, _vp(arrs[0]), _vp(arrs[1]), _vp(arrs[2]), int(n)),
               "oracle_grid_set_channels")
        self._channels = tuple(a is not None for a in arrs)

    def export_channels(self) -> dict:
        n = self.num_tets
        have = getattr(self, "_channels", (False, False, False))
        out = {k: (np.empty(n, np.float32) if h else None) for k, h in zip(("temperature", "albedo", "g"), have)}
        _check(lib().oracle_grid_export_channels(self._h, _vp(out["temperature"]), _vp(out["albedo"]), _vp(out["g"])),
               "oracle_grid_export_channels")
        return out

    def set_density_model(self, model: int, density=None, n: int = 0, scale: float = 1.0):
        """Extinction inside each tet (leb.c item 9): 0 constant, 1 linear
        between trilinear vertex samples, 2 voxel lookup."""
        d = None if density is None else np.ascontiguousarray(density, np.float32).reshape(-1)
        assert d is None or d.size == n ** 3
        _check(lib().oracle_grid_set_density_model(self._h, _vp(d), int(n), float(scale), int(model)),
               "oracle_grid_set_density_model")
        self._model = int(model)

    def export_density_model(self) -> dict:
        """Per-tet majorant and (linear model) coefficients (c0, gx, gy, gz)."""
        n = self.num_tets
        model = getattr(self, "_model", 0)
        out = dict(majorant=np.empty(n, np.float32), coef=np.empty((n, 4), np.float32) if model == 1 else None)
        _check(lib().oracle_grid_export_density_model(self._h, _vp(out["majorant"]), _vp(out["coef"])),
               "oracle_grid_export_density_model")
        return out

    def locate(self, pts: np.ndarray) -> np.ndarray:
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        out = np.empty(len(pts), np.int64)
        _check(lib().oracle_locate(self._h, len(pts), _vp(pts), _vp(out)), "oracle_locate")
        return out

    def walk(self, o, d, start: int, max_out: int = 100000):
        o = np.ascontiguousarray(o, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        tets = np.empty(max_out, np.int64)
        faces = np.empty(max_out, np.int32)
        tex = np.empty(max_out, np.float32)
        n = ctypes.c_int32()
        _check(lib().oracle_walk(self._h, _vp(o), _vp(d), int(start), max_out, _vp(tets), _vp(faces), _vp(tex),
                                 ctypes.byref(n)), "oracle_walk")
        k = n.value
        return tets[:k], faces[:k], tex[:k]

    def render(self, camera: dict, medium: dict, light: dict, spp: int, seed: int, render: dict | None = None,
               pixels: np.ndarray | None = None, threads: int = 1):
        """Average radiance per pixel: (H, W, 3) for the whole image, or
        (len(pixels), 3) for a pixel subset.  Returns (image, stats)."""
        cam = make_cam(camera)
        ro = make_render_opts(render or {})
        st = ORenderStats()
        if pixels is not None:
            pixels = np.ascontiguousarray(pixels, np.int32)
            out = np.empty((len(pixels), 3), np.float32)
            npx = len(pixels)
        else:
            out = np.empty((cam.height, cam.width, 3), np.float32)
            npx = 0
        _check(lib().oracle_tet_render(self._h, ctypes.byref(cam), ctypes.byref(make_medium(medium)),
                                       ctypes.byref(make_light(light)), int(spp), int(seed), ctypes.byref(ro),
                                       _vp(pixels), npx, _vp(out), ctypes.byref(st), int(threads)),
               "oracle_tet_render")
        return out, st.as_dict()


    def nrc_render(self, camera: dict, medium: dict, light: dict, spp: int, seed: int, params, render=None,
                   truncate_bounce: int = 2, sigma_ref: float = 1.0, bf16: bool = True, pixels=None,
                   threads: int = 1):
        """Truncated render with the radiance cache `params` (17,603
        values): every path stops at real vertex `truncate_bounce` and adds
        the throughput reaching it times the cache's estimate."""
        cam = make_cam(camera)
        ro = make_render_opts(render or {})
        st = ORenderStats()
        params = np.ascontiguousarray(params, np.float64)
        assert params.size == N_PARAMS
        if pixels is not None:
            pixels = np.ascontiguousarray(pixels, np.int32)
            out = np.empty((len(pixels), 3), np.float32)
            npx = len(pixels)
        else:
            out = np.empty((cam.height, cam.width, 3), np.float32)
            npx = 0
        _check(lib().oracle_nrc_render(self._h, ctypes.byref(cam), ctypes.byref(make_medium(medium)),
                                       ctypes.byref(make_light(light)), int(spp), int(seed), ctypes.byref(ro),
                                       _vp(params), int(bool(bf16)), int(truncate_bounce), float(sigma_ref),
                                       _vp(pixels), npx, _vp(out), ctypes.byref(st), int(threads)),
               "oracle_nrc_render")
        return out, st.as_dict()

    def nrc_collect(self, camera: dict, medium: dict, light: dict, frame_seed: int, n_paths: int,
                    max_vertices: int = 4, render=None, threads: int = 1) -> dict:
        """Training records of one frame (see oracle_nrc_collect): pos,
        dir, sigma, target, tag, plus each path's pixel and radiance."""
        cam = make_cam(camera)
        ro = make_render_opts(render or {})
        cap = max(1, n_paths * max_vertices)
        r = dict(pos=np.empty((cap, 3), np.float32), dir=np.empty((cap, 3), np.float32),
                 sigma=np.empty(cap, np.float32), target=np.empty((cap, 3), np.float32), tag=np.empty(cap, np.int32),
                 path_pixel=np.empty(max(1, n_paths), np.int32), path_L=np.empty((max(1, n_paths), 3), np.float32))
        cnt = ctypes.c_int64()
        _check(lib().oracle_nrc_collect(self._h, ctypes.byref(cam), ctypes.byref(make_medium(medium)),
                                        ctypes.byref(make_light(light)), int(frame_seed), ctypes.byref(ro),
                                        int(n_paths), int(max_vertices), _vp(r["pos"]), _vp(r["dir"]),
                                        _vp(r["sigma"]), _vp(r["target"]), _vp(r["tag"]), ctypes.byref(cnt),
                                        _vp(r["path_pixel"]), _vp(r["path_L"]), int(threads)), "oracle_nrc_collect")
        c = cnt.value
        for k in ("pos", "dir", "sigma", "target", "tag"):
            r[k] = r[k][:c]
        r["path_pixel"] = r["path_pixel"][:n_paths]
        r["path_L"] = r["path_L"][:n_paths]
        return r


def densify(coords: np.ndarray, values: np.ndarray, n: int) -> np.ndarray:
    """The dense n^3 volume (x fastest) a sparse volume describes: zero
    outside its 8^3 bricks, brick (bx, by, bz) holding voxels 8 bx .. 8 bx
    + 7 along x (and likewise in y, z), its 512 values x fastest."""
    out = np.zeros((n, n, n), np.float32)  # [z, y, x]
    for (bx, by, bz), v in zip(np.asarray(coords).reshape(-1, 3), np.asarray(values).reshape(-1, 512)):
        out[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8] = v.reshape(8, 8, 8)
    return out.reshape(-1)


def leb_build(density: np.ndarray, n: int, camera: dict, build: dict) -> Grid:
    density = np.ascontiguousarray(density, np.float32)
    assert density.size == n ** 3
    h = ctypes.c_void_p()
    cam = make_cam(camera)
    bo = make_build_opts(build)
    _check(lib().oracle_leb_build(_vp(density), int(n), ctypes.byref(cam), ctypes.byref(bo), ctypes.byref(h)),
           "oracle_leb_build")
    return Grid(h)


def leb_build_status(density: np.ndarray, n: int, camera: dict, build: dict) -> int:
    """Status code of a build (0 = ok), freeing the grid."""
    density = np.ascontiguousarray(density, np.float32)
    h = ctypes.c_void_p()
    rc = lib().oracle_leb_build(_vp(density), int(n), ctypes.byref(make_cam(camera)),
                                ctypes.byref(make_build_opts(build)), ctypes.byref(h))
    if rc == 0:
        lib().oracle_grid_free(h)
    return rc


def box_stats(density: np.ndarray, n: int, lo, hi):
    density = np.ascontiguousarray(density, np.float32)
    lo = np.ascontiguousarray(lo, np.int32)
    hi = np.ascontiguousarray(hi, np.int32)
    mn, mx = ctypes.c_float(), ctypes.c_float()
    s, c = ctypes.c_double(), ctypes.c_double()
    _check(lib().oracle_box_stats(_vp(density), n, _vp(lo), _vp(hi), ctypes.byref(mn), ctypes.byref(mx),
                                  ctypes.byref(s), ctypes.byref(c)), "oracle_box_stats")
    return mn.value, mx.value, s.value, c.value


def want(density, n, camera, build, verts, depth, ids) -> np.ndarray:
    density = np.ascontiguousarray(density, np.float32)
    verts = np.ascontiguousarray(verts, np.int32)
    depth = np.ascontiguousarray(depth, np.int32)
    ids = np.ascontiguousarray(ids, np.uint64)
    out = np.empty(len(depth), np.uint8)
    _check(lib().oracle_want(_vp(density), n, ctypes.byref(make_cam(camera)), ctypes.byref(make_build_opts(build)),
                             len(depth), _vp(verts), _vp(depth), _vp(ids), _vp(out)), "oracle_want")
    return out.astype(bool)


def dda_render(density, n, density_scale, camera, medium, light, spp, seed, render=None, pixels=None, threads=1):
    density = np.ascontiguousarray(density, np.float32)
    cam = make_cam(camera)
    ro = make_render_opts(render or {})
    st = ORenderStats()
    if pixels is not None:
        pixels = np.ascontiguousarray(pixels, np.int32)
        out = np.empty((len(pixels), 3), np.float32)
        npx = len(pixels)
    else:
        out = np.empty((cam.height, cam.width, 3), np.float32)
        npx = 0
    _check(lib().oracle_dda_render(_vp(density), int(n), float(density_scale), ctypes.byref(cam),
                                   ctypes.byref(make_medium(medium)), ctypes.byref(make_light(light)), int(spp),
                                   int(seed), ctypes.byref(ro), _vp(pixels), npx, _vp(out), ctypes.byref(st),
                                   int(threads)), "oracle_dda_render")
    return out, st.as_dict()


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.empty(4, np.uint32)
    lib().oracle_philox4x32_10(_vp(c), _vp(k), _vp(o))
    return o


def uniform(seed, pixel, sample, bounce, stream, draw) -> float:
    return float(lib().oracle_uniform(seed, pixel, sample, bounce, stream, draw))


def hg_sample_mu(g, u) -> float:
    return float(lib().oracle_hg_sample_mu(g, u))


def neglog1m(u) -> float:
    return float(lib().oracle_neglog1m(u))


def expneg(x) -> float:
    return float(lib().oracle_expneg(x))


def sincos2pi(u):
    c, s = ctypes.c_float(), ctypes.c_float()
    lib().oracle_sincos2pi(u, ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def hg_eval(g, mu) -> float:
    return float(lib().oracle_hg_eval(g, mu))


def hg_direction(d, g, u1, u2) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float32)
    o = np.empty(3, np.float32)
    lib().oracle_hg_direction(_vp(d), g, u1, u2, _vp(o))
    return o


def camera_ray(camera: dict, px, py, u0, u1):
    o = np.empty(3, np.float32)
    d = np.empty(3, np.float32)
    lib().oracle_camera_ray(ctypes.byref(make_cam(camera)), px, py, u0, u1, _vp(o), _vp(d))
    return o, d


def bf16_round(x) -> np.ndarray:
    """bfloat16 rounding (nearest, ties to even) of FP32 values, as FP32."""
    x = np.ascontiguousarray(x, np.float32).reshape(-1)
    f = lib().oracle_bf16_round
    return np.array([f(float(v)) for v in x], np.float32)


def nrc_encode(pos, dirs, sigma, sigma_ref: float) -> np.ndarray:
    pos = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
    dirs = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
    sg = np.ascontiguousarray(sigma, np.float32).reshape(-1)
    out = np.empty((len(pos), N_FEATS), np.float32)
    _check(lib().oracle_nrc_encode(len(pos), _vp(pos), _vp(dirs), _vp(sg), float(sigma_ref), _vp(out)),
           "oracle_nrc_encode")
    return out


def mlp_forward(params, x, bf16: bool = False) -> np.ndarray:
    params = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, N_FEATS)
    y = np.empty((len(x), 3), np.float64)
    _check(lib().oracle_mlp_forward(_vp(params), len(x), _vp(x), _vp(y), int(bool(bf16))), "oracle_mlp_forward")
    return y


def mlp_backward(params, x, dy, bf16: bool = False):
    params = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, N_FEATS)
    dy = np.ascontiguousarray(dy, np.float64).reshape(-1, 3)
    y = np.empty((len(x), 3), np.float64)
    g = np.empty(N_PARAMS, np.float64)
    _check(lib().oracle_mlp_backward(_vp(params), len(x), _vp(x), _vp(dy), _vp(y), _vp(g), int(bool(bf16))),
           "oracle_mlp_backward")
    return y, g


def ema_step(ema, params, beta, step):
    """One step of the weight average (in place on `ema`); returns the
    bias-corrected weights."""
    assert ema.dtype == np.float64 and ema.flags.c_contiguous
    params = np.ascontiguousarray(params, np.float64)
    out = np.empty_like(ema)
    _check(lib().oracle_ema_step(len(ema), _vp(ema), _vp(params), float(beta), int(step), _vp(out)),
           "oracle_ema_step")
    return out


def nrc_eval_point(params, p, d, sigma, sigma_ref, bf16: bool = True) -> np.ndarray:
    params = np.ascontiguousarray(params, np.float64)
    p = np.ascontiguousarray(p, np.float32)
    d = np.ascontiguousarray(d, np.float32)
    out = np.empty(3, np.float32)
    lib().oracle_nrc_eval_point(_vp(params), int(bool(bf16)), float(sigma_ref), _vp(p), _vp(d), float(sigma),
                                _vp(out))
    return out


def train_pixel(frame_seed: int, j: int, npix: int) -> int:
    return int(lib().oracle_train_pixel(int(frame_seed), int(j), int(npix)))


def nrc_loss_grad(y, target):
    y = np.ascontiguousarray(y, np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(target, np.float64).reshape(-1, 3)
    loss = ctypes.c_double()
    dy = np.empty_like(y)
    _check(lib().oracle_nrc_loss_grad(len(y), _vp(y), _vp(t), ctypes.byref(loss), _vp(dy)), "oracle_nrc_loss_grad")
    return loss.value, dy


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.99, eps=1e-8):
    for a in (params, grads, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _check(lib().oracle_adam_step(len(params), _vp(params), _vp(grads), _vp(m), _vp(v), int(step), lr, beta1, beta2,
                                  eps), "oracle_adam_step")
