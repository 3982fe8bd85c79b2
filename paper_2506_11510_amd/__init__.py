"""Adaptive tetrahedral grids for volumetric path tracing on MI355X (gfx950).

Python face of libtetvol.so (include/tetvol.h): argument marshalling around
the C ABI.  The LEB grid build, the tet walk, delta tracking, scattering and
the radiance cache all run in the library's HIP kernels; torch tensors only
hold device memory and supply streams.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import TetError, check, lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream) if torch.cuda.is_available() else None


def _ptr(t):
    """(pointer, on_device) of a contiguous torch tensor or numpy array."""
    if isinstance(t, np.ndarray):
        assert t.flags.c_contiguous
        return ctypes.c_void_p(t.ctypes.data), 0
    assert t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr()), int(t.is_cuda)


def density_struct(density, n: int, density_scale: float = 1.0) -> _abi.TetDensity:
    p, dev = _ptr(density)
    return _abi.TetDensity(p, int(n), dev, float(density_scale))


class Grid:
    """A device-resident tet grid (owns the library handle)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                lib().tet_grid_free(h)
            except Exception:  # interpreter shutdown: the library is already gone
                pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n = ctypes.c_int64()
        d = ctypes.c_int32()
        st = _abi.TetBuildStats()
        check(lib().tet_grid_info(self._h, ctypes.byref(n), ctypes.byref(d), ctypes.byref(st)), "tet_grid_info")
        return {**st.as_dict(), "num_tets": n.value, "max_depth": d.value}

    @property
    def num_tets(self) -> int:
        return self.info()["num_tets"]

    def update(self, density, n: int, camera: dict, target_cell_px: float = 1.0, build: dict | None = None,
               density_scale: float | None = None) -> "Grid":
        """leb_update: rebuilds this grid in place for a new camera (same
        result as leb_build with these arguments), seeded from its current
        tree.  Returns self."""
        b = dict(build or {})
        scale = b.pop("density_scale", 1.0) if density_scale is None else density_scale
        target = b.pop("target_px", target_cell_px)
        b.pop("shuffle_seed", None)
        ds = density_struct(density, n, scale)
        cam = _abi.make_camera(camera)
        opts = _abi.make_build_opts(b)
        check(lib().leb_update(self._h, ctypes.byref(ds), ctypes.byref(cam), float(target), ctypes.byref(opts),
                               _stream()), "leb_update")
        self.__dict__.pop("_model", None)
        return self

    def update_sparse(self, coords, values, n: int, camera: dict, target_cell_px: float = 1.0,
                      build: dict | None = None, density_scale: float | None = None) -> "Grid":
        """leb_update_sparse: the same from 8^3 bricks (see leb_build_sparse)."""
        b = dict(build or {})
        scale = b.pop("density_scale", 1.0) if density_scale is None else density_scale
        target = b.pop("target_px", target_cell_px)
        b.pop("shuffle_seed", None)
        sd, _keep = _sparse_struct(coords, values, n, scale)
        cam = _abi.make_camera(camera)
        opts = _abi.make_build_opts(b)
        check(lib().leb_update_sparse(self._h, ctypes.byref(sd), ctypes.byref(cam), float(target),
                                      ctypes.byref(opts), _stream()), "leb_update_sparse")
        self.__dict__.pop("_model", None)
        return self

    def export(self, device: bool = False, fields=("ids", "nbr", "sigma", "majorant", "verts")) -> dict:
        """Copies of ids, neighbour links, extinction, majorant, vertices:
        numpy arrays, or CUDA tensors with device=True (ids and links as
        int64 / int32 bit patterns); only the listed fields."""
        n = self.num_tets
        shapes = dict(ids=(n,), nbr=(n, 4), sigma=(n,), majorant=(n,), verts=(n, 4, 3))
        if device:
            import torch
            dt = dict(ids=torch.int64, nbr=torch.int32, sigma=torch.float32, majorant=torch.float32,
                      verts=torch.int32)
            out = {k: torch.empty(shapes[k], dtype=dt[k], device="cuda") for k in fields}
            ptr = {k: ctypes.c_void_p(v.data_ptr()) for k, v in out.items()}
        else:
            dt = dict(ids=np.uint64, nbr=np.uint32, sigma=np.float32, majorant=np.float32, verts=np.int32)
            out = {k: np.empty(shapes[k], dt[k]) for k in fields}
            ptr = {k: ctypes.c_void_p(v.ctypes.data) for k, v in out.items()}
        check(lib().tet_grid_export(self._h, ptr.get("ids"), ptr.get("nbr"), ptr.get("sigma"), ptr.get("majorant"),
                                    ptr.get("verts"), int(device), _stream()), "tet_grid_export")
        return out

    def set_channels(self, n: int, temperature=None, albedo=None, g=None):
        """Extra per-tet channels from n^3 FP32 grids (x fastest; numpy
        arrays or CUDA tensors, all on one side; None = absent): each tet
        gets the mean over its voxel box.  Renders use them with
        render option channels=1 (emission = per-unit-temperature RGB)."""
        arrs = [temperature, albedo, g]
        dev = any(a is not None and not isinstance(a, np.ndarray) for a in arrs)
        keep, ptrs = [], []
        for a in arrs:
            if a is None:
                ptrs.append(None)
                continue
            if dev:
                a = a.contiguous().float().reshape(-1)
                ptrs.append(a.data_ptr())
            else:
                a = np.ascontiguousarray(a, np.float32).reshape(-1)
                ptrs.append(a.ctypes.data)
            assert a.shape[0] == n ** 3
            keep.append(a)
        c = _abi.TetChannels(ptrs[0], ptrs[1], ptrs[2], int(n), int(dev))
        check(lib().tet_grid_set_channels(self._h, ctypes.byref(c), _stream()), "tet_grid_set_channels")
        self._channels = tuple(a is not None for a in arrs)

    def export_faces(self, layout: int = 48) -> dict:
        """Face data of the 48- or 32-byte traversal records: codes (n, 4)
        uint8, offsets (n, 4) int32 (lattice units), links (n, 4) uint32."""
        n = self.num_tets
        out = dict(codes=np.empty((n, 4), np.uint8), offsets=np.empty((n, 4), np.int32),
                   links=np.empty((n, 4), np.uint32))
        check(lib().tet_grid_export_faces(self._h, int(layout), out["codes"].ctypes.data, out["offsets"].ctypes.data,
                                          out["links"].ctypes.data, 0, _stream()), "tet_grid_export_faces")
        return out

    def export_channels(self) -> dict:
        """Per-tet channel values (numpy float32; None for absent ones)."""
        n = self.num_tets
        have = getattr(self, "_channels", (False, False, False))
        out = {k: (np.empty(n, np.float32) if h else None) for k, h in zip(("temperature", "albedo", "g"), have)}
        ptr = [None if v is None else ctypes.c_void_p(v.ctypes.data) for v in out.values()]
        check(lib().tet_grid_export_channels(self._h, ptr[0], ptr[1], ptr[2], 0), "tet_grid_export_channels")
        return out

    def set_density_model(self, model: int, density=None, n: int = 0, scale: float = 1.0):
        """Extinction inside each tet: 0 constant (the build's), 1 linear
        between trilinear vertex samples of `density` (n^3, x fastest;
        numpy or CUDA tensor), 2 voxel lookup in it; `scale` multiplies
        the density."""
        if model == 0 and density is None:
            ds = None
        else:
            if not isinstance(density, np.ndarray):
                density = density.contiguous().float().reshape(-1)
            else:
                density = np.ascontiguousarray(density, np.float32).reshape(-1)
            assert density.shape[0] == n ** 3
            ds = density_struct(density, n, scale)
        check(lib().tet_grid_set_density_model(self._h, ctypes.byref(ds) if ds is not None else None, int(model),
                                               _stream()), "tet_grid_set_density_model")
        self._model = int(model)

    def export_density_model(self) -> dict:
        """Per-tet majorant and (linear model) coefficients (c0, gx, gy, gz),
        numpy float32."""
        n = self.num_tets
        model = getattr(self, "_model", 0)
        out = dict(majorant=np.empty(n, np.float32), coef=np.empty((n, 4), np.float32) if model == 1 else None)
        ptr = [None if v is None else ctypes.c_void_p(v.ctypes.data) for v in out.values()]
        check(lib().tet_grid_export_density_model(self._h, ptr[0], ptr[1], 0), "tet_grid_export_density_model")
        return out

    def locate(self, pts):
        """Tet index of each point (torch CUDA tensor (N,3) float32 -> int64
        tensor, or numpy on the host)."""
        if isinstance(pts, np.ndarray):
            pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
            out = np.empty(len(pts), np.int64)
            check(lib().tet_locate(self._h, pts.ctypes.data, len(pts), out.ctypes.data, 0, _stream()), "tet_locate")
            return out
        import torch
        pts = pts.contiguous().float().reshape(-1, 3)
        out = torch.empty(pts.shape[0], dtype=torch.int64, device=pts.device)
        check(lib().tet_locate(self._h, ctypes.c_void_p(pts.data_ptr()), pts.shape[0],
                               ctypes.c_void_p(out.data_ptr()), 1, _stream()), "tet_locate")
        return out


def leb_build(density, n: int, camera: dict, target_cell_px: float = 1.0, build: dict | None = None,
              density_scale: float | None = None) -> Grid:
    """Builds the adaptive conforming tet grid from an n^3 density (torch CUDA
    tensor or numpy array, x fastest)."""
    b = dict(build or {})
    scale = b.pop("density_scale", 1.0) if density_scale is None else density_scale
    target = b.pop("target_px", target_cell_px)
    for k in ("shuffle_seed",):
        b.pop(k, None)
    ds = density_struct(density, n, scale)
    cam = _abi.make_camera(camera)
    opts = _abi.make_build_opts(b)
    h = ctypes.c_void_p()
    check(lib().leb_build(ctypes.byref(ds), ctypes.byref(cam), float(target), ctypes.byref(opts), _stream(),
                          ctypes.byref(h)), "leb_build")
    return Grid(h)


def _sparse_struct(coords, values, n: int, scale: float):
    """(tet_sparse_density, the contiguous arrays it points into)."""
    if isinstance(coords, np.ndarray):
        coords = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
        values = np.ascontiguousarray(values, np.float32).reshape(-1, 512)
    else:
        coords = coords.contiguous().int().reshape(-1, 3)
        values = values.contiguous().float().reshape(-1, 512)
    assert coords.shape[0] == values.shape[0]
    pc, dev_c = _ptr(coords)
    pv, dev_v = _ptr(values)
    assert dev_c == dev_v
    return _abi.TetSparseDensity(pc, pv, int(coords.shape[0]), int(n), dev_c, float(scale)), (coords, values)


def leb_build_sparse(coords, values, n: int, camera: dict, target_cell_px: float = 1.0, build: dict | None = None,
                     density_scale: float | None = None) -> Grid:
    """The same build from a sparse volume: `coords` (B, 3) int32 brick
    positions (voxel / 8) and `values` (B, 512) float32 voxels of each 8^3
    brick, x fastest; both numpy arrays or both CUDA tensors."""
    b = dict(build or {})
    scale = b.pop("density_scale", 1.0) if density_scale is None else density_scale
    target = b.pop("target_px", target_cell_px)
    b.pop("shuffle_seed", None)
    sd, _keep = _sparse_struct(coords, values, n, scale)
    cam = _abi.make_camera(camera)
    opts = _abi.make_build_opts(b)
    h = ctypes.c_void_p()
    check(lib().leb_build_sparse(ctypes.byref(sd), ctypes.byref(cam), float(target), ctypes.byref(opts), _stream(),
                                 ctypes.byref(h)), "leb_build_sparse")
    return Grid(h)


def render(grid: Grid, camera: dict, medium: dict, light: dict, spp: int, seed: int, render: dict | None = None,
           out=None):
    """Renders (H, W, 3) float32 radiance into a torch CUDA tensor.  Returns
    (image, stats)."""
    import torch
    cam = _abi.make_camera(camera)
    if out is None:
        out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")
    st = _abi.TetRenderStats()
    p, dev = _ptr(out)
    check(lib().tet_render(grid.handle, ctypes.byref(cam), ctypes.byref(_abi.make_medium(medium)),
                           ctypes.byref(_abi.make_light(light)), int(spp), int(seed),
                           ctypes.byref(_abi.make_render_opts(render)), p, dev, _stream(), ctypes.byref(st)),
          "tet_render")
    return out, st.as_dict()


def render_noalloc(grid: Grid, camera: dict, medium: dict, light: dict, spp: int, seed: int,
                   render: dict | None = None, out=None):
    """tet_render_noalloc: the same render with the library's fixed scratch
    (no device allocation inside the call) into a torch CUDA tensor `out`
    (allocated here when None); launches on the current stream without
    waiting.  Returns the image."""
    import torch
    cam = _abi.make_camera(camera)
    if out is None:
        out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")
    assert out.is_cuda and out.is_contiguous() and out.numel() == cam.height * cam.width * 3
    check(lib().tet_render_noalloc(grid.handle, ctypes.byref(cam), ctypes.byref(_abi.make_medium(medium)),
                                   ctypes.byref(_abi.make_light(light)), int(spp), int(seed),
                                   ctypes.byref(_abi.make_render_opts(render)), ctypes.c_void_p(out.data_ptr()),
                                   _stream()), "tet_render_noalloc")
    return out


def dda_render(density, n: int, density_scale: float, camera: dict, medium: dict, light: dict, spp: int, seed: int,
               render: dict | None = None, out=None):
    """Same integrator on the regular voxel grid (regular-grid reference)."""
    import torch
    cam = _abi.make_camera(camera)
    if out is None:
        out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda")
    st = _abi.TetRenderStats()
    ds = density_struct(density, n, density_scale)
    p, dev = _ptr(out)
    check(lib().dda_render(ctypes.byref(ds), ctypes.byref(cam), ctypes.byref(_abi.make_medium(medium)),
                           ctypes.byref(_abi.make_light(light)), int(spp), int(seed),
                           ctypes.byref(_abi.make_render_opts(render)), p, dev, _stream(), ctypes.byref(st)),
          "dda_render")
    return out, st.as_dict()


TUNED_FIELDS = ("waves_per_simd", "event_wait", "batch_items", "block_size", "record_layout", "samples_per_item")


def autotune(grid: Grid, camera: dict, medium: dict, light: dict, render: dict | None = None, probe_spp: int = 2,
             probe_repeats: int = 2, cache_path: str | None = None):
    """Launch options for this frame chosen by the library's autotuner:
    returns (render options dict = `render` with the tuned fields, probe ms)."""
    o = _abi.make_render_opts(render)
    ao = _abi.TetAutotuneOpts(int(probe_spp), int(probe_repeats),
                              cache_path.encode() if cache_path else None)
    ms = ctypes.c_double()
    check(lib().tet_autotune(grid.handle, ctypes.byref(_abi.make_camera(camera)),
                             ctypes.byref(_abi.make_medium(medium)), ctypes.byref(_abi.make_light(light)),
                             ctypes.byref(ao), ctypes.byref(o), _stream(), ctypes.byref(ms)), "tet_autotune")
    out = dict(render or {})
    out.update({k: int(getattr(o, k)) for k in TUNED_FIELDS})
    return out, ms.value


class _SceneArrays:
    """ctypes arrays describing a batch of scenes (kept alive with it)."""

    def __init__(self, grids, cameras, media, lights, spp, outs):
        import torch
        n = len(grids)
        assert n == len(cameras) == len(media) == len(lights) == len(spp)
        self.n = n
        self.grids = list(grids)
        self.grid_ptrs = (ctypes.c_void_p * n)(*[g.handle for g in grids])
        self.cams = (_abi.TetCamera * n)(*[_abi.make_camera(c) for c in cameras])
        self.media = (_abi.TetMedium * n)(*[_abi.make_medium(m) for m in media])
        self.lights = (_abi.TetLight * n)(*[_abi.make_light(l) for l in lights])
        self.spp = (ctypes.c_int32 * n)(*[int(x) for x in spp])
        if outs is None:
            outs = [torch.empty((c["height"], c["width"], 3), dtype=torch.float32, device="cuda") for c in cameras]
        for o, c in zip(outs, cameras):
            assert o.is_cuda and o.is_contiguous() and o.numel() == c["width"] * c["height"] * 3
        self.outs = list(outs)
        self.out_ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])


def render_batch(grids, cameras, media, lights, spp, seeds, render: dict | None = None, outs=None):
    """Renders a batch of scenes with one persistent launch; returns (list
    of (H, W, 3) CUDA tensors, batch stats)."""
    a = _SceneArrays(grids, cameras, media, lights, spp, outs)
    sd = (ctypes.c_uint64 * a.n)(*[int(x) for x in seeds])
    st = _abi.TetRenderStats()
    check(lib().tet_render_batch(a.n, a.grid_ptrs, a.cams, a.media, a.lights, a.spp, sd,
                                 ctypes.byref(_abi.make_render_opts(render)), a.out_ptrs, _stream(),
                                 ctypes.byref(st)), "tet_render_batch")
    return a.outs, st.as_dict()


class Batch:
    """A batch of scenes captured once as a HIP graph frame; render(seeds)
    replays it into the same output tensors."""

    def __init__(self, grids, cameras, media, lights, spp, render: dict | None = None, outs=None):
        self._a = _SceneArrays(grids, cameras, media, lights, spp, outs)
        h = ctypes.c_void_p()
        check(lib().tet_batch_create(self._a.n, self._a.grid_ptrs, self._a.cams, self._a.media, self._a.lights,
                                     self._a.spp, ctypes.byref(_abi.make_render_opts(render)), self._a.out_ptrs,
                                     ctypes.byref(h)), "tet_batch_create")
        self._h = h

    @property
    def outs(self):
        return self._a.outs

    def render(self, seeds) -> dict:
        sd = (ctypes.c_uint64 * self._a.n)(*[int(x) for x in seeds])
        st = _abi.TetRenderStats()
        check(lib().tet_batch_render(self._h, sd, _stream(), ctypes.byref(st)), "tet_batch_render")
        return st.as_dict()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                lib().tet_batch_free(h)
            except Exception:
                pass


N_PARAMS = 17603  # radiance-cache parameters (76 -> 64 x 4 -> 3, with biases)


def _dev(a, dtype, shape):
    """A contiguous CUDA float32/int32 tensor of `shape` from a tensor or array."""
    import torch
    t = torch.as_tensor(a, dtype=dtype)
    if not t.is_cuda:
        t = t.cuda()
    return t.contiguous().reshape(shape)


class Nrc:
    """Learned radiance cache (include/tetvol.h, tet_nrc_*): a handle to the
    network, its FP32 master weights and Adam state on the device."""

    def __init__(self, opts: dict | None = None):
        o = _abi.make_nrc_opts(opts)
        h = ctypes.c_void_p()
        check(lib().tet_nrc_create(ctypes.byref(o), ctypes.byref(h)), "tet_nrc_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                lib().tet_nrc_free(h)
            except Exception:
                pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        o = _abi.TetNrcOpts()
        steps = ctypes.c_int64()
        check(lib().tet_nrc_info(self._h, ctypes.byref(o), ctypes.byref(steps)), "tet_nrc_info")
        return {**o.as_dict(), "adam_steps": steps.value}

    def export(self) -> np.ndarray:
        p = np.empty(N_PARAMS, np.float32)
        check(lib().tet_nrc_export(self._h, p.ctypes.data, 0, _stream()), "tet_nrc_export")
        return p

    def export_inference(self) -> np.ndarray:
        """The weights queries use (the bias-corrected average when ema > 0)."""
        p = np.empty(N_PARAMS, np.float32)
        check(lib().tet_nrc_export_inference(self._h, p.ctypes.data, 0, _stream()), "tet_nrc_export_inference")
        return p

    def load(self, params) -> None:
        """Sets the master weights (17,603 FP32) and resets Adam."""
        p = np.ascontiguousarray(params, np.float32).reshape(-1)
        assert p.size == N_PARAMS
        check(lib().tet_nrc_import(self._h, p.ctypes.data, 0, _stream()), "tet_nrc_import")

    def infer(self, pos, dirs, sigma):
        """Network outputs (unclamped) at points: CUDA tensors in and out."""
        import torch
        pos = _dev(pos, torch.float32, (-1, 3))
        n = pos.shape[0]
        dirs = _dev(dirs, torch.float32, (n, 3))
        sigma = _dev(sigma, torch.float32, (n,))
        y = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
        check(lib().tet_nrc_infer(self._h, n, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(dirs.data_ptr()),
                                  ctypes.c_void_p(sigma.data_ptr()), ctypes.c_void_p(y.data_ptr()), 1, _stream()),
              "tet_nrc_infer")
        return y

    def forward_backward(self, feats, dy):
        """(y, grads) for explicit features (B x 76) and output gradients."""
        import torch
        feats = _dev(feats, torch.float32, (-1, 76))
        n = feats.shape[0]
        dy = _dev(dy, torch.float32, (n, 3))
        y = torch.empty((n, 3), dtype=torch.float32, device=feats.device)
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=feats.device)
        check(lib().tet_nrc_forward_backward(self._h, n, ctypes.c_void_p(feats.data_ptr()),
                                             ctypes.c_void_p(dy.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                             ctypes.c_void_p(g.data_ptr()), 1, _stream()), "tet_nrc_forward_backward")
        return y, g

    def train_batch(self, pos, dirs, sigma, target) -> float:
        """One Adam step on explicit records; returns the loss before it."""
        import torch
        pos = _dev(pos, torch.float32, (-1, 3))
        n = pos.shape[0]
        dirs = _dev(dirs, torch.float32, (n, 3))
        sigma = _dev(sigma, torch.float32, (n,))
        target = _dev(target, torch.float32, (n, 3))
        loss = ctypes.c_float()
        check(lib().tet_nrc_train_batch(self._h, n, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(dirs.data_ptr()),
                                        ctypes.c_void_p(sigma.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                        ctypes.byref(loss), 1, _stream()), "tet_nrc_train_batch")
        return loss.value

    def collect(self, grid: Grid, camera: dict, medium: dict, light: dict, frame_seed: int,
                render: dict | None = None) -> dict:
        """The frame's training records (host arrays): pos, dir, sigma,
        target, tag."""
        info = self.info()
        cap = info["train_paths"] * info["train_vertices"]
        r = dict(pos=np.empty((cap, 3), np.float32), dir=np.empty((cap, 3), np.float32),
                 sigma=np.empty(cap, np.float32), target=np.empty((cap, 3), np.float32), tag=np.empty(cap, np.int32))
        cnt = ctypes.c_int64()
        check(lib().tet_nrc_collect(self._h, grid.handle, ctypes.byref(_abi.make_camera(camera)),
                                    ctypes.byref(_abi.make_medium(medium)), ctypes.byref(_abi.make_light(light)),
                                    int(frame_seed), ctypes.byref(_abi.make_render_opts(render)),
                                    r["pos"].ctypes.data, r["dir"].ctypes.data, r["sigma"].ctypes.data,
                                    r["target"].ctypes.data, r["tag"].ctypes.data, cap, ctypes.byref(cnt), 0,
                                    _stream()), "tet_nrc_collect")
        return {k: v[:cnt.value] for k, v in r.items()}

    def train_frame(self, grid: Grid, camera: dict, medium: dict, light: dict, frame_seed: int,
                    render: dict | None = None) -> dict:
        st = _abi.TetNrcStats()
        check(lib().tet_nrc_train_frame(self._h, grid.handle, ctypes.byref(_abi.make_camera(camera)),
                                        ctypes.byref(_abi.make_medium(medium)), ctypes.byref(_abi.make_light(light)),
                                        int(frame_seed), ctypes.byref(_abi.make_render_opts(render)), _stream(),
                                        ctypes.byref(st)), "tet_nrc_train_frame")
        return st.as_dict()


FUNCTIONS = {"neglog1m": 0, "expneg": 1, "sincos2pi": 2, "hg_pdf": 3, "hg_mu": 4}


def eval_functions(name: str, a, b=None) -> np.ndarray:
    """The tracer's device elementary function `name` (a key of FUNCTIONS)
    at host arguments a (and g = b for the HG functions); FP32 results,
    (n, 2) = (cos, sin) for sincos2pi."""
    fn = FUNCTIONS[name]
    a = np.ascontiguousarray(a, np.float32).ravel()
    bb = None if b is None else np.ascontiguousarray(np.broadcast_to(np.float32(b) if np.isscalar(b) else b, a.shape),
                                                     np.float32)
    out = np.empty((len(a), 2) if fn == 2 else len(a), np.float32)
    check(lib().tet_eval_functions(fn, len(a), a.ctypes.data, None if bb is None else bb.ctypes.data,
                                   out.ctypes.data, 0, _stream()), "tet_eval_functions")
    return out


def release_cache():
    lib().tet_release_cache()


__all__ = ["Grid", "Nrc", "Batch", "render_batch", "autotune", "N_PARAMS", "TetError", "leb_build", "leb_build_sparse", "render", "dda_render", "release_cache", "lib"]
