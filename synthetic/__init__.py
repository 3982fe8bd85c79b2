"""Seeded synthetic inputs (density volumes and scene descriptions).

The paper renders OpenVDB production assets (a cloud and an explosion) that
are not available here; these seeded volumes stand in for them with the
shapes and sizes the workloads call for.  This module holds none of the
rendering method's arithmetic: both the oracle and the GPU path take its
output as plain input.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> None:
    """Compile the generator library (host C, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           os.path.join(_HERE, "gen.c"), "-o", _SO + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        f32p = ctypes.POINTER(ctypes.c_float)
        lib.synth_blobs.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, f32p]
        lib.synth_cloud_raw.argtypes = [ctypes.c_uint64, ctypes.c_int32, f32p]
        lib.synth_plume_raw.argtypes = [ctypes.c_uint64, ctypes.c_int32, f32p]
        lib.synth_threshold.argtypes = [f32p, ctypes.c_int64, ctypes.c_double, ctypes.c_double]
        lib.synth_threshold.restype = None
        _lib = lib
    return _lib


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def blobs(seed: int, n: int, nblobs: int = 8) -> np.ndarray:
    """Sum of `nblobs` seeded Gaussian blobs on an n^3 grid (float32,
    x fastest): centres U[0.2,0.8]^3, std-devs U[0.05,0.2], peaks U[2,10]."""
    out = np.empty(n * n * n, dtype=np.float32)
    _load().synth_blobs(seed, n, nblobs, _fptr(out))
    return out


def _threshold(raw: np.ndarray, keep_fraction: float, peak: float) -> np.ndarray:
    """Keep the top `keep_fraction` of voxels (value minus the cut), scaled so
    that the maximum is `peak`."""
    cut = np.partition(raw, int((1.0 - keep_fraction) * raw.size))[int((1.0 - keep_fraction) * raw.size)]
    v = np.maximum(raw - cut, 0.0).astype(np.float32)
    m = float(v.max())
    if m > 0:
        v *= np.float32(peak / m)
    return v


def cloud(seed: int, n: int = 256, keep_fraction: float = 0.2, peak: float = 20.0) -> np.ndarray:
    """fBm cloud (6 octaves gradient noise, ellipsoidal falloff), cut at the
    (1 - keep_fraction) quantile and scaled to `peak` extinction."""
    raw = np.empty(n * n * n, dtype=np.float32)
    _load().synth_cloud_raw(seed, n, _fptr(raw))
    return _threshold(raw, keep_fraction, peak)


def plume(seed: int, n: int = 1024, keep_fraction: float = 0.05, peak: float = 50.0) -> np.ndarray:
    """Smoke plume (curl-advected fBm, height falloff), ~5 % occupancy.  The
    cut and scaling run in place in C (the 1024^3 volume is 4 GiB)."""
    raw = np.empty(n * n * n, dtype=np.float32)
    L = _load()
    L.synth_plume_raw(seed, n, _fptr(raw))
    L.synth_threshold(_fptr(raw), raw.size, ctypes.c_double(keep_fraction), ctypes.c_double(peak))
    return raw


def channels(seed: int, n: int) -> dict:
    """Seeded extra-channel fields on an n^3 grid (float32, x fastest):
    temperature >= 0 (a few hot blobs, peak ~4), albedo in [0.35, 1] and
    phase parameter g in [-0.4, 0.85], both varying smoothly through the
    cube."""
    hot = blobs(seed, n, 4)
    temperature = (4.0 * hot / max(float(hot.max()), 1e-6)).astype(np.float32)
    a = blobs(seed + 1, n, 6)
    albedo = (0.35 + 0.65 * a / max(float(a.max()), 1e-6)).astype(np.float32)
    b = blobs(seed + 2, n, 6)
    g = (-0.4 + 1.25 * b / max(float(b.max()), 1e-6)).astype(np.float32)
    return dict(temperature=temperature, albedo=np.clip(albedo, 0.0, 1.0), g=np.clip(g, -0.4, 0.85))


def bricks(density: np.ndarray, n: int, keep_empty: int = 0, seed: int = 0):
    """Sparse (OpenVDB-like leaf) form of an n^3 volume: the 8^3 bricks that
    hold a nonzero voxel, as (coords (B, 3) int32 in brick units, values
    (B, 512) float32, x fastest), in a seeded random order; `keep_empty`
    all-zero bricks are listed too (a sparse file may carry them)."""
    nb = n // 8
    v = np.asarray(density, np.float32).reshape(nb, 8, nb, 8, nb, 8)  # [bz, z, by, y, bx, x]
    v = v.transpose(0, 2, 4, 1, 3, 5).reshape(nb * nb * nb, 512)  # brick (bz, by, bx), voxel (z, y, x)
    occupied = np.flatnonzero(v.any(axis=1))
    rng = np.random.default_rng(seed)
    empty = np.setdiff1d(np.arange(nb ** 3), occupied)
    pick = np.concatenate([occupied, rng.choice(empty, size=min(keep_empty, len(empty)), replace=False)])
    pick = pick[rng.permutation(len(pick))]
    coords = np.stack([pick % nb, (pick // nb) % nb, pick // (nb * nb)], axis=1).astype(np.int32)
    return coords, np.ascontiguousarray(v[pick])


def _unit(v):
    l = math.sqrt(sum(x * x for x in v))
    return [x / l for x in v]


LIGHT_DEFAULT = dict(sun_dir=_unit([0.3, 0.8, -0.5]), sun_irradiance=[3.0, 2.9, 2.7],
                     env_radiance=[0.25, 0.30, 0.40])


def scene(name: str, **over) -> dict:
    """Scene description: density + camera + medium + light + build/render
    options.  Names: 'tiny' (blobs, uniform depth 9, 64^2, 16 spp),
    'cloud' (256^3 fBm cloud, adaptive, 1024^2, 32 spp), 'plume'
    (1024^3 plume, 85.7 M tets at tau 0.2, 64 bounces), 'plume_small' (the
    same plume generator and settings at 256^3), or 'blobs_adaptive' (small
    adaptive test scene)."""
    if name == "tiny":
        s = dict(density_fn=lambda: blobs(0, 64), n=64,
                 camera=dict(pos=[0.5, 0.5, -1.2], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=40.0,
                             width=64, height=64),
                 medium=dict(albedo=0.9, g=0.3), light=dict(LIGHT_DEFAULT),
                 build=dict(want_mode=1, uniform_depth=9, max_depth=9, majorant_mode=0, variation_tau=0.0,
                            target_px=1.0, density_scale=1.0, max_tets=1 << 20),
                 render=dict(spp=16, max_bounces=8, transmittance=0, max_steps_per_path=(1 << 31) - 1))
    elif name == "cloud":
        s = dict(density_fn=lambda: cloud(1, 256), n=256,
                 camera=dict(pos=[0.5, 0.45, -0.9], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=45.0,
                             width=1024, height=1024),
                 medium=dict(albedo=0.9, g=0.3), light=dict(LIGHT_DEFAULT),
                 build=dict(want_mode=0, uniform_depth=0, max_depth=24, majorant_mode=0, variation_tau=0.2,
                            target_px=1.0, density_scale=1.0, max_tets=1 << 26),
                 render=dict(spp=32, max_bounces=32, transmittance=0, max_steps_per_path=(1 << 31) - 1))
    elif name == "plume":
        s = dict(density_fn=lambda: plume(2, 1024), n=1024,
                 camera=dict(pos=[0.5, 0.45, -0.9], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=45.0,
                             width=1024, height=1024),
                 medium=dict(albedo=0.95, g=0.6), light=dict(LIGHT_DEFAULT),
                 build=dict(want_mode=0, uniform_depth=0, max_depth=30, majorant_mode=0, variation_tau=0.2,
                            target_px=1.0, density_scale=1.0, max_tets=1 << 27),
                 render=dict(spp=32, max_bounces=64, transmittance=0, max_steps_per_path=(1 << 31) - 1))
    elif name == "plume_small":
        s = scene("plume")
        s["density_fn"] = lambda: plume(2, 256)
        s["n"] = 256
    elif name == "blobs_adaptive":
        s = dict(density_fn=lambda: blobs(3, 32), n=32,
                 camera=dict(pos=[0.4, 0.6, -1.0], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=40.0,
                             width=48, height=40),
                 medium=dict(albedo=0.8, g=-0.2), light=dict(LIGHT_DEFAULT),
                 build=dict(want_mode=0, uniform_depth=0, max_depth=15, majorant_mode=1, variation_tau=0.3,
                            target_px=2.0, density_scale=1.5, max_tets=1 << 22),
                 render=dict(spp=8, max_bounces=6, transmittance=0, max_steps_per_path=(1 << 31) - 1))
    else:
        raise KeyError(name)
    for k, v in over.items():
        if isinstance(v, dict) and isinstance(s.get(k), dict):
            s[k] = {**s[k], **v}
        else:
            s[k] = v
    return s


def camera_path(cam: dict, count: int, degrees_per_frame: float = 2.0, dolly_per_frame: float = 0.0) -> list:
    """`count` cameras of a scripted move (frame 0 = `cam`): the position
    turned about the vertical axis through look_at by `degrees_per_frame`
    each frame, and moved toward look_at by `dolly_per_frame` of its
    distance each frame; positions rounded to FP32, other fields as `cam`."""
    out = []
    c = np.array(cam["look_at"], np.float64)
    p0 = np.array(cam["pos"], np.float64) - c
    for f in range(count):
        a = math.radians(degrees_per_frame * f)
        r = (1.0 - dolly_per_frame) ** f
        x = (p0[0] * math.cos(a) + p0[2] * math.sin(a)) * r
        z = (-p0[0] * math.sin(a) + p0[2] * math.cos(a)) * r
        pos = [float(np.float32(c[0] + x)), float(np.float32(c[1] + p0[1] * r)), float(np.float32(c[2] + z))]
        out.append(dict(cam, pos=pos))
    return out


def scene_batch(count: int = 64, first_seed: int = 100) -> list:
    """A batch of small scenes for batched rendering: scene i has seed
    first_seed + i; even i are Gaussian blobs at 64^3 on a uniform depth-9
    grid (3,072 tets), odd i fBm clouds at 64^3, 128^3 or 256^3 on adaptive
    grids; the camera orbits the cube (angle 2 pi i / count); images of 64,
    128, 256 or 512 pixels square and 4, 8, 16, 32 or 64 spp, cycling."""
    out = []
    for i in range(count):
        seed = first_seed + i
        ang = 2.0 * math.pi * i / count
        size = [64, 128, 256, 512][i % 4]
        spp = [4, 8, 16, 32, 64][i % 5]
        cam = dict(pos=[0.5 + 1.4 * math.sin(ang), 0.45 + 0.1 * math.cos(3 * ang), 0.5 - 1.4 * math.cos(ang)],
                   look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=42.0, width=size, height=size)
        if i % 2 == 0:
            n = 64
            fn = (lambda sd: (lambda: blobs(sd, 64)))(seed)
            build = dict(want_mode=1, uniform_depth=9, max_depth=9, majorant_mode=0, variation_tau=0.0,
                         target_px=1.0, density_scale=1.0, max_tets=1 << 20)
        else:
            n = [64, 128, 256][(i // 2) % 3]
            fn = (lambda sd, nn: (lambda: cloud(sd, nn)))(seed, n)
            build = dict(want_mode=0, uniform_depth=0, max_depth=24, majorant_mode=0, variation_tau=0.2,
                         target_px=1.0, density_scale=1.0, max_tets=1 << 24)
        out.append(dict(density_fn=fn, n=n, camera=cam, medium=dict(albedo=0.9, g=0.3), light=dict(LIGHT_DEFAULT),
                        build=build, render=dict(spp=spp, max_bounces=16, transmittance=0,
                                                 max_steps_per_path=(1 << 31) - 1), seed=seed))
    return out
